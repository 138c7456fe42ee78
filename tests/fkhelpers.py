"""Helpers shared by the GPU tests: run a chain through the C ABI on device
tensors and compare with the oracle."""
import numpy as np
import torch

import paper_2508_07071_amd as fk

NP_OUT = {"f32": np.float32, "f16": np.float16}


def device():
    return torch.device("cuda:0")


def to_dev(frames):
    return [torch.from_numpy(np.ascontiguousarray(f)).to(device()) for f in frames]


def alloc_outs(chain, items):
    dt = fk.TORCH_DTYPE[chain["write"]["dtype"]]
    # poison outputs with NaN so unwritten elements are caught
    return [torch.full(fk.out_shape(chain, it), float("nan"), dtype=dt, device=device()) for it in items]


class Plan:
    """A plan handle with the chain descriptor it was built from."""

    def __init__(self, chain, max_batch, **opts):
        self.chain = chain
        self.desc = fk.chain_desc(chain)
        self.h = fk.fk_plan_create(self.desc, max_batch, fk.plan_opts(**opts))

    def run(self, dframes, items, outs=None, stream=None):
        outs = outs if outs is not None else alloc_outs(self.chain, items)
        arr = fk.make_items(self.chain, dframes, items, outs)
        fk.fk_run(self.h, arr, len(items), fk.stream_handle(stream))
        return outs

    def run_unfused(self, dframes, items, outs=None):
        outs = outs if outs is not None else alloc_outs(self.chain, items)
        arr = fk.make_items(self.chain, dframes, items, outs)
        nbytes = fk.fk_unfused_scratch_bytes(self.h, arr, len(items))
        scratch = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device())
        fk.fk_run_unfused(self.h, arr, len(items), scratch.data_ptr(), nbytes, fk.stream_handle())
        return outs

    def set_config(self, t, k):
        fk.fk_plan_set_config(self.h, fk.fk_launch_config(t, k))

    def close(self):
        if self.h:
            fk.fk_plan_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def host(outs):
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def assert_bitexact(g, r, what=""):
    g = np.asarray(g)
    r = np.asarray(r)
    assert g.shape == r.shape, (what, g.shape, r.shape)
    assert g.dtype == r.dtype, (what, g.dtype, r.dtype)
    bits = {np.dtype(np.float16): np.uint16, np.dtype(np.float32): np.uint32, np.dtype(np.float64): np.uint64}
    gv, rv = g.view(bits[g.dtype]), r.view(bits[r.dtype])
    bad = np.flatnonzero(gv.ravel() != rv.ravel())
    # NaN == NaN regardless of payload
    if bad.size:
        both_nan = np.isnan(g.ravel()[bad]) & np.isnan(r.ravel()[bad])
        bad = bad[~both_nan]
    assert bad.size == 0, f"{what}: {bad.size} elements differ, first at {bad[:5]}: " \
                          f"{g.ravel()[bad[:5]]} vs {r.ravel()[bad[:5]]}"


def assert_close(g, ref, s_floor=None, rel=1e-5, what=""):
    """|g - r| <= rel * max(|r|, s) per element; s = the oracle's largest
    intermediate magnitude for that element, or the constant s_floor; NaN
    must match NaN.  fp16 outputs get the fp16 rounding on top."""
    g = np.asarray(g).astype(np.float64)
    r = np.asarray(ref["out"]).astype(np.float64)
    s = np.full_like(r, s_floor) if s_floor is not None else ref["smax"].astype(np.float64)
    tol = rel * np.maximum(np.abs(r), s)
    if ref["out"].dtype == np.float16:
        tol = tol + np.abs(r) * 2.0 ** -10 + 2.0 ** -24
    nan = np.isnan(r)
    assert np.array_equal(np.isnan(g), nan), f"{what}: NaN pattern differs"
    with np.errstate(invalid="ignore"):
        err = np.abs(g - r)
    err[nan] = 0
    if ref["out"].dtype == np.float16:
        # at the fp16 overflow boundary one side may round to +-inf, the other
        # to +-65504: both mean "out of fp16 range" with the same sign
        big = (np.abs(r) >= 65504) & (np.abs(g) >= 65504) & (np.sign(r) == np.sign(g))
        err[big] = 0
    bad = err > tol
    assert not bad.any(), f"{what}: {bad.sum()} elements beyond tolerance, worst {err.max():.3g} " \
                          f"(tol there {tol.ravel()[np.argmax(err)]:.3g})"
