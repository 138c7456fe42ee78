"""Parity with the oracle at the shapes of the paper's parameter sweeps:
1-D fp32 arrays with 100 Mul+Add pairs through the loop op (data size),
batches of 60x120 single-channel images through Read -> Cast -> Mul -> Sub
-> Div -> Write for eight input/output types, two of them computing in
double (data type) and up to 1191
images (plain-read horizontal fusion)."""
import numpy as np
import pytest

import datagen
import oracle
import paper_2508_07071_amd as fk
from fkhelpers import Plan, assert_bitexact, assert_close, host, to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def both_modes(cfg, what, sample=None, static=None, rel=1e-5):
    items = cfg["items"]
    idx = list(range(len(items))) if sample is None else sample
    refs = oracle.run_chain(cfg["chain"], cfg["frames"], [items[i] for i in idx])
    dframes = to_dev(cfg["frames"])
    for strict in (True, False):
        with Plan(cfg["chain"], len(items), strict=strict) as p:
            if static is not None:
                assert fk.fk_plan_get_tier(p.h) == int(static)
            outs = host(p.run(dframes, items))
        for i, r in zip(idx, refs):
            if strict:
                assert_bitexact(outs[i], r["out"], f"{what} strict item {i}")
            else:
                assert_close(outs[i], r, rel=rel, what=f"{what} item {i}")


@pytest.mark.parametrize("n", [100, 4096, 282370])
def test_data_size_fp32_loop_chain(n):
    say("data size", n)
    both_modes(datagen.data_size_case(n, seed=n % 97), f"n={n}", static=True)


@pytest.mark.parametrize("din,dout", [("u8", "f32"), ("u8", "f16"), ("f16", "f32"), ("f16", "f16"),
                                      ("f32", "f32"), ("f32", "f16"), ("f32", "f64"), ("f64", "f64")])
def test_cast_chain_data_types_batch50(din, dout):
    say("data types", din, "->", dout)
    both_modes(datagen.cast_chain_batch(50, din, dout, seed=3), f"{din}->{dout}",
               rel=1e-13 if dout == "f64" else 1e-5)


def test_plain_batch_1191_images_sampled():
    say("plain-read batch 1191")
    cfg = datagen.cast_chain_batch(1191, seed=4)
    both_modes(cfg, "B=1191", sample=[0, 1, 500, 1189, 1190])


@pytest.mark.parametrize("batch", [625, 1191])
def test_plain_batch_one_output_tensor_chunked(batch):
    """Items written into one output tensor at a constant stride: a batch
    above one launch's kernel-argument capacity (312 items) goes out as
    consecutive kernel-argument launches.  The items on both sides of every
    launch boundary, and a last launch of one item (625 = 2 x 312 + 1),
    match the oracle."""
    import torch
    from fkhelpers import device
    say("plain-read batch, one output tensor", batch)
    cfg = datagen.cast_chain_batch(batch, seed=5)
    items = cfg["items"]
    idx = sorted({0, batch - 1} | {b for k in range(312, batch, 312) for b in (k - 1, k)})
    refs = oracle.run_chain(cfg["chain"], cfg["frames"], [items[i] for i in idx])
    dframes = to_dev(cfg["frames"])
    shape = fk.out_shape(cfg["chain"], items[0])
    for strict in (True, False):
        big = torch.full((batch,) + tuple(shape), float("nan"), dtype=torch.float32, device=device())
        with Plan(cfg["chain"], batch, strict=strict) as p:
            outs = host(p.run(dframes, items, outs=[big[b] for b in range(batch)]))
        for i, r in zip(idx, refs):
            if strict:
                assert_bitexact(outs[i], r["out"], f"B={batch} strict item {i}")
            else:
                assert_close(outs[i], r, what=f"B={batch} item {i}")
        assert not np.isnan(np.stack(outs)).any(), "an item was not written"


@pytest.mark.parametrize("per_op", [1, 7, 100, 500])
def test_instructions_per_op_fused_and_one_kernel_per_op(per_op):
    """500 multiplications as ops of `per_op` instructions (looped Mul ops):
    the fused run matches the oracle bit for bit, and so does the unfused
    baseline in both of its loop forms (one kernel per looped op, or one
    kernel per multiplication)."""
    say("instructions per op", per_op)
    cfg = datagen.instructions_per_op_case(per_op, n_elems=3 * 4096 + 4096, seed=per_op)
    ref = oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"])[0]["out"]
    dframes = to_dev(cfg["frames"])
    for one_kernel in (True, False):
        if not one_kernel and per_op > 100:
            continue  # 500 launches: covered by the smaller cases
        with Plan(cfg["chain"], 1, strict=True, unfused_loop_kernel=one_kernel) as p:
            fused = host(p.run(dframes, cfg["items"]))[0]
            unfused = host(p.run_unfused(dframes, cfg["items"]))[0]
        assert_bitexact(fused, ref, f"fused per_op={per_op}")
        assert_bitexact(unfused, ref, f"unfused per_op={per_op} one_kernel={one_kernel}")
