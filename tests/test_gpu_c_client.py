"""The C ABI from plain C on the GPU: tests/c_client/fk_client (C11, links
libfkmi.so and the HIP runtime, no Python or torch) runs the normalisation
chain over uneven crops of one frame in one launch; its outputs match the
oracle bit for bit in the strict mode and within the tolerance in the
contracted mode.  The client prints its fp32 constants as hexadecimal
floats, from which the oracle's chain is rebuilt."""
import os
import subprocess
import sys

import numpy as np
import pytest

import datagen
import oracle
from fkhelpers import assert_bitexact, assert_close

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "c_client"))
import build_client  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def client():
    if not os.path.exists(build_client.BIN):
        build_client.build()
    return build_client.BIN


def constants(stdout):
    got = {}
    for line in stdout.splitlines():
        k, *v = line.split()
        if k in ("scale", "mean", "std"):
            got[k] = [float.fromhex(x) for x in v]
    return got


@pytest.mark.parametrize("strict", [1, 0])
def test_c_client_matches_oracle(tmp_path, strict):
    say("C client, strict", strict)
    g = datagen.rng(31)
    H, W, OW, OH = 270, 480, 64, 128
    frame = datagen.frame(g, H, W, 3)
    crops = datagen.random_crops(g, 9, W, H, lo=2, hi=260, out=(OW, OH))
    crops.append({"frame": 0, "x": W - 1, "y": H - 1, "w": 1, "h": 1, "out_w": OW, "out_h": OH})
    (tmp_path / "frame.u8").write_bytes(frame.tobytes())
    (tmp_path / "crops.txt").write_text("".join(f"{c['x']} {c['y']} {c['w']} {c['h']}\n" for c in crops))
    out = tmp_path / "out.f32"
    r = subprocess.run([client(), str(tmp_path / "frame.u8"), str(W), str(H), str(OW), str(OH), str(strict),
                        str(tmp_path / "crops.txt"), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    k = constants(r.stdout)
    chain = {"read": {"kind": "crop_resize", "dtype": "u8", "channels": 3, "out_w": OW, "out_h": OH},
             "ops": [{"kind": "swap", "k": []}, {"kind": "cvt", "k": []}, {"kind": "mul", "k": k["scale"]},
                     {"kind": "sub", "k": k["mean"]}, {"kind": "div", "k": k["std"]}],
             "write": {"dtype": "f32", "layout": "planar"}}
    refs = oracle.run_chain(chain, [frame], crops)
    got = np.fromfile(out, dtype=np.float32).reshape(len(crops), 3, OH, OW)
    for b, ref in enumerate(refs):
        if strict:
            assert_bitexact(got[b], ref["out"], f"C client item {b}")
        else:
            assert_close(got[b], ref, what=f"C client item {b}")
