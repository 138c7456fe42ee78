"""Host-side logic of the cost-model driver (no GPU): dataset sizing,
targets, the quality measure and shard loading."""
import os
import tempfile

import numpy as np

import datagen
from paper_2508_07071_amd import costmodel as cm


def test_fit_spec_caps_input_and_output_bytes():
    g = datagen.rng(0)
    for _ in range(300):
        spec = cm.fit_spec(datagen.random_chain_spec(g))
        ch = spec["chain"]
        C = ch["read"]["channels"]
        fh, fw = spec["frame_hw"]
        B = len(spec["items"])
        assert B == spec["batch"] >= 1
        assert B * fw * fh * C * cm._esize(ch["read"]["dtype"]) <= cm.ARENA_IN
        out = max(it["out_w"] * it["out_h"] for it in spec["items"]) * C * cm._esize(ch["write"]["dtype"])
        assert B * out <= cm.ARENA_OUT
        for it in spec["items"]:
            assert 0 <= it["x"] and it["x"] + it["w"] <= fw and 0 <= it["y"] and it["y"] + it["h"] <= fh


def test_targets_and_quality():
    t = np.array([[2.0, 1.0, 4.0], [3.0, 6.0, 3.0]])
    y = cm.targets_from_times(t)
    np.testing.assert_allclose(y, np.log([[2, 1, 4], [1, 2, 1]]), rtol=1e-6)
    np.testing.assert_allclose(cm.quality(t, np.array([1, 0])), [1.0, 1.0])
    np.testing.assert_allclose(cm.quality(t, np.array([2, 1])), [0.25, 0.5])
    s = cm.summarize([1.0, 0.5])
    assert abs(s["geomean"] - np.sqrt(0.5)) < 1e-12 and s["frac_within_10pct"] == 0.5


def test_shards_concatenate_in_start_order():
    with tempfile.TemporaryDirectory() as d:
        paths = []
        for start, val in ((5, 2.0), (0, 1.0)):
            p = os.path.join(d, f"s{start}.npz")
            np.savez(p, features=np.full((5, 32), val, np.float32), times_ms=np.full((5, 20), val, np.float32),
                     default_idx=np.zeros(5, np.int32), meta=np.array(["{}"] * 5), start=np.array(start))
            paths.append(p)
        data = cm.load_shards(paths)
    assert data["features"].shape == (10, 32)
    assert data["features"][0, 0] == 1.0 and data["features"][9, 0] == 2.0


def test_random_chain_specs_are_deterministic():
    a = [datagen.random_chain_spec(datagen.rng(3)) for _ in range(1)]
    b = [datagen.random_chain_spec(datagen.rng(3)) for _ in range(1)]
    assert a == b
