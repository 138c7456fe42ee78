"""The cost model's GPU kernels (forward, backward, Adam) against the CPU
oracle in fp64, and the model's C ABI around them."""
import os
import tempfile

import numpy as np
import pytest
import torch

import datagen
import paper_2508_07071_amd as fk
from fkhelpers import Plan, alloc_outs, to_dev
from oracle import mlp

pytestmark = pytest.mark.gpu
F, O = fk.FK_MODEL_FEATURES, fk.FK_MODEL_OUTPUTS


def say(*a):
    print("[case]", *a, flush=True)


def dims(h):
    return [F, h, h, h, O]


def close(g, r, rel=2e-4, what=""):
    g = np.asarray(g, np.float64)
    r = np.asarray(r, np.float64)
    scale = max(np.abs(r).max(), 1e-30)
    err = np.abs(g - r)
    tol = rel * np.maximum(np.abs(r), 0.01 * scale)
    assert np.all(err <= tol), f"{what}: worst {err.max():.3g} at {np.argmax(err)} (scale {scale:.3g})"


@pytest.mark.parametrize("hidden,n", [(16, 37), (128, 300)])
def test_loss_and_gradients_match_oracle(hidden, n):
    say("loss/grad", hidden, n)
    g = np.random.default_rng(hidden + n)
    X = g.normal(size=(n, F)).astype(np.float32)
    T = g.normal(size=(n, O)).astype(np.float32)
    m = fk.fk_model_create(hidden, 11)
    try:
        p = fk.fk_model_get_params(m)
        assert p.size == mlp.n_params(dims(hidden))
        loss, grad = fk.fk_model_loss_grad(m, X, T)
    finally:
        fk.fk_model_destroy(m)
    rl, rg = mlp.loss_grad(p.astype(np.float64), dims(hidden), X.astype(np.float64), T.astype(np.float64))
    assert loss == pytest.approx(rl, rel=1e-5)
    close(grad, rg, what="gradient")


def test_forward_with_normalisation_matches_oracle():
    say("forward + normalisation")
    g = np.random.default_rng(5)
    X = (g.normal(size=(70, F)) * 3 + 2).astype(np.float32)
    mean = g.normal(size=F).astype(np.float32)
    std = g.uniform(0.5, 2.0, size=F).astype(np.float32)
    m = fk.fk_model_create(64, 3)
    try:
        fk.fk_model_set_normalization(m, mean, std)
        p = fk.fk_model_get_params(m)
        y = fk.fk_model_predict_batch(m, X)
        mm, ss = fk.fk_model_get_normalization(m)
    finally:
        fk.fk_model_destroy(m)
    np.testing.assert_array_equal(mm, mean)
    Xs = (X - mean) / std  # the library standardises in fp32 on the host
    r = mlp.forward(p.astype(np.float64), dims(64), Xs.astype(np.float64))[-1]
    close(y, r, rel=1e-4, what="forward")


def test_one_full_batch_adam_step_matches_oracle():
    say("one Adam step")
    g = np.random.default_rng(8)
    n = 64
    X = g.normal(size=(n, F)).astype(np.float32)
    T = g.normal(size=(n, O)).astype(np.float32)
    lr = 1e-3
    m = fk.fk_model_create(32, 4)
    try:
        p0 = fk.fk_model_get_params(m).astype(np.float64)
        fk.fk_model_train(m, X, T, epochs=1, batch=n, lr=lr, seed=0)
        p1 = fk.fk_model_get_params(m).astype(np.float64)
        mean, std = fk.fk_model_get_normalization(m)
    finally:
        fk.fk_model_destroy(m)
    Xs = ((X - mean) / std).astype(np.float64)
    _, grad = mlp.loss_grad(p0, dims(32), Xs, T.astype(np.float64))
    pr, _, _ = mlp.adam_step(p0, grad, np.zeros_like(p0), np.zeros_like(p0), 1, lr)
    # step 1 moves each parameter by ~lr * sign(g): compare where g is not
    # within rounding of zero
    big = np.abs(grad) > 1e-4 * np.abs(grad).max()
    np.testing.assert_allclose((p1 - p0)[big], (pr - p0)[big], rtol=1e-3, atol=1e-7)
    assert np.all(np.abs(p1 - p0) <= lr * 1.001 + 1e-7)


def test_training_fits_a_smooth_target():
    say("training reduces loss")
    g = np.random.default_rng(9)
    X = g.normal(size=(2048, F)).astype(np.float32)
    W = g.normal(size=(F, O)) / np.sqrt(F)
    T = np.tanh(X @ W).astype(np.float32)
    m = fk.fk_model_create(64, 1)
    try:
        curve = fk.fk_model_train(m, X, T, epochs=60, batch=256, lr=3e-3, seed=2)
    finally:
        fk.fk_model_destroy(m)
    assert curve[-1] < 0.1 * curve[0], curve


def test_save_load_roundtrip_is_bitwise():
    say("save/load")
    g = np.random.default_rng(10)
    X = g.normal(size=(20, F)).astype(np.float32)
    T = g.normal(size=(20, O)).astype(np.float32)
    m = fk.fk_model_create(48, 6)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.bin")
        try:
            fk.fk_model_train(m, X, T, epochs=3, batch=8, lr=1e-3, seed=1)
            y0 = fk.fk_model_predict_batch(m, X)
            fk.fk_model_save(m, path)
        finally:
            fk.fk_model_destroy(m)
        m2 = fk.fk_model_load(path)
        try:
            y1 = fk.fk_model_predict_batch(m2, X)
        finally:
            fk.fk_model_destroy(m2)
    np.testing.assert_array_equal(y0, y1)


def test_features_and_model_choice_for_a_plan():
    say("features / plan_use_model")
    cfg = datagen.config2(8, seed=1)
    dframes = to_dev(cfg["frames"])
    m = fk.fk_model_create(32, 2)
    try:
        with Plan(cfg["chain"], 8) as p:
            outs = alloc_outs(cfg["chain"], cfg["items"])
            arr = fk.make_items(cfg["chain"], dframes, cfg["items"], outs)
            f = fk.fk_model_features(p.h, arr, 8)
            assert f[0] == 1.0 and f[1] == 1.0 and f[5] == 1.0  # crop_resize, u8, 3 channels
            assert f[8] == 1.0 and f[7] == 0.0  # planar fp32
            assert f[9] == pytest.approx(3.0)  # log2(batch)
            assert f[10] == pytest.approx(np.log2(8 * 64 * 128))
            assert f[26] == 1.0  # compile-time chain
            fk.fk_plan_use_model(p.h, m, arr, 8)
            c = fk.fk_plan_get_config(p.h)
            assert (c.block_threads, c.coarsen) in [(s.block_threads, s.coarsen) for s in fk.fk_autotune_space()]
            p.run(dframes, cfg["items"], outs=outs)
            torch.cuda.synchronize()
            assert not torch.isnan(outs[0]).any()
    finally:
        fk.fk_model_destroy(m)


def test_raw_kernels_forward_mse_backward_step_match_oracle():
    """The network's kernels called one by one on device arrays: forward
    (every hidden layer), MSE and its gradient, backward, and two Adam
    steps, each against the fp64 oracle given the same inputs."""
    say("raw forward/mse/backward/step")
    hidden, n, lr = 48, 53, 2e-3
    g = np.random.default_rng(12)
    X = g.normal(size=(n, F)).astype(np.float32)
    T = g.normal(size=(n, O)).astype(np.float32)
    dev = torch.device("cuda:0")
    dX, dT = torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev)
    m = fk.fk_model_create(hidden, 13)
    try:
        p0 = fk.fk_model_get_params(m).astype(np.float64)
        ws = torch.full((fk.fk_mlp_workspace_floats(m, n),), float("nan"), device=dev)
        assert ws.numel() == n * (3 * hidden + 2 * max(hidden, O))
        dY = torch.empty(n, O, device=dev)
        fk.fk_mlp_forward(m, dX, ws, dY)
        dDY = torch.empty(n, O, device=dev)
        dL = torch.empty(1, device=dev)
        fk.fk_mlp_mse(dY, dT, dDY, dL)
        dG = torch.full((p0.size,), float("nan"), device=dev)
        fk.fk_mlp_backward(m, dX, ws, dDY, dG)
        torch.cuda.synchronize()
        acts = mlp.forward(p0, dims(hidden), X.astype(np.float64))
        hid = ws[:3 * n * hidden].view(3, n, hidden).cpu().numpy()
        for l in range(3):
            close(hid[l], acts[l + 1], rel=1e-4, what=f"hidden layer {l}")
        close(dY.cpu().numpy(), acts[-1], rel=1e-4, what="forward")
        rl, rg = mlp.loss_grad(p0, dims(hidden), X.astype(np.float64), T.astype(np.float64))
        assert float(dL.item()) == pytest.approx(rl, rel=1e-5)
        y64 = acts[-1]
        close(dDY.cpu().numpy(), 2.0 * (y64 - T) / y64.size, rel=2e-4, what="dY")
        grad = dG.cpu().numpy().astype(np.float64)
        close(grad, rg, what="gradient")
        # two Adam steps along the kernels' own gradient
        pr, mr, vr = p0, np.zeros_like(p0), np.zeros_like(p0)
        for t in (1, 2):
            fk.fk_mlp_step(m, dG, lr)
            torch.cuda.synchronize()
            pr, mr, vr = mlp.adam_step(pr, grad, mr, vr, t, lr)
            pg = fk.fk_model_get_params(m).astype(np.float64)
            np.testing.assert_allclose(pg, pr, rtol=0, atol=2e-7 + 1e-4 * lr, err_msg=f"Adam step {t}")
    finally:
        fk.fk_model_destroy(m)


def test_device_training_equals_host_training():
    """fk_model_train (host arrays) and fk_model_train_device (device
    arrays on the caller's stream) run the same steps: same normalisation,
    same loss curve and the same parameters, bit for bit."""
    say("train_device == train")
    g = np.random.default_rng(14)
    n = 700
    X = (g.normal(size=(n, F)) * 2 + 1).astype(np.float32)
    T = np.tanh(X[:, :O]).astype(np.float32)
    dev = torch.device("cuda:0")
    a = fk.fk_model_create(32, 5)
    b = fk.fk_model_create(32, 5)
    try:
        curve_a = fk.fk_model_train(a, X, T, epochs=4, batch=64, lr=1e-3, seed=9)
        dX, dT = torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev)
        dC = torch.zeros(4, device=dev)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            fk.fk_model_train_device(b, dX, dT, epochs=4, batch=64, lr=1e-3, seed=9, d_loss_curve=dC, stream=s)
        # reading the parameters waits for the queued training
        pb = fk.fk_model_get_params(b)
        s.synchronize()
        curve_b = dC.cpu().numpy()
        pa = fk.fk_model_get_params(a)
        na, nb = fk.fk_model_get_normalization(a), fk.fk_model_get_normalization(b)
    finally:
        fk.fk_model_destroy(a)
        fk.fk_model_destroy(b)
    np.testing.assert_array_equal(na[0], nb[0])
    np.testing.assert_array_equal(na[1], nb[1])
    np.testing.assert_array_equal(curve_a, curve_b)
    np.testing.assert_array_equal(pa, pb)
    # the normalisation is the features' mean and (population) std
    np.testing.assert_allclose(na[0], X.astype(np.float64).mean(axis=0), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(na[1], X.astype(np.float64).std(axis=0), rtol=1e-5)
