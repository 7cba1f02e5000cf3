"""Surrogate network kernels (BF16 MFMA GEMMs, SiLU, MSE, Adam) against the
FP64 numpy reference, and the surrogate pipeline (batched SEM data,
training, ensemble indicator, SEM fallback) at a reduced size.

Bars: BF16 forward / parameter gradients within 2e-2 / 3e-2 relative L2 of
FP64 (BF16 operands, FP32 accumulation); Adam within 1e-5 (FP32 arithmetic).
The trained network's own accuracy is stated, not pinned."""
import time

import numpy as np
import pytest

import workloads as W
from oracle import mlp_ref as M
from tests.gpu_common import rel_l2

pytestmark = pytest.mark.gpu


def _net(widths, batch, seed=0):
    from paper_2606_12850_amd.surrogate import MLP
    return MLP(widths, batch, seed)


@pytest.mark.parametrize("widths,batch", [([64, 128, 96, 200], 37), ([5, 70, 3], 1), ([64, 512, 512, 512, 24576], 128),
                                          ([64, 512, 20000], 520)])
def test_forward_backward_vs_fp64(widths, batch):
    import torch
    rng = np.random.default_rng(1)
    net = _net(widths, batch)
    theta = (M.he_uniform(widths, 3) + 0.01 * rng.standard_normal(M.num_params(widths))).astype(np.float32)
    net.set_params(theta)
    x = rng.standard_normal((batch, widths[0])).astype(np.float32)
    t = rng.standard_normal((batch, widths[-1])).astype(np.float32)
    xd = torch.from_numpy(x).cuda(); td = torch.from_numpy(t).cuda()
    y = net.forward(xd)
    torch.cuda.synchronize()
    yr, cache = M.forward(theta.astype(np.float64), widths, x.astype(np.float64))
    ferr = rel_l2(y.cpu().numpy(), yr)
    import paper_2606_12850_amd as P
    dy = torch.empty_like(y)
    loss = P.semx_mlp_mse(net.net, y, td, y.numel(), dy)
    lr_, dyr = M.mse(yr, t)
    P.semx_mlp_backward(net.net, dy, batch)
    g = np.zeros(net.nparam, np.float32)
    P.semx_mlp_get_grads(net.net, g)
    gr = M.backward(theta.astype(np.float64), widths, cache, dyr)
    gerr = rel_l2(g, gr)
    print(f"widths {widths} batch {batch}: forward rel L2 {ferr:.2e}, loss {loss:.6e} vs {lr_:.6e}, grad rel L2 {gerr:.2e}")
    assert ferr <= 2e-2
    assert abs(loss - lr_) <= 3e-2 * lr_
    assert gerr <= 3e-2
    net.close()


def test_adam_matches_reference():
    import torch
    import paper_2606_12850_amd as P
    widths = [8, 16, 4]
    net = _net(widths, 8)
    theta = M.he_uniform(widths, 2).astype(np.float32)
    net.set_params(theta)
    x = torch.randn(8, 8, device="cuda"); t = torch.randn(8, 4, device="cuda")
    th = theta.astype(np.float64); m = np.zeros_like(th); v = np.zeros_like(th)
    for step in range(1, 4):
        y = net.forward(x); dy = torch.empty_like(y)
        P.semx_mlp_mse(net.net, y, t, y.numel(), dy, want_loss=False)
        P.semx_mlp_backward(net.net, dy, 8)
        g = np.zeros(net.nparam, np.float32)
        P.semx_mlp_get_grads(net.net, g)
        P.semx_mlp_adam(net.net, 1e-2, 0.9, 0.999, 1e-8, step)
        th, m, v = M.adam(th, g.astype(np.float64), m, v, step, 1e-2)
        np.testing.assert_allclose(net.params(), th, rtol=1e-5, atol=1e-6)
    net.close()


def test_training_follows_fp64_trajectory():
    """Surrogate.fit on the GPU against the same training run in FP64 numpy
    (same initial weights, normalisation, minibatch order, cosine learning
    rate and Adam): the losses along the way agree to BF16 accuracy."""
    import torch
    from paper_2606_12850_amd.surrogate import Surrogate, cosine_lr
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, (512, 16))
    A = rng.standard_normal((16, 40))
    Y = np.tanh(X @ A) + 0.1 * (X[:, :1] ** 2)
    widths = [16, 64, 64, 40]
    s = Surrogate(16, 40, hidden=(64, 64), members=1, max_batch=512)
    theta = s.members[0].params().astype(np.float64)
    Xn = (X - X.mean(0)) / (X.std(0) + 1e-12)
    Yn = (Y - Y.mean(0)) / (Y.std(0) + 1e-30)
    Xd = torch.from_numpy(Xn.astype(np.float32)).cuda()
    Yd = torch.from_numpy(Yn.astype(np.float32)).cuda()
    losses = {}
    for ep in (5, 20, 60):
        s.fit(X, Y, epochs=ep, batch=64)
        losses[ep] = s.members[0].loss(Xd, Yd)
        s.members[0].set_params(theta.astype(np.float32))
        s.members[0].step = 0
    ref = {}
    for ep in (5, 20, 60):
        th = theta.copy(); m = np.zeros_like(th); v = np.zeros_like(th)
        r = np.random.default_rng(0); total = ep * 8; step = 0
        for _ in range(ep):
            perm = r.permutation(512)
            for b in range(8):
                idx = perm[b * 64:(b + 1) * 64]
                y, cache = M.forward(th, widths, Xn[idx])
                _, dy = M.mse(y, Yn[idx])
                g = M.backward(th, widths, cache, dy)
                step += 1
                th, m, v = M.adam(th, g, m, v, step, cosine_lr(step - 1, total, 1e-3, 1e-5))
        ref[ep] = M.mse(M.forward(th, widths, Xn)[0], Yn)[0]
    l0 = M.mse(M.forward(theta, widths, Xn)[0], Yn)[0]
    print(f"loss at start {l0:.4e}; GPU {losses}; FP64 {ref}")
    for ep in ref:
        assert abs(losses[ep] - ref[ep]) <= 0.05 * ref[ep]
    assert ref[60] < 0.2 * l0
    s.close()


def test_resample_is_linear_interpolation():
    from paper_2606_12850_amd.surrogate import resample
    nt, nout = 800, 512
    t = np.arange(1, nt + 1) * 1.0
    s = 3.0 * t + 2.0          # linear in time: interpolation is exact
    r = resample(s[None], nout)[0]
    tj = (np.arange(nout) + 1.0) * nt / nout
    np.testing.assert_allclose(r, 3.0 * tj + 2.0, rtol=1e-12)


def test_surrogate_pipeline_with_fallback():
    """Reduced-size surrogate: 8^3 mesh, 3 Hz Ricker, 200 steps -> 100
    samples, 16 receivers; train on 4096 models, calibrate on 128, test on
    256.  States the surrogate error and the fallback outcome; checks that
    the SEM fallback keeps every flagged model at the SEM answer, that the
    trained network beats the mean seismogram, that most models are accepted
    at the 5 % tolerance (measured: 1024 training models leave the mean error
    at 6.4 % and flag 98 %; 4096 bring it to 2.4 % and flag 9 %), and that
    surrogate + fallback is cheaper than SEM for all test models (training
    excluded) at a final mean error within the tolerance."""
    import torch
    from paper_2606_12850_amd.surrogate import BatchedSEM, Surrogate, rel_err, resample
    mesh = W.box_mesh(8, 5, 4000.0)
    basis = W.fourier_modes(mesh)
    nt, nout, f0 = 200, 100, 3.0
    dt = 0.01  # below Courant 0.4: min GLL spacing 0.1727 h = 86 m, vp <= 3300 m/s
    se, sx = W.center_vertex_source(mesh)
    re, rx = W.top_receivers_grid(mesh, 4)
    stf = W.ricker(f0, 1.2 / f0, dt, nt + 1)[None, :]
    sem = BatchedSEM(mesh, se, sx, [[0.0, 0.0, 1.0]], stf, re, rx, dt, nt, batch=64)
    model_fn = lambda a: W.perturbed_models(mesh, basis, a)
    A_tr = W.perturbation_coefficients(basis, range(0, 4096))
    A_va = W.perturbation_coefficients(basis, range(5000, 5128))
    A_te = W.perturbation_coefficients(basis, range(10000, 10256))
    Y_tr4 = resample(sem.run_models(model_fn, A_tr), nout)
    Y_tr = Y_tr4.reshape(len(A_tr), -1)
    Y_va = resample(sem.run_models(model_fn, A_va), nout).reshape(len(A_va), -1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Y_te = resample(sem.run_models(model_fn, A_te), nout).reshape(len(A_te), -1)
    t_sem = time.perf_counter() - t0
    s = Surrogate(64, Y_tr.shape[1], hidden=(256, 256, 256), members=4, max_batch=512)
    s.fit(A_tr, Y_tr4, epochs=120, batch=64)
    cal = s.calibrate(A_va, Y_va, tol=0.05)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred, ind = s.predict(A_te)
    flag = ind > s.threshold
    fallback = pred.copy()
    if flag.any():
        fallback[flag] = resample(sem.run_models(model_fn, A_te[flag]), nout).reshape(int(flag.sum()), -1)
    torch.cuda.synchronize()
    t_sur = time.perf_counter() - t0
    e_sur = rel_err(pred, Y_te)
    e_fin = rel_err(fallback, Y_te)
    print(f"surrogate test error mean {e_sur.mean():.3e} max {e_sur.max():.3e}; calibration {cal}; "
          f"flagged {flag.mean():.2%}; final error mean {e_fin.mean():.3e} max {e_fin.max():.3e}; "
          f"time surrogate+fallback {t_sur:.3f} s vs SEM {t_sem:.3f} s")
    e_mean = rel_err(np.broadcast_to(Y_tr.mean(0), Y_te.shape), Y_te)
    print(f"mean-seismogram error {e_mean.mean():.3e}")
    assert np.all(np.isfinite(pred))
    assert e_sur.mean() < 0.5 * e_mean.mean()
    assert np.all(e_fin[flag] <= 1e-6)          # flagged models carry the SEM answer
    assert e_fin.mean() <= e_sur.mean() + 1e-12
    assert flag.mean() < 0.5                    # most models accepted
    assert e_fin.mean() <= 0.05
    assert t_sur < t_sem                        # the gain, unconditionally
    s.close(); sem.close()


def test_affine_and_ensemble_kernels_match_numpy():
    """The surrogate's normalisation (column-wise affine map) and ensemble
    statistics (mean in physical units, unbiased spread, the indicator
    ||scale * std|| / ||mean||) against FP64 numpy on the same data."""
    import torch
    import paper_2606_12850_amd as P
    rng = np.random.default_rng(21)
    M, S, C = 4, 37, 1000
    net = P.semx_mlp_create([8, 8], 16, torch.cuda.current_stream())
    try:
        x = rng.standard_normal((S, C)).astype(np.float32)
        a = rng.uniform(0.5, 2.0, C).astype(np.float32)
        b = rng.standard_normal(C).astype(np.float32)
        dev = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()
        xd, y = dev(x), torch.empty((S, C), device="cuda")
        P.semx_mlp_affine(net, xd, S, C, dev(a), dev(b), y)
        P.semx_mlp_affine(net, xd, S, C, dev(a), dev(b), xd)          # in place
        ref = a[None].astype(np.float64) * x + b[None]
        torch.cuda.synchronize()
        assert np.abs(y.cpu().numpy() - ref).max() <= 1e-5 * np.abs(ref).max()
        assert np.array_equal(y.cpu().numpy(), xd.cpu().numpy())
        p = rng.standard_normal((M, S, C)).astype(np.float32)
        mean, ind = torch.empty((S, C), device="cuda"), torch.empty(S, device="cuda")
        P.semx_mlp_ensemble(net, dev(p), M, S, C, dev(a), dev(b), mean, ind)
        torch.cuda.synchronize()
        p64 = p.astype(np.float64)
        mref = a * p64.mean(0) + b
        sref = a * p64.std(0, ddof=1)
        iref = np.linalg.norm(sref, axis=1) / np.linalg.norm(mref, axis=1)
        assert np.abs(mean.cpu().numpy() - mref).max() <= 1e-5 * np.abs(mref).max()
        np.testing.assert_allclose(ind.cpu().numpy(), iref, rtol=1e-5)
        # one member: zero spread
        P.semx_mlp_ensemble(net, dev(p[:1]), 1, S, C, dev(a), dev(b), mean, ind)
        torch.cuda.synchronize()
        assert np.all(ind.cpu().numpy() == 0.0)
        with pytest.raises(P.SemxError):
            P.semx_mlp_ensemble(net, dev(p), 0, S, C, dev(a), dev(b), mean, ind)
    finally:
        P.semx_mlp_destroy(net)
