"""GPU discrete adjoint (sensitivity kernels K_lambda, K_mu, K_rho) against
the FP64 oracle's adjoint and against FP64 central finite differences of the
misfit.  Bar: relative difference <= 1e-3 (FP32 adjoint vs FP64 references)."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import rel_l2

pytestmark = pytest.mark.gpu


def _problem(n=4, ne=(3, 3, 2), nt=80, jitter=0.12, seed=0, L=2000.0):
    m = W.box_mesh(ne, n, L, jitter=jitter, seed=seed)
    lam, mu, rho = W.layered_model(m, vp_layers=(3000.0, 2500.0), grf_amp=0.05, grf_seed=seed,
                                   grf_corr_elems=1.0)
    dt = 2e-3
    se = np.array([m.nspec // 2], np.int32); sx = np.array([[0.3, -0.2, 0.4]]); sd = np.array([[0.3, 0.2, 1.0]])
    stf = W.ricker(25.0, 0.04, dt, nt + 1)[None, :]
    re, rx = W.top_receivers_grid(m, 2)
    return dict(m=m, lam=lam, mu=mu, rho=rho, dt=dt, nt=nt, se=se, sx=sx, sd=sd, stf=stf, re=re, rx=rx)


def _oracle_chi(orc, Pb, lam, mu, rho, data):
    m = Pb["m"]
    gam, jac, _ = orc.geometry(m.n, m.elem_vert, m.vert)
    s = orc.forward(m.n, m.ibool, gam, jac, lam, mu, rho, m.nglob, Pb["dt"], Pb["nt"], Pb["se"], Pb["sx"],
                    Pb["sd"], Pb["stf"], Pb["re"], Pb["rx"])["seis"]
    return orc.misfit(s, data, Pb["dt"]), s


def _gpu_op(Pb, every=25, geometry=None):
    from paper_2606_12850_amd.autograd import SeismogramOperator
    return SeismogramOperator(Pb["m"], Pb["se"], Pb["sx"], Pb["sd"], Pb["stf"], Pb["re"], Pb["rx"], Pb["dt"],
                              Pb["nt"], checkpoint_every=every, geometry=geometry)


@pytest.mark.parametrize("geometry", ["stored", "trilinear"])
def test_adjoint_vs_oracle_and_fd(orc, geometry):
    import torch
    import paper_2606_12850_amd as P
    Pb = _problem(seed=1)
    m = Pb["m"]
    _, data = _oracle_chi(orc, Pb, Pb["lam"] * 1.03, Pb["mu"] * 0.97, Pb["rho"], np.zeros((4, 3, Pb["nt"])))
    chi0, s0 = _oracle_chi(orc, Pb, Pb["lam"], Pb["mu"], Pb["rho"], data)
    gseis = Pb["dt"] * (s0 - data)
    gam, jac, _ = orc.geometry(m.n, m.elem_vert, m.vert)
    rl, rm, rr = orc.adjoint(m.n, m.ibool, gam, jac, Pb["lam"], Pb["mu"], Pb["rho"], m.nglob, Pb["dt"], Pb["nt"],
                             Pb["se"], Pb["sx"], Pb["sd"], Pb["stf"], Pb["re"], Pb["rx"], gseis)
    op = _gpu_op(Pb, every=25, geometry=P.SEMX_GEOM_STORED if geometry == "stored" else P.SEMX_GEOM_TRILINEAR)
    seis = op.run(Pb["lam"], Pb["mu"], Pb["rho"])
    torch.cuda.synchronize()
    assert rel_l2(seis[0].cpu().numpy(), s0) < 1e-4
    gl, gm, gr = (t[0].cpu().numpy().astype(np.float64) for t in op.gradient(torch.from_numpy(gseis[None])))
    for name, a, b in (("lambda", gl, rl), ("mu", gm, rm), ("rho", gr, rr)):
        err = rel_l2(a, b)
        print(f"{geometry} K_{name}: rel L2 vs oracle adjoint {err:.2e}")
        assert err <= 1e-3, (name, err)
    # directional derivatives against FP64 central differences
    rng = np.random.default_rng(7)
    for k in range(4):
        dl = Pb["lam"] * rng.standard_normal(Pb["lam"].shape)
        dm = Pb["mu"] * rng.standard_normal(Pb["mu"].shape)
        dr = Pb["rho"] * rng.standard_normal(Pb["rho"].shape)
        eps = 1e-6
        cp, _ = _oracle_chi(orc, Pb, Pb["lam"] + eps * dl, Pb["mu"] + eps * dm, Pb["rho"] + eps * dr, data)
        cm, _ = _oracle_chi(orc, Pb, Pb["lam"] - eps * dl, Pb["mu"] - eps * dm, Pb["rho"] - eps * dr, data)
        fd = (cp - cm) / (2 * eps)
        ad = np.sum(gl * dl) + np.sum(gm * dm) + np.sum(gr * dr)
        print(f"{geometry} direction {k}: adjoint {ad:.6e} FD {fd:.6e} rel {abs(ad - fd) / abs(fd):.2e}")
        assert abs(ad - fd) <= 1e-3 * abs(fd)
    op.solver.close()


def test_checkpoint_interval_does_not_change_gradient():
    import torch
    Pb = _problem(seed=2, nt=60)
    g = torch.from_numpy(np.random.default_rng(0).standard_normal((1, 4, 3, Pb["nt"])).astype(np.float32))
    res = []
    for every in (7, 60, 100):
        op = _gpu_op(Pb, every=every)
        op.run(Pb["lam"], Pb["mu"], Pb["rho"])
        res.append([t.cpu().numpy() for t in op.gradient(g)])
        op.solver.close()
    for r in res[1:]:
        for a, b in zip(res[0], r):
            np.testing.assert_array_equal(a, b)


def test_autograd_function_matches_direct_adjoint():
    import torch
    from paper_2606_12850_amd.autograd import SemForward
    Pb = _problem(seed=3, nt=50)
    op = _gpu_op(Pb, every=10)
    lam = torch.tensor(Pb["lam"], requires_grad=True)
    mu = torch.tensor(Pb["mu"], requires_grad=True)
    rho = torch.tensor(Pb["rho"], requires_grad=True)
    seis = SemForward.apply(lam, mu, rho, op)
    target = torch.zeros_like(seis)
    chi = 0.5 * Pb["dt"] * torch.sum((seis.double() - target.double()) ** 2)
    gl, gm, gr = torch.autograd.grad(chi, (lam, mu, rho))
    op2 = _gpu_op(Pb, every=10)
    s2 = op2.run(Pb["lam"], Pb["mu"], Pb["rho"])
    dl, dm, dr = op2.gradient(Pb["dt"] * s2)
    for a, b in ((gl, dl), (gm, dm), (gr, dr)):
        np.testing.assert_allclose(a.numpy(), b[0].double().cpu().numpy(), rtol=1e-5, atol=1e-30)
    assert torch.isfinite(gl).all() and gl.abs().max() > 0
    op.solver.close(); op2.solver.close()


def test_adjoint_requires_checkpoints():
    import torch
    import paper_2606_12850_amd as P
    Pb = _problem(seed=4, nt=20)
    op = _gpu_op(Pb, every=0)
    op.run(Pb["lam"], Pb["mu"], Pb["rho"])
    with pytest.raises(P.SemxError) as ei:
        op.gradient(torch.zeros((1, 4, 3, Pb["nt"])))
    assert ei.value.code == P.SEMX_ESTATE
    op.solver.close()


def test_adjoint_checkpoints_follow_the_run():
    """Checkpoints belong to the run that saved them.  A new model with a
    different batch size, uploaded on a checkpointed context, starts a new
    run (checkpoint 0 saved at upload): its gradient equals a fresh
    context's.  After semx_set_state or semx_set_sources the old run's
    checkpoints are refused (SEMX_ESTATE) instead of being replayed."""
    import torch
    import paper_2606_12850_amd as P
    Pb = _problem(seed=5, nt=40)
    g1 = torch.from_numpy(np.random.default_rng(1).standard_normal((1, 4, 3, Pb["nt"])).astype(np.float32))
    op = _gpu_op(Pb, every=10)
    op.run(Pb["lam"], Pb["mu"], Pb["rho"])
    op.gradient(g1)
    s = op.solver
    # two models sharing the mesh, uploaded on the same context, stepped without semx_reset
    lam2 = np.stack([Pb["lam"], 1.02 * Pb["lam"]]); mu2 = np.stack([Pb["mu"], Pb["mu"]])
    rho2 = np.stack([Pb["rho"], 0.99 * Pb["rho"]])
    s.upload_model(lam2, mu2, rho2)
    P.semx_step(s.ctx, Pb["nt"])
    g2 = torch.from_numpy(np.random.default_rng(2).standard_normal((2, 4, 3, Pb["nt"])).astype(np.float32)).cuda()
    shape = (2, Pb["m"].nspec, Pb["m"].n ** 3)
    got = [torch.empty(shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    P.semx_adjoint(s.ctx, g2, Pb["nt"], *got)
    op2 = _gpu_op(Pb, every=10)
    op2.run(lam2, mu2, rho2)
    ref = op2.gradient(g2)
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    # a new state or new sources: the saved checkpoints are not of this run
    u = s.empty_field(); v = s.empty_field(); a = s.empty_field()
    it = P.semx_get_state(s.ctx, u, v, a)
    P.semx_set_state(s.ctx, u, v, a, it)
    with pytest.raises(P.SemxError) as ei:
        P.semx_adjoint(s.ctx, g2, Pb["nt"], *got)
    assert ei.value.code == P.SEMX_ESTATE
    P.semx_reset(s.ctx)
    P.semx_step(s.ctx, Pb["nt"])
    P.semx_set_sources(s.ctx, *op.src)
    with pytest.raises(P.SemxError) as ei:
        P.semx_adjoint(s.ctx, g2, Pb["nt"], *got)
    assert ei.value.code == P.SEMX_ESTATE
    op.solver.close(); op2.solver.close()


def test_autograd_backward_refuses_a_later_forward():
    """backward of a graph whose operator has since run another forward raises
    (its checkpoints are of the later run)."""
    import torch
    from paper_2606_12850_amd.autograd import SemForward
    Pb = _problem(seed=6, nt=30)
    op = _gpu_op(Pb, every=10)
    lam = torch.tensor(Pb["lam"], requires_grad=True)
    seis = SemForward.apply(lam, torch.tensor(Pb["mu"]), torch.tensor(Pb["rho"]), op)
    op.run(Pb["lam"] * 1.01, Pb["mu"], Pb["rho"])   # e.g. a finite-difference probe
    with pytest.raises(RuntimeError, match="another forward"):
        torch.sum(seis.double() ** 2).backward()
    op.solver.close()


@pytest.mark.parametrize("n,geometry", [(12, "stored"), (16, "trilinear")])
def test_adjoint_high_order(orc, n, geometry):
    """NGLL 12 and 16 (the column kernels): sensitivity kernels against the
    oracle adjoint and one FP64 central-difference direction."""
    import torch
    import paper_2606_12850_amd as P
    Pb = _problem(n=n, ne=(2, 2, 1), nt=60, seed=3)
    Pb["dt"] = 1e-3
    Pb["stf"] = W.ricker(25.0, 0.04, Pb["dt"], Pb["nt"] + 1)[None, :]
    m = Pb["m"]
    _, data = _oracle_chi(orc, Pb, Pb["lam"] * 1.03, Pb["mu"] * 0.97, Pb["rho"], np.zeros((4, 3, Pb["nt"])))
    chi0, s0 = _oracle_chi(orc, Pb, Pb["lam"], Pb["mu"], Pb["rho"], data)
    gseis = Pb["dt"] * (s0 - data)
    gam, jac, _ = orc.geometry(m.n, m.elem_vert, m.vert)
    rl, rm, rr = orc.adjoint(m.n, m.ibool, gam, jac, Pb["lam"], Pb["mu"], Pb["rho"], m.nglob, Pb["dt"], Pb["nt"],
                             Pb["se"], Pb["sx"], Pb["sd"], Pb["stf"], Pb["re"], Pb["rx"], gseis)
    op = _gpu_op(Pb, every=20, geometry=P.SEMX_GEOM_STORED if geometry == "stored" else P.SEMX_GEOM_TRILINEAR)
    seis = op.run(Pb["lam"], Pb["mu"], Pb["rho"])
    torch.cuda.synchronize()
    assert rel_l2(seis[0].cpu().numpy(), s0) < 1e-4
    gl, gm, gr = (t[0].cpu().numpy().astype(np.float64) for t in op.gradient(torch.from_numpy(gseis[None])))
    for name, a, b in (("lambda", gl, rl), ("mu", gm, rm), ("rho", gr, rr)):
        err = rel_l2(a, b)
        print(f"NGLL {n} {geometry} K_{name}: rel L2 vs oracle adjoint {err:.2e}")
        assert err <= 1e-3, (name, err)
    rng = np.random.default_rng(9)
    dl = Pb["lam"] * rng.standard_normal(Pb["lam"].shape)
    dm = Pb["mu"] * rng.standard_normal(Pb["mu"].shape)
    dr = Pb["rho"] * rng.standard_normal(Pb["rho"].shape)
    eps = 1e-6
    cp, _ = _oracle_chi(orc, Pb, Pb["lam"] + eps * dl, Pb["mu"] + eps * dm, Pb["rho"] + eps * dr, data)
    cm, _ = _oracle_chi(orc, Pb, Pb["lam"] - eps * dl, Pb["mu"] - eps * dm, Pb["rho"] - eps * dr, data)
    fd = (cp - cm) / (2 * eps)
    ad = np.sum(gl * dl) + np.sum(gm * dm) + np.sum(gr * dr)
    print(f"NGLL {n} direction: adjoint {ad:.6e} FD {fd:.6e} rel {abs(ad - fd) / abs(fd):.2e}")
    assert abs(ad - fd) <= 1e-3 * abs(fd)
    op.solver.close()
