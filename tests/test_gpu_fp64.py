"""FP64 storage (semx_set_storage(SEMX_F64)) against the FP64 oracle (GPU).

Both sides compute the same discrete operator and time loop in FP64; they
differ only in the order of the sums (the library's LDS contractions and
colour-ordered or atomic assembly against the oracle's element loop).  The
force therefore agrees to FP64 rounding times the cancellation of the
operator: bound 1e-12 relative L2 (the FP32 path's bar is 1e-5).
Seismograms after 200 / 1000 steps: 1e-10 (rounding differences grow at most
linearly over a stable run: 1000 steps x ~1e-13)."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import oracle_geometry, rel_l2, smooth_field

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-12
TOL_SEIS64 = 1e-10


def solver64(n):
    import paper_2606_12850_amd as P
    return P.Solver(n, storage=P.SEMX_F64)


def gpu_force64(s, u_np):
    import torch
    u = torch.from_numpy(np.ascontiguousarray(u_np, dtype=np.float64)).to(s.device)
    f = s.apply_force(u)
    torch.cuda.synchronize()
    return f.cpu().numpy()


@pytest.mark.parametrize("n", [2, 3, 5, 8, 10])
def test_fp64_force_matches_oracle(orc, n):
    import paper_2606_12850_amd as P
    ne = (3, 2, 3) if n <= 5 else (2, 2, 2)
    mesh = W.box_mesh(ne, n, 4000.0, jitter=0.1, seed=5)
    lam, mu, rho = W.layered_model(mesh, grf_amp=0.05, grf_seed=3, grf_corr_elems=1.5)
    gam, jac, _ = oracle_geometry(orc, mesh)
    s = solver64(n)
    s.upload_mesh(mesh)
    s.upload_model(lam, mu, rho)
    for label, u in (("random", np.random.default_rng(1).uniform(-1, 1, (mesh.nglob, 3))),
                     ("smooth", smooth_field(orc, mesh))):
        ref = orc.force(n, mesh.ibool, gam, jac, lam, mu, u, mesh.nglob)
        out = {}
        for asm in (P.SEMX_ASM_COLORED, P.SEMX_ASM_ATOMIC):
            s.set_mode(P.SEMX_C_F32, asm)
            out[asm] = gpu_force64(s, u)
            err = rel_l2(out[asm], ref)
            print(f"fp64 n={n} {label} asm={asm}: rel L2 vs oracle = {err:.3e}")
            assert err <= TOL_F64
        s.set_mode(P.SEMX_C_F32, P.SEMX_ASM_COLORED)
        assert np.array_equal(gpu_force64(s, u), out[P.SEMX_ASM_COLORED])  # deterministic
    s.close()


def test_fp64_batched_models(orc):
    n = 4
    mesh = W.box_mesh((2, 3, 2), n, 3000.0, jitter=0.1, seed=11)
    models = [W.layered_model(mesh, grf_amp=0.05, grf_seed=k, grf_corr_elems=1.5) for k in (1, 2)]
    lam = np.stack([m[0] for m in models]); mu = np.stack([m[1] for m in models]); rho = np.stack([m[2] for m in models])
    gam, jac, _ = oracle_geometry(orc, mesh)
    u = np.random.default_rng(4).uniform(-1, 1, (2, mesh.nglob, 3))
    s = solver64(n)
    s.upload_mesh(mesh)
    s.upload_model(lam, mu, rho)
    got = gpu_force64(s, u)
    for k in range(2):
        ref = orc.force(n, mesh.ibool, gam, jac, lam[k], mu[k], u[k], mesh.nglob)
        assert rel_l2(got[k], ref) <= TOL_F64
    s.close()


def run_oracle(orc, wl):
    m = wl.mesh
    gam, jac, _ = oracle_geometry(orc, m)
    return orc.forward(m.n, m.ibool, gam, jac, wl.lam, wl.mu, wl.rho, m.nglob, wl.dt, wl.nt, wl.src_elem,
                       wl.src_xi, wl.src_dir, wl.stf, wl.rec_elem, wl.rec_xi)["seis"]


@pytest.mark.parametrize("nt", [200, 1000])
def test_fp64_cube_seismograms(orc, nt):
    """Homogeneous 4 km cube, 4^3 elements, NGLL 5, Ricker 10 Hz, Courant 0.4,
    in FP64 on both sides."""
    import paper_2606_12850_amd as P
    wl = W.cube_homogeneous(ne=4, n=5, nt=nt)
    ref = run_oracle(orc, wl)
    for asm in (P.SEMX_ASM_COLORED, P.SEMX_ASM_ATOMIC):
        s = solver64(5)
        s.upload_mesh(wl.mesh)
        s.upload_model(wl.lam, wl.mu, wl.rho)
        s.set_mode(P.SEMX_C_F32, asm)
        s.setup_run(wl)
        s.step(wl.nt)
        got = s.seismograms()
        s.close()
        assert got.dtype == np.float64
        err = rel_l2(got, ref)
        print(f"fp64 cube nt={nt} asm={asm}: seismogram rel L2 = {err:.3e}")
        assert err <= TOL_SEIS64


def test_fp64_layered_jittered_seismograms(orc):
    from tests.test_gpu_timeloop import cfl_dt
    nt = 600
    wl = W.layered_jittered(ne=6, n=5, nt=nt, dt=1.0, jitter=0.1, nrec=8)
    wl.dt = cfl_dt(orc, wl.mesh, wl.lam, wl.mu, wl.rho)
    wl.stf = W.ricker(10.0, 0.12, wl.dt, nt + 1)[None, :]
    ref = run_oracle(orc, wl)
    s = solver64(5)
    s.upload_mesh(wl.mesh)
    s.upload_model(wl.lam, wl.mu, wl.rho)
    s.setup_run(wl)
    s.step(nt)
    err = rel_l2(s.seismograms(), ref)
    s.close()
    print(f"fp64 layered jittered 6^3 nt={nt}: rel L2 = {err:.3e}")
    assert err <= TOL_SEIS64


def test_fp64_state_roundtrip_and_energy():
    """Checkpoint and restore reproduce the run bitwise, and with it the
    discrete energy tracked on the last step (deterministic FP64 sums); a
    restored state has no tracked half step until it steps."""
    import torch
    import paper_2606_12850_amd as P
    wl = W.cube_homogeneous(ne=3, n=4, nt=60, dt=0.02)
    s = solver64(4)
    s.upload_mesh(wl.mesh)
    s.upload_model(wl.lam, wl.mu, wl.rho)
    s.setup_run(wl)
    s.step(30)
    shape = (wl.mesh.nglob, 3)
    u, v, a = (torch.zeros(shape, dtype=torch.float64, device="cuda") for _ in range(3))
    it = P.semx_get_state_f64(s.ctx, u, v, a)
    s.step(30)
    first = s.seismograms()
    e1 = P.semx_energy(s.ctx)
    P.semx_set_state_f64(s.ctx, u, v, a, it)
    with pytest.raises(P.SemxError) as ei:
        P.semx_energy(s.ctx)
    assert ei.value.code == P.SEMX_ESTATE
    s.step(30)
    assert np.array_equal(s.seismograms(), first)
    assert P.semx_energy(s.ctx) == e1
    s.close()


def test_fp64_energy_identity_per_step(orc):
    """The discrete energy balance of the scheme, step by step in FP64 storage,
    while the source acts: E^{n+1/2} - E^{n-1/2} = 1/2 (u^{n+1} - u^{n-1})^T f_src^n
    to 1e-12 of E; and E^{n+1/2} and the work against the oracle's to 1e-10.
    The same balance in FP32 storage is reported (its rounding drift)."""
    import paper_2606_12850_amd as P
    wl = W.layered_jittered(ne=4, n=5, nt=60, dt=1.0, jitter=0.1)
    from tests.test_gpu_timeloop import cfl_dt
    wl.dt = cfl_dt(orc, wl.mesh, wl.lam, wl.mu, wl.rho)
    wl.stf = W.ricker(10.0, 0.12, wl.dt, wl.nt + 1)[None, :]
    m = wl.mesh
    gam, jac, _ = orc.geometry(5, m.elem_vert, m.vert)
    ref = orc.forward(5, m.ibool, gam, jac, wl.lam, wl.mu, wl.rho, m.nglob, wl.dt, wl.nt, wl.src_elem, wl.src_xi,
                      wl.src_dir, wl.stf, wl.rec_elem, wl.rec_xi, want_energy=True)
    res = {}
    for storage in ("f64", "f32"):
        s = solver64(5) if storage == "f64" else P.Solver(5)
        s.upload_mesh(m)
        s.upload_model(wl.lam, wl.mu, wl.rho)
        s.setup_run(wl)
        E, Wk = [], []
        for _ in range(wl.nt):
            s.step(1)
            k, p, w = P.semx_energy(s.ctx, with_work=True)
            E.append(k + p); Wk.append(w)
        s.close()
        E, Wk = np.array(E), np.array(Wk)
        scale = np.abs(E).max()
        bal = np.abs(np.diff(E) - np.diff(Wk)).max() / scale
        e_or = np.abs(E - ref["energy"]).max() / scale
        w_or = np.abs(Wk - np.cumsum(ref["work"])).max() / scale
        res[storage] = (bal, e_or, w_or)
        print(f"{storage}: max |dE - dW| / max E = {bal:.2e}; vs oracle: E {e_or:.2e}, work {w_or:.2e}")
    assert res["f64"][0] <= 1e-12
    assert res["f64"][1] <= 1e-10 and res["f64"][2] <= 1e-10
    assert res["f32"][1] <= 1e-4


def test_fp64_mode_errors():
    import torch
    import paper_2606_12850_amd as P
    wl = W.cube_homogeneous(ne=2, n=4, nt=5, dt=0.02)
    s = solver64(4)
    s.upload_mesh(wl.mesh)
    s.upload_model(wl.lam, wl.mu, wl.rho)
    u32 = torch.zeros((wl.mesh.nglob, 3), dtype=torch.float32, device="cuda")
    for call in (lambda: P.semx_apply_force(s.ctx, u32, u32.clone()),
                 lambda: P.semx_get_state(s.ctx, u32),
                 lambda: P.semx_set_state(s.ctx, u32, u32, u32, 0),
                 lambda: P.semx_set_checkpointing(s.ctx, 10),
                 lambda: P.semx_set_storage(s.ctx, P.SEMX_F32)):
        with pytest.raises(P.SemxError) as ei:
            call()
        assert ei.value.code == P.SEMX_ESTATE
    with pytest.raises(P.SemxError) as ei:
        P.semx_set_mode(s.ctx, P.SEMX_C_BF16, P.SEMX_ASM_COLORED)
    assert ei.value.code == P.SEMX_EINVAL
    s.close()
    # the FP64 entry points need FP64 storage
    s32 = P.Solver(4)
    s32.upload_mesh(wl.mesh)
    s32.upload_model(wl.lam, wl.mu, wl.rho)
    u64 = torch.zeros((wl.mesh.nglob, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(P.SemxError) as ei:
        P.semx_apply_force_f64(s32.ctx, u64, u64.clone())
    assert ei.value.code == P.SEMX_ESTATE
    with pytest.raises(P.SemxError) as ei:
        P.semx_set_storage(s32.ctx, 7)
    assert ei.value.code == P.SEMX_EINVAL
    s32.close()
