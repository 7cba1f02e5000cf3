"""High orders NGLL 11..16 (polynomial degree up to 15) against the FP64
oracle (GPU): the column kernel (NGLL 11..12) and the matrix-core tile
kernel (NGLL 13..16, padded tiles below 16; 16-bit operands from NGLL 11).

Bars as for the lower orders: force 1e-5 relative L2 (FP32), seismograms
1e-4 after the run.  The meshes are small (NGLL 16 has 4096 points per
element) and cover the three geometry paths, both assemblies, a mesh with
both element kinds, and batched models."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import gpu_force, make_solver, oracle_geometry, rel_l2, smooth_field

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5
TOL_SEIS = 1e-4


@pytest.mark.parametrize("n", [11, 12, 13, 14, 15, 16])
def test_high_order_force_parity(orc, n):
    import paper_2606_12850_amd as P
    rng = np.random.default_rng(n)
    for jitter in (0.1, 0.0):
        mesh = W.box_mesh((2, 2, 2) if n >= 14 else (3, 2, 2), n, 4000.0, jitter=jitter, seed=23)
        lam, mu, rho = W.layered_model(mesh, grf_amp=0.05, grf_seed=n, grf_corr_elems=1.5)
        gam, jac, _ = oracle_geometry(orc, mesh)
        s = make_solver(n)
        info = s.upload_mesh(mesh)
        assert (info["nirregular"] == 0) == (jitter == 0.0)
        s.upload_model(lam, mu, rho)
        geos = ("stored", "trilinear") if jitter else ("regular",)
        for u in (rng.uniform(-1, 1, (mesh.nglob, 3)), smooth_field(orc, mesh)):
            u32 = u.astype(np.float32).astype(np.float64)
            ref = orc.force(n, mesh.ibool, gam, jac, lam, mu, u32, mesh.nglob)
            for geo in geos:
                if geo != "regular":
                    P.semx_set_geometry(s.ctx, P.SEMX_GEOM_STORED if geo == "stored" else P.SEMX_GEOM_TRILINEAR)
                out = {}
                for asm in (P.SEMX_ASM_COLORED, P.SEMX_ASM_ATOMIC):
                    s.set_mode(P.SEMX_C_F32, asm)
                    out[asm] = gpu_force(s, u32)
                    err = rel_l2(out[asm], ref)
                    print(f"n={n} {geo} asm={asm}: rel L2 = {err:.3e}")
                    assert err <= TOL_F32, (geo, asm, err)
                s.set_mode(P.SEMX_C_F32, P.SEMX_ASM_COLORED)
                assert np.array_equal(gpu_force(s, u32), out[P.SEMX_ASM_COLORED])
        s.close()


def test_high_order_mixed_kinds_and_batched_models(orc):
    import paper_2606_12850_amd as P
    n = 12
    mesh = W.box_mesh((3, 2, 2), n, 3000.0)
    mesh.vert[1 + 4 * (1 + 3 * 1)] += np.array([40.0, -30.0, 20.0])  # elements around it become irregular
    models = [W.layered_model(mesh, grf_amp=0.05, grf_seed=k, grf_corr_elems=1.5) for k in (1, 2)]
    lam = np.stack([m[0] for m in models]); mu = np.stack([m[1] for m in models]); rho = np.stack([m[2] for m in models])
    gam, jac, _ = oracle_geometry(orc, mesh)
    s = make_solver(n)
    info = s.upload_mesh(mesh)
    assert info["nirregular"] > 0 and info["nregular"] > 0
    s.upload_model(lam, mu, rho)
    u = np.random.default_rng(5).uniform(-1, 1, (2, mesh.nglob, 3)).astype(np.float32).astype(np.float64)
    got = gpu_force(s, u)
    for k in range(2):
        ref = orc.force(n, mesh.ibool, gam, jac, lam[k], mu[k], u[k], mesh.nglob)
        assert rel_l2(got[k], ref) <= TOL_F32
    s.close()


@pytest.mark.parametrize("n", [12, 16])
def test_high_order_seismograms(orc, n):
    """A 2^3-element homogeneous cube at NGLL 12 and 16: Ricker source at the
    centre vertex, receivers on the top face, 200 steps at Courant 0.4."""
    import paper_2606_12850_amd as P
    from tests.test_gpu_timeloop import cfl_dt
    nt = 200
    wl = W.cube_homogeneous(ne=2, n=n, nt=nt, dt=1.0)
    wl.dt = cfl_dt(orc, wl.mesh, wl.lam, wl.mu, wl.rho)
    wl.stf = W.ricker(10.0, 0.12, wl.dt, nt + 1)[None, :]
    m = wl.mesh
    gam, jac, _ = oracle_geometry(orc, m)
    ref = orc.forward(n, m.ibool, gam, jac, wl.lam, wl.mu, wl.rho, m.nglob, wl.dt, nt, wl.src_elem, wl.src_xi,
                      wl.src_dir, wl.stf, wl.rec_elem, wl.rec_xi)["seis"]
    for asm in (P.SEMX_ASM_COLORED, P.SEMX_ASM_ATOMIC):
        s = make_solver(n)
        s.upload_mesh(m)
        s.upload_model(wl.lam, wl.mu, wl.rho)
        s.set_mode(P.SEMX_C_F32, asm)
        s.setup_run(wl)
        s.step(nt)
        err = rel_l2(s.seismograms(), ref)
        s.close()
        print(f"n={n} asm={asm}: seismogram rel L2 = {err:.3e}")
        assert err <= TOL_SEIS


def test_ngll16_matrix_core_mode_is_the_fp32_path():
    """At NGLL 16 the FP32 path already contracts on the matrix cores with
    FP32 operands: SEMX_C_MFMA_F32 selects the same kernel (identical bits)."""
    import paper_2606_12850_amd as P
    mesh = W.box_mesh((2, 2, 1), 16, 3000.0, jitter=0.1, seed=4)
    lam, mu, rho = W.layered_model(mesh, grf_amp=0.05, grf_seed=2, grf_corr_elems=1.5)
    s = make_solver(16)
    s.upload_mesh(mesh)
    s.upload_model(lam, mu, rho)
    u = np.random.default_rng(8).uniform(-1, 1, (mesh.nglob, 3))
    s.set_mode(P.SEMX_C_F32, P.SEMX_ASM_COLORED)
    a = gpu_force(s, u)
    s.set_mode(P.SEMX_C_MFMA_F32, P.SEMX_ASM_COLORED)
    assert np.array_equal(gpu_force(s, u), a)
    s.close()


def test_high_order_limits():
    """FP64 storage stops at NGLL 10 and says so; checkpointing for the
    adjoint and 16-bit matrix-core operands are accepted at NGLL 12."""
    import paper_2606_12850_amd as P
    mesh = W.box_mesh((1, 1, 1), 12, 1000.0)
    lam, mu, rho = W.homogeneous_model(mesh)
    s = make_solver(12)
    with pytest.raises(P.SemxError) as ei:
        P.semx_set_storage(s.ctx, P.SEMX_F64)
    assert ei.value.code == P.SEMX_EINVAL
    s.upload_mesh(mesh)
    s.upload_model(lam, mu, rho)
    P.semx_set_checkpointing(s.ctx, 10)
    P.semx_set_checkpointing(s.ctx, 0)
    # the matrix-core tile kernel covers NGLL 11..16, so 16-bit operands are accepted here
    P.semx_set_mode(s.ctx, P.SEMX_C_BF16, P.SEMX_ASM_COLORED)
    s.close()
    with pytest.raises(P.SemxError):
        P.Solver(17)
