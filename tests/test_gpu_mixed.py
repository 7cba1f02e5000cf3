"""Matrix-core force operator (BF16 / FP16 MFMA operands with FP32
accumulation; FP32 MFMA operands): error against the FP64 oracle, stated per
case.  The FP32-operand matrix-core path is held to the FP32 force bar
(1e-5 relative L2).

Parity here is unpinned beyond the stated bounds: the expected relative
error is set by the operand precision (BF16 8-bit, FP16 11-bit significand)
times the cancellation of the operator, so the bounds below are loose
ceilings, not tolerances of the method.  A random field has no
cancellation: its ceiling is the same at every order.  A smooth field's
derivatives are small against the rounding of the operands times the row
sums of |D| (the infinity norm of D: 51 at NGLL 8, 245 at NGLL 16), so
beyond NGLL 8 its ceiling scales with that norm.  Exact properties are
checked exactly: a rigid translation gives zero force (operand offset), and
the result does not depend on the assembly mode beyond FP32 rounding."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import gpu_force, make_solver, oracle_geometry, rel_l2, smooth_field

pytestmark = pytest.mark.gpu

BOUND = {"bf16": 5e-2, "f16": 5e-3, "mf32": 1e-5}


def _dnorm(orc, n):
    return float(np.abs(np.asarray(orc.dmatrix(n)).reshape(n, n)).sum(axis=1).max())


def _cprec(P, prec):
    return {"bf16": P.SEMX_C_BF16, "f16": P.SEMX_C_F16, "mf32": P.SEMX_C_MFMA_F32}[prec]


@pytest.mark.parametrize("prec", ["bf16", "f16", "mf32"])
@pytest.mark.parametrize("n", [4, 5, 6, 7, 8, 11, 14, 16])
@pytest.mark.parametrize("geometry", ["stored", "trilinear"])
def test_mixed_force_error(orc, n, prec, geometry):
    import paper_2606_12850_amd as P
    mesh = W.box_mesh((3, 2, 3) if n <= 6 else ((2, 2, 2) if n <= 8 else (2, 2, 1)), n, 4000.0, jitter=0.1, seed=5)
    lam, mu, rho = W.layered_model(mesh, grf_amp=0.05, grf_seed=3, grf_corr_elems=1.5)
    gam, jac, _ = oracle_geometry(orc, mesh)
    s = make_solver(n)
    s.upload_mesh(mesh)
    s.upload_model(lam, mu, rho)
    P.semx_set_geometry(s.ctx, P.SEMX_GEOM_STORED if geometry == "stored" else P.SEMX_GEOM_TRILINEAR)
    cprec = _cprec(P, prec)
    for label, u in (("random", np.random.default_rng(1).uniform(-1, 1, (mesh.nglob, 3))),
                     ("smooth", smooth_field(orc, mesh))):
        u32 = u.astype(np.float32).astype(np.float64)
        ref = orc.force(n, mesh.ibool, gam, jac, lam, mu, u32, mesh.nglob)
        errs = {}
        for asm in (P.SEMX_ASM_COLORED, P.SEMX_ASM_ATOMIC):
            s.set_mode(cprec, asm)
            errs[asm] = rel_l2(gpu_force(s, u32), ref)
        bound = BOUND[prec]
        if label == "smooth" and prec != "mf32":
            bound *= max(1.0, _dnorm(orc, n) / _dnorm(orc, 8))
        print(f"mixed {prec} n={n} {geometry} {label}: rel L2 vs FP64 = {errs[P.SEMX_ASM_COLORED]:.3e} "
              f"(ceiling {bound:.1e})")
        assert errs[P.SEMX_ASM_COLORED] <= bound
        assert abs(errs[P.SEMX_ASM_ATOMIC] - errs[P.SEMX_ASM_COLORED]) <= 1e-6 + 1e-3 * errs[P.SEMX_ASM_COLORED]
    s.close()


@pytest.mark.parametrize("prec", ["bf16", "f16"])
@pytest.mark.parametrize("n", [5, 16])
def test_mixed_rigid_translation_is_exactly_zero(prec, n):
    import paper_2606_12850_amd as P
    mesh = W.box_mesh((3, 3, 2) if n == 5 else (2, 1, 2), n, 4000.0, jitter=0.1, seed=9)
    lam, mu, rho = W.homogeneous_model(mesh)
    s = make_solver(n)
    s.upload_mesh(mesh)
    s.upload_model(lam, mu, rho)
    s.set_mode(P.SEMX_C_BF16 if prec == "bf16" else P.SEMX_C_F16, P.SEMX_ASM_COLORED)
    u = np.tile(np.array([[1.5e-7, -2.25e-7, 3.0e-7]]), (mesh.nglob, 1))
    f = gpu_force(s, u)
    assert np.all(f == 0.0)
    s.close()


def test_mixed_rejects_unsupported_order():
    import paper_2606_12850_amd as P
    s = make_solver(9)
    for cp in (P.SEMX_C_BF16, P.SEMX_C_F16, P.SEMX_C_MFMA_F32):
        with pytest.raises(P.SemxError) as ei:
            P.semx_set_mode(s.ctx, cp, P.SEMX_ASM_COLORED)
        assert ei.value.code == P.SEMX_EINVAL
    s.close()


@pytest.mark.parametrize("prec", ["bf16", "f16", "mf32"])
def test_mixed_seismograms(orc, prec):
    """Seismogram error of a whole run with mixed-precision contractions.

    BF16 / FP16: the error against the FP64 oracle is reported, not gated
    (their parity is unpinned: the per-apply force error of the operand
    precision accumulates through 400 steps as a frequency shift whose size
    depends on the spectrum of the run).  The only gate is that the run stays
    a bounded, finite seismogram (relative error below 1).  FP32 operands on
    the matrix cores keep the FP32 seismogram bar."""
    import paper_2606_12850_amd as P
    wl = W.cube_homogeneous(ne=4, n=5, nt=400)
    m = wl.mesh
    gam, jac, _ = oracle_geometry(orc, m)
    ref = orc.forward(5, m.ibool, gam, jac, wl.lam, wl.mu, wl.rho, m.nglob, wl.dt, wl.nt, wl.src_elem, wl.src_xi,
                      wl.src_dir, wl.stf, wl.rec_elem, wl.rec_xi)["seis"]
    s = make_solver(5)
    s.upload_mesh(m)
    s.upload_model(wl.lam, wl.mu, wl.rho)
    s.set_mode(_cprec(P, prec), P.SEMX_ASM_COLORED)
    s.setup_run(wl)
    s.step(wl.nt)
    err = rel_l2(s.seismograms(), ref)
    print(f"mixed {prec} cube 400 steps: seismogram rel L2 vs FP64 = {err:.3e}")
    assert np.all(np.isfinite(s.seismograms()))
    assert err <= (1e-4 if prec == "mf32" else 1.0)
    s.close()
