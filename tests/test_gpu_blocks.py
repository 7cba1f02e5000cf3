"""GPU parity of the 2 x 2 x 2 element-block force kernel (NGLL 2..5).

The block kernel gathers each node of a block of eight elements once,
sums the elements' shared nodes in a fixed order and writes each node once;
it must give the FP32 force of the per-element kernel up to the order of
floating-point summation, and the FP64 oracle's force within the FP32 bar
(1e-5 relative L2).  Meshes that do not decompose into blocks (an odd
element count along an axis) must fall back to the per-element kernel.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import gpu_force, make_solver, oracle_geometry, rel_l2, smooth_field

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


@pytest.mark.parametrize("geometry", ["stored", "trilinear"])
@pytest.mark.parametrize("n,ne,jitter", [(5, 4, 0.1), (5, (2, 4, 6), 0.1), (5, 4, 0.0), (4, (4, 2, 4), 0.1),
                                         (3, (2, 2, 4), 0.1), (2, (6, 4, 2), 0.1)])
def test_block_force_parity(orc, n, ne, jitter, geometry):
    import paper_2606_12850_amd as P
    mesh = W.box_mesh(ne, n, 4000.0, jitter=jitter, seed=31)
    lam, mu, rho = W.layered_model(mesh, grf_amp=0.05, grf_seed=7, grf_corr_elems=1.5)
    gam, jac, _ = oracle_geometry(orc, mesh)
    s = make_solver(n)
    s.upload_mesh(mesh)
    s.upload_model(lam, mu, rho)
    s.set_mode(P.SEMX_C_F32, P.SEMX_ASM_COLORED)
    P.semx_set_geometry(s.ctx, P.SEMX_GEOM_STORED if geometry == "stored" else P.SEMX_GEOM_TRILINEAR)
    rng = np.random.default_rng(11)
    for u in (rng.uniform(-1, 1, (mesh.nglob, 3)), smooth_field(orc, mesh)):
        u32 = u.astype(np.float32).astype(np.float64)
        f_ref = orc.force(n, mesh.ibool, gam, jac, lam, mu, u32, mesh.nglob)
        assert P.semx_set_blocks(s.ctx, P.SEMX_BLOCKS_ON)
        f_blk = gpu_force(s, u32)
        f_blk2 = gpu_force(s, u32)               # first-touch stores: a second pass overwrites
        assert not P.semx_set_blocks(s.ctx, P.SEMX_BLOCKS_OFF)
        f_el = gpu_force(s, u32)
        e_ref, e_el = rel_l2(f_blk, f_ref), rel_l2(f_blk, f_el)
        print(f"blocks n={n} ne={ne} {geometry}: vs oracle {e_ref:.3e}, vs per-element {e_el:.3e}")
        assert e_ref <= TOL_F32, e_ref
        assert e_el <= 2e-6, e_el
        assert np.array_equal(f_blk, f_blk2)      # deterministic
    # the automatic mode takes the blocks on the stored-Gamma path of irregular elements only
    auto = P.semx_set_blocks(s.ctx, P.SEMX_BLOCKS_AUTO)
    assert auto == (geometry == "stored" and jitter > 0.0)
    s.close()


def test_block_batched_models(orc):
    """Two models sharing the mesh: each model's force matches its oracle."""
    import paper_2606_12850_amd as P
    import torch
    n = 5
    mesh = W.box_mesh(4, n, 4000.0, jitter=0.1, seed=5)
    gam, jac, _ = oracle_geometry(orc, mesh)
    models = [W.layered_model(mesh, grf_amp=0.05, grf_seed=sd, grf_corr_elems=1.5) for sd in (1, 2)]
    s = make_solver(n)
    s.upload_mesh(mesh)
    s.upload_model(np.stack([m[0] for m in models]), np.stack([m[1] for m in models]),
                   np.stack([m[2] for m in models]))
    s.set_mode(P.SEMX_C_F32, P.SEMX_ASM_COLORED)
    assert P.semx_set_blocks(s.ctx, P.SEMX_BLOCKS_ON)
    u = np.random.default_rng(4).uniform(-1, 1, (2, mesh.nglob, 3)).astype(np.float32)
    ut = torch.from_numpy(u).to(s.device)
    f = torch.empty_like(ut)
    P.semx_apply_force(s.ctx, ut, f)
    torch.cuda.synchronize()
    f = f.cpu().numpy().astype(np.float64)
    for k, (lam, mu, rho) in enumerate(models):
        f_ref = orc.force(n, mesh.ibool, gam, jac, lam, mu, u[k].astype(np.float64), mesh.nglob)
        assert rel_l2(f[k], f_ref) <= TOL_F32
    s.close()


@pytest.mark.parametrize("n,ne", [(5, 3), (5, (4, 4, 3)), (6, 4)])
def test_block_fallback(n, ne):
    """An odd element count along an axis, or NGLL above 5: no blocks."""
    import paper_2606_12850_amd as P
    mesh = W.box_mesh(ne, n, 4000.0, jitter=0.1, seed=2)
    lam, mu, rho = W.layered_model(mesh)
    s = make_solver(n)
    s.upload_mesh(mesh)
    s.upload_model(lam, mu, rho)
    s.set_mode(P.SEMX_C_F32, P.SEMX_ASM_COLORED)
    assert not P.semx_set_blocks(s.ctx, P.SEMX_BLOCKS_ON)
    with pytest.raises(P.SemxError):
        P.semx_set_blocks(s.ctx, 3)
    s.close()
