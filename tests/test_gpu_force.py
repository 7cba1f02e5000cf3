"""GPU parity of the FP32 force operator f = -K u against the FP64 oracle.

Bar: relative L2 error <= 1e-5 over all degrees of freedom for the FP32
path (the stated tolerance of the FP32 force apply), on random and smooth
displacements, for every NGLL, both assembly modes and both geometry paths.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import gpu_force, make_solver, oracle_geometry, rel_l2, smooth_field

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


def _hetero_model(mesh, seed):
    lam, mu, rho = W.layered_model(mesh, grf_amp=0.05, grf_seed=seed, grf_corr_elems=1.5)
    return lam, mu, rho


CASES = [
    # (name, ne, n, jitter)
    ("regular_cube_n5", 4, 5, 0.0),
    ("jittered_ragged_n5", (7, 5, 3), 5, 0.1),
    ("jittered_n4", (5, 4, 3), 4, 0.1),
    ("jittered_n3", (4, 3, 5), 3, 0.1),
    ("jittered_n6", (3, 4, 3), 6, 0.1),
    ("jittered_n7", (3, 3, 2), 7, 0.1),
    ("jittered_n8", (2, 3, 2), 8, 0.1),
    ("jittered_n9", (2, 2, 2), 9, 0.1),
    ("regular_n9", (3, 2, 2), 9, 0.0),
    ("jittered_n10", (2, 2, 2), 10, 0.1),
    ("regular_n2", (5, 3, 4), 2, 0.0),
]


@pytest.mark.parametrize("geometry", ["stored", "trilinear"])
@pytest.mark.parametrize("assembly", ["colored", "atomic"])
@pytest.mark.parametrize("name,ne,n,jitter", CASES, ids=[c[0] for c in CASES])
def test_force_parity(orc, name, ne, n, jitter, assembly, geometry):
    import paper_2606_12850_amd as P
    if jitter == 0.0 and geometry == "trilinear":
        pytest.skip("regular meshes use the per-element path in both geometry modes")
    mesh = W.box_mesh(ne, n, 4000.0, jitter=jitter, seed=17)
    lam, mu, rho = _hetero_model(mesh, 5)
    gam, jac, _ = oracle_geometry(orc, mesh)
    s = make_solver(n)
    info = s.upload_mesh(mesh)
    if jitter == 0.0:
        assert info["nirregular"] == 0
    else:
        assert info["nregular"] == 0
    s.upload_model(lam, mu, rho)
    s.set_mode(P.SEMX_C_F32, P.SEMX_ASM_COLORED if assembly == "colored" else P.SEMX_ASM_ATOMIC)
    P.semx_set_geometry(s.ctx, P.SEMX_GEOM_STORED if geometry == "stored" else P.SEMX_GEOM_TRILINEAR)
    rng = np.random.default_rng(3)
    for u in (rng.uniform(-1, 1, (mesh.nglob, 3)), smooth_field(orc, mesh)):
        u32 = u.astype(np.float32).astype(np.float64)   # both sides see the same FP32 input
        f_ref = orc.force(n, mesh.ibool, gam, jac, lam, mu, u32, mesh.nglob)
        f_gpu = gpu_force(s, u32)
        err = rel_l2(f_gpu, f_ref)
        print(f"{name} {assembly} n={n}: rel L2 = {err:.3e}")
        assert err <= TOL_F32, err
    s.close()


def test_force_mixed_regular_irregular(orc):
    """A mesh with both element kinds runs the two specialised paths."""
    import paper_2606_12850_amd as P
    mesh = W.box_mesh((4, 3, 3), 5, 4000.0)
    # move one interior vertex: the 8 elements around it become irregular
    mesh.vert[1 + 5 * (1 + 4 * 1)] += np.array([60.0, -40.0, 30.0])
    lam, mu, rho = _hetero_model(mesh, 9)
    gam, jac, _ = oracle_geometry(orc, mesh)
    s = make_solver(5)
    info = s.upload_mesh(mesh)
    assert info["nirregular"] == 8 and info["nregular"] == mesh.nspec - 8
    s.upload_model(lam, mu, rho)
    u = np.random.default_rng(4).uniform(-1, 1, (mesh.nglob, 3)).astype(np.float32).astype(np.float64)
    f_ref = orc.force(5, mesh.ibool, gam, jac, lam, mu, u, mesh.nglob)
    for asm in (P.SEMX_ASM_COLORED, P.SEMX_ASM_ATOMIC):
        s.set_mode(P.SEMX_C_F32, asm)
        assert rel_l2(gpu_force(s, u), f_ref) <= TOL_F32
    s.close()


def test_rigid_modes_and_symmetry_on_gpu(orc):
    mesh = W.box_mesh((4, 4, 3), 5, 4000.0, jitter=0.1, seed=3)
    lam, mu, rho = _hetero_model(mesh, 2)
    gam, jac, xyz = oracle_geometry(orc, mesh)
    s = make_solver(5)
    s.upload_mesh(mesh)
    s.upload_model(lam, mu, rho)
    rng = np.random.default_rng(5)
    ur = rng.uniform(-1, 1, (mesh.nglob, 3))
    fr = gpu_force(s, ur)
    kscale = np.linalg.norm(fr) / np.linalg.norm(ur)
    f = gpu_force(s, np.ones((mesh.nglob, 3)))
    # FP32 rounding of the contraction only: D 1 = 0 is not exact in FP32
    assert np.linalg.norm(f) <= 1e-5 * kscale * np.sqrt(3 * mesh.nglob)
    u = rng.uniform(-1, 1, (mesh.nglob, 3)); v = rng.uniform(-1, 1, (mesh.nglob, 3))
    fu, fv = gpu_force(s, u), gpu_force(s, v)
    a, b = np.sum(u * fv), np.sum(v * fu)
    assert abs(a - b) <= 1e-5 * np.linalg.norm(fu) * np.linalg.norm(v)
    s.close()


def test_colored_is_deterministic_atomic_within_tolerance():
    import torch
    import paper_2606_12850_amd as P
    mesh = W.box_mesh((6, 5, 4), 5, 4000.0, jitter=0.1, seed=8)
    lam, mu, rho = _hetero_model(mesh, 1)
    s = make_solver(5)
    s.upload_mesh(mesh)
    s.upload_model(lam, mu, rho)
    u = torch.rand((mesh.nglob, 3), device=s.device) - 0.5
    s.set_mode(P.SEMX_C_F32, P.SEMX_ASM_COLORED)
    f1 = s.apply_force(u).clone(); f2 = s.apply_force(u).clone()
    assert torch.equal(f1, f2)
    s.set_mode(P.SEMX_C_F32, P.SEMX_ASM_ATOMIC)
    fa = s.apply_force(u)
    torch.cuda.synchronize()
    assert (torch.linalg.norm(fa - f1) / torch.linalg.norm(f1)).item() < 1e-6
    s.close()


def test_empty_and_error_paths():
    import paper_2606_12850_amd as P
    s = make_solver(5)
    with pytest.raises(P.SemxError) as ei:
        P.semx_apply_force(s.ctx, None, None)
    assert ei.value.code == P.SEMX_ESTATE
    mesh = W.box_mesh(2, 5, 1000.0)
    bad = mesh.ibool.copy(); bad[0, 0] = mesh.nglob
    with pytest.raises(P.SemxError) as ei:
        P.semx_upload_mesh(s.ctx, bad, mesh.vert, mesh.elem_vert, mesh.nglob)
    assert ei.value.code == P.SEMX_EINVAL
    ev = mesh.elem_vert.copy(); ev[:, [0, 1]] = ev[:, [1, 0]]
    with pytest.raises(P.SemxError) as ei:
        P.semx_upload_mesh(s.ctx, mesh.ibool, mesh.vert, ev, mesh.nglob)
    assert ei.value.code == P.SEMX_EGEOM
    s.upload_mesh(mesh)
    lam, mu, rho = W.homogeneous_model(mesh)
    with pytest.raises(P.SemxError) as ei:
        P.semx_upload_model(s.ctx, lam, -mu, rho)
    assert ei.value.code == P.SEMX_EINVAL
    s.upload_model(lam, mu, rho)
    with pytest.raises(P.SemxError) as ei:
        P.semx_step(s.ctx, 1)  # no dt yet
    assert ei.value.code == P.SEMX_ESTATE
    with pytest.raises(P.SemxError):
        P.semx_set_dt(s.ctx, -1.0)
    # an element repeating a node (periodic, one element wide) cannot be coloured
    pm = W.box_mesh((1, 2, 2), 3, 1000.0, periodic=True)
    s3 = make_solver(3)
    s3.upload_mesh(pm)
    with pytest.raises(P.SemxError):
        P.semx_set_mode(s3.ctx, P.SEMX_C_F32, P.SEMX_ASM_COLORED)
    s3.close()
    s.close()


def test_periodic_atomic_matches_oracle(orc):
    """Wrap-around numbering (a periodic box) through the atomic path."""
    import paper_2606_12850_amd as P
    mesh = W.box_mesh((1, 3, 2), 4, 1200.0, periodic=True)
    lam, mu, rho = W.homogeneous_model(mesh)
    gam, jac, _ = oracle_geometry(orc, mesh)
    s = make_solver(4)
    s.upload_mesh(mesh)
    s.upload_model(lam, mu, rho)
    P.semx_set_mode(s.ctx, P.SEMX_C_F32, P.SEMX_ASM_ATOMIC)
    u = np.random.default_rng(0).uniform(-1, 1, (mesh.nglob, 3)).astype(np.float32).astype(np.float64)
    f_ref = orc.force(4, mesh.ibool, gam, jac, lam, mu, u, mesh.nglob)
    assert rel_l2(gpu_force(s, u), f_ref) <= TOL_F32
    s.close()


def test_stream_bandwidth_reference():
    """The library's streaming copy gives a bandwidth between a plausible
    floor and the published 8 TB/s peak, and rejects bad sizes."""
    import paper_2606_12850_amd as P
    s = make_solver(4)
    bw = P.semx_stream_bandwidth(s.ctx, 256 << 20, 5)
    print(f"stream copy: {bw:.0f} GB/s")
    assert 500.0 < bw < 8000.0 * 1.05
    for nbytes, reps in ((0, 1), (100, 1), (1 << 20, 0)):
        with pytest.raises(P.SemxError) as ei:
            P.semx_stream_bandwidth(s.ctx, nbytes, reps)
        assert ei.value.code == P.SEMX_EINVAL
    s.close()


def test_force_timing_stride():
    """semx_set_timing(k) event-times force passes 0, k, 2k, ... (k = 1: all,
    0: none) and counts the colour launches inside them; the summed
    durations are positive."""
    import torch
    import paper_2606_12850_amd as P
    mesh = W.box_mesh(4, 4, 400.0, jitter=0.1, seed=3)
    lam, mu, rho = W.homogeneous_model(mesh)
    s = make_solver(4)
    info = s.upload_mesh(mesh)
    s.upload_model(lam, mu, rho)
    assert info["ncolors"] == 8
    u = torch.rand((mesh.nglob, 3), device="cuda")
    f = torch.empty_like(u)
    for stride, expect in ((1, 40), (2, 24), (3, 16), (0, 0)):  # passes 0..4, 8 launches each
        P.semx_set_timing(s.ctx, stride)
        for _ in range(5):  # 5 applies x 8 colour launches
            P.semx_apply_force(s.ctx, u, f)
        n, ms = P.semx_force_timing(s.ctx)
        assert n == expect, (stride, n)
        assert (ms > 0) == (expect > 0)
    with pytest.raises(P.SemxError) as ei:
        P.semx_set_timing(s.ctx, -1)
    assert ei.value.code == P.SEMX_EINVAL
    s.close()


def test_force_skeleton():
    """The memory skeleton of the coloured force pass (same launches, loads
    and stores, no arithmetic) runs on every geometry path, takes no longer
    than the force pass itself, leaves the operator unchanged, and rejects
    the contexts it does not cover."""
    import torch
    import paper_2606_12850_amd as P
    mesh = W.box_mesh(32, 5, 4000.0, jitter=0.1, seed=3)
    lam, mu, rho = _hetero_model(mesh, 4)
    s = make_solver(5)
    s.upload_mesh(mesh)
    s.upload_model(lam, mu, rho)
    u = torch.rand((mesh.nglob, 3), device="cuda")
    f = torch.empty_like(u)
    for geometry in (P.SEMX_GEOM_STORED, P.SEMX_GEOM_TRILINEAR):
        P.semx_set_geometry(s.ctx, geometry)
        P.semx_apply_force(s.ctx, u, f)
        f0 = f.clone()
        sk = P.semx_force_skeleton(s.ctx, u, f, 20)
        P.semx_set_timing(s.ctx, 1)
        for _ in range(20):
            P.semx_apply_force(s.ctx, u, f)
        _, ms = P.semx_force_timing(s.ctx)
        P.semx_set_timing(s.ctx, 0)
        torch.cuda.synchronize()
        print(f"geometry {geometry}: skeleton {sk * 1e3:.1f} us, force pass {ms / 20 * 1e3:.1f} us per pass")
        assert 0.0 < sk <= 1.1 * ms / 20
        assert torch.equal(f, f0)
    for bad in (0, -3):
        with pytest.raises(P.SemxError) as ei:
            P.semx_force_skeleton(s.ctx, u, f, bad)
        assert ei.value.code == P.SEMX_EINVAL
    with pytest.raises(P.SemxError) as ei:
        P.semx_force_skeleton(s.ctx, u, u, 1)
    assert ei.value.code == P.SEMX_EINVAL
    s.set_mode(P.SEMX_C_F32, P.SEMX_ASM_ATOMIC)
    with pytest.raises(P.SemxError) as ei:
        P.semx_force_skeleton(s.ctx, u, f, 1)
    assert ei.value.code == P.SEMX_ESTATE
    s.close()
    # batched models (one grid row per model)
    m2 = W.box_mesh((6, 5, 4), 5, 1000.0, jitter=0.1, seed=8)
    models = [_hetero_model(m2, k) for k in (1, 2)]
    s = make_solver(5)
    s.upload_mesh(m2)
    s.upload_model(*(np.stack([m[i] for m in models]) for i in range(3)))
    u = torch.rand((2, m2.nglob, 3), device="cuda")
    f = torch.empty_like(u)
    P.semx_apply_force(s.ctx, u, f)
    f0 = f.clone()
    assert P.semx_force_skeleton(s.ctx, u, f, 3) > 0.0
    P.semx_apply_force(s.ctx, u, f)
    torch.cuda.synchronize()
    assert torch.equal(f, f0)
    s.close()
    # the column kernels (NGLL 11-16): skeleton on a jittered mesh, then the
    # operator is unchanged
    for n in (11, 16):
        mh = W.box_mesh((4, 4, 2), n, 1000.0, jitter=0.1, seed=5)
        s = make_solver(n)
        s.upload_mesh(mh)
        s.upload_model(*_hetero_model(mh, 6))
        u = torch.rand((mh.nglob, 3), device="cuda")
        f = torch.empty_like(u)
        for geometry in (P.SEMX_GEOM_STORED, P.SEMX_GEOM_TRILINEAR):
            P.semx_set_geometry(s.ctx, geometry)
            P.semx_apply_force(s.ctx, u, f)
            f0 = f.clone()
            assert P.semx_force_skeleton(s.ctx, u, f, 3) > 0.0
            P.semx_apply_force(s.ctx, u, f)
            torch.cuda.synchronize()
            assert torch.equal(f, f0)
        s.close()
    # acoustic physics has no skeleton
    ma = W.box_mesh(2, 5, 1000.0)
    s = P.Solver(5, physics=P.SEMX_ACOUSTIC)
    s.upload_mesh(ma)
    s.upload_model_acoustic(np.full((ma.nspec, 125), 2.25e9), np.full((ma.nspec, 125), 1000.0))
    u = torch.zeros(ma.nglob, device="cuda")
    with pytest.raises(P.SemxError) as ei:
        P.semx_force_skeleton(s.ctx, u, torch.empty_like(u), 1)
    assert ei.value.code == P.SEMX_ESTATE
    s.close()


def _degenerate_meshes(n):
    """One element (regular, then with a displaced corner) and a strip of
    four elements one element wide (displaced corner): the smallest grids,
    with one and two colours."""
    import dataclasses
    out = []
    for ne, distort in (((1, 1, 1), False), ((1, 1, 1), True), ((1, 1, 4), True)):
        mesh = W.box_mesh(ne, n, 1000.0)
        if distort:
            vert = mesh.vert.copy()
            c = int(np.argmax(vert.sum(axis=1)))
            vert[c] += np.array([0.07, -0.05, 0.06]) * (np.array(mesh.L) / np.array(ne))
            mesh = dataclasses.replace(mesh, vert=vert)
        out.append((ne, distort, mesh))
    return out


@pytest.mark.parametrize("n", [2, 5, 10, 11, 16])
def test_force_degenerate_meshes(orc, n):
    """Single-element and one-element-wide meshes at the orders where the
    kernel changes (one lane per point up to NGLL 10, the column kernel from
    11, its DPP rows at 16): every assembly and geometry mode against the
    oracle."""
    import paper_2606_12850_amd as P
    rng = np.random.default_rng(40 + n)
    for ne, distort, mesh in _degenerate_meshes(n):
        lam, mu, rho = _hetero_model(mesh, 1)
        gam, jac, _ = oracle_geometry(orc, mesh)
        u = rng.uniform(-1, 1, (mesh.nglob, 3)).astype(np.float32).astype(np.float64)
        f_ref = orc.force(n, mesh.ibool, gam, jac, lam, mu, u, mesh.nglob)
        s = make_solver(n)
        info = s.upload_mesh(mesh)
        assert (info["nirregular"] > 0) == distort
        s.upload_model(lam, mu, rho)
        for geometry in (P.SEMX_GEOM_STORED, P.SEMX_GEOM_TRILINEAR):
            P.semx_set_geometry(s.ctx, geometry)
            for assembly in (P.SEMX_ASM_COLORED, P.SEMX_ASM_ATOMIC):
                s.set_mode(P.SEMX_C_F32, assembly)
                err = rel_l2(gpu_force(s, u), f_ref)
                print(f"n={n} ne={ne} distorted={distort} geometry={geometry} assembly={assembly}: {err:.2e}")
                assert err <= TOL_F32, (ne, distort, geometry, assembly, err)
        s.close()


def test_zero_steps_and_silent_run():
    """semx_step(0) changes nothing; with no sources and no receivers a run
    from rest stays exactly at rest and the time index advances."""
    import torch
    import paper_2606_12850_amd as P
    mesh = W.box_mesh((3, 2, 2), 5, 1000.0, jitter=0.1, seed=3)
    lam, mu, rho = _hetero_model(mesh, 2)
    s = make_solver(5)
    s.upload_mesh(mesh)
    s.upload_model(lam, mu, rho)
    P.semx_set_dt(s.ctx, P.semx_cfl_dt(s.ctx, 0.4))
    P.semx_reset(s.ctx)
    P.semx_step(s.ctx, 0)
    assert P.semx_time_index(s.ctx) == 0
    P.semx_step(s.ctx, 25)
    assert P.semx_time_index(s.ctx) == 25
    u = s.empty_field(); v = s.empty_field(); a = s.empty_field()
    assert P.semx_get_state(s.ctx, u, v, a) == 25
    torch.cuda.synchronize()
    for x in (u, v, a):
        assert int(torch.count_nonzero(x)) == 0
    s.close()


@pytest.mark.parametrize("renumber", ["reversed", "x_reversed", "scrambled"])
def test_force_parity_renumbered_nodes(orc, renumber):
    """Node numberings the affine path must handle: all strides negative
    (g -> G - 1 - g), one negative stride (x reversed), and a random
    permutation (no element affine: node numbers streamed).  The force of
    each must equal the oracle's on the same numbering; a wrong node span in
    the affine buffer reads would return zeros instead of u or f."""
    import paper_2606_12850_amd as P
    n = 5
    base = W.box_mesh(4, n, 4000.0, jitter=0.1, seed=23)
    Gx = 4 * (n - 1) + 1
    g = np.arange(base.nglob)
    if renumber == "reversed":
        perm = base.nglob - 1 - g
    elif renumber == "x_reversed":
        X, rest = g % Gx, g // Gx
        perm = (Gx - 1 - X) + Gx * rest
    else:
        perm = np.random.default_rng(5).permutation(base.nglob)
    mesh = base
    mesh.ibool = perm[base.ibool].astype(np.int32)
    lam, mu, rho = _hetero_model(mesh, 12)
    gam, jac, _ = oracle_geometry(orc, mesh)
    for geometry in ("trilinear", "stored"):
        for blocks in (P.SEMX_BLOCKS_OFF, P.SEMX_BLOCKS_ON):
            s = make_solver(n)
            s.upload_mesh(mesh)
            s.upload_model(lam, mu, rho)
            s.set_mode(P.SEMX_C_F32, P.SEMX_ASM_COLORED)
            P.semx_set_geometry(s.ctx, P.SEMX_GEOM_STORED if geometry == "stored" else P.SEMX_GEOM_TRILINEAR)
            active = P.semx_set_blocks(s.ctx, blocks)
            assert active == (blocks == P.SEMX_BLOCKS_ON and renumber != "scrambled")
            u = np.random.default_rng(8).uniform(-1, 1, (mesh.nglob, 3)).astype(np.float32).astype(np.float64)
            f_ref = orc.force(n, mesh.ibool, gam, jac, lam, mu, u, mesh.nglob)
            err = rel_l2(gpu_force(s, u), f_ref)
            print(f"{renumber} {geometry} blocks={active}: rel L2 = {err:.3e}")
            assert err <= TOL_F32, err
            s.close()
