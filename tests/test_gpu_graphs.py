"""Graph-captured time stepping equals direct stepping bitwise.

With semx_set_graphs(ctx, G) a long semx_step() call records G steps once as
a HIP graph and launches it for the middle of the call; the source, receiver
and source-work kernels read the time index from a device counter.  The
same sequence of calls, with eager work between them (state and energy
reads), must give the same state, energies and seismograms to the bit as
direct stepping, on every path the time loop takes: coloured and atomic
assembly (atomic to rounding: its summation order is the hardware's),
the element-block kernel, trilinear geometry, batched models,
acoustic physics, and steps past the recorded length.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import rel_l2

pytestmark = pytest.mark.gpu

# call lengths: a fresh graph-eligible call, a short direct call, then long
# calls that replay the graph many times, 2 chunks exactly, and one that is
# one step too short for graphs
CALLS = [90, 3, 200, 35, 33]
NT_REC = 300          # receivers record 300 of the 361 steps
CHUNK = 16


def _run(case, chunk):
    import torch
    import paper_2606_12850_amd as P
    n = 5
    acoustic = case == "acoustic"
    mesh = W.box_mesh(4, n, 4000.0, jitter=0.1, seed=3)
    s = P.Solver(n, physics=P.SEMX_ACOUSTIC) if acoustic else P.Solver(n)
    s.upload_mesh(mesh)
    if acoustic:
        rng = np.random.default_rng(5)
        shape = (mesh.nspec, n ** 3)
        s.upload_model_acoustic(2.25e9 * (1 + 0.1 * rng.uniform(-1, 1, shape)), np.full(shape, 1000.0))
    elif case == "batched":
        ms = [W.layered_model(mesh, grf_amp=0.05, grf_seed=sd) for sd in (1, 2)]
        s.upload_model(*(np.stack([m[k] for m in ms]) for k in range(3)))
    else:
        s.upload_model(*W.layered_model(mesh, grf_amp=0.05, grf_seed=1))
    if case == "atomic":
        s.set_mode(P.SEMX_C_F32, P.SEMX_ASM_ATOMIC)
    if case == "blocks":
        assert P.semx_set_blocks(s.ctx, P.SEMX_BLOCKS_ON)
    if case == "trilinear":
        P.semx_set_geometry(s.ctx, P.SEMX_GEOM_TRILINEAR)
    dt = 0.5 * P.semx_cfl_dt(s.ctx, 0.4)
    f0 = 0.25 / (20 * dt)
    stf = W.ricker(f0, 1.2 / f0, dt, NT_REC + 1)[None, :] * 1e9
    se, sx = W.center_vertex_source(mesh)
    re, rx = W.top_receivers_line(mesh, 6)
    P.semx_set_sources(s.ctx, se, sx, None if acoustic else np.array([[0.3, -0.2, 1.0]]), stf.astype(np.float32))
    P.semx_set_receivers(s.ctx, re, rx, NT_REC)
    s.nrec, s.nt_max = len(re), NT_REC
    P.semx_set_dt(s.ctx, dt)
    P.semx_reset(s.ctx)
    P.semx_set_graphs(s.ctx, chunk)
    trace = []
    for k in CALLS:
        s.step(k)
        u, v, a = s.empty_field(), s.empty_field(), s.empty_field()
        it = P.semx_get_state(s.ctx, u, v, a)
        torch.cuda.synchronize()
        trace.append((it, P.semx_energy(s.ctx, with_work=True), u.cpu().numpy(), v.cpu().numpy(), a.cpu().numpy()))
    seis = s.seismograms()
    s.close()
    return trace, seis


@pytest.mark.parametrize("case", ["colored", "blocks", "trilinear", "batched", "acoustic"])
def test_graph_steps_bitwise(case):
    eager, seis_e = _run(case, 0)
    graph, seis_g = _run(case, CHUNK)
    assert np.abs(seis_e).max() > 0
    for (it_e, en_e, *st_e), (it_g, en_g, *st_g) in zip(eager, graph):
        assert it_e == it_g
        assert en_e == en_g, (en_e, en_g)
        for x, y in zip(st_e, st_g):
            np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(seis_e, seis_g)
    print(f"graphs {case}: bitwise over {sum(CALLS)} steps, it = {graph[-1][0]}")


def test_graph_steps_atomic():
    """Atomic assembly adds element contributions in hardware order, so two
    direct runs already differ by rounding: the graph run must agree with the
    direct run to that level (FP32 rounding grown over the steps)."""
    eager, seis_e = _run("atomic", 0)
    graph, seis_g = _run("atomic", CHUNK)
    for (it_e, en_e, *st_e), (it_g, en_g, *st_g) in zip(eager, graph):
        assert it_e == it_g
        np.testing.assert_allclose(en_g, en_e, rtol=1e-6)
        for x, y in zip(st_e, st_g):
            assert rel_l2(y, x) <= 1e-5
    err = rel_l2(seis_g, seis_e)
    print(f"graphs atomic: seismograms rel L2 {err:.2e} against direct stepping")
    assert err <= 1e-5


def test_graph_chunk_limits():
    import paper_2606_12850_amd as P
    s = P.Solver(5)
    for bad in (-1, 4097):
        with pytest.raises(P.SemxError):
            P.semx_set_graphs(s.ctx, bad)
    P.semx_set_graphs(s.ctx, 4096)
    P.semx_set_graphs(s.ctx, 0)
    s.close()
