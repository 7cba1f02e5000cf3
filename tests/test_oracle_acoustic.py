"""Pins of the FP64 acoustic oracle (no GPU): the scalar operator against an
independent bilinear form, closed-form fields and invariants; the 1-D rod
against the independent 1-D Bloch relation and the closed-form half-line
solution; the 3-D rod against the 1-D rod."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import acoustic as A
from tests import indep


def _mesh(ne, n, L, jitter=0.0, seed=3):
    m = W.box_mesh(ne, n, L, jitter=jitter, seed=seed)
    gam, jac, xyz = A.O.geometry(n, m.elem_vert, m.vert)
    return m, gam, jac, xyz


def _node_xyz(m, xyz):
    X = np.zeros((m.nglob, 3))
    X[m.ibool.ravel()] = xyz.reshape(-1, 3)
    return X


@pytest.mark.parametrize("n", [2, 3, 4])
def test_force_matches_independent_bilinear_form(n):
    """f = -K p with K from sum W / rho grad phi_a . grad phi_b evaluated by an
    independent numpy geometry (jittered mesh, varying rho)."""
    m, gam, jac, _ = _mesh((2, 2, 1), n, (200.0, 150.0, 100.0), jitter=0.15)
    rng = np.random.default_rng(n)
    rho = rng.uniform(800.0, 1200.0, (m.nspec, n ** 3))
    K = indep.dense_stiffness_acoustic(n, m.ibool, m.elem_vert, m.vert, rho, m.nglob)
    p = rng.uniform(-1, 1, m.nglob)
    f = A.force(n, m.ibool, gam, jac, rho, p, m.nglob)
    np.testing.assert_allclose(f, -K @ p, rtol=0, atol=1e-12 * np.abs(K @ p).max())
    # symmetric, positive semi-definite, constants the only null space
    np.testing.assert_allclose(K, K.T, rtol=0, atol=1e-12 * np.abs(K).max())
    ev = np.linalg.eigvalsh(K)
    assert ev[0] > -1e-10 * ev[-1] and ev[1] > 1e-8 * ev[-1]


@pytest.mark.parametrize("n", [4, 5])
def test_constant_field_has_no_force(n):
    m, gam, jac, _ = _mesh((3, 2, 2), n, 300.0, jitter=0.1)
    rho = np.full((m.nspec, n ** 3), A.RHO)
    f0 = A.force(n, m.ibool, gam, jac, rho, np.full(m.nglob, 3.7), m.nglob)
    fr = A.force(n, m.ibool, gam, jac, rho, np.random.default_rng(1).uniform(-1, 1, m.nglob), m.nglob)
    assert np.abs(f0).max() <= 1e-13 * np.abs(fr).max()


@pytest.mark.parametrize("n", [3, 5])
def test_linear_field_patch_test(n):
    """p = a x on a jittered box (flat faces): zero force at interior nodes;
    on the faces x = 0 and x = Lx the force is the boundary flux
    -(a/rho) n_x times the face quadrature weight of the node."""
    ne = (3, 3, 2)
    L = (300.0, 240.0, 180.0)
    m, gam, jac, xyz = _mesh(ne, n, L, jitter=0.12)
    X = _node_xyz(m, xyz)
    a = 2.5
    rho = np.full((m.nspec, n ** 3), A.RHO)
    f = A.force(n, m.ibool, gam, jac, rho, a * X[:, 0], m.nglob)
    _, w = A.O.gll(n)
    N = n - 1

    def face_w(nel, h):
        out = np.zeros(nel * N + 1)
        for e in range(nel):
            out[e * N:e * N + n] += 0.5 * h * w
        return out

    wy = face_w(ne[1], L[1] / ne[1]); wz = face_w(ne[2], L[2] / ne[2])
    Gx, Gy = ne[0] * N + 1, ne[1] * N + 1
    g = np.arange(m.nglob)
    gx, gy, gz = g % Gx, (g // Gx) % Gy, g // (Gx * Gy)
    expect = np.zeros(m.nglob)
    expect[gx == 0] = a / A.RHO * wy[gy[gx == 0]] * wz[gz[gx == 0]]
    expect[gx == Gx - 1] = -a / A.RHO * wy[gy[gx == Gx - 1]] * wz[gz[gx == Gx - 1]]
    np.testing.assert_allclose(f, expect, rtol=0, atol=1e-12 * np.abs(expect).max())


@pytest.mark.parametrize("n", [4, 6])
def test_rod_reduces_to_1d_operator(n):
    """A field constant over the cross-section of a one-element rod: the 3-D
    force is the 1-D force times the face quadrature weight of the node, and
    so is the mass."""
    ne, h, hy, hz = 5, 40.0, 25.0, 30.0
    m, gam, jac, xyz = _mesh((ne, 1, 1), n, (ne * h, hy, hz), jitter=0.0)
    x1, M1, K1 = A.rod_operator(n, h, ne)
    rng = np.random.default_rng(n)
    p1 = rng.uniform(-1, 1, len(x1))
    N = n - 1
    Gx, Gy = ne * N + 1, n
    g = np.arange(m.nglob)
    gx, gy, gz = g % Gx, (g // Gx) % Gy, g // (Gx * Gy)
    _, w = A.O.gll(n)
    face = 0.25 * hy * hz * w[gy] * w[gz]
    f3 = A.force(n, m.ibool, gam, jac, np.full((m.nspec, n ** 3), A.RHO), p1[gx], m.nglob)
    np.testing.assert_allclose(f3, -(K1 @ p1)[gx] * face, rtol=0, atol=1e-12 * np.abs(f3).max())
    kappa = np.full((m.nspec, n ** 3), A.RHO * A.VP ** 2)
    np.testing.assert_allclose(A.mass(n, m.ibool, jac, kappa, m.nglob), M1[gx] * face, rtol=1e-13)


@pytest.mark.parametrize("n", [3, 5, 8])
def test_periodic_1d_spectrum_contains_bloch_branch(n):
    """Eigenvalues of M^-1 K of the periodic 1-D operator include
    omega(k)^2 of the independent 1-D GLL Bloch relation at every
    k = 2 pi m / (ne h)."""
    ne, h = 8, 50.0
    _, Mg, K = A.rod_operator(n, h, ne, periodic=True)
    ev = np.sort(np.linalg.eigvalsh(K.toarray() / np.sqrt(np.outer(Mg, Mg))))
    for mm in range(0, 4):
        k = 2.0 * math.pi * mm / (ne * h)
        om = indep.sem1d_bloch_omega(n, h, A.VP, k)
        assert np.min(np.abs(ev - om * om)) <= 1e-9 * ev[-1], (mm, om)


def test_rod_matches_closed_form_when_resolved():
    """Degree 8, 10 points per shortest wavelength at 2.5 f0, dt = 2e-5 s:
    the rod's trace at 300 m equals the half-line solution to 1e-9 in the
    waveform error (Ricker delay 1.6 / f0, so the source tail before t = 0
    is below 1e-10)."""
    t0 = 1.6 / A.F0
    err = A.rod_error(9, 24.0, x_rec=300.0, dt=2e-5, t0=t0)
    assert err < 1e-9, err


def test_rod_time_error_is_second_order():
    """With space resolved, halving dt divides the waveform error by 16
    (phase error of the central difference ~ (omega dt)^2 / 24 per cycle,
    error ~ phase^2)."""
    t0 = 1.6 / A.F0
    e1 = A.rod_error(9, 24.0, x_rec=1500.0, dt=4e-4, t0=t0)
    e2 = A.rod_error(9, 24.0, x_rec=1500.0, dt=2e-4, t0=t0)
    assert 12.0 < e1 / e2 < 20.0, (e1, e2)


def test_3d_rod_run_equals_1d_rod_run():
    """The 3-D oracle's time loop on a one-element rod with a plane source
    (one point source per end-face node, amplitude the face quadrature
    weight) and a receiver on the axis gives the 1-D rod's trace."""
    n, h, x_rec = 4, 50.0, 100.0
    t_end = A.window(x_rec)
    ne, nt = A.rod_setup(n, h, x_rec, t_end)
    hy = hz = 40.0
    m, gam, jac, _ = _mesh((ne, 1, 1), n, (ne * h, hy, hz))
    _, w = A.O.gll(n)
    xi, _ = A.O.gll(n)
    jj, kk = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    src_xi = np.stack([-np.ones(n * n), xi[jj.ravel()], xi[kk.ravel()]], axis=1)
    amp = 0.25 * hy * hz * w[jj.ravel()] * w[kk.ravel()]
    stf = amp[:, None] * A.ricker(np.arange(nt + 1) * A.DT)[None, :]
    e = int(x_rec // h)
    rec_xi = np.array([[2.0 * (x_rec - e * h) / h - 1.0, 0.3, -0.2]])
    kappa = np.full((m.nspec, n ** 3), A.RHO * A.VP ** 2)
    rho = np.full((m.nspec, n ** 3), A.RHO)
    out = A.forward(n, m.ibool, gam, jac, kappa, rho, m.nglob, A.DT, nt, np.zeros(n * n, np.int32), src_xi,
                    stf, np.array([e], np.int32), rec_xi)
    t, tr = A.rod_run(n, h, x_rec, t_end)
    np.testing.assert_allclose(out["seis"][0], tr, rtol=0, atol=1e-10 * np.abs(tr).max())


def test_forward_conserves_energy_after_the_source():
    n = 4
    m, gam, jac, _ = _mesh((2, 2, 2), n, 200.0, jitter=0.1)
    rng = np.random.default_rng(7)
    kappa = A.RHO * A.VP ** 2 * rng.uniform(0.8, 1.2, (m.nspec, n ** 3))
    rho = A.RHO * rng.uniform(0.8, 1.2, (m.nspec, n ** 3))
    nt = 300
    stf = np.zeros((1, nt + 1)); stf[0, :20] = A.ricker(np.arange(20) * 2e-4, 200.0, 0.002)
    out = A.forward(n, m.ibool, gam, jac, kappa, rho, m.nglob, 2e-4, nt, np.array([3], np.int32),
                    np.array([[0.1, -0.3, 0.5]]), stf, np.array([0], np.int32), np.array([[0.0, 0.0, 0.0]]),
                    want_energy=True)
    E = out["energy"][25:]
    assert E[0] > 0
    np.testing.assert_allclose(E, E[0], rtol=1e-12)


def test_equal_accuracy_table_reproducible():
    """tests/golden/acoustic_iso.json (written by make_acoustic_iso.py from
    this oracle): one entry recomputed, and the time-step check on the two
    sides of the bound (dt = 1e-4 s passes the 1 % relative L2 error on a
    resolved mesh, 2e-4 s does not: the paper's choice of dt)."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "acoustic_iso.json")))
    assert A.rod_error(16, 130.0) == pytest.approx(g["orders"]["16"]["errors"]["130"], rel=1e-9)
    ts = g["time_step_check"]
    assert ts["0.0001"] <= g["bound_ratio"] < ts["0.0002"]
    for key in ("5", "8", "16"):
        assert g["orders"][key]["error_at_h_max"] <= g["bound_ratio"]


def test_source_receiver_reciprocity():
    """p recorded at B for a source at A equals p at A for the same source at
    B (jittered mesh, varying kappa and rho), to rounding."""
    n = 4
    m, gam, jac, _ = _mesh((2, 2, 2), n, (300.0, 260.0, 220.0), jitter=0.12, seed=11)
    rng = np.random.default_rng(4)
    kappa = A.RHO * A.VP ** 2 * rng.uniform(0.8, 1.2, (m.nspec, n ** 3))
    rho = A.RHO * rng.uniform(0.8, 1.2, (m.nspec, n ** 3))
    ea, xa = np.array([1], np.int32), np.array([[0.31, -0.42, 0.17]])
    eb, xb = np.array([6], np.int32), np.array([[-0.25, 0.38, -0.61]])
    dt, nt = 2e-4, 1000  # A and B are about 207 m apart: the wave arrives after 0.14 s
    stf = W.ricker(30.0, 0.04, dt, nt + 1)[None, :]
    ab = A.forward(n, m.ibool, gam, jac, kappa, rho, m.nglob, dt, nt, ea, xa, stf, eb, xb)["seis"][0]
    ba = A.forward(n, m.ibool, gam, jac, kappa, rho, m.nglob, dt, nt, eb, xb, stf, ea, xa)["seis"][0]
    assert np.abs(ab).max() > 0
    np.testing.assert_allclose(ab, ba, rtol=0, atol=1e-10 * np.abs(ab).max())
