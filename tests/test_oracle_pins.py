"""Pins of the FP64 oracle against closed forms, invariants and independent
re-derivations (no GPU).  Each test names what fixes the expected value."""
import numpy as np
import pytest

import workloads as W
from tests import indep


# --- GLL nodes, weights, Lagrange basis (Sec. II-B) -------------------------

def test_gll_closed_forms(orc):
    xi, w = orc.gll(4)
    s = 1.0 / np.sqrt(5.0)
    np.testing.assert_allclose(xi, [-1, -s, s, 1], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], rtol=0, atol=1e-15)
    xi, w = orc.gll(5)
    s = np.sqrt(3.0 / 7.0)
    np.testing.assert_allclose(xi, [-1, -s, 0, s, 1], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", range(2, 17))
def test_gll_weights_and_exactness(orc, n):
    xi, w = orc.gll(n)
    N = n - 1
    assert abs(w.sum() - 2.0) <= 4 * n * np.finfo(float).eps
    np.testing.assert_allclose(xi, -xi[::-1], atol=0)
    for k in range(0, 2 * N):  # exact up to degree 2N-1
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.dot(w, xi ** k) - exact) < 1e-14
    if N >= 1:  # and not beyond: degree 2N is integrated with an error
        assert abs(np.dot(w, xi ** (2 * N)) - 2.0 / (2 * N + 1)) > 1e-10
    xr, wr = indep.gll_numpy(n)
    np.testing.assert_allclose(xi, xr, atol=1e-14)
    np.testing.assert_allclose(w, wr, atol=1e-13)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8, 9, 12, 16])
def test_dmatrix(orc, n):
    D = orc.dmatrix(n)
    xi, _ = orc.gll(n)
    N = n - 1
    # exact differentiation of every polynomial of degree <= N
    for k in range(0, N + 1):
        exact = k * xi ** (k - 1) if k > 0 else np.zeros(n)
        np.testing.assert_allclose(D @ xi ** k, exact, atol=1e-12 * max(k, 1) * n)
    np.testing.assert_allclose(D @ np.ones(n), 0.0, atol=1e-12 * n)
    # corner entries of the GLL differentiation matrix: -+N(N+1)/4
    assert abs(D[0, 0] + N * (N + 1) / 4.0) < 1e-11 * n * n
    assert abs(D[N, N] - N * (N + 1) / 4.0) < 1e-11 * n * n
    # independent barycentric evaluation
    np.testing.assert_allclose(D, indep.dmatrix_barycentric(indep.gll_numpy(n)[0]), atol=1e-11 * n * n)


@pytest.mark.parametrize("n", [3, 5, 8])
def test_lagrange_kronecker_and_interpolation(orc, n):
    xi, _ = orc.gll(n)
    for b in range(n):
        np.testing.assert_allclose(orc.lagrange(n, xi[b]), np.eye(n)[b], atol=1e-14)
    rng = np.random.default_rng(0)
    c = rng.standard_normal(n)  # random polynomial of degree N
    for x in rng.uniform(-1, 1, 5):
        l = orc.lagrange(n, x)
        assert abs(np.dot(l, np.polyval(c, xi)) - np.polyval(c, x)) < 1e-12
        dl = orc.lagrange_deriv(n, x)
        assert abs(np.dot(dl, np.polyval(c, xi)) - np.polyval(np.polyder(c), x)) < 1e-11


# --- Geometry and mass ------------------------------------------------------

def test_geometry_affine(orc):
    m = W.box_mesh((2, 3, 1), 5, L=(1000.0, 600.0, 250.0))
    gam, jac, xyz = orc.geometry(5, m.elem_vert, m.vert)
    hx, hy, hz = 500.0, 200.0, 250.0
    np.testing.assert_allclose(jac, hx * hy * hz / 8.0, rtol=1e-14)
    G = np.zeros((3, 3)); G[0, 0] = 2 / hx; G[1, 1] = 2 / hy; G[2, 2] = 2 / hz
    np.testing.assert_allclose(gam, np.broadcast_to(G, gam.shape), atol=1e-17)


def test_geometry_jittered_matches_numpy_and_vertices(orc):
    m = W.box_mesh(3, 5, 4000.0, jitter=0.1, seed=7)
    gam, jac, xyz = orc.geometry(5, m.elem_vert, m.vert)
    J, det, gi, xr = indep.geometry_numpy(5, m.elem_vert, m.vert)
    np.testing.assert_allclose(jac, det, rtol=1e-13)
    np.testing.assert_allclose(gam, gi, rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(xyz, xr, rtol=1e-13, atol=1e-9)
    # corner GLL points reproduce the element vertices
    n = 5
    for v in range(8):
        a, b, c = v & 1, (v >> 1) & 1, (v >> 2) & 1
        q = a * (n - 1) + n * (b * (n - 1) + n * c * (n - 1))
        np.testing.assert_allclose(xyz[:, q, :], m.vert[m.elem_vert[:, v]], atol=1e-9)
    # Gamma J = I
    np.testing.assert_allclose(np.einsum("eqdb,eqbc->eqdc", gam, J), np.broadcast_to(np.eye(3), J.shape), atol=1e-12)


@pytest.mark.parametrize("n", [3, 5, 7])
def test_volume_and_mass(orc, n):
    # flat boundary faces: total volume is exactly L^3 even with jitter
    m = W.box_mesh(3, n, 4000.0, jitter=0.1, seed=3)
    gam, jac, _ = orc.geometry(n, m.elem_vert, m.vert)
    xi, w = orc.gll(n)
    w3 = np.einsum("k,j,i->kji", w, w, w).ravel()
    assert abs(np.sum(jac * w3) / 4000.0 ** 3 - 1.0) < 1e-13
    lam, mu, rho = W.homogeneous_model(m)
    M = orc.mass(n, m.ibool, jac, rho, m.nglob)
    assert np.all(M > 0)
    assert abs(M.sum() / (2500.0 * 4000.0 ** 3) - 1.0) < 1e-13
    np.testing.assert_allclose(M, indep.mass_numpy(n, m.ibool, m.elem_vert, m.vert, rho, m.nglob), rtol=1e-12)


def test_geometry_rejects_inverted_element(orc):
    m = W.box_mesh(1, 3, 100.0)
    ev = m.elem_vert.copy()
    ev[:, [0, 1]] = ev[:, [1, 0]]  # mirror: det J < 0
    with pytest.raises(ValueError):
        orc.geometry(3, ev, m.vert)


# --- Internal force f = -K u -------------------------------------------------

def _setup(orc, ne=3, n=5, jitter=0.1, seed=11, hetero=True):
    m = W.box_mesh(ne, n, 4000.0, jitter=jitter, seed=seed)
    gam, jac, xyz = orc.geometry(n, m.elem_vert, m.vert)
    lam, mu, rho = W.homogeneous_model(m)
    if hetero:
        rng = np.random.default_rng(seed)
        lam = lam * rng.uniform(0.5, 1.5, lam.shape)
        mu = mu * rng.uniform(0.5, 1.5, mu.shape)
    return m, gam, jac, xyz, lam, mu, rho


def test_force_rigid_modes(orc):
    m, gam, jac, xyz, lam, mu, rho = _setup(orc)
    # global coordinates of the nodes
    X = np.zeros((m.nglob, 3)); X[m.ibool.ravel()] = xyz.reshape(-1, 3)
    scale = None
    rng = np.random.default_rng(1)
    ur = rng.standard_normal((m.nglob, 3))
    fr = orc.force(5, m.ibool, gam, jac, lam, mu, ur, m.nglob)
    scale = np.linalg.norm(fr) / np.linalg.norm(ur)   # ~ |K|
    for t in np.eye(3):
        f = orc.force(5, m.ibool, gam, jac, lam, mu, np.broadcast_to(t, (m.nglob, 3)), m.nglob)
        assert np.linalg.norm(f) <= 1e-12 * scale * np.sqrt(m.nglob)
    for om in np.eye(3):
        u = np.cross(om, X - 2000.0)   # infinitesimal rotation omega x x
        f = orc.force(5, m.ibool, gam, jac, lam, mu, u, m.nglob)
        assert np.linalg.norm(f) <= 1e-12 * scale * np.linalg.norm(u)


def test_force_matches_bilinear_form(orc):
    """-v^T f(u) equals the symmetric bilinear form computed independently."""
    m, gam, jac, xyz, lam, mu, rho = _setup(orc, ne=2, seed=5)
    rng = np.random.default_rng(2)
    for _ in range(3):
        u = rng.standard_normal((m.nglob, 3)); v = rng.standard_normal((m.nglob, 3))
        f = orc.force(5, m.ibool, gam, jac, lam, mu, u, m.nglob)
        a = indep.bilinear(5, m.ibool, m.elem_vert, m.vert, lam, mu, u, v)
        assert abs(-np.sum(v * f) - a) <= 1e-12 * abs(a) + 1e-12 * np.linalg.norm(f) * np.linalg.norm(v)


def test_force_symmetric_psd(orc):
    m, gam, jac, xyz, lam, mu, rho = _setup(orc, ne=3, seed=9)
    rng = np.random.default_rng(3)
    u = rng.standard_normal((m.nglob, 3)); v = rng.standard_normal((m.nglob, 3))
    fu = orc.force(5, m.ibool, gam, jac, lam, mu, u, m.nglob)
    fv = orc.force(5, m.ibool, gam, jac, lam, mu, v, m.nglob)
    a, b = np.sum(u * fv), np.sum(v * fu)
    assert abs(a - b) <= 1e-13 * np.linalg.norm(fu) * np.linalg.norm(v)
    assert -np.sum(u * fu) > 0 and -np.sum(v * fv) > 0


def test_force_dense_matrix_bruteforce(orc):
    """Column-by-column K from the bilinear form equals -f(e_col) (1 jittered element + neighbour)."""
    m = W.box_mesh((2, 1, 1), 3, L=(2000.0, 1000.0, 1000.0), jitter=0.0)
    m.vert[m.elem_vert[0, 7]] += np.array([40.0, -30.0, 25.0])  # distort one shared-free vertex
    gam, jac, _ = orc.geometry(3, m.elem_vert, m.vert)
    lam, mu, rho = W.homogeneous_model(m)
    rng = np.random.default_rng(4)
    lam = lam * rng.uniform(0.5, 1.5, lam.shape); mu = mu * rng.uniform(0.5, 1.5, mu.shape)
    K = indep.dense_stiffness(3, m.ibool, m.elem_vert, m.vert, lam, mu, m.nglob)
    u = rng.standard_normal((m.nglob, 3))
    f = orc.force(3, m.ibool, gam, jac, lam, mu, u, m.nglob)
    np.testing.assert_allclose(-f.ravel(), K @ u.ravel(), rtol=1e-11, atol=1e-11 * np.abs(K).max() * np.abs(u).max())


def test_patch_test_affine_field(orc):
    """Affine u = A x in a homogeneous medium: zero force at interior nodes;
    boundary nodes get -sigma n times the integral of their basis function
    over the (flat, regular) boundary faces."""
    n = 4
    m = W.box_mesh(3, n, 3000.0, jitter=0.12, seed=21)
    gam, jac, xyz = orc.geometry(n, m.elem_vert, m.vert)
    lam, mu, rho = W.homogeneous_model(m)
    X = np.zeros((m.nglob, 3)); X[m.ibool.ravel()] = xyz.reshape(-1, 3)
    A = np.random.default_rng(8).standard_normal((3, 3)) * 1e-3
    u = X @ A.T
    f = orc.force(n, m.ibool, gam, jac, lam, mu, u, m.nglob)
    eps = 0.5 * (A + A.T)
    sig = lam.flat[0] * np.trace(A) * np.eye(3) + 2 * mu.flat[0] * eps
    _, w = indep.gll_numpy(n)
    h = 1000.0
    expect = np.zeros((m.nglob, 3))
    N = n - 1
    G = 3 * N + 1
    # six flat faces of the cube, each tiled by 3x3 element faces of area h^2
    for axis in range(3):
        for side, normal_sign in ((0, -1.0), (G - 1, 1.0)):
            nvec = np.zeros(3); nvec[axis] = normal_sign
            trac = sig @ nvec
            others = [a for a in range(3) if a != axis]
            for e1 in range(3):
                for e2 in range(3):
                    for a in range(n):
                        for b in range(n):
                            idx = [0, 0, 0]
                            idx[axis] = side
                            idx[others[0]] = e1 * N + a
                            idx[others[1]] = e2 * N + b
                            g = idx[0] + G * (idx[1] + G * idx[2])
                            expect[g] -= w[a] * w[b] * (h / 2) ** 2 * trac
    scale = np.abs(expect).max()
    np.testing.assert_allclose(f, expect, atol=1e-11 * scale)


@pytest.mark.parametrize("n,tol", [(5, 2e-5), (6, 2e-7), (8, 1e-10)])
def test_lame_mode_rayleigh_quotient(orc, n, tol):
    """Free-cube Lame mode u = (cos ax sin ay, -sin ax cos ay, 0), a = pi/L,
    is traction free with omega^2 = 2 a^2 mu / rho; the discrete Rayleigh
    quotient converges to it spectrally in n."""
    L = 4000.0
    m = W.box_mesh(4, n, L)
    gam, jac, xyz = orc.geometry(n, m.elem_vert, m.vert)
    lam, mu, rho = W.homogeneous_model(m)
    X = np.zeros((m.nglob, 3)); X[m.ibool.ravel()] = xyz.reshape(-1, 3)
    a = np.pi / L
    u = np.stack([np.cos(a * X[:, 0]) * np.sin(a * X[:, 1]), -np.sin(a * X[:, 0]) * np.cos(a * X[:, 1]),
                  np.zeros(m.nglob)], axis=1)
    f = orc.force(n, m.ibool, gam, jac, lam, mu, u, m.nglob)
    M = orc.mass(n, m.ibool, jac, rho, m.nglob)
    rq = -np.sum(u * f) / np.sum(M[:, None] * u * u)
    w2 = 2 * a * a * mu.flat[0] / rho.flat[0]
    assert abs(rq / w2 - 1.0) < tol
    # frequency of the first Lame mode of the 4 km homogeneous cube: vs / (sqrt(2) L)
    assert abs(np.sqrt(w2) / (2 * np.pi) - 1732.0 / (np.sqrt(2) * L)) < 1e-12


# --- Time loop ----------------------------------------------------------------

def test_energy_identity(orc):
    """E^{n+1/2} - E^{n-1/2} = 1/2 (u^{n+1} - u^{n-1})^T f_src^n to rounding."""
    wl = W.cube_homogeneous(ne=3, n=4, nt=60, dt=0.02)
    m = wl.mesh
    gam, jac, _ = orc.geometry(4, m.elem_vert, m.vert)
    out = orc.forward(4, m.ibool, gam, jac, wl.lam, wl.mu, wl.rho, m.nglob, wl.dt, wl.nt,
                      wl.src_elem, wl.src_xi, wl.src_dir, wl.stf, wl.rec_elem, wl.rec_xi,
                      want_energy=True)
    E, Wk = out["energy"], out["work"]
    scale = np.abs(E).max()
    assert scale > 0
    d = np.diff(E) - Wk[1:]
    assert np.abs(d).max() <= 1e-11 * scale
    # after the wavelet has decayed the energy is conserved and positive
    assert np.all(E[-10:] > 0)


def test_time_loop_vs_dense_central_difference(orc):
    """Newmark run == central differences M(u+ - 2u + u-) = dt^2 (f_src - K u)
    with K and M built independently (tiny mesh)."""
    n = 3
    m = W.box_mesh((2, 1, 1), n, L=(2000.0, 1000.0, 1000.0), jitter=0.0)
    m.vert[m.elem_vert[0, 7]] += np.array([40.0, -30.0, 25.0])
    gam, jac, _ = orc.geometry(n, m.elem_vert, m.vert)
    lam, mu, rho = W.homogeneous_model(m)
    nt, dt = 40, 0.01
    se = np.array([1], np.int32); sx = np.array([[0.3, -0.2, 0.1]])
    sd = np.array([[0.2, 0.5, 1.0]])
    stf = W.ricker(8.0, 0.1, dt, nt + 1)[None, :]
    re = np.array([0, 1], np.int32); rx = np.array([[0.5, 0.5, 1.0], [-1.0, 1.0, -1.0]])
    out = orc.forward(n, m.ibool, gam, jac, lam, mu, rho, m.nglob, dt, nt, se, sx, sd, stf, re, rx,
                      want_history=True)
    K = indep.dense_stiffness(n, m.ibool, m.elem_vert, m.vert, lam, mu, m.nglob)
    M = np.repeat(indep.mass_numpy(n, m.ibool, m.elem_vert, m.vert, rho, m.nglob), 3)
    xi, _ = indep.gll_numpy(n)

    def lag(x):
        return np.array([np.prod([(x - xi[mm]) / (xi[a] - xi[mm]) for mm in range(n) if mm != a]) for a in range(n)])

    def pt_weights(r):
        lx, ly, lz = lag(r[0]), lag(r[1]), lag(r[2])
        return np.einsum("k,j,i->kji", lz, ly, lx).ravel()

    fvec = np.zeros((nt + 1, m.nglob, 3))
    wsrc = pt_weights(sx[0])
    for t in range(nt + 1):
        np.add.at(fvec[t], m.ibool[1], stf[0, t] * wsrc[:, None] * sd[0][None, :])
    fvec = fvec.reshape(nt + 1, -1)
    u = np.zeros((nt + 1, 3 * m.nglob))
    u[1] = 0.5 * dt * dt * fvec[0] / M
    for t in range(1, nt):
        u[t + 1] = 2 * u[t] - u[t - 1] + dt * dt * (fvec[t] - K @ u[t]) / M
    np.testing.assert_allclose(out["uhist"].reshape(nt + 1, -1), u, rtol=1e-9, atol=1e-9 * np.abs(u).max())
    # receivers: Lagrange interpolation of the nodal displacement
    for r in range(2):
        wr = pt_weights(rx[r])
        s = np.einsum("q,tqc->ct", wr, u.reshape(nt + 1, m.nglob, 3)[:, m.ibool[re[r]], :])[:, 1:]
        np.testing.assert_allclose(out["seis"][r], s, rtol=1e-9, atol=1e-9 * np.abs(s).max())


def test_node_receiver_reads_node(orc):
    wl = W.cube_homogeneous(ne=2, n=5, nt=20, dt=0.02)
    m = wl.mesh
    gam, jac, _ = orc.geometry(5, m.elem_vert, m.vert)
    re = np.array([3], np.int32); rx = np.array([[-1.0, 1.0, 1.0]])
    out = orc.forward(5, m.ibool, gam, jac, wl.lam, wl.mu, wl.rho, m.nglob, wl.dt, wl.nt,
                      wl.src_elem, wl.src_xi, wl.src_dir, wl.stf, re, rx, want_history=True)
    q = 0 + 5 * (4 + 5 * 4)
    g = m.ibool[3, q]
    np.testing.assert_array_equal(out["seis"][0], out["uhist"][1:, g, :].T)


def _reciprocity_problem(n=4):
    m = W.box_mesh((2, 2, 2), n, (300.0, 260.0, 220.0), jitter=0.12, seed=11)
    rng = np.random.default_rng(2)
    shape = (m.nspec, n ** 3)
    lam = 7.5e9 * rng.uniform(0.8, 1.2, shape)
    mu = 7.5e9 * rng.uniform(0.8, 1.2, shape)
    rho = 2500.0 * rng.uniform(0.8, 1.2, shape)
    pa = (np.array([1], np.int32), np.array([[0.31, -0.42, 0.17]]))   # interior points only
    pb = (np.array([6], np.int32), np.array([[-0.25, 0.38, -0.61]]))
    return m, lam, mu, rho, pa, pb


def test_source_receiver_reciprocity(orc):
    """G_ij(B, A) = G_ji(A, B): the component i recorded at B for a force
    along j at A equals the component j at A for a force along i at B, to
    rounding, because K and M are symmetric and the source injects with the
    transpose of the receiver interpolation (same Lagrange weights).  A
    source or receiver weighted differently, or a non-symmetric operator,
    breaks it."""
    m, lam, mu, rho, (ea, xa), (eb, xb) = _reciprocity_problem()
    gam, jac, _ = orc.geometry(m.n, m.elem_vert, m.vert)
    dt, nt = 2e-4, 800  # A and B are about 207 m apart: P arrives after 0.07 s, S after 0.12 s
    stf = W.ricker(30.0, 0.04, dt, nt + 1)[None, :]
    for i, j in ((0, 2), (1, 1), (2, 0)):
        dj = np.eye(3)[[j]]; di = np.eye(3)[[i]]
        ab = orc.forward(m.n, m.ibool, gam, jac, lam, mu, rho, m.nglob, dt, nt, ea, xa, dj, stf, eb, xb)["seis"][0, i]
        ba = orc.forward(m.n, m.ibool, gam, jac, lam, mu, rho, m.nglob, dt, nt, eb, xb, di, stf, ea, xa)["seis"][0, j]
        assert np.abs(ab).max() > 0
        np.testing.assert_allclose(ab, ba, rtol=0, atol=1e-10 * np.abs(ab).max())
