"""FP64 CPU oracle for the scalar (acoustic) SEM operator and for the
paper's equal-accuracy (h, p) experiment -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may import this module; the HIP library never does and
shares no code with it.  GLL nodes, weights, D and the per-point geometry
come from :mod:`oracle.oracle` (the pinned C oracle).

Reading of the acoustic problem.  The paper selects its equal-accuracy
(h, p) pairs with SPECFEM3D's acoustic solver in a homogeneous medium
(Sec. V-C): density 1000 kg/m^3, P speed 1500 m/s, a 20 Hz Ricker source,
second-order Newmark, the waveform error in the energy norm after 8 s of
propagation, dt = 1e-4 s.  The field is taken here as the pressure p of

    (1/kappa) p_tt = div(rho^-1 grad p) + s(t) delta(x - x_s),
    kappa = rho c^2,

whose GLL weak form (Sec. II-B quadrature) gives the lumped mass
M_g = sum_{(e,q) -> g} W_q / kappa_q and the stiffness
K_gh = sum_e sum_q W_q rho_q^-1 grad phi_g . grad phi_h, W_q = w_i w_j w_k det J:
the elastic operator's three forward and three transpose contractions with
one component and the flux (W / rho) Gamma^T Gamma grad_ref p in place of the
stress.

The propagation experiment is run in a rod: one element in y and z, natural
(zero-flux) boundaries everywhere, a uniform plane source on the end face
x = 0.  A field that is constant over the cross-section stays so, and the 3-D
GLL operator restricted to such fields is the 1-D GLL operator along x
(mass and stiffness both carry the same face quadrature weights), so the rod
reproduces axis-direction propagation exactly; the paper records its
stations along one axis.  Its closed-form solution is the half-line Green's
function: for a boundary source s(t) on a zero-flux end,
p(x, t) = rho c S(t - x / c) with S' = s, and for the Ricker
s(t) = (1 - 2 a (t - t0)^2) exp(-a (t - t0)^2), a = (pi f0)^2,
S(t) = (t - t0) exp(-a (t - t0)^2).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from oracle import oracle as O

# The paper's acoustic medium and source (Sec. V-C).
RHO = 1000.0
VP = 1500.0
F0 = 20.0
DT = 1e-4
T_PROP = 8.0
EPS = 0.01


def _reshape(n: int, a):
    """[nspec, n^3] in local order q = i + n (j + n k) -> [nspec, k, j, i]."""
    return a.reshape(a.shape[0], n, n, n)


# ---------------------------------------------------------------------------
# 3-D operator
# ---------------------------------------------------------------------------

def weights3(n: int, jac):
    """W_q = w_i w_j w_k det J_q, [nspec, n^3]."""
    _, w = O.gll(n)
    wq = (w[None, None, :] * w[None, :, None] * w[:, None, None]).ravel()  # [k][j][i]
    return wq[None, :] * jac


def force(n: int, ibool, gam, jac, rho, p, nglob: int):
    """f = -K p for the scalar operator, [nglob] (FP64).

    For every element and point: reference derivatives of p with D along
    xi, eta, zeta (Sec. II-B), the physical gradient through Gamma = J^-1,
    the flux Phi_d = (W / rho) sum_b grad_b Gamma_db, the transpose
    contractions with D^T, and the scatter-add into f."""
    D = O.dmatrix(n)
    ib = np.asarray(ibool)
    P = _reshape(n, np.asarray(p, dtype=np.float64)[ib])
    dxi = np.einsum("ia,ekja->ekji", D, P)
    deta = np.einsum("ja,ekai->ekji", D, P)
    dzeta = np.einsum("ka,eaji->ekji", D, P)
    nspec = ib.shape[0]
    dref = np.stack([dxi.reshape(nspec, -1), deta.reshape(nspec, -1), dzeta.reshape(nspec, -1)], axis=-1)
    grad = np.einsum("eqd,eqdb->eqb", dref, gam)
    wr = weights3(n, jac) / np.asarray(rho, dtype=np.float64)
    phi = np.einsum("eqb,eqdb->eqd", grad, gam) * wr[..., None]
    px = _reshape(n, phi[..., 0]); py = _reshape(n, phi[..., 1]); pz = _reshape(n, phi[..., 2])
    F = -(np.einsum("ai,ekja->ekji", D, px) + np.einsum("aj,ekai->ekji", D, py)
          + np.einsum("ak,eaji->ekji", D, pz))
    f = np.zeros(nglob)
    np.add.at(f, ib.ravel(), F.reshape(-1))
    return f


def mass(n: int, ibool, jac, kappa, nglob: int):
    """M_g = sum W / kappa (the lumped GLL mass with density 1/kappa)."""
    return O.mass(n, ibool, jac, 1.0 / np.asarray(kappa, dtype=np.float64), nglob)


def interp_weights(n: int, ibool, elem, xi):
    """Nodes and Lagrange weights l_i l_j l_k (Sec. II-B product formula) of
    points given as (element, reference coordinates): ([m, n^3], [m, n^3])."""
    ib = np.asarray(ibool)
    nodes = np.zeros((len(elem), n ** 3), dtype=np.int64)
    wts = np.zeros((len(elem), n ** 3))
    for r, (e, x) in enumerate(zip(elem, np.asarray(xi, dtype=np.float64).reshape(-1, 3))):
        lx, ly, lz = (O.lagrange(n, float(v)) for v in x)
        nodes[r] = ib[e]
        wts[r] = (lz[:, None, None] * ly[None, :, None] * lx[None, None, :]).ravel()
    return nodes, wts


def forward(n: int, ibool, gam, jac, kappa, rho, nglob: int, dt: float, nt: int,
            src_elem, src_xi, stf, rec_elem, rec_xi, want_energy: bool = False):
    """Explicit Newmark run (beta = 0, gamma = 1/2; Sec. V-C second-order
    Newmark) of the scalar problem from rest, in the order: predict
    u += dt v + dt^2/2 a, v += dt/2 a; f = -K u + f_src(t_{n+1});
    a = M^-1 f; v += dt/2 a; record.  Point sources inject
    stf[s, m] l(x_s) at the nodes of their element; ``stf`` is
    [nsrc, nt + 1] sampled at t_m = m dt.  Returns ``seis`` [nrec, nt]
    (the field after each step) and, with ``want_energy``, the discrete
    energy of each step, which stays constant while no source acts."""
    minv = 1.0 / mass(n, ibool, jac, kappa, nglob)
    sn, sw = interp_weights(n, ibool, src_elem, src_xi) if len(src_elem) else (None, None)
    rn, rw = interp_weights(n, ibool, rec_elem, rec_xi)
    stf = np.asarray(stf, dtype=np.float64).reshape(len(src_elem), nt + 1) if len(src_elem) else None
    M = 1.0 / minv

    def fsrc(m):
        f = np.zeros(nglob)
        if stf is not None:
            np.add.at(f, sn.ravel(), (stf[:, m][:, None] * sw).ravel())
        return f

    u = np.zeros(nglob); v = np.zeros(nglob)
    a = minv * fsrc(0)
    fint = np.zeros(nglob)  # -K u^0
    seis = np.zeros((len(rec_elem), nt))
    energy = np.zeros(nt) if want_energy else None
    for m in range(nt):
        u_old, f_old = u, fint
        u = u + dt * v + 0.5 * dt * dt * a
        v = v + 0.5 * dt * a
        fint = force(n, ibool, gam, jac, rho, u, nglob)
        a = minv * (fint + fsrc(m + 1))
        v = v + 0.5 * dt * a
        seis[:, m] = (u[rn] * rw).sum(axis=1)
        if want_energy:
            # E^{m+1/2} = 1/2 vh^T M vh + 1/2 (u^{m+1})^T K u^m, vh = (u^{m+1} - u^m) / dt:
            # constant while no source acts
            vh = (u - u_old) / dt
            energy[m] = 0.5 * float(np.sum(M * vh * vh)) - 0.5 * float(np.dot(u, f_old))
    out = {"seis": seis}
    if want_energy:
        out["energy"] = energy
    return out


# ---------------------------------------------------------------------------
# 1-D rod (axis propagation) and the closed-form solution
# ---------------------------------------------------------------------------

def rod_operator(n: int, h: float, ne: int, c: float = VP, rho: float = RHO, periodic: bool = False):
    """1-D GLL operator on [0, ne h]: node coordinates x [ne N + 1] (ne N
    when ``periodic``: the last node wraps onto the first), lumped mass M
    (density 1/kappa) and the sparse stiffness K (weight 1/rho), element by
    element: M_e = (h/2) w / kappa, K_e = (2/h) rho^-1 D^T diag(w) D."""
    N = n - 1
    xi, w = O.gll(n)
    D = O.dmatrix(n)
    kappa = rho * c * c
    G = ne * N if periodic else ne * N + 1
    x = np.empty(G)
    Mg = np.zeros(G)
    ke = (2.0 / h) / rho * (D.T @ np.diag(w) @ D)
    rows, cols, vals = [], [], []
    for e in range(ne):
        g = (e * N + np.arange(n)) % G
        x[g[:-1]] = e * h + 0.5 * h * (xi[:-1] + 1.0)
        if not periodic and e == ne - 1:
            x[g[-1]] = ne * h
        Mg[g] += 0.5 * h * w / kappa
        rows.append(np.repeat(g, n)); cols.append(np.tile(g, n)); vals.append(ke.ravel())
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(G, G))
    return x, Mg, K


def ricker(t, f0: float = F0, t0: float | None = None):
    """s(t) = (1 - 2 a tau^2) exp(-a tau^2), a = (pi f0)^2, tau = t - t0 (t0 = 1.2 / f0)."""
    t0 = 1.2 / f0 if t0 is None else t0
    a = (math.pi * f0) ** 2
    tau = np.asarray(t, dtype=np.float64) - t0
    return (1.0 - 2.0 * a * tau * tau) * np.exp(-a * tau * tau)


def rod_analytic(x: float, t, c: float = VP, rho: float = RHO, f0: float = F0, t0: float | None = None):
    """Closed-form field of a Ricker boundary source on the zero-flux end of
    a half-line: p = rho c S(t - x/c), S(tau) = (tau - t0) exp(-a (tau - t0)^2)."""
    t0 = 1.2 / f0 if t0 is None else t0
    a = (math.pi * f0) ** 2
    tau = np.asarray(t, dtype=np.float64) - x / c - t0
    return rho * c * tau * np.exp(-a * tau * tau)


def rod_setup(n: int, h: float, x_rec: float, t_end: float, dt: float = DT, c: float = VP, f0: float = F0):
    """Rod length, element count and step count for a station at x_rec
    recorded until t_end: the rod reaches past the station far enough that
    the echo from its far end (path 2 L - x_rec) arrives after t_end."""
    length = max(0.5 * (x_rec + c * t_end) + 2.4 * c / f0, x_rec + 2.0 * h)
    ne = int(math.ceil(length / h))
    nt = int(math.ceil(t_end / dt - 1e-9))
    return ne, nt


def rod_run(n: int, h: float, x_rec: float, t_end: float, dt: float = DT, c: float = VP,
            rho: float = RHO, f0: float = F0, t0: float | None = None):
    """FP64 Newmark run of the 1-D rod (same step order as :func:`forward`)
    with the plane Ricker source (unit force per unit area) on the node
    x = 0; returns (t [nt], trace at x_rec [nt]) with t_m = (m + 1) dt."""
    ne, nt = rod_setup(n, h, x_rec, t_end, dt, c, f0)
    x, Mg, K = rod_operator(n, h, ne, c, rho)
    minv = 1.0 / Mg
    # receiver: Lagrange weights inside its element
    N = n - 1
    e = min(int(x_rec // h), ne - 1)
    lw = O.lagrange(n, 2.0 * (x_rec - e * h) / h - 1.0)
    rn = e * N + np.arange(n)
    s = ricker(np.arange(nt + 1) * dt, f0, t0)
    u = np.zeros(len(x)); v = np.zeros(len(x))
    a = np.zeros(len(x)); a[0] = minv[0] * s[0]
    tr = np.zeros(nt)
    hdt, hdt2 = 0.5 * dt, 0.5 * dt * dt
    for m in range(nt):
        u += dt * v + hdt2 * a
        v += hdt * a
        f = -(K @ u)
        f[0] += s[m + 1]
        a = minv * f
        v += hdt * a
        tr[m] = lw @ u[rn]
    return (np.arange(nt) + 1) * dt, tr


def energy_error(w, w_th) -> float:
    """The paper's waveform error: int (w - w_th)^2 dt / int w_th^2 dt
    (uniform samples, so the dt cancels)."""
    w = np.asarray(w, dtype=np.float64); w_th = np.asarray(w_th, dtype=np.float64)
    return float(np.sum((w - w_th) ** 2) / np.sum(w_th ** 2))


def window(x_rec: float, c: float = VP, f0: float = F0, t0: float | None = None) -> float:
    """End of the recording at a station x_rec: the direct pulse has passed
    (its peak, at x_rec / c + t0, lies 1.2 / f0 + 1 / f0 earlier)."""
    t0 = 1.2 / f0 if t0 is None else t0
    return x_rec / c + t0 + 1.2 / f0 + 1.0 / f0


def rod_error(n: int, h: float, x_rec: float = VP * T_PROP, dt: float = DT, t0: float | None = None) -> float:
    """Energy-norm error of the rod's trace at x_rec against the closed form."""
    t, tr = rod_run(n, h, x_rec, window(x_rec, t0=t0), dt, t0=t0)
    return energy_error(tr, rod_analytic(x_rec, t, t0=t0))


def iso_h(n: int, hs, eps: float = EPS, x_rec: float = VP * T_PROP, dt: float = DT):
    """Largest element size among the ascending candidates ``hs`` whose rod
    error stays below ``eps``, scanning upwards until the first failure;
    returns (h, {h: error})."""
    errs = {}
    best = None
    for h in sorted(hs):
        errs[h] = rod_error(n, h, x_rec, dt)
        if errs[h] < eps:
            best = h
        else:
            break
    return best, errs
