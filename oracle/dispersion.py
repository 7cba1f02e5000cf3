"""Bloch dispersion analysis of the SEM elastic operator -- TEST INFRASTRUCTURE.

Plane waves on the infinite lattice of identical cubic elements of side h:
restricted to Bloch-periodic fields, u(x + h e_a) = exp(i k_a h) u(x), the
semi-discrete operator M u'' = -K u (Sec. II-B: GLL quadrature, lumped mass,
stiffness of the weak form) becomes a 3N^3 x 3N^3 Hermitian generalized
eigenproblem K(k) U = omega^2 M(k) U for each wave vector k.  It is
assembled from one element's stiffness (columns of the oracle's force
operator) and lumped mass, so its eigenvalues are the exact frequencies of
the discrete operator the oracle implements.  Only tests use this module.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.linalg

from . import oracle as O


def _cube(n: int, h: float):
    """One cubic element of side h: identity numbering, corners a + 2b + 4c."""
    n3 = n ** 3
    ibool = np.arange(n3, dtype=np.int32)[None, :]
    vert = np.array([[a * h, b * h, c * h] for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=np.float64)
    elem_vert = np.arange(8, dtype=np.int32)[None, :]
    return ibool, vert, elem_vert


def element_matrices(n: int, h: float, lam: float, mu: float, rho: float):
    """Element stiffness K_e [3 n^3, 3 n^3] (K u = -f, component fastest) and
    lumped mass m_e [n^3] of a homogeneous cubic element."""
    n3 = n ** 3
    ibool, vert, elem_vert = _cube(n, h)
    gam, jac, _ = O.geometry(n, elem_vert, vert)
    L = np.full((1, n3), float(lam))
    Mu = np.full((1, n3), float(mu))
    R = np.full((1, n3), float(rho))
    K = np.zeros((3 * n3, 3 * n3))
    u = np.zeros((n3, 3))
    for col in range(3 * n3):
        u.flat[col] = 1.0
        K[:, col] = -O.force(n, ibool, gam, jac, L, Mu, u, n3).ravel()
        u.flat[col] = 0.0
    m = O.mass(n, ibool, jac, R, n3)
    return K, m


def cell_map(n: int):
    """For each element-local point q: its node in the periodic cell
    r = (i mod N, j mod N, k mod N) and the cell offset (i // N, j // N, k // N)."""
    N = n - 1
    q = np.arange(n ** 3)
    i, j, k = q % n, (q // n) % n, q // (n * n)
    r = (i % N) + N * ((j % N) + N * (k % N))
    off = np.stack([i // N, j // N, k // N], axis=1)
    return r, off


def cell_coordinates(n: int, h: float):
    """Coordinates of the N^3 cell nodes inside the cell [0, h)^3."""
    xi, _ = O.gll(n)
    x = (xi[:-1] + 1.0) * 0.5 * h
    N = n - 1
    r = np.arange(N ** 3)
    return np.stack([x[r % N], x[(r // N) % N], x[r // (N * N)]], axis=1)


def bloch_modes(n: int, h: float, Ke, me, kvec):
    """Frequencies omega (ascending) and M-orthonormal eigenvectors
    [3 N^3, 3 N^3] (cell node fastest in blocks of 3 components) of the
    Bloch-reduced operator at wave vector kvec."""
    N = n - 1
    r, off = cell_map(n)
    ph = np.exp(1j * h * (off @ np.asarray(kvec, dtype=np.float64)))
    n3, nr = n ** 3, N ** 3
    P = np.zeros((3 * n3, 3 * nr), dtype=np.complex128)
    q = np.arange(n3)
    for c in range(3):
        P[3 * q + c, 3 * r + c] = ph
    Kr = P.conj().T @ Ke @ P
    Kr = 0.5 * (Kr + Kr.conj().T)
    mr = np.zeros(nr)
    np.add.at(mr, r, me)
    Mr = np.repeat(mr, 3)
    w2, V = scipy.linalg.eigh(Kr, np.diag(Mr))
    return np.sqrt(np.clip(w2, 0.0, None)), V, Mr


def plane_wave(n: int, h: float, kvec, pol):
    """pol * exp(i k.x) sampled at the cell nodes (3 N^3, component fastest)."""
    x = cell_coordinates(n, h)
    return (np.exp(1j * (x @ np.asarray(kvec, dtype=np.float64)))[:, None]
            * np.asarray(pol, dtype=np.float64)[None, :]).ravel()


def on_zone_boundary(kvec, h: float, tol: float = 1e-9) -> bool:
    """k and -k are the same Bloch vector when every k_a h is a multiple of pi."""
    t = np.asarray(kvec, dtype=np.float64) * h / np.pi
    return bool(np.all(np.abs(t - np.round(t)) <= tol))


def _eigenspaces(w, rtol=1e-8):
    """Index groups of equal frequency (degenerate eigenspaces: the two S
    polarisations on a symmetry axis, the cubic images of a mode)."""
    groups, j = [], 0
    scale = max(float(w[-1]), 1e-300)
    while j < len(w):
        m = j + 1
        while m < len(w) and w[m] - w[j] <= rtol * scale:
            m += 1
        groups.append(np.arange(j, m))
        j = m
    return groups


def plane_wave_branches(n: int, h: float, Ke, me, kvec, pols, share: float = 0.1):
    """The discrete modes that carry the plane wave pols[0] * exp(i k.x),
    the polarisations `pols` being orthonormal and spanning the wave type
    (one for P, the two transverse ones for S).

    Every eigenspace gets the M-weighted squared overlap with the span of
    the plane waves pol * exp(i k.x), pol in pols, per polarisation; those
    holding at least `share` of it are the wave's branches: one travelling
    mode per polarisation (both quasi-S polarisations for S) or, on a zone
    boundary, two standing modes of slightly different frequency, while the
    sampling error of the plane wave on the GLL nodes leaves O(1e-3) in the
    others.  Returns (branches, captured): branches is a list of (omega,
    mode, weight, weight0) sorted by omega, `mode` the M-normalised
    M-projection of the plane wave pols[0] * exp(i k.x) onto the eigenspace,
    `weight` the eigenspace's share of the span, `weight0` its share of
    pols[0] * exp(i k.x) alone (`mode` is meaningful where weight0 is not
    negligible); captured is the total share of the branches (1 up to the
    sampling error)."""
    w, V, Mr = bloch_modes(n, h, Ke, me, kvec)
    pws = [plane_wave(n, h, kvec, pol) for pol in pols]
    coef = [V.conj().T @ (Mr * pw) / np.sqrt(np.sum(Mr * np.abs(pw) ** 2)) for pw in pws]
    branches, captured = [], 0.0
    for g in _eigenspaces(w):
        wt = sum(float(np.sum(np.abs(c[g]) ** 2)) for c in coef) / len(pols)
        if wt < share:
            continue
        v = V[:, g] @ coef[0][g]
        nv = np.sqrt(np.real(np.vdot(v, Mr * v)))
        wt0 = float(np.sum(np.abs(coef[0][g]) ** 2))
        branches.append((float(np.mean(w[g])), v / nv if nv > 0 else v, wt, wt0))
        captured += wt
    return sorted(branches, key=lambda t: t[0]), captured


def wave(direction, wave_type: str, lam: float, mu: float, rho: float):
    """Unit propagation direction, polarisations and continuum speed of a P
    or S plane wave in the isotropic medium."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    if wave_type == "P":
        return d, [d], float(np.sqrt((lam + 2.0 * mu) / rho))
    t1 = np.cross(d, [0.0, 0.0, 1.0]) if abs(d[2]) < 0.9 else np.cross(d, [1.0, 0.0, 0.0])
    t1 = t1 / np.linalg.norm(t1)
    t2 = np.cross(d, t1)
    return d, [t1, t2], float(np.sqrt(mu / rho))


def dispersion_error(n: int, h: float, lam: float, mu: float, rho: float, direction, ppw: float,
                     wave_type: str, Ke=None, me=None):
    """Relative frequency error omega_h / (c |k|) - 1 of a P or S plane wave
    along `direction` with ppw points per wavelength (average GLL spacing
    h / N along the propagation direction).

    Returns a dict: `error`, the overlap-weighted mean over the wave's
    branches; `branches`, the error of each branch (two quasi-S
    polarisations; two standing modes per polarisation on a zone boundary);
    `captured`; `boundary`."""
    N = n - 1
    d, pols, c = wave(direction, wave_type, lam, mu, rho)
    kmag = 2.0 * np.pi * N / (ppw * h)
    if Ke is None:
        Ke, me = element_matrices(n, h, lam, mu, rho)
    br, captured = plane_wave_branches(n, h, Ke, me, kmag * d, pols)
    errs = np.array([b[0] / (c * kmag) - 1.0 for b in br])
    wts = np.array([b[2] for b in br])
    return {"error": float(np.sum(wts * errs) / np.sum(wts)), "branches": [float(e) for e in errs],
            "captured": captured, "boundary": on_zone_boundary(kmag * d, h)}


def mode_on_lattice(n: int, h: float, v, kvec, gx, gy, gz):
    """A Bloch eigenvector v (3 N^3, component fastest) extended to the
    points with global lattice coordinates (gx, gy, gz) of a periodic box of
    cubic elements of side h: complex field [npts, 3]."""
    N = n - 1
    gx, gy, gz = (np.asarray(a, dtype=np.int64) for a in (gx, gy, gz))
    r = (gx % N) + N * ((gy % N) + N * (gz % N))
    cell = np.stack([gx // N, gy // N, gz // N], axis=-1).astype(np.float64)
    ph = np.exp(1j * h * (cell @ np.asarray(kvec, dtype=np.float64)))
    return np.asarray(v).reshape(N ** 3, 3)[r] * ph[..., None]


def lattice_coordinates(n: int, h: float, gx, gy, gz):
    """Physical coordinates of GLL lattice points (gx, gy, gz) of a regular
    box of cubic elements of side h."""
    xi, _ = O.gll(n)
    N = n - 1
    t = 0.5 * (xi[:N] + 1.0) * h

    def axis(g):
        g = np.asarray(g, dtype=np.int64)
        return (g // N) * h + t[g % N]
    return np.stack([axis(gx), axis(gy), axis(gz)], axis=-1)


def periodic_plane_wave(mesh, lam: float, mu: float, rho: float, m, wave_type: str, elem=None):
    """A P or S plane wave on a periodic box of cubic elements, with wave
    vector k = 2 pi m / L (m integer per axis, so the wave wraps).

    Returns a dict: `u0` [nglob, 3], the wave pol * cos(k.x) sampled at the
    GLL nodes; `w` [nglob, 3], M times the real part of the Bloch mode that
    carries it (projecting a displacement on `w` keeps that mode's
    coefficient only: every other eigenvector of M^{-1} K is M-orthogonal to
    it); `omega_h`, its Bloch frequency; `c`, `k` (|k|), `ppw`, `captured`."""
    n = mesh.n
    h = mesh.h[0]
    if not (mesh.periodic and np.allclose(mesh.h, h) and mesh.jitter == 0.0):
        raise ValueError("periodic_plane_wave: needs a periodic box of undistorted cubic elements")
    kvec = 2.0 * np.pi * np.asarray(m, dtype=np.float64) / np.asarray(mesh.L)
    kmag = float(np.linalg.norm(kvec))
    if on_zone_boundary(kvec, h):
        raise ValueError("periodic_plane_wave: k on a Brillouin-zone boundary")
    _, pols, c = wave(kvec, wave_type, lam, mu, rho)
    Ke, me = elem if elem is not None else element_matrices(n, h, lam, mu, rho)
    branches, captured = plane_wave_branches(n, h, Ke, me, kvec, pols)
    # the branch that carries the initialised polarisation pols[0]
    omega_h, v, _, _ = max(branches, key=lambda b: b[3])
    G = np.zeros((mesh.nglob, 3), dtype=np.int64)
    gx, gy, gz = mesh.lattice_index()
    Gs = (mesh.nex * (n - 1), mesh.ney * (n - 1), mesh.nez * (n - 1))
    for a, g in enumerate((gx, gy, gz)):
        G[mesh.ibool.ravel(), a] = g.ravel() % Gs[a]
    phi = mode_on_lattice(n, h, v, kvec, G[:, 0], G[:, 1], G[:, 2])
    X = lattice_coordinates(n, h, G[:, 0], G[:, 1], G[:, 2])
    u0 = np.cos(X @ kvec)[:, None] * pols[0][None, :]
    _, jac, _ = O.geometry(n, mesh.elem_vert, mesh.vert)
    mass = O.mass(n, mesh.ibool, jac, np.full(mesh.ibool.shape, float(rho)), mesh.nglob)
    w = mass[:, None] * np.real(phi)
    N = n - 1
    return {"u0": u0, "w": w, "omega_h": omega_h, "c": c, "k": kmag,
            "ppw": 2.0 * np.pi / kmag / (h / N), "captured": captured}


def fit_frequency(s, dt: float):
    """Frequencies of a single-mode series s_n of the explicit Newmark
    scheme (beta = 0, gamma = 1/2).  For n >= 1 the scheme satisfies
    u_{n+1} - 2 u_n + u_{n-1} = dt^2 a_n with a_n = -omega_h^2 u_n on a mode,
    so s_{n+1} + s_{n-1} = 2 C s_n with C = 1 - omega_h^2 dt^2 / 2; C is fitted
    by least squares over n >= 1.  Returns (omega_h, the frequency of the
    operator, and acos(C) / dt, that of the time-discrete run)."""
    s = np.asarray(s, dtype=np.float64)
    mid = s[1:-1]
    C = float(np.dot(s[2:] + s[:-2], mid) / (2.0 * np.dot(mid, mid)))
    return float(np.sqrt(2.0 * (1.0 - C)) / dt), float(np.arccos(C) / dt)


def newmark_free(mesh, lam, mu, rho, u0, dt: float, nt: int, weights):
    """Explicit Newmark (beta = 0, gamma = 1/2) from displacement u0 at rest,
    no sources, with the oracle's FP64 force and lumped mass; returns the
    projections sum(weights * u_n) for n = 0..nt."""
    n = mesh.n
    gam, jac, _ = O.geometry(n, mesh.elem_vert, mesh.vert)
    shape = mesh.ibool.shape
    L, Mu, R = (np.full(shape, float(x)) for x in (lam, mu, rho))
    minv = 1.0 / O.mass(n, mesh.ibool, jac, R, mesh.nglob)
    u = np.array(u0, dtype=np.float64)
    v = np.zeros_like(u)
    a = np.zeros_like(u)
    out = [float(np.sum(weights * u))]
    for _ in range(nt):
        u = u + dt * v + 0.5 * dt * dt * a
        v = v + 0.5 * dt * a
        a = minv[:, None] * O.force(n, mesh.ibool, gam, jac, L, Mu, u, mesh.nglob)
        v = v + 0.5 * dt * a
        out.append(float(np.sum(weights * u)))
    return np.array(out)


def table(ns=(4, 5, 6, 7, 8, 9), ppw: float = 5.0, vp: float = 3000.0, vs: float = 1732.0,
          rho: float = 2500.0, directions=((1, 0, 0), (1, 1, 1))):
    """Relative dispersion errors of P and S waves at `ppw` points per
    wavelength for each order: rows (n, direction, wave, error, branch
    errors, on a zone boundary)."""
    mu = rho * vs * vs
    lam = rho * vp * vp - 2.0 * mu
    rows = []
    for n in ns:
        Ke, me = element_matrices(n, 100.0, lam, mu, rho)
        for d in directions:
            for wt in "PS":
                r = dispersion_error(n, 100.0, lam, mu, rho, d, ppw, wt, Ke, me)
                rows.append((n, tuple(d), wt, r["error"], r["branches"], r["boundary"]))
    return rows


if __name__ == "__main__":
    for n, d, wt, e, br, bd in table():
        extra = "  standing modes " + ", ".join(f"{b:+.3e}" for b in br) if bd else ""
        print(f"n={n} {d} {wt}: {e:+.3e}{extra}")


@functools.lru_cache(maxsize=None)
def _axis_element(n: int):
    """GLL nodes, weights and the 1-D element stiffness (h = c = 1)."""
    xi, w = O.gll(n)
    D = O.dmatrix(n)  # D[a, b] = l'_b(xi_a)
    return xi, w, 2.0 * (D.T * w) @ D


def axis_omega(n: int, kh: float) -> float:
    """omega h / c of the plane wave exp(i k x) along a lattice axis, for
    the 1-D GLL spectral element lattice (element size h, lumped GLL mass,
    weak-form stiffness): the N x N Bloch problem.  A P or S wave along an
    axis of the 3-D operator reduces exactly to it (cross-axis terms cancel
    between periodic neighbours), for every wave speed c."""
    N = n - 1
    xi, w, Ke = _axis_element(n)
    me = 0.5 * w
    r = np.arange(n) % N
    ph = np.exp(1j * kh * (np.arange(n) // N))
    P = np.zeros((n, N), dtype=np.complex128)
    P[np.arange(n), r] = ph
    Kr = P.conj().T @ Ke @ P
    mr = np.bincount(r, weights=me, minlength=N)
    s = 1.0 / np.sqrt(mr)
    A = s[:, None] * Kr * s[None, :]
    ev, V = np.linalg.eigh(0.5 * (A + A.conj().T))
    x = 0.5 * (xi[:N] + 1.0)
    pw = np.sqrt(mr) * np.exp(1j * kh * x)
    j = int(np.argmax(np.abs(V.conj().T @ pw)))
    return float(np.sqrt(max(ev[j], 0.0)))


def axis_error(n: int, ppw: float) -> float:
    """Relative phase-velocity error omega_h / (c k) - 1 along a lattice axis
    at ppw GLL points per wavelength (average spacing h / N)."""
    kh = 2.0 * np.pi * (n - 1) / ppw
    return axis_omega(n, kh) / kh - 1.0


def iso_accuracy_ppw(n: int, eps: float, lo: float = 2.0, hi: float = 2000.0) -> float:
    """Fewest points per wavelength at which |axis_error| stays <= eps for
    every finer resolution.  The error is smooth except next to the
    Brillouin-zone boundaries k h = m pi (ppw = 2N/m), where the travelling
    branch bends towards a small band gap; candidates are a geometric grid
    plus points packed log-densely on both sides of every boundary, and the
    last candidate above eps is refined by bisection towards the next one."""
    N = n - 1
    cand = list(np.geomspace(lo, hi, 4000))
    for m in range(1, N):
        pb = 2.0 * N / m
        for d in np.geomspace(1e-7, 3e-2, 40):
            cand += [pb * (1.0 - d), pb * (1.0 + d)]
    cand = np.array(sorted(p for p in cand if lo <= p <= hi))
    bad = np.array([abs(axis_error(n, p)) > eps for p in cand])
    if bad[-1]:
        raise ValueError(f"iso_accuracy_ppw: error above {eps} at {hi} ppw")
    if not bad.any():
        return float(lo)
    last = int(np.nonzero(bad)[0][-1])
    a, b = cand[last], cand[last + 1]  # error > eps at a, <= eps at b
    for _ in range(60):
        mid = 0.5 * (a + b)
        if abs(axis_error(n, mid)) > eps:
            a = mid
        else:
            b = mid
    return float(b)


def axis_mode(n: int, kh: float):
    """axis_omega with its mode: (omega h / c, v, mr), v the M-normalised
    Bloch eigenvector over the N cell nodes of the 1-D lattice (h = c = 1)
    and mr the lumped cell mass."""
    N = n - 1
    xi, w, Ke = _axis_element(n)
    r = np.arange(n) % N
    ph = np.exp(1j * kh * (np.arange(n) // N))
    P = np.zeros((n, N), dtype=np.complex128)
    P[np.arange(n), r] = ph
    Kr = P.conj().T @ Ke @ P
    mr = np.bincount(r, weights=0.5 * w, minlength=N)
    s = 1.0 / np.sqrt(mr)
    A = s[:, None] * Kr * s[None, :]
    ev, V = np.linalg.eigh(0.5 * (A + A.conj().T))
    x = 0.5 * (xi[:N] + 1.0)
    pw = np.sqrt(mr) * np.exp(1j * kh * x)
    j = int(np.argmax(np.abs(V.conj().T @ pw)))
    return float(np.sqrt(max(ev[j], 0.0))), s * V[:, j], mr


def periodic_axis_wave(mesh, lam: float, mu: float, rho: float, m: int, wave_type: str):
    """periodic_plane_wave for a wave along x (k = 2 pi m / L_x) from the 1-D
    Bloch analysis, for any order: the 3-D mode of an axis wave is the 1-D
    mode, uniform across the axis, times the polarisation (x for P, y for
    S).  Returns the same dict as periodic_plane_wave."""
    n = mesh.n
    N = n - 1
    h = mesh.h[0]
    if not (mesh.periodic and np.allclose(mesh.h, h) and mesh.jitter == 0.0):
        raise ValueError("periodic_axis_wave: needs a periodic box of undistorted cubic elements")
    k = 2.0 * np.pi * m / mesh.L[0]
    kh = k * h
    t = kh / np.pi
    if abs(t - round(t)) < 1e-9:
        raise ValueError("periodic_axis_wave: k on a Brillouin-zone boundary")
    pol = np.array([1.0, 0.0, 0.0]) if wave_type == "P" else np.array([0.0, 1.0, 0.0])
    c = float(np.sqrt((lam + 2.0 * mu) / rho)) if wave_type == "P" else float(np.sqrt(mu / rho))
    w1, v, _ = axis_mode(n, kh)
    G = np.zeros(mesh.nglob, dtype=np.int64)
    gx, _, _ = mesh.lattice_index()
    G[mesh.ibool.ravel()] = gx.ravel() % (mesh.nex * N)
    phi = v[G % N] * np.exp(1j * kh * (G // N))
    xi, _ = O.gll(n)
    X = (G // N) * h + 0.5 * (xi[:N][G % N] + 1.0) * h
    u0 = np.cos(k * X)[:, None] * pol[None, :]
    _, jac, _ = O.geometry(n, mesh.elem_vert, mesh.vert)
    mass = O.mass(n, mesh.ibool, jac, np.full(mesh.ibool.shape, float(rho)), mesh.nglob)
    wts = (mass * np.real(phi))[:, None] * pol[None, :]
    return {"u0": u0, "w": wts, "omega_h": w1 * c / h, "c": c, "k": k, "ppw": 2.0 * np.pi / k / (h / N),
            "captured": None}
