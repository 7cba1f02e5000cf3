"""Seeded synthetic inputs for the SEM elastic operator.

This module builds meshes, material fields, source wavelets and
source/receiver placements.  It holds none of the method's arithmetic (no GLL
points, no Jacobians, no operator): it only produces the plain arrays that
both the HIP library and the FP64 oracle take as inputs, so that the two sides
see identical data.

Conventions (also those of the library's C interface):

* element e = ex + nex*(ey + ney*ez); local point q = i + n*(j + n*k);
* structured global numbering g = (ex*N+i) + Gx*((ey*N+j) + Gy*(ez*N+k)),
  Gx = nex*N + 1, with N = n - 1 (``periodic=True`` wraps the lattice);
* corner v = a + 2b + 4c of an element sits at reference (2a-1, 2b-1, 2c-1);
* vertices are stored [nvert, 3] in FP64, z up, domain [0, Lx]x[0, Ly]x[0, Lz].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    n: int
    nex: int
    ney: int
    nez: int
    L: tuple
    ibool: np.ndarray        # int32 [nspec, n^3]
    vert: np.ndarray         # float64 [nvert, 3]
    elem_vert: np.ndarray    # int32 [nspec, 8]
    nglob: int
    jitter: float = 0.0
    periodic: bool = False
    meta: dict = field(default_factory=dict)

    @property
    def nspec(self) -> int:
        return self.ibool.shape[0]

    @property
    def h(self):
        return (self.L[0] / self.nex, self.L[1] / self.ney, self.L[2] / self.nez)

    def lattice_index(self):
        """(gx, gy, gz) lattice coordinates of every element-local point, [nspec, n^3] each."""
        N = self.n - 1
        e = np.arange(self.nspec)
        ex = e % self.nex
        ey = (e // self.nex) % self.ney
        ez = e // (self.nex * self.ney)
        q = np.arange(self.n ** 3)
        i = q % self.n
        j = (q // self.n) % self.n
        k = q // (self.n * self.n)
        gx = ex[:, None] * N + i[None, :]
        gy = ey[:, None] * N + j[None, :]
        gz = ez[:, None] * N + k[None, :]
        return gx, gy, gz


def box_mesh(ne, n: int, L=4000.0, jitter: float = 0.0, seed: int = 0,
             periodic: bool = False) -> Mesh:
    """Structured hexahedral box of ne = (nex, ney, nez) (or an int) elements.

    ``jitter`` moves every interior vertex of the (ne+1)^3 lattice by an
    independent U(-jitter*h, +jitter*h) per coordinate (seeded); boundary
    vertices stay put so the faces remain flat.
    """
    if np.isscalar(ne):
        ne = (int(ne),) * 3
    nex, ney, nez = (int(x) for x in ne)
    if np.isscalar(L):
        L = (float(L),) * 3
    L = tuple(float(x) for x in L)
    N = n - 1
    if periodic:
        Gx, Gy, Gz = nex * N, ney * N, nez * N
    else:
        Gx, Gy, Gz = nex * N + 1, ney * N + 1, nez * N + 1
    nglob = Gx * Gy * Gz

    e = np.arange(nex * ney * nez, dtype=np.int64)
    ex = e % nex
    ey = (e // nex) % ney
    ez = e // (nex * ney)
    q = np.arange(n ** 3)
    i = q % n
    j = (q // n) % n
    k = q // (n * n)
    gx = ex[:, None] * N + i[None, :]
    gy = ey[:, None] * N + j[None, :]
    gz = ez[:, None] * N + k[None, :]
    if periodic:
        gx %= Gx; gy %= Gy; gz %= Gz
    ibool = (gx + Gx * (gy + Gy * gz)).astype(np.int32)

    vx, vy, vz = nex + 1, ney + 1, nez + 1
    I, J, K = np.meshgrid(np.arange(vx), np.arange(vy), np.arange(vz), indexing="ij")
    I = I.transpose(2, 1, 0).ravel(); J = J.transpose(2, 1, 0).ravel(); K = K.transpose(2, 1, 0).ravel()
    h = (L[0] / nex, L[1] / ney, L[2] / nez)
    vert = np.stack([I * h[0], J * h[1], K * h[2]], axis=1).astype(np.float64)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter, jitter, size=vert.shape) * np.array(h)
        interior = (I > 0) & (I < nex) & (J > 0) & (J < ney) & (K > 0) & (K < nez)
        vert[interior] += d[interior]
    corners = []
    for c in range(2):
        for b in range(2):
            for a in range(2):
                corners.append((ex + a) + vx * ((ey + b) + vy * (ez + c)))
    elem_vert = np.stack(corners, axis=1).astype(np.int32)
    return Mesh(n=n, nex=nex, ney=ney, nez=nez, L=L, ibool=ibool, vert=vert,
                elem_vert=elem_vert, nglob=int(nglob), jitter=jitter, periodic=periodic)


def lame(vp, vs, rho):
    """Lame parameters from wave speeds: lambda = rho (vp^2 - 2 vs^2), mu = rho vs^2."""
    vp = np.asarray(vp, dtype=np.float64); vs = np.asarray(vs, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    return rho * (vp * vp - 2.0 * vs * vs), rho * vs * vs


def homogeneous_model(mesh: Mesh, vp=3000.0, vs=1732.0, rho=2500.0):
    """lambda, mu, rho per element-local point, [nspec, n^3] each (FP64)."""
    shape = (mesh.nspec, mesh.n ** 3)
    lam, mu = lame(vp, vs, rho)
    return (np.full(shape, float(lam)), np.full(shape, float(mu)), np.full(shape, float(rho)))


def gaussian_random_field(shape, corr_len: float, seed: int) -> np.ndarray:
    """Seeded white noise filtered by a Gaussian kernel of correlation length
    ``corr_len`` lattice steps (covariance ~ exp(-r^2/corr_len^2)), scaled so
    that max |field| = 1 exactly."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(shape)
    F = np.fft.rfftn(z)
    ks = [np.fft.fftfreq(s) for s in shape[:-1]] + [np.fft.rfftfreq(shape[-1])]
    K2 = np.zeros(F.shape)
    for ax, kk in enumerate(ks):
        sh = [1] * len(shape)
        sh[ax] = -1
        K2 = K2 + (2 * np.pi * kk.reshape(sh)) ** 2
    # Fourier transform of exp(-r^2/l^2) ~ exp(-k^2 l^2 / 4); amplitude filter is its sqrt
    F *= np.exp(-K2 * corr_len ** 2 / 8.0)
    out = np.fft.irfftn(F, s=shape, axes=list(range(len(shape))))
    return out / np.max(np.abs(out))


def layered_model(mesh: Mesh, vp_layers=(6000.0, 4000.0, 2500.0), vpvs=1.73, rho=2500.0,
                  grf_amp: float = 0.0, grf_seed: int = 12850, grf_corr_elems: float = 4.0,
                  anomaly: dict | None = None):
    """Flat layers of equal thickness, listed bottom to top.

    A point belongs to the layer of its element's vertical index (interfaces
    on element faces, element layer index = floor(ez * nlayers / nez)).
    ``grf_amp`` multiplies vp and vs by (1 + grf_amp * field) with the field
    of :func:`gaussian_random_field` on the global lattice (so shared nodes
    agree); correlation length ``grf_corr_elems`` elements.  ``anomaly`` =
    {"center": (x,y,z), "radius": R, "amp": a} multiplies vp, vs by
    (1 + a exp(-|x-c|^2/R^2)), evaluated at the nominal lattice position
    (gx h/N, gy h/N, gz h/N) of each point (equispaced, so shared nodes agree).
    """
    n3 = mesh.n ** 3
    e = np.arange(mesh.nspec)
    ez = e // (mesh.nex * mesh.ney)
    nl = len(vp_layers)
    layer = (ez * nl) // mesh.nez
    vp = np.asarray(vp_layers, dtype=np.float64)[layer][:, None] * np.ones((1, n3))
    if grf_amp:
        N = mesh.n - 1
        shape = (mesh.nez * N + 1, mesh.ney * N + 1, mesh.nex * N + 1)
        fld = gaussian_random_field(shape, grf_corr_elems * N, grf_seed).ravel()
        gx, gy, gz = mesh.lattice_index()
        lat = gx + shape[2] * (gy + shape[1] * gz)
        vp = vp * (1.0 + grf_amp * fld[lat])
    if anomaly is not None:
        N = mesh.n - 1
        gx, gy, gz = mesh.lattice_index()
        h = mesh.h
        c = np.asarray(anomaly["center"], dtype=np.float64)
        r2 = ((gx * h[0] / N - c[0]) ** 2 + (gy * h[1] / N - c[1]) ** 2
              + (gz * h[2] / N - c[2]) ** 2)
        vp = vp * (1.0 + anomaly["amp"] * np.exp(-r2 / anomaly["radius"] ** 2))
    vs = vp / vpvs
    rho_a = np.full_like(vp, float(rho))
    lam, mu = lame(vp, vs, rho_a)
    return lam, mu, rho_a


def ricker(f0: float, t0: float, dt: float, nsamples: int, amp: float = 1.0) -> np.ndarray:
    """Ricker wavelet A (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2) at t_m = m dt."""
    t = np.arange(nsamples) * dt
    a = (np.pi * f0 * (t - t0)) ** 2
    return amp * (1.0 - 2.0 * a) * np.exp(-a)


def locate_regular(mesh: Mesh, x, y, z):
    """Element and reference coordinates of physical points in an unjittered
    box (or on the flat top face of a jittered one: ``z = Lz``).  Points on an
    element boundary go to the lowest-index element that holds them."""
    pts = np.stack(np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float),
                                       np.asarray(z, float)), axis=-1).reshape(-1, 3)
    h = np.array(mesh.h)
    nel = np.array([mesh.nex, mesh.ney, mesh.nez])
    s = pts / h
    idx = np.floor(s).astype(np.int64)
    # lowest-index owner: a point exactly on a face belongs to the element below it
    on_face = (s == idx) & (idx > 0)
    idx = np.where(on_face, idx - 1, idx)
    idx = np.clip(idx, 0, nel - 1)
    ref = 2.0 * (s - idx) - 1.0
    ref = np.clip(ref, -1.0, 1.0)
    elem = idx[:, 0] + mesh.nex * (idx[:, 1] + mesh.ney * idx[:, 2])
    return elem.astype(np.int32), ref


def top_receivers_line(mesh: Mesh, count: int = 8):
    """``count`` receivers on the top face along y = Ly/2 at x = (k + 1/2) Lx/count."""
    x = (np.arange(count) + 0.5) * mesh.L[0] / count
    return locate_regular(mesh, x, np.full(count, mesh.L[1] / 2), np.full(count, mesh.L[2]))


def top_receivers_grid(mesh: Mesh, m: int):
    """m x m receivers on the top face at ((a+1/2) Lx/m, (b+1/2) Ly/m, Lz)."""
    a = (np.arange(m) + 0.5) / m
    X, Y = np.meshgrid(a * mesh.L[0], a * mesh.L[1], indexing="xy")
    return locate_regular(mesh, X.ravel(), Y.ravel(), np.full(m * m, mesh.L[2]))


def center_vertex_source(mesh: Mesh):
    """The lattice vertex nearest the domain centre, as (element, reference
    coordinates) of the lowest-index element holding it."""
    cx, cy, cz = mesh.nex // 2, mesh.ney // 2, mesh.nez // 2
    ex, ey, ez = max(cx - 1, 0), max(cy - 1, 0), max(cz - 1, 0)
    ref = np.array([[1.0 if cx > 0 else -1.0, 1.0 if cy > 0 else -1.0, 1.0 if cz > 0 else -1.0]])
    return np.array([ex + mesh.nex * (ey + mesh.ney * ez)], dtype=np.int32), ref


@dataclass
class Workload:
    """A complete synthetic run: mesh, model, sources, receivers, time axis."""
    name: str
    mesh: Mesh
    lam: np.ndarray
    mu: np.ndarray
    rho: np.ndarray
    dt: float
    nt: int
    src_elem: np.ndarray
    src_xi: np.ndarray
    src_dir: np.ndarray
    stf: np.ndarray          # [nsrc, nt+1]
    rec_elem: np.ndarray
    rec_xi: np.ndarray


def cube_homogeneous(ne=4, n=5, nt=200, dt=0.0230231, f0=10.0, jitter=0.0, seed=2606,
                     nrec=8) -> Workload:
    """Homogeneous isotropic cube, 4 km side (vp 3000, vs 1732, rho 2500), free
    surfaces, vertical Ricker point force (f0 Hz, t0 = 1.2/f0) at the centre
    vertex, ``nrec`` receivers on the top face.  Defaults: 4^3 elements,
    NGLL = 5, 200 steps, dt of Courant number 0.4."""
    m = box_mesh(ne, n, 4000.0, jitter=jitter, seed=seed)
    lam, mu, rho = homogeneous_model(m)
    se, sx = center_vertex_source(m)
    re, rx = top_receivers_line(m, nrec)
    stf = ricker(f0, 1.2 / f0, dt, nt + 1)[None, :]
    return Workload("cube_homogeneous", m, lam, mu, rho, dt, nt, se, sx,
                    np.array([[0.0, 0.0, 1.0]]), stf, re, rx)


def layered_jittered(ne=64, n=5, nt=2000, dt=None, f0=10.0, jitter=0.10, seed=2606,
                     grf_seed=12850, grf_amp=0.05, nrec=8) -> Workload:
    """Layered elastic cube (vp 6000/4000/2500 bottom to top, vp/vs = 1.73,
    rho 2500), interior vertices jittered +-``jitter``*h, +-5% Gaussian
    random field of correlation length 4 elements.  ``dt`` must be given by
    the caller (it depends on the discretisation)."""
    m = box_mesh(ne, n, 4000.0, jitter=jitter, seed=seed)
    lam, mu, rho = layered_model(m, grf_amp=grf_amp, grf_seed=grf_seed)
    se, sx = center_vertex_source(m)
    re, rx = top_receivers_line(m, nrec)
    dt = float(dt) if dt is not None else 1e-4
    stf = ricker(f0, 1.2 / f0, dt, nt + 1)[None, :]
    return Workload("layered_jittered", m, lam, mu, rho, dt, nt, se, sx,
                    np.array([[0.0, 0.0, 1.0]]), stf, re, rx)


def adjoint_layered(ne=32, n=5, nt=1000, dt=None, f0=10.0, anomaly: bool = True, nrec_side=8) -> Workload:
    """Layered cube (vp 6000/4000/2500 m/s bottom to top, vp/vs 1.73, rho 2500)
    on a regular ne^3 mesh, optionally with a -5% Gaussian velocity anomaly of
    radius 0.2 L at the centre; vertical Ricker source at (L/2, L/2, 0.2 L);
    nrec_side^2 receivers on the top face.  ``dt`` must be set by the caller
    (it depends on the discretisation)."""
    L = 4000.0
    m = box_mesh(ne, n, L)
    an = {"center": (L / 2, L / 2, L / 2), "radius": 0.2 * L, "amp": -0.05} if anomaly else None
    lam, mu, rho = layered_model(m, anomaly=an)
    se, sx = locate_regular(m, L / 2, L / 2, 0.2 * L)
    re, rx = top_receivers_grid(m, nrec_side)
    dt = float(dt) if dt is not None else 1e-3
    stf = ricker(f0, 1.2 / f0, dt, nt + 1)[None, :]
    return Workload("adjoint_layered", m, lam, mu, rho, dt, nt, se, sx, np.array([[0.0, 0.0, 1.0]]), stf, re, rx)


def fourier_modes(mesh: Mesh, nmodes_per_axis: int = 4):
    """Cosine modes b_pqr(x) = cos(p pi x/Lx) cos(q pi y/Ly) cos(r pi z/Lz),
    p, q, r in 0..nmodes_per_axis-1, at the nominal lattice position
    (gx h/N, gy h/N, gz h/N) of every element-local point: [nspec*n^3, nmodes^3]."""
    N = mesh.n - 1
    gx, gy, gz = mesh.lattice_index()
    h = mesh.h
    X = (gx * h[0] / N).ravel(); Y = (gy * h[1] / N).ravel(); Z = (gz * h[2] / N).ravel()
    k = np.arange(nmodes_per_axis)
    cx = np.cos(np.pi * np.outer(X, k) / mesh.L[0])
    cy = np.cos(np.pi * np.outer(Y, k) / mesh.L[1])
    cz = np.cos(np.pi * np.outer(Z, k) / mesh.L[2])
    B = (cz[:, :, None, None] * cy[:, None, :, None] * cx[:, None, None, :]).reshape(X.size, -1)
    return B


def perturbation_coefficients(basis, seeds, amp: float = 0.10):
    """For each seed: c ~ U(-1, 1)^64 (seeded), S = basis c, scaled so that
    max |S| over the points is amp; returns the effective coefficients
    a = amp c / max|S| [len(seeds), 64] (the perturbation is basis @ a)."""
    out = np.empty((len(seeds), basis.shape[1]))
    for t, s in enumerate(seeds):
        c = np.random.default_rng(int(s)).uniform(-1.0, 1.0, basis.shape[1])
        S = basis @ c
        out[t] = amp * c / np.max(np.abs(S))
    return out


def perturbed_models(mesh: Mesh, basis, coeffs, vp=3000.0, vs=1732.0, rho=2500.0):
    """lambda (1 + delta), mu (1 + delta), rho for delta = basis @ a, per model:
    arrays [nmodels, nspec, n^3] on the homogeneous background."""
    lam0, mu0 = lame(vp, vs, rho)
    delta = (basis @ np.asarray(coeffs).T).T.reshape(len(coeffs), mesh.nspec, mesh.n ** 3)
    lam = float(lam0) * (1.0 + delta)
    mu = float(mu0) * (1.0 + delta)
    return lam, mu, np.full_like(lam, float(rho))


@dataclass
class Rod:
    """The acoustic equal-accuracy workload: a rod of ``ne`` elements of size
    h along x and one element (side ``section``) across, natural boundaries
    everywhere; a plane source on the end face x = 0 given as one point
    source per face node; one receiver on the axis at ``x_rec``."""
    mesh: Mesh
    h: float
    section: float
    nt: int
    dt: float
    src_elem: np.ndarray   # [n^2] int32 (element 0)
    src_xi: np.ndarray     # [n^2, 3] reference coordinates (-1, xi_j, xi_k)
    src_amp: np.ndarray    # [n^2] face quadrature weight of each face node
    rec_elem: np.ndarray   # [1]
    rec_xi: np.ndarray     # [1, 3]
    stf: np.ndarray        # [n^2, nt + 1] amplitude x Ricker at t_m = m dt


def acoustic_rod(n: int, h: float, x_rec: float, t_end: float, gll_xi, gll_w, dt: float = 1e-4,
                 c: float = 1500.0, f0: float = 20.0, t0: float | None = None, section: float | None = None) -> Rod:
    """Inputs of the acoustic rod run.  The rod reaches past the station far
    enough that the echo of its far end (path 2 L - x_rec) arrives 2.4 / f0
    after t_end; the run has ceil(t_end / dt) steps.  ``gll_xi``, ``gll_w``
    are the caller's GLL nodes and weights for n points (the face node
    positions and their quadrature weights (section/2)^2 w_j w_k)."""
    t0 = 1.2 / f0 if t0 is None else t0
    section = h if section is None else float(section)
    length = max(0.5 * (x_rec + c * t_end) + 2.4 * c / f0, x_rec + 2.0 * h)
    ne = int(np.ceil(length / h))
    nt = int(np.ceil(t_end / dt - 1e-9))
    mesh = box_mesh((ne, 1, 1), n, (ne * h, section, section))
    xi = np.asarray(gll_xi, dtype=np.float64); w = np.asarray(gll_w, dtype=np.float64)
    jj, kk = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    src_xi = np.stack([-np.ones(n * n), xi[jj.ravel()], xi[kk.ravel()]], axis=1)
    amp = 0.25 * section * section * w[jj.ravel()] * w[kk.ravel()]
    e = min(int(x_rec // h), ne - 1)
    rec_xi = np.array([[2.0 * (x_rec - e * h) / h - 1.0, 0.0, 0.0]])
    stf = amp[:, None] * ricker(f0, t0, dt, nt + 1)[None, :]
    return Rod(mesh=mesh, h=float(h), section=section, nt=nt, dt=float(dt),
               src_elem=np.zeros(n * n, dtype=np.int32), src_xi=src_xi, src_amp=amp,
               rec_elem=np.array([e], dtype=np.int32), rec_xi=rec_xi, stf=stf)
