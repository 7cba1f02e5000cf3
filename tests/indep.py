"""Independent numpy re-derivations used to pin the oracle.

Nothing here calls the oracle: GLL points come from numpy's Legendre module,
the differentiation matrix from the barycentric formula, the geometry from a
numpy evaluation of the trilinear map with ``numpy.linalg.inv``, and the
stiffness from the symmetric bilinear form
  a(u, v) = sum_{e,q} w_q detJ_q [lambda div u div v + 2 mu eps(u):eps(v)],
which the paper's weak form (Sec. II-B) reduces to for isotropic Hooke's law.
A mistake in the oracle's flux form (dropped term, wrong sign, transposed
inverse Jacobian) makes the two disagree.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_numpy(n):
    N = n - 1
    cN = np.zeros(N + 1); cN[N] = 1.0
    inner = np.sort(np.real(npleg.legroots(npleg.legder(cN)))) if N >= 2 else np.array([])
    xi = np.concatenate([[-1.0], inner, [1.0]])
    PN = npleg.legval(xi, cN)
    w = 2.0 / (N * (N + 1) * PN ** 2)
    return xi, w


def dmatrix_barycentric(xi):
    n = len(xi)
    lam = np.array([1.0 / np.prod([xi[a] - xi[m] for m in range(n) if m != a]) for a in range(n)])
    D = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            if a != b:
                D[a, b] = (lam[b] / lam[a]) / (xi[a] - xi[b])
        D[a, a] = -np.sum(D[a, :])
    return D


def geometry_numpy(n, elem_vert, vert):
    """J[e,q,a,b] = dx_a/dxi_b, det J, Gamma = inv(J), xyz; q = i + n(j + n k)."""
    xi, _ = gll_numpy(n)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    r = np.stack([xi[i.ravel()], xi[j.ravel()], xi[k.ravel()]], axis=1)  # [n3, 3]
    s = np.array([[(v & 1) * 2 - 1, ((v >> 1) & 1) * 2 - 1, ((v >> 2) & 1) * 2 - 1] for v in range(8)], float)
    f = 1.0 + r[:, None, :] * s[None, :, :]                 # [n3, 8, 3]
    Nv = f.prod(axis=2) / 8.0                                # [n3, 8]
    dN = np.stack([s[None, :, 0] * f[:, :, 1] * f[:, :, 2],
                   f[:, :, 0] * s[None, :, 1] * f[:, :, 2],
                   f[:, :, 0] * f[:, :, 1] * s[None, :, 2]], axis=2) / 8.0  # [n3, 8, 3]
    X = vert[elem_vert]                                      # [E, 8, 3]
    xyz = np.einsum("qv,eva->eqa", Nv, X)
    J = np.einsum("qvb,eva->eqab", dN, X)
    det = np.linalg.det(J)
    gam = np.linalg.inv(J)   # gam[e,q,d,b] = dxi_d/dx_b
    return J, det, gam, xyz


def grad_at_points(n, ibool, u, gam):
    """g[e,q,c,b] = du_c/dx_b at every element-local point."""
    xi, _ = gll_numpy(n)
    D = dmatrix_barycentric(xi)
    E = ibool.shape[0]
    ue = u[ibool].reshape(E, n, n, n, 3)           # [e,k,j,i,c]
    dxi = np.einsum("ia,ekjac->ekjic", D, ue)
    deta = np.einsum("ja,ekaic->ekjic", D, ue)
    dzeta = np.einsum("ka,eajic->ekjic", D, ue)
    dref = np.stack([dxi, deta, dzeta], axis=-1).reshape(E, n ** 3, 3, 3)  # [e,q,c,d]
    return np.einsum("eqcd,eqdb->eqcb", dref, gam)


def bilinear(n, ibool, elem_vert, vert, lam, mu, u, v):
    _, det, gam, _ = geometry_numpy(n, elem_vert, vert)
    _, w = gll_numpy(n)
    w3 = np.einsum("k,j,i->kji", w, w, w).ravel()
    gu = grad_at_points(n, ibool, u, gam)
    gv = grad_at_points(n, ibool, v, gam)
    eu = 0.5 * (gu + np.swapaxes(gu, -1, -2))
    ev = 0.5 * (gv + np.swapaxes(gv, -1, -2))
    divu = np.trace(gu, axis1=-2, axis2=-1)
    divv = np.trace(gv, axis1=-2, axis2=-1)
    dens = lam * divu * divv + 2.0 * mu * np.einsum("eqab,eqab->eq", eu, ev)
    return float(np.sum(w3[None, :] * det * dens))


def dense_stiffness(n, ibool, elem_vert, vert, lam, mu, nglob):
    """K (3 nglob x 3 nglob) from the bilinear form, column by column (tiny meshes only)."""
    m = 3 * nglob
    _, det, gam, _ = geometry_numpy(n, elem_vert, vert)
    _, w = gll_numpy(n)
    w3 = np.einsum("k,j,i->kji", w, w, w).ravel()
    grads = []
    for col in range(m):
        u = np.zeros(m); u[col] = 1.0
        g = grad_at_points(n, ibool, u.reshape(nglob, 3), gam)
        grads.append(g)
    G = np.stack(grads)                      # [m, e, q, c, b]
    eps = 0.5 * (G + np.swapaxes(G, -1, -2))
    div = np.trace(G, axis1=-2, axis2=-1)    # [m, e, q]
    W = (w3[None, :] * det)
    K = (np.einsum("aeq,beq,eq->ab", div, div, W * lam)
         + 2.0 * np.einsum("aeqcd,beqcd,eq->ab", eps, eps, W * mu))
    return K


def mass_numpy(n, ibool, elem_vert, vert, rho, nglob):
    _, det, _, _ = geometry_numpy(n, elem_vert, vert)
    _, w = gll_numpy(n)
    w3 = np.einsum("k,j,i->kji", w, w, w).ravel()
    M = np.zeros(nglob)
    np.add.at(M, ibool.ravel(), (rho * det * w3[None, :]).ravel())
    return M


def sem1d_bloch_omega(n, h, c, k):
    """Frequency of the plane-wave branch exp(i k x) of the 1-D GLL spectral
    element discretisation of u'' = c^2 u'' on a uniform lattice of side h
    (lumped GLL mass, exact GLL stiffness), from the N x N Bloch system."""
    N = n - 1
    xi, w = gll_numpy(n)
    D = dmatrix_barycentric(xi)
    Ke = (2.0 / h) * c * c * (D.T * w) @ D
    me = 0.5 * h * w
    r = np.arange(n) % N
    ph = np.exp(1j * k * h * (np.arange(n) // N))
    P = np.zeros((n, N), dtype=np.complex128)
    P[np.arange(n), r] = ph
    Kr = P.conj().T @ Ke @ P
    mr = np.zeros(N)
    np.add.at(mr, r, me)
    ev, V = np.linalg.eigh(Kr / np.sqrt(np.outer(mr, mr)))
    x = 0.5 * (xi[:N] + 1.0) * h
    pw = np.sqrt(mr) * np.exp(1j * k * x)
    j = int(np.argmax(np.abs(V.conj().T @ pw)))
    return float(np.sqrt(max(ev[j], 0.0)))


def dense_stiffness_acoustic(n, ibool, elem_vert, vert, rho, nglob):
    """Scalar stiffness K_ab = sum_{e,q} w_q detJ_q / rho_q grad phi_a . grad phi_b
    (nglob x nglob), from the bilinear form, column by column (tiny meshes only)."""
    _, det, gam, _ = geometry_numpy(n, elem_vert, vert)
    _, w = gll_numpy(n)
    w3 = np.einsum("k,j,i->kji", w, w, w).ravel()
    grads = []
    for col in range(nglob):
        u = np.zeros((nglob, 3)); u[col, 0] = 1.0
        grads.append(grad_at_points(n, ibool, u, gam)[:, :, 0, :])  # [e, q, b]
    G = np.stack(grads)
    return np.einsum("aeqb,ceqb,eq->ac", G, G, w3[None, :] * det / rho)
