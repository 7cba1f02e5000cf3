"""FP64 CPU oracle for the SEM elastic operator -- TEST INFRASTRUCTURE.

This module is the independent reference that the HIP library is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may import it; the product path never does, and the two
share no code (the arithmetic lives in ``semx_oracle.c``, plain C in FP64,
compiled by :func:`build`).  Each wrapper names the passage of the paper
("High-Order Spectral Element Methods for Wave Propagation on ARM Multicore
CPU with SME") that its C function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "semx_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile ``semx_oracle.c`` into ``liboracle.so`` (gcc, -O3, OpenMP, no fast-math, no
    -march=native: the same build also runs on the GPU host, whose CPU may differ)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        i64 = ctypes.c_int64
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_gll.argtypes = [ctypes.c_int, _dp, _dp]
        L.orc_gll.restype = ctypes.c_int
        L.orc_lagrange.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _dp]
        L.orc_lagrange_deriv.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _dp]
        L.orc_dmatrix.argtypes = [ctypes.c_int, _dp, _dp]
        L.orc_geometry.argtypes = [ctypes.c_int, i64, _ip, _dp, _dp, _dp, ctypes.c_void_p]
        L.orc_geometry.restype = ctypes.c_int
        L.orc_mass.argtypes = [ctypes.c_int, i64, i64, _ip, _dp, _dp, _dp]
        L.orc_force.argtypes = [ctypes.c_int, i64, i64, _ip, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_forward.argtypes = [ctypes.c_int, i64, i64, _ip, _dp, _dp, _dp, _dp, _dp,
                                  ctypes.c_double, i64,
                                  ctypes.c_int, _ip, _dp, _dp, _dp,
                                  ctypes.c_int, _ip, _dp,
                                  _dp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_forward.restype = ctypes.c_int
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def num_threads() -> int:
    """OpenMP threads used by the oracle's element loops."""
    return int(lib().orc_num_threads())


def gll(n: int):
    """GLL nodes and weights (Sec. II-B): xi ascending, w."""
    xi = np.zeros(n); w = np.zeros(n)
    if lib().orc_gll(n, xi, w) != 0:
        raise ValueError(f"n={n} outside [2, 16]")
    return xi, w


def lagrange(n: int, x: float):
    """l_a(x) for a = 0..n-1 by the product formula of Sec. II-B."""
    xi, _ = gll(n)
    out = np.zeros(n)
    lib().orc_lagrange(n, xi, float(x), out)
    return out


def lagrange_deriv(n: int, x: float):
    xi, _ = gll(n)
    out = np.zeros(n)
    lib().orc_lagrange_deriv(n, xi, float(x), out)
    return out


def dmatrix(n: int):
    """D[a, b] = l'_b(xi_a) (Sec. II-B, xi-derivative)."""
    xi, _ = gll(n)
    D = np.zeros(n * n)
    lib().orc_dmatrix(n, xi, D)
    return D.reshape(n, n)


def geometry(n: int, elem_vert, vert):
    """Per-point Gamma = J^{-1} [nspec, n^3, 3, 3], det J [nspec, n^3], xyz [nspec, n^3, 3]."""
    ev = _i32(elem_vert); vt = _f64(vert)
    nspec = ev.shape[0]
    n3 = n ** 3
    gam = np.zeros(nspec * n3 * 9); jac = np.zeros(nspec * n3); xyz = np.zeros(nspec * n3 * 3)
    rc = lib().orc_geometry(n, nspec, ev.ravel(), vt.ravel(), gam, jac, xyz.ctypes.data)
    if rc == -1:
        raise ValueError("non-positive Jacobian determinant")
    return gam.reshape(nspec, n3, 3, 3), jac.reshape(nspec, n3), xyz.reshape(nspec, n3, 3)


def mass(n: int, ibool, jac, rho, nglob: int):
    """Lumped GLL mass M_g (Sec. II-B)."""
    ib = _i32(ibool)
    out = np.zeros(nglob)
    lib().orc_mass(n, ib.shape[0], nglob, ib.ravel(), _f64(jac).ravel(), _f64(rho).ravel(), out)
    return out


def force(n: int, ibool, gam, jac, lam, mu, u, nglob: int):
    """f = -K u, [nglob, 3] (Sec. II-B, stiffness term of the weak form)."""
    ib = _i32(ibool)
    f = np.zeros(nglob * 3)
    lib().orc_force(n, ib.shape[0], nglob, ib.ravel(), _f64(gam).ravel(), _f64(jac).ravel(),
                    _f64(lam).ravel(), _f64(mu).ravel(), _f64(u).ravel(), f)
    return f.reshape(nglob, 3)


def forward(n: int, ibool, gam, jac, lam, mu, rho, nglob: int, dt: float, nt: int,
            src_elem, src_xi, src_dir, stf, rec_elem, rec_xi,
            want_energy: bool = False, want_history: bool = False):
    """Explicit Newmark run (Sec. V-C: second-order Newmark) with point forces and receivers.

    Returns a dict with ``seis`` [nrec, 3, nt] (displacement after each step)
    and optionally ``energy``/``work`` [nt] and ``uhist`` [nt+1, nglob, 3].
    """
    ib = _i32(ibool)
    nsrc = len(src_elem); nrec = len(rec_elem)
    stf = _f64(stf).reshape(nsrc, nt + 1) if nsrc else np.zeros((0, nt + 1))
    seis = np.zeros(max(nrec, 1) * 3 * nt)
    energy = np.zeros(nt) if want_energy else None
    work = np.zeros(nt) if want_energy else None
    uhist = np.zeros((nt + 1) * nglob * 3) if want_history else None
    rc = lib().orc_forward(
        n, ib.shape[0], nglob, ib.ravel(), _f64(gam).ravel(), _f64(jac).ravel(),
        _f64(lam).ravel(), _f64(mu).ravel(), _f64(rho).ravel(), float(dt), int(nt),
        nsrc, _i32(src_elem).ravel() if nsrc else np.zeros(1, np.int32),
        _f64(src_xi).ravel() if nsrc else np.zeros(3), _f64(src_dir).ravel() if nsrc else np.zeros(3),
        stf.ravel() if nsrc else np.zeros(1),
        nrec, _i32(rec_elem).ravel() if nrec else np.zeros(1, np.int32),
        _f64(rec_xi).ravel() if nrec else np.zeros(3),
        seis,
        energy.ctypes.data if energy is not None else None,
        work.ctypes.data if work is not None else None,
        uhist.ctypes.data if uhist is not None else None)
    if rc != 0:
        raise RuntimeError(f"orc_forward failed ({rc})")
    out = {"seis": seis[: nrec * 3 * nt].reshape(nrec, 3, nt)}
    if want_energy:
        out["energy"] = energy
        out["work"] = work
    if want_history:
        out["uhist"] = uhist.reshape(nt + 1, nglob, 3)
    return out


def adjoint(n: int, ibool, gam, jac, lam, mu, rho, nglob: int, dt: float, nt: int,
            src_elem, src_xi, src_dir, stf, rec_elem, rec_xi, gseis):
    """Exact discrete-adjoint gradient of a seismogram functional chi through
    the Newmark run of :func:`forward`, given gseis = d chi / d seis
    [nrec, 3, nt].  Returns (d chi/d lambda, d chi/d mu, d chi/d rho), each
    [nspec, n^3] per element-local point."""
    L = lib()
    if not getattr(L, "_adj_sig", False):
        i64 = ctypes.c_int64
        L.orc_adjoint.argtypes = [ctypes.c_int, i64, i64, _ip, _dp, _dp, _dp, _dp, _dp,
                                  ctypes.c_double, i64,
                                  ctypes.c_int, _ip, _dp, _dp, _dp,
                                  ctypes.c_int, _ip, _dp, _dp, _dp, _dp, _dp]
        L.orc_adjoint.restype = ctypes.c_int
        L._adj_sig = True
    ib = _i32(ibool)
    nspec = ib.shape[0]
    n3 = n ** 3
    nsrc = len(src_elem); nrec = len(rec_elem)
    stf = _f64(stf).reshape(nsrc, nt + 1)
    gl = np.zeros(nspec * n3); gm = np.zeros(nspec * n3); gr = np.zeros(nspec * n3)
    rc = L.orc_adjoint(n, nspec, nglob, ib.ravel(), _f64(gam).ravel(), _f64(jac).ravel(),
                       _f64(lam).ravel(), _f64(mu).ravel(), _f64(rho).ravel(), float(dt), int(nt),
                       nsrc, _i32(src_elem).ravel(), _f64(src_xi).ravel(), _f64(src_dir).ravel(),
                       stf.ravel(), nrec, _i32(rec_elem).ravel(), _f64(rec_xi).ravel(),
                       _f64(gseis).ravel(), gl, gm, gr)
    if rc != 0:
        raise RuntimeError(f"orc_adjoint failed ({rc})")
    return gl.reshape(nspec, n3), gm.reshape(nspec, n3), gr.reshape(nspec, n3)


def misfit(seis, data, dt: float) -> float:
    """L2 seismogram misfit chi = 1/2 dt sum (s - d)^2."""
    return 0.5 * dt * float(np.sum((np.asarray(seis) - np.asarray(data)) ** 2))
