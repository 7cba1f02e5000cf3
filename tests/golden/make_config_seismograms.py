"""Write the FP64 oracle's seismograms for the time-loop parity tests at the
workloads' own sizes (tests/test_gpu_config_parity.py).  Calls only
``oracle/`` and the seeded input generators in ``workloads/``.

Cases (all NGLL 5, vertical Ricker point force 10 Hz with t0 = 0.12 s,
dt = 0.4 x smallest GLL-point spacing / largest P speed, from the oracle's
geometry):
  layered16  16^3 jittered (+-10 % h, seed 2606) layered cube with the +-5 %
             random field, centre source, 8 top receivers, 1000 steps; also
             the discrete energy and the source work of every step;
  adjoint32  32^3 regular layered cube with the -5 % Gaussian anomaly,
             source at (L/2, L/2, 0.2 L), 8 x 8 top receivers, 1000 steps;
  layered64  64^3 jittered layered cube (the throughput workload), centre
             source, 8 top receivers, 2000 steps (about 20 minutes on 8 cores).

Usage: python tests/golden/make_config_seismograms.py [case ...]
Seismograms are stored in FP32 (rounding 6e-8 relative, far below the 1e-4
bar); dt, the energies and a fingerprint of the inputs in FP64.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402

NT = {"layered16": 1000, "adjoint32": 1000, "layered64": 2000}


def workload(case: str) -> W.Workload:
    nt = NT[case]
    if case == "layered16":
        return W.layered_jittered(ne=16, n=5, nt=nt, dt=1.0, jitter=0.10, seed=2606, grf_seed=12850, nrec=8)
    if case == "adjoint32":
        return W.adjoint_layered(ne=32, n=5, nt=nt, dt=1.0, anomaly=True)
    if case == "layered64":
        return W.layered_jittered(ne=64, n=5, nt=nt, dt=1.0, jitter=0.10, seed=2606, grf_seed=12850, nrec=8)
    raise KeyError(case)


def cfl_dt(mesh, lam, mu, rho, xyz, courant: float = 0.4) -> float:
    """dt = courant x (smallest distance between GLL points adjacent along a
    reference axis) / (largest P speed)."""
    n = mesh.n
    x = xyz.reshape(mesh.nspec, n, n, n, 3)
    d = min(np.linalg.norm(np.diff(x, axis=ax), axis=-1).min() for ax in (1, 2, 3))
    vp = np.sqrt((lam + 2.0 * mu) / rho).max()
    return float(courant * d / vp)


def fingerprint(wl: W.Workload) -> str:
    h = hashlib.sha256()
    for a in (wl.mesh.vert, wl.mesh.ibool, wl.lam, wl.mu, wl.rho, wl.src_xi, wl.rec_xi):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


def prepare(case: str):
    """The case's workload with the oracle's dt and Ricker (shared with the tests)."""
    wl = workload(case)
    gam, jac, xyz = O.geometry(5, wl.mesh.elem_vert, wl.mesh.vert)
    wl.dt = cfl_dt(wl.mesh, wl.lam, wl.mu, wl.rho, xyz)
    wl.stf = W.ricker(10.0, 0.12, wl.dt, wl.nt + 1)[None, :]
    return wl, gam, jac


def make(case: str) -> str:
    t0 = time.time()
    wl, gam, jac = prepare(case)
    m = wl.mesh
    out = O.forward(5, m.ibool, gam, jac, wl.lam, wl.mu, wl.rho, m.nglob, wl.dt, wl.nt,
                    wl.src_elem, wl.src_xi, wl.src_dir, wl.stf, wl.rec_elem, wl.rec_xi,
                    want_energy=(case == "layered16"))
    extra = {}
    if "energy" in out:
        extra = {"energy": out["energy"], "work": out["work"]}
    path = os.path.join(HERE, f"seis_{case}.npz")
    np.savez_compressed(path, seis=out["seis"].astype(np.float32), dt=np.float64(wl.dt), nt=np.int64(wl.nt),
                        fingerprint=np.array(fingerprint(wl)), **extra)
    print(f"{case}: nspec {m.nspec}, nglob {m.nglob}, dt {wl.dt:.6g}, {wl.nt} steps, "
          f"peak |s| {np.abs(out['seis']).max():.3e}, {time.time() - t0:.0f} s -> {path}", flush=True)
    return path


if __name__ == "__main__":
    for c in (sys.argv[1:] or list(NT)):
        make(c)
