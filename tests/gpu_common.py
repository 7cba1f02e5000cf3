"""Shared helpers for the GPU parity tests: build inputs once, run the
library through its C ABI, run the oracle on the same inputs."""
from __future__ import annotations

import numpy as np

import workloads as W


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64); b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make_solver(n):
    import paper_2606_12850_amd as P
    return P.Solver(n)


def oracle_geometry(orc, mesh):
    return orc.geometry(mesh.n, mesh.elem_vert, mesh.vert)


def smooth_field(orc, mesh, seed=0):
    """A smooth displacement: sum of a few long-wavelength sines at the GLL
    node coordinates (oracle geometry)."""
    _, _, xyz = oracle_geometry(orc, mesh)
    X = np.zeros((mesh.nglob, 3)); X[mesh.ibool.ravel()] = xyz.reshape(-1, 3)
    rng = np.random.default_rng(seed)
    L = np.array(mesh.L)
    u = np.zeros((mesh.nglob, 3))
    for _ in range(4):
        k = rng.integers(1, 3, size=3) * np.pi / L
        ph = rng.uniform(0, 2 * np.pi, 3)
        amp = rng.standard_normal(3)
        u += amp[None, :] * np.sin(X @ k + ph[0])[:, None] * np.cos(X[:, 0] * k[1] + ph[1])[:, None]
    return u * 1e-6


def gpu_force(solver, u_np, nmodels=1):
    import torch
    u = torch.from_numpy(np.ascontiguousarray(u_np, dtype=np.float32)).to(solver.device)
    f = solver.apply_force(u)
    torch.cuda.synchronize()
    return f.cpu().numpy().astype(np.float64)
