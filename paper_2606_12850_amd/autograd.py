"""torch.autograd bridge: seismograms as a differentiable function of the
elastic model (lambda, mu, rho per element-local point).

The forward pass runs the library's explicit Newmark loop with forward
checkpoints; the backward pass calls the library's discrete adjoint
(``semx_adjoint``), which recomputes the forward segment by segment and
returns d chi/d lambda, d chi/d mu, d chi/d rho.  Only marshalling happens
here.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (SEMX_C_F32, Solver, semx_adjoint, semx_read_seismograms, semx_reset,
               semx_set_checkpointing, semx_set_dt, semx_set_receivers, semx_set_sources, semx_step)


class SeismogramOperator:
    """A mesh with fixed sources, receivers, dt and step count on one context."""

    def __init__(self, mesh, src_elem, src_xi, src_dir, stf, rec_elem, rec_xi, dt: float, nt: int,
                 ngll: int | None = None, checkpoint_every: int = 100, geometry: int | None = None,
                 device: str = "cuda:0"):
        self.solver = Solver(ngll or mesh.n, device)
        self.solver.upload_mesh(mesh)
        if geometry is not None:
            from . import semx_set_geometry
            semx_set_geometry(self.solver.ctx, geometry)
        self.mesh = mesh
        self.src = (np.asarray(src_elem, np.int32), np.asarray(src_xi, float), np.asarray(src_dir, float),
                    np.asarray(stf, np.float32))
        self.rec = (np.asarray(rec_elem, np.int32), np.asarray(rec_xi, float))
        self.dt = float(dt)
        self.nt = int(nt)
        self.every = int(checkpoint_every)
        self.nmodels = 0
        self.runs = 0  # forward runs so far: the adjoint replays only the latest

    def run(self, lam, mu, rho):
        """Upload the model, run nt steps with checkpoints, return seismograms
        as a device tensor [nmodels, nrec, 3, nt] (nmodels = 1 squeezed)."""
        s = self.solver
        s.upload_model(lam, mu, rho)
        self.nmodels = s.nmodels
        semx_set_sources(s.ctx, *self.src)
        semx_set_receivers(s.ctx, self.rec[0], self.rec[1], self.nt)
        semx_set_dt(s.ctx, self.dt)
        semx_set_checkpointing(s.ctx, self.every)
        semx_reset(s.ctx)
        semx_step(s.ctx, self.nt)
        self.runs += 1
        out = torch.empty((self.nmodels, len(self.rec[0]), 3, self.nt), dtype=torch.float32, device=s.device)
        semx_read_seismograms(s.ctx, out, True)
        return out

    def gradient(self, gseis):
        """d chi/d (lambda, mu, rho) [nmodels, nspec, n^3] from d chi/d seis."""
        s = self.solver
        g = gseis.to(device=s.device, dtype=torch.float32).reshape(self.nmodels, len(self.rec[0]), 3, self.nt)
        g = g.contiguous()
        shape = (self.nmodels, self.mesh.nspec, self.mesh.n ** 3)
        gl = torch.empty(shape, dtype=torch.float64, device=s.device)
        gm = torch.empty_like(gl)
        gr = torch.empty_like(gl)
        semx_adjoint(s.ctx, g, self.nt, gl, gm, gr)
        return gl, gm, gr


class SemForward(torch.autograd.Function):
    """seis = SemForward.apply(lam, mu, rho, op): lam, mu, rho are CPU float64
    tensors [nspec, n^3] (or [nmodels, nspec, n^3]); seis is a float32 device
    tensor [nrec, 3, nt] (or with a leading model axis)."""

    @staticmethod
    def forward(ctx, lam, mu, rho, op: SeismogramOperator):
        squeeze = lam.dim() == 2
        seis = op.run(lam.detach().cpu().numpy(), mu.detach().cpu().numpy(), rho.detach().cpu().numpy())
        ctx.op = op
        ctx.run = op.runs
        ctx.squeeze = squeeze
        ctx.dev = lam.device
        return seis[0] if squeeze else seis

    @staticmethod
    def backward(ctx, gseis):
        op = ctx.op
        if op.runs != ctx.run:
            raise RuntimeError("SemForward.backward: the operator ran another forward since this graph was built; "
                               "its checkpoints are of that run (use one operator per graph, or run backward first)")
        g = gseis.unsqueeze(0) if ctx.squeeze else gseis
        gl, gm, gr = op.gradient(g)
        outs = []
        for t in (gl, gm, gr):
            t = t.to(device=ctx.dev, dtype=torch.float64)
            outs.append(t[0] if ctx.squeeze else t)
        return outs[0], outs[1], outs[2], None
