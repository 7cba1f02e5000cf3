"""Learned surrogate for receiver seismograms, with the SEM solve as fallback
and as the reference for its error.

* Training data come from batched SEM runs of the library (many models
  sharing one mesh in one context, ``nmodels`` > 1).
* The network is an MLP (SiLU hidden layers, linear output) trained on the
  GPU by the library's own kernels (``semx_mlp_*``: BF16 matrix-core GEMMs
  with FP32 accumulation, FP32 master weights, Adam).
* An ensemble of such networks provides an error indicator (the spread of
  the members); inputs whose indicator exceeds a threshold calibrated on
  validation data are sent to the SEM solver instead.

Only marshalling, the training-set statistics and bookkeeping happen in
Python; normalisation, the ensemble statistics and the indicator run in the
library's kernels.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import (Solver, semx_mlp_adam, semx_mlp_affine, semx_mlp_backward, semx_mlp_create, semx_mlp_destroy,
               semx_mlp_ensemble, semx_mlp_forward, semx_mlp_get_params, semx_mlp_mse, semx_mlp_num_params,
               semx_mlp_set_params, semx_read_seismograms, semx_reset, semx_set_dt, semx_set_receivers,
               semx_set_sources, semx_step)


class BatchedSEM:
    """Seismograms of many models on one mesh: models run ``batch`` at a time
    as one multi-model context (shared geometry, per-model lambda, mu, rho)."""

    def __init__(self, mesh, src_elem, src_xi, src_dir, stf, rec_elem, rec_xi, dt: float, nt: int,
                 batch: int = 64, device: str = "cuda:0"):
        self.solver = Solver(mesh.n, device)
        self.solver.upload_mesh(mesh)
        self.mesh = mesh
        self.src = (np.asarray(src_elem, np.int32), np.asarray(src_xi, float), np.asarray(src_dir, float),
                    np.asarray(stf, np.float32))
        self.rec = (np.asarray(rec_elem, np.int32), np.asarray(rec_xi, float))
        self.dt, self.nt, self.batch = float(dt), int(nt), int(batch)

    def run(self, lam, mu, rho):
        """lam, mu, rho [B, nspec, n^3] -> seismograms [B, nrec, 3, nt] (host FP32)."""
        s = self.solver
        s.upload_model(lam, mu, rho)
        semx_set_sources(s.ctx, *self.src)
        semx_set_receivers(s.ctx, self.rec[0], self.rec[1], self.nt)
        semx_set_dt(s.ctx, self.dt)
        semx_reset(s.ctx)
        semx_step(s.ctx, self.nt)
        out = np.zeros((s.nmodels, len(self.rec[0]), 3, self.nt), np.float32)
        semx_read_seismograms(s.ctx, out, False)
        return out

    def run_models(self, model_fn, coeffs):
        """model_fn(coeff_block) -> (lam, mu, rho); all coefficient rows."""
        outs = []
        for b0 in range(0, len(coeffs), self.batch):
            lam, mu, rho = model_fn(coeffs[b0:b0 + self.batch])
            outs.append(self.run(lam, mu, rho))
        return np.concatenate(outs, axis=0)

    def close(self):
        self.solver.close()


def resample(seis, nout: int):
    """Linear interpolation of [..., nt] samples at t_n = n dt (n = 1..nt)
    onto t_j = (j+1) T / nout, T = nt dt (j = 0..nout-1)."""
    nt = seis.shape[-1]
    tj = (np.arange(nout) + 1.0) * nt / nout
    lo = np.clip(np.floor(tj).astype(int), 1, nt - 1)
    w = tj - lo
    a = seis[..., lo - 1]
    b = seis[..., lo]
    return (1.0 - w) * a + w * b


def he_uniform(widths, seed: int) -> np.ndarray:
    """Packed initial parameters: W_l ~ U(-sqrt(6/fan_in), sqrt(6/fan_in)), b_l = 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(len(widths) - 1):
        lim = math.sqrt(6.0 / widths[l])
        parts.append(rng.uniform(-lim, lim, widths[l + 1] * widths[l]).astype(np.float32))
        parts.append(np.zeros(widths[l + 1], np.float32))
    return np.concatenate(parts)


class MLP:
    """An MLP whose forward, backward, loss and Adam step run in the library."""

    def __init__(self, widths, max_batch: int, seed: int = 0, device: str = "cuda:0"):
        self.widths = list(widths)
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.net = semx_mlp_create(self.widths, max_batch, self.stream)
        self.nparam = semx_mlp_num_params(self.net)
        semx_mlp_set_params(self.net, he_uniform(self.widths, seed))
        self.step = 0

    def close(self):
        if getattr(self, "net", None) is not None:
            semx_mlp_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.zeros(self.nparam, np.float32)
        semx_mlp_get_params(self.net, out)
        return out

    def set_params(self, theta):
        semx_mlp_set_params(self.net, theta)

    def forward(self, x):
        y = torch.empty((x.shape[0], self.widths[-1]), dtype=torch.float32, device=self.device)
        semx_mlp_forward(self.net, x, x.shape[0], y)
        return y

    def train_step(self, x, t, lr: float) -> float:
        y = self.forward(x)
        dy = torch.empty_like(y)
        loss = semx_mlp_mse(self.net, y, t, y.numel(), dy, want_loss=False)
        semx_mlp_backward(self.net, dy, x.shape[0])
        self.step += 1
        semx_mlp_adam(self.net, lr, 0.9, 0.999, 1e-8, self.step)
        return loss

    def loss(self, x, t) -> float:
        y = self.forward(x)
        return semx_mlp_mse(self.net, y, t, y.numel())


def cosine_lr(step, total, lr0=1e-3, lr1=1e-5):
    return lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * min(step, total) / max(total, 1)))


class Surrogate:
    """Ensemble of MLPs predicting normalised seismograms from model coefficients."""

    def __init__(self, n_in: int, n_out: int, hidden=(512, 512, 512), members: int = 4, max_batch: int = 4096,
                 seed: int = 0, device: str = "cuda:0"):
        self.widths = [n_in, *hidden, n_out]
        self.members = [MLP(self.widths, max_batch, seed + 1000 * k, device) for k in range(members)]
        self.device = torch.device(device)
        self.x_mu = self.x_sd = self.y_mu = self.y_sd = None
        self.threshold = None

    def close(self):
        for m in self.members:
            m.close()

    def fit(self, X, Y, epochs: int = 300, batch: int = 128, lr0: float = 1e-3, lr1: float = 1e-5, seed: int = 0,
            log=None):
        """X [S, n_in]; Y [S, nrec, ncomp, nt] seismograms (targets normalised
        by the training-set mean per sample and the std per (receiver,
        component) over models and time, so quiet samples are not
        amplified) or Y [S, n_out] (std per output)."""
        self.x_mu, self.x_sd = X.mean(0), X.std(0) + 1e-12
        if Y.ndim == 4:
            sd = Y.std(axis=(0, 3), keepdims=True)[0]  # [nrec, ncomp, 1]
            sd = np.broadcast_to(sd + 1e-30 + 1e-6 * sd.max(), Y.shape[1:]).reshape(-1)
            Y = Y.reshape(Y.shape[0], -1)
        else:
            sd = Y.std(0) + 1e-30
        self.y_mu = Y.mean(0)
        self.y_sd = sd
        S = X.shape[0]
        net0 = self.members[0].net
        Xn = self._dev(X)
        semx_mlp_affine(net0, Xn, S, X.shape[1], self._dev(1.0 / self.x_sd), self._dev(-self.x_mu / self.x_sd), Xn)
        Yn = self._dev(Y)
        semx_mlp_affine(net0, Yn, S, Y.shape[1], self._dev(1.0 / self.y_sd), self._dev(-self.y_mu / self.y_sd), Yn)
        steps_per_epoch = max(1, S // batch)
        total = epochs * steps_per_epoch
        rng = np.random.default_rng(seed)
        t0 = time.perf_counter()
        for k, m in enumerate(self.members):
            step = 0
            for ep in range(epochs):
                perm = torch.from_numpy(rng.permutation(S)).to(self.device)
                for b in range(steps_per_epoch):
                    idx = perm[b * batch:(b + 1) * batch]
                    m.train_step(Xn[idx].contiguous(), Yn[idx].contiguous(), cosine_lr(step, total, lr0, lr1))
                    step += 1
                if log is not None and (ep + 1) % max(1, epochs // 5) == 0:
                    log(f"member {k} epoch {ep + 1}: train loss {m.loss(Xn[:min(S, 1024)], Yn[:min(S, 1024)]):.4e}")
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def _dev(self, a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(self.device)

    def predict(self, X):
        """Mean prediction (physical units) and spread indicator
        ||std|| / ||mean|| per input.  The input normalisation, the members'
        forward passes, the ensemble mean, its mapping back to physical
        units and the indicator all run in the library's kernels."""
        net0 = self.members[0].net
        S, n_in = X.shape
        x = self._dev(X)
        xs, xb = self._dev(1.0 / self.x_sd), self._dev(-self.x_mu / self.x_sd)
        semx_mlp_affine(net0, x, S, n_in, xs, xb, x)  # (x - mean) / std in place
        n_out = self.widths[-1]
        preds = torch.empty((len(self.members), S, n_out), dtype=torch.float32, device=self.device)
        for k, m in enumerate(self.members):
            for b in range(0, S, 4096):
                nb = min(4096, S - b)
                semx_mlp_forward(m.net, x[b:b + nb], nb, preds[k, b:b + nb])
        mean = torch.empty((S, n_out), dtype=torch.float32, device=self.device)
        ind = torch.empty(S, dtype=torch.float32, device=self.device)
        semx_mlp_ensemble(net0, preds, len(self.members), S, n_out, self._dev(self.y_sd), self._dev(self.y_mu),
                          mean, ind)
        torch.cuda.synchronize(self.device)
        return mean.cpu().numpy(), ind.cpu().numpy().astype(np.float64)

    def calibrate(self, X, Y, tol: float = 0.05):
        """Smallest indicator threshold that flags every validation input whose
        true relative error exceeds tol."""
        pred, ind = self.predict(X)
        err = rel_err(pred, Y)
        bad = err > tol
        self.threshold = float(ind[bad].min()) * (1 - 1e-6) if bad.any() else float(ind.max()) * (1 + 1e-6)
        return {"val_err_mean": float(err.mean()), "val_err_max": float(err.max()),
                "val_frac_above_tol": float(bad.mean()), "threshold": self.threshold}


def rel_err(pred, ref):
    a = pred.reshape(pred.shape[0], -1).astype(np.float64)
    b = ref.reshape(ref.shape[0], -1).astype(np.float64)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)
