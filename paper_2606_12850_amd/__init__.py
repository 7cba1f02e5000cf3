"""semx: spectral-element elastic wave operator for AMD Instinct MI355X.

Thin Python binding of ``libsemx.so`` (HIP, gfx950).  Every function named
``semx_*`` below marshals its arguments and calls the C function of the same
name declared in ``include/semx.h``; all arithmetic runs in the library's
kernels.  PyTorch is used only for device memory and the HIP stream.  There
is no CPU fallback: if the library is missing or fails to load, importing the
binding's entry points raises.

:class:`Solver` is a small convenience wrapper around one context.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsemx.so")

SEMX_OK = 0
SEMX_EINVAL = -1
SEMX_ESTATE = -2
SEMX_EGEOM = -3
SEMX_EUNSTABLE = -4
SEMX_EHIP = -5
SEMX_ENOMEM = -6
SEMX_ENUMERIC = -7

SEMX_C_F32 = 0
SEMX_C_BF16 = 1
SEMX_C_F16 = 2
SEMX_C_MFMA_F32 = 3
SEMX_ASM_COLORED = 0
SEMX_ASM_ATOMIC = 1
SEMX_GEOM_STORED = 0
SEMX_GEOM_TRILINEAR = 1
SEMX_BLOCKS_OFF, SEMX_BLOCKS_AUTO, SEMX_BLOCKS_ON = 0, 1, 2
SEMX_F32 = 0
SEMX_F64 = 1
SEMX_ELASTIC = 0
SEMX_ACOUSTIC = 1

_ERRNAMES = {-1: "EINVAL", -2: "ESTATE", -3: "EGEOM", -4: "EUNSTABLE", -5: "EHIP", -6: "ENOMEM",
             -7: "ENUMERIC"}

_lib = None

_vp = ctypes.c_void_p
_i32 = ctypes.c_int
_i64 = ctypes.c_int64
_f64 = ctypes.c_double

# name -> argtypes (all return int unless listed in _RESTYPE)
_SIGS = {
    "semx_create": [ctypes.POINTER(_vp), _i32, _vp],
    "semx_destroy": [_vp],
    "semx_last_error": [_vp],
    "semx_upload_mesh": [_vp, _i64, _i64, _vp, _i64, _vp, _vp],
    "semx_set_coloring": [_vp, _i32, _vp, _vp],
    "semx_get_coloring": [_vp, ctypes.POINTER(_i32), _vp, _vp],
    "semx_mesh_info": [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i32)],
    "semx_upload_model": [_vp, _i32, _vp, _vp, _vp],
    "semx_set_mode": [_vp, _i32, _i32],
    "semx_apply_force": [_vp, _vp, _vp],
    "semx_set_dt": [_vp, _f64],
    "semx_cfl_dt": [_vp, _f64, ctypes.POINTER(_f64)],
    "semx_max_eigenvalue": [_vp, _i32, ctypes.POINTER(_f64)],
    "semx_set_sources": [_vp, _i32, _vp, _vp, _vp, _i64, _vp],
    "semx_set_receivers": [_vp, _i32, _vp, _vp, _i64],
    "semx_reset": [_vp],
    "semx_step": [_vp, _i64],
    "semx_time_index": [_vp, ctypes.POINTER(_i64)],
    "semx_read_seismograms": [_vp, _vp, _i32],
    "semx_get_state": [_vp, _vp, _vp, _vp, ctypes.POINTER(_i64)],
    "semx_set_state": [_vp, _vp, _vp, _vp, _i64],
    "semx_energy": [_vp, ctypes.POINTER(_f64), ctypes.POINTER(_f64), ctypes.POINTER(_f64)],
    "semx_set_watchdog": [_vp, _i64, _f64],
    "semx_set_geometry": [_vp, _i32],
    "semx_set_blocks": [_vp, _i32, ctypes.c_void_p],
    "semx_set_graphs": [_vp, _i32],
    "semx_set_checkpointing": [_vp, _i64],
    "semx_adjoint": [_vp, _vp, _i64, _vp, _vp, _vp],
    "semx_mlp_create": [ctypes.POINTER(_vp), _i32, _vp, _i32, _vp],
    "semx_mlp_destroy": [_vp],
    "semx_mlp_last_error": [_vp],
    "semx_mlp_num_params": [_vp, ctypes.POINTER(_i64)],
    "semx_mlp_set_params": [_vp, _vp],
    "semx_mlp_get_params": [_vp, _vp],
    "semx_mlp_get_grads": [_vp, _vp],
    "semx_mlp_forward": [_vp, _vp, _i32, _vp],
    "semx_mlp_forward_noalloc": [_vp, _vp, _i32, _vp],
    "semx_mlp_backward": [_vp, _vp, _i32],
    "semx_mlp_mse": [_vp, _vp, _vp, _i64, _vp, ctypes.POINTER(_f64)],
    "semx_mlp_adam": [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _i64],
    "semx_mlp_affine": [_vp, _vp, _i64, _i32, _vp, _vp, _vp],
    "semx_mlp_ensemble": [_vp, _vp, _i32, _i64, _i32, _vp, _vp, _vp, _vp],
    "semx_set_storage": [_vp, _i32],
    "semx_apply_force_f64": [_vp, _vp, _vp],
    "semx_set_sources_f64": [_vp, _i32, _vp, _vp, _vp, _i64, _vp],
    "semx_read_seismograms_f64": [_vp, _vp, _i32],
    "semx_get_state_f64": [_vp, _vp, _vp, _vp, ctypes.POINTER(_i64)],
    "semx_set_state_f64": [_vp, _vp, _vp, _vp, _i64],
    "semx_stream_bandwidth": [_vp, _i64, _i32, ctypes.POINTER(_f64)],
    "semx_force_skeleton": [_vp, _vp, _vp, _i32, ctypes.POINTER(_f64)],
    "semx_set_timing": [_vp, _i32],
    "semx_set_physics": [_vp, _i32],
    "semx_upload_model_acoustic": [_vp, _i32, _vp, _vp],
    "semx_gll": [_i32, _vp, _vp],
    "semx_force_timing": [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_f64)],
}
_RESTYPE = {"semx_last_error": ctypes.c_char_p, "semx_mlp_last_error": ctypes.c_char_p}


def lib():
    """Load ``libsemx.so`` (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with __graft_entry__.build() "
                              "or python -m paper_2606_12850_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue  # optional export set not built into this library
            fn.argtypes = args
            fn.restype = _RESTYPE.get(name, ctypes.c_int)
        _lib = L
    return _lib


def exported_symbols():
    """Names of the C entry points present in the loaded library."""
    L = lib()
    return sorted(n for n in _SIGS if getattr(L, n, None) is not None)


class SemxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"semx error {code} ({_ERRNAMES.get(code, '?')}): {msg}")
        self.code = code


def _ptr(x):
    """Pointer of a numpy array or torch tensor (or None)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


def _check(ctx, rc):
    if rc != SEMX_OK:
        msg = lib().semx_last_error(ctx)
        raise SemxError(rc, msg.decode() if msg else "")
    return rc


# ---- one function per C entry point ------------------------------------------

def semx_create(ngll: int, stream=None):
    h = _vp()
    s = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    rc = lib().semx_create(ctypes.byref(h), int(ngll), s)
    if rc != SEMX_OK:
        raise SemxError(rc, "semx_create failed")
    return h


def semx_destroy(ctx):
    return lib().semx_destroy(ctx)


def semx_last_error(ctx) -> str:
    m = lib().semx_last_error(ctx)
    return m.decode() if m else ""


def semx_upload_mesh(ctx, ibool, vert, elem_vert, nglob: int):
    ib = np.ascontiguousarray(ibool, dtype=np.int32)
    vt = np.ascontiguousarray(vert, dtype=np.float64)
    ev = np.ascontiguousarray(elem_vert, dtype=np.int32)
    return _check(ctx, lib().semx_upload_mesh(ctx, ib.shape[0], int(nglob), _ptr(ib), vt.shape[0], _ptr(vt), _ptr(ev)))


def semx_set_coloring(ctx, color_ptr, elem_order):
    cp = np.ascontiguousarray(color_ptr, dtype=np.int32)
    eo = np.ascontiguousarray(elem_order, dtype=np.int32)
    return _check(ctx, lib().semx_set_coloring(ctx, len(cp) - 1, _ptr(cp), _ptr(eo)))


def semx_get_coloring(ctx, nspec: int):
    nc = _i32()
    _check(ctx, lib().semx_get_coloring(ctx, ctypes.byref(nc), None, None))
    cp = np.zeros(nc.value + 1, np.int32)
    eo = np.zeros(nspec, np.int32)
    if nc.value:
        _check(ctx, lib().semx_get_coloring(ctx, ctypes.byref(nc), _ptr(cp), _ptr(eo)))
    return cp, eo


def semx_mesh_info(ctx):
    r, i, c = _i64(), _i64(), _i32()
    _check(ctx, lib().semx_mesh_info(ctx, ctypes.byref(r), ctypes.byref(i), ctypes.byref(c)))
    return {"nregular": r.value, "nirregular": i.value, "ncolors": c.value}


def semx_upload_model(ctx, lam, mu, rho):
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    nm = lam.shape[0] if lam.ndim == 3 else 1
    return _check(ctx, lib().semx_upload_model(ctx, nm, _ptr(lam), _ptr(mu), _ptr(rho)))


def semx_set_physics(ctx, physics: int):
    return _check(ctx, lib().semx_set_physics(ctx, int(physics)))


def semx_upload_model_acoustic(ctx, kappa, rho):
    kappa = np.ascontiguousarray(kappa, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    nm = kappa.shape[0] if kappa.ndim == 3 else 1
    return _check(ctx, lib().semx_upload_model_acoustic(ctx, nm, _ptr(kappa), _ptr(rho)))


def semx_gll(ngll: int):
    """The library's GLL nodes and weights (FP64 numpy arrays)."""
    xi = np.zeros(int(ngll)); w = np.zeros(int(ngll))
    rc = lib().semx_gll(int(ngll), _ptr(xi), _ptr(w))
    if rc != SEMX_OK:
        raise SemxError(rc, f"semx_gll: ngll={ngll} outside [2, 16]")
    return xi, w


def semx_set_mode(ctx, contraction: int, assembly: int):
    return _check(ctx, lib().semx_set_mode(ctx, int(contraction), int(assembly)))


def semx_apply_force(ctx, u, f):
    return _check(ctx, lib().semx_apply_force(ctx, _ptr(u), _ptr(f)))


def semx_set_dt(ctx, dt: float):
    return _check(ctx, lib().semx_set_dt(ctx, float(dt)))


def semx_cfl_dt(ctx, courant: float) -> float:
    out = _f64()
    _check(ctx, lib().semx_cfl_dt(ctx, float(courant), ctypes.byref(out)))
    return out.value


def semx_max_eigenvalue(ctx, iters: int) -> float:
    out = _f64()
    _check(ctx, lib().semx_max_eigenvalue(ctx, int(iters), ctypes.byref(out)))
    return out.value


def semx_set_sources(ctx, elem, xi, direction, stf):
    """``direction`` may be None for the acoustic physics."""
    el = np.ascontiguousarray(elem, dtype=np.int32)
    x = np.ascontiguousarray(xi, dtype=np.float64)
    d = None if direction is None else np.ascontiguousarray(direction, dtype=np.float64)
    s = np.ascontiguousarray(stf, dtype=np.float32)
    nsrc = len(el)
    nstf = s.shape[-1] if nsrc else 0
    return _check(ctx, lib().semx_set_sources(ctx, nsrc, _ptr(el), _ptr(x), None if d is None else _ptr(d),
                                              nstf, _ptr(s)))


def semx_set_sources_f64(ctx, elem, xi, direction, stf):
    el = np.ascontiguousarray(elem, dtype=np.int32)
    x = np.ascontiguousarray(xi, dtype=np.float64)
    d = np.ascontiguousarray(direction, dtype=np.float64)
    s = np.ascontiguousarray(stf, dtype=np.float64)
    nsrc = len(el)
    nstf = s.shape[-1] if nsrc else 0
    return _check(ctx, lib().semx_set_sources_f64(ctx, nsrc, _ptr(el), _ptr(x), _ptr(d), nstf, _ptr(s)))


def semx_set_receivers(ctx, elem, xi, nt_max: int):
    el = np.ascontiguousarray(elem, dtype=np.int32)
    x = np.ascontiguousarray(xi, dtype=np.float64)
    return _check(ctx, lib().semx_set_receivers(ctx, len(el), _ptr(el), _ptr(x), int(nt_max)))


def semx_reset(ctx):
    return _check(ctx, lib().semx_reset(ctx))


def semx_step(ctx, nsteps: int):
    return _check(ctx, lib().semx_step(ctx, int(nsteps)))


def semx_time_index(ctx) -> int:
    it = _i64()
    _check(ctx, lib().semx_time_index(ctx, ctypes.byref(it)))
    return it.value


def semx_read_seismograms(ctx, out, on_device: bool):
    return _check(ctx, lib().semx_read_seismograms(ctx, _ptr(out), 1 if on_device else 0))


def semx_get_state(ctx, u=None, v=None, a=None) -> int:
    it = _i64()
    _check(ctx, lib().semx_get_state(ctx, _ptr(u), _ptr(v), _ptr(a), ctypes.byref(it)))
    return it.value


def semx_set_state(ctx, u, v, a, it: int):
    return _check(ctx, lib().semx_set_state(ctx, _ptr(u), _ptr(v), _ptr(a), int(it)))


def semx_set_storage(ctx, storage: int):
    return _check(ctx, lib().semx_set_storage(ctx, int(storage)))


def semx_apply_force_f64(ctx, u, f):
    return _check(ctx, lib().semx_apply_force_f64(ctx, _ptr(u), _ptr(f)))


def semx_read_seismograms_f64(ctx, out, on_device: bool):
    return _check(ctx, lib().semx_read_seismograms_f64(ctx, _ptr(out), 1 if on_device else 0))


def semx_get_state_f64(ctx, u=None, v=None, a=None) -> int:
    it = _i64()
    _check(ctx, lib().semx_get_state_f64(ctx, _ptr(u), _ptr(v), _ptr(a), ctypes.byref(it)))
    return it.value


def semx_set_state_f64(ctx, u, v, a, it: int):
    return _check(ctx, lib().semx_set_state_f64(ctx, _ptr(u), _ptr(v), _ptr(a), int(it)))


def semx_stream_bandwidth(ctx, nbytes: int, reps: int) -> float:
    out = _f64()
    _check(ctx, lib().semx_stream_bandwidth(ctx, int(nbytes), int(reps), ctypes.byref(out)))
    return out.value


def semx_force_skeleton(ctx, u, f, reps: int) -> float:
    """Milliseconds per pass of the force pass's memory skeleton (f is overwritten)."""
    out = _f64()
    _check(ctx, lib().semx_force_skeleton(ctx, _ptr(u), _ptr(f), int(reps), ctypes.byref(out)))
    return out.value


def semx_energy(ctx, with_work: bool = False):
    """(kinetic, potential) of E^{n+1/2} at the current time index, plus the
    summed source work when ``with_work``."""
    k, p, w = _f64(), _f64(), _f64()
    _check(ctx, lib().semx_energy(ctx, ctypes.byref(k), ctypes.byref(p), ctypes.byref(w)))
    return (k.value, p.value, w.value) if with_work else (k.value, p.value)


def semx_set_watchdog(ctx, interval: int, max_energy: float = 0.0):
    return _check(ctx, lib().semx_set_watchdog(ctx, int(interval), float(max_energy)))


def semx_set_geometry(ctx, mode: int):
    return _check(ctx, lib().semx_set_geometry(ctx, int(mode)))


def semx_set_blocks(ctx, mode: int) -> bool:
    """Mode of the 2 x 2 x 2 element-block force kernel (SEMX_BLOCKS_OFF /
    _AUTO / _ON); returns whether the next coloured FP32 force pass uses it."""
    active = ctypes.c_int(0)
    _check(ctx, lib().semx_set_blocks(ctx, int(mode), ctypes.byref(active)))
    return bool(active.value)


def semx_set_graphs(ctx, chunk: int):
    """Steps per captured HIP graph in semx_step (0: direct launches)."""
    return _check(ctx, lib().semx_set_graphs(ctx, int(chunk)))


def semx_set_checkpointing(ctx, every: int):
    return _check(ctx, lib().semx_set_checkpointing(ctx, int(every)))


def semx_adjoint(ctx, gseis, nt: int, g_lambda, g_mu, g_rho):
    """d chi/d (lambda, mu, rho) into the three device arrays, from d chi/d seis."""
    return _check(ctx, lib().semx_adjoint(ctx, _ptr(gseis), int(nt), _ptr(g_lambda), _ptr(g_mu), _ptr(g_rho)))


def _mcheck(net, rc):
    if rc != SEMX_OK:
        msg = lib().semx_mlp_last_error(net)
        raise SemxError(rc, msg.decode() if msg else "")
    return rc


def semx_mlp_create(widths, max_batch: int, stream=None):
    h = _vp()
    w = np.ascontiguousarray(widths, dtype=np.int32)
    s = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    rc = lib().semx_mlp_create(ctypes.byref(h), len(w) - 1, _ptr(w), int(max_batch), s)
    if rc != SEMX_OK:
        raise SemxError(rc, "semx_mlp_create failed")
    return h


def semx_mlp_destroy(net):
    return lib().semx_mlp_destroy(net)


def semx_mlp_last_error(net) -> str:
    m = lib().semx_mlp_last_error(net)
    return m.decode() if m else ""


def semx_mlp_num_params(net) -> int:
    n = _i64()
    _mcheck(net, lib().semx_mlp_num_params(net, ctypes.byref(n)))
    return n.value


def semx_mlp_set_params(net, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    return _mcheck(net, lib().semx_mlp_set_params(net, _ptr(p)))


def semx_mlp_get_params(net, out):
    return _mcheck(net, lib().semx_mlp_get_params(net, _ptr(out)))


def semx_mlp_get_grads(net, out):
    return _mcheck(net, lib().semx_mlp_get_grads(net, _ptr(out)))


def semx_mlp_forward(net, x, batch: int, y):
    return _mcheck(net, lib().semx_mlp_forward(net, _ptr(x), int(batch), _ptr(y)))


def semx_mlp_forward_noalloc(net, x, batch: int, y):
    return _mcheck(net, lib().semx_mlp_forward_noalloc(net, _ptr(x), int(batch), _ptr(y)))


def semx_mlp_backward(net, dy, batch: int):
    return _mcheck(net, lib().semx_mlp_backward(net, _ptr(dy), int(batch)))


def semx_mlp_mse(net, y, t, n: int, dy=None, want_loss: bool = True):
    loss = _f64()
    _mcheck(net, lib().semx_mlp_mse(net, _ptr(y), _ptr(t), int(n), _ptr(dy), ctypes.byref(loss) if want_loss else None))
    return loss.value


def semx_mlp_adam(net, lr: float, beta1: float, beta2: float, eps: float, step: int):
    return _mcheck(net, lib().semx_mlp_adam(net, float(lr), float(beta1), float(beta2), float(eps), int(step)))


def semx_mlp_affine(net, x, rows: int, cols: int, scale, shift, y):
    """y[r][c] = scale[c] x[r][c] + shift[c] on device FP32 buffers (x may be y)."""
    return _mcheck(net, lib().semx_mlp_affine(net, _ptr(x), int(rows), int(cols), _ptr(scale), _ptr(shift), _ptr(y)))


def semx_mlp_ensemble(net, preds, members: int, rows: int, cols: int, scale, shift, mean, indicator):
    """Ensemble mean (physical units) and spread indicator of preds [members][rows][cols]."""
    return _mcheck(net, lib().semx_mlp_ensemble(net, _ptr(preds), int(members), int(rows), int(cols), _ptr(scale),
                                                _ptr(shift), _ptr(mean), _ptr(indicator)))


def semx_set_timing(ctx, stride=1):
    """Event-time every ``stride``-th force launch (True = every launch, 0 / False = off)."""
    return _check(ctx, lib().semx_set_timing(ctx, int(stride)))


def semx_force_timing(ctx):
    """(launches, total_ms) of force kernels since the last read."""
    n, ms = _i64(), _f64()
    _check(ctx, lib().semx_force_timing(ctx, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


# ---- convenience wrapper -------------------------------------------------------

class Solver:
    """One library context bound to torch's current HIP stream on ``device``;
    ``storage`` SEMX_F32 (default) or SEMX_F64 (fields and time loop in FP64)."""

    def __init__(self, ngll: int, device: str = "cuda:0", storage: int = SEMX_F32, physics: int = SEMX_ELASTIC):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.ctx = semx_create(ngll, self.stream)
        self.storage = storage
        if storage != SEMX_F32:
            semx_set_storage(self.ctx, storage)
        self.physics = physics
        self.ncomp = 1 if physics == SEMX_ACOUSTIC else 3
        if physics != SEMX_ELASTIC:
            semx_set_physics(self.ctx, physics)
        self.n = ngll
        self.nspec = self.nglob = self.nmodels = 0
        self.nrec = 0
        self.nt_max = 0

    def close(self):
        if getattr(self, "ctx", None) is not None:
            semx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upload_mesh(self, mesh):
        semx_upload_mesh(self.ctx, mesh.ibool, mesh.vert, mesh.elem_vert, mesh.nglob)
        self.nspec, self.nglob = mesh.nspec, mesh.nglob
        return semx_mesh_info(self.ctx)

    def upload_model(self, lam, mu, rho):
        lam = np.asarray(lam)
        self.nmodels = lam.shape[0] if lam.ndim == 3 else 1
        semx_upload_model(self.ctx, lam, mu, rho)

    def upload_model_acoustic(self, kappa, rho):
        kappa = np.asarray(kappa)
        self.nmodels = kappa.shape[0] if kappa.ndim == 3 else 1
        semx_upload_model_acoustic(self.ctx, kappa, rho)

    def set_mode(self, contraction=SEMX_C_F32, assembly=SEMX_ASM_COLORED):
        semx_set_mode(self.ctx, contraction, assembly)

    def empty_field(self):
        per = (self.nglob, 3) if self.ncomp == 3 else (self.nglob,)
        shape = (self.nmodels,) + per if self.nmodels > 1 else per
        dt = self.torch.float64 if self.storage == SEMX_F64 else self.torch.float32
        return self.torch.zeros(shape, dtype=dt, device=self.device)

    def apply_force(self, u, out=None):
        f = self.empty_field() if out is None else out
        if self.storage == SEMX_F64:
            semx_apply_force_f64(self.ctx, u, f)
        else:
            semx_apply_force(self.ctx, u, f)
        return f

    def setup_run(self, wl, dt=None):
        """Sources, receivers and dt from a workloads.Workload."""
        if self.storage == SEMX_F64:
            semx_set_sources_f64(self.ctx, wl.src_elem, wl.src_xi, wl.src_dir, wl.stf)
        else:
            semx_set_sources(self.ctx, wl.src_elem, wl.src_xi, wl.src_dir, wl.stf.astype(np.float32))
        semx_set_receivers(self.ctx, wl.rec_elem, wl.rec_xi, wl.nt)
        self.nrec, self.nt_max = len(wl.rec_elem), wl.nt
        semx_set_dt(self.ctx, wl.dt if dt is None else dt)
        semx_reset(self.ctx)

    def step(self, nsteps: int):
        semx_step(self.ctx, nsteps)

    def seismograms(self):
        if self.storage == SEMX_F64:
            out = np.zeros((max(self.nmodels, 1), self.nrec, self.ncomp, self.nt_max), np.float64)
            semx_read_seismograms_f64(self.ctx, out, False)
        else:
            out = np.zeros((max(self.nmodels, 1), self.nrec, self.ncomp, self.nt_max), np.float32)
            semx_read_seismograms(self.ctx, out, False)
        return out if self.nmodels > 1 else out[0]
