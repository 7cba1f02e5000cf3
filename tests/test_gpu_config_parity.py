"""Seismogram parity of the FP32 time loop against the FP64 oracle at the
workloads' own sizes.

The expected seismograms come from ``tests/golden/make_config_seismograms.py``
(the oracle only); the inputs are regenerated here from the same seeds and
checked against the stored fingerprint.  Bar: relative L2 <= 1e-4 over all
receivers, components and samples (the stated seismogram tolerance after
1000 steps; the 64^3 case runs its 2000 steps).

  layered16  16^3 jittered layered cube, 8 receivers, 1000 steps (coloured and atomic)
  adjoint32  32^3 layered cube with the -5 % anomaly, 64 receivers, 1000 steps
  layered64  64^3 jittered layered cube, 8 receivers, 2000 steps; the error
             over the first 100 steps is reported too (those samples are
             exactly zero on both sides: the first arrival reaches the
             receivers later, so the 2000-step figure is the one that counts)
"""
import os
import sys

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import rel_l2

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_config_seismograms as G  # noqa: E402

TOL_SEIS = 1e-4


def _golden(case):
    path = os.path.join(HERE, "golden", f"seis_{case}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (python tests/golden/make_config_seismograms.py {case})")
    return np.load(path)


def _run(case, assembly=None):
    import paper_2606_12850_amd as P
    g = _golden(case)
    wl = G.workload(case)
    assert G.fingerprint(wl) == str(g["fingerprint"]), "inputs differ from the ones the oracle ran"
    wl.dt = float(g["dt"])
    wl.stf = W.ricker(10.0, 0.12, wl.dt, wl.nt + 1)[None, :]
    s = P.Solver(5)
    s.upload_mesh(wl.mesh)
    s.upload_model(wl.lam, wl.mu, wl.rho)
    if assembly is not None:
        s.set_mode(P.SEMX_C_F32, assembly)
    s.setup_run(wl)
    s.step(wl.nt)
    seis = s.seismograms()
    s.close()
    return seis, g["seis"].astype(np.float64), g


@pytest.mark.parametrize("assembly", ["colored", "atomic"])
def test_layered16_1000_steps(assembly):
    import paper_2606_12850_amd as P
    seis, ref, _ = _run("layered16", P.SEMX_ASM_COLORED if assembly == "colored" else P.SEMX_ASM_ATOMIC)
    err = rel_l2(seis, ref)
    print(f"layered 16^3 jittered, 1000 steps, {assembly}: rel L2 {err:.3e}")
    assert err <= TOL_SEIS


def test_adjoint32_1000_steps():
    seis, ref, _ = _run("adjoint32")
    err = rel_l2(seis, ref)
    per_rec = [rel_l2(seis[r], ref[r]) for r in range(ref.shape[0])]
    print(f"layered 32^3 + anomaly, 64 receivers, 1000 steps: rel L2 {err:.3e} "
          f"(worst receiver {max(per_rec):.3e})")
    assert err <= TOL_SEIS


def test_layered64_2000_steps():
    seis, ref, _ = _run("layered64")
    err = rel_l2(seis, ref)
    err100 = rel_l2(seis[..., :100], ref[..., :100])
    print(f"layered 64^3 jittered, 8 receivers: 2000 steps rel L2 {err:.3e}; first 100 steps {err100:.3e} "
          f"(peak |s| over them {np.abs(ref[..., :100]).max():.2e} of {np.abs(ref).max():.2e})")
    assert err <= TOL_SEIS
