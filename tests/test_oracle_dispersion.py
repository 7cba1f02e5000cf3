"""Pins of the oracle's Bloch dispersion analysis (no GPU).

The Bloch eigenproblem is assembled from the oracle's own element force, so
these tests pin that operator through its plane-wave spectrum:
  * linear elements (N = 1) with lumped mass reduce, for waves along a
    lattice axis, to the 1-D lattice omega = (2 c / h) sin(k h / 2);
  * for every order, a P or S wave along a lattice axis reduces exactly to the
    1-D GLL spectral element problem (the cross-axis terms telescope to zero
    across periodic neighbours), re-derived independently in tests/indep.py;
  * the relative error decays like (k h)^{2N} (spectral accuracy of GLL
    elements with lumped mass, Sec. II-B; the paper's dispersion study relies
    on it), and at long wavelength every direction propagates at the
    continuum P and S speeds of isotropic Hooke's law;
  * k = 0 leaves exactly the three rigid translations at zero frequency.
"""
import numpy as np
import pytest

from oracle import dispersion as Dp
from tests import indep

H = 100.0
# vp/vs = 2.5, so lambda != mu: a swapped pair of Lame moduli changes both speeds
RHO = 2200.0
VP, VS = 4000.0, 1600.0
MU = RHO * VS * VS
LAM = RHO * VP * VP - 2.0 * MU


def main_branch(branches):
    return max(branches, key=lambda b: b[2])[0]


@pytest.fixture(scope="module")
def elem():
    cache = {}

    def get(n):
        if n not in cache:
            cache[n] = Dp.element_matrices(n, H, LAM, MU, RHO)
        return cache[n]
    return get


def test_element_stiffness_symmetric_psd(elem):
    for n in (2, 4):
        K, m = elem(n)
        assert np.max(np.abs(K - K.T)) <= 1e-12 * np.max(np.abs(K))
        ev = np.linalg.eigvalsh(0.5 * (K + K.T))
        assert ev[0] >= -1e-10 * ev[-1]
        assert np.all(m > 0) and abs(m.sum() - RHO * H ** 3) <= 1e-9 * RHO * H ** 3


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_linear_element_closed_form(elem, axis):
    K, m = elem(2)
    cp, cs = VP, VS
    for kh in (0.3, 1.0, 2.5):
        kvec = np.zeros(3); kvec[axis] = kh / H
        pol_s = np.zeros(3); pol_s[(axis + 1) % 3] = 1.0
        pol_p = np.zeros(3); pol_p[axis] = 1.0
        wp = main_branch(Dp.plane_wave_branches(2, H, K, m, kvec, [pol_p])[0])
        ws = main_branch(Dp.plane_wave_branches(2, H, K, m, kvec, [pol_s])[0])
        np.testing.assert_allclose(wp, 2 * cp / H * np.sin(kh / 2), rtol=1e-12)
        np.testing.assert_allclose(ws, 2 * cs / H * np.sin(kh / 2), rtol=1e-12)


@pytest.mark.parametrize("n", [3, 4, 5, 6, 7, 8])
def test_axis_waves_equal_1d_sem(elem, n):
    K, m = elem(n)
    for kh in (0.7, 1.9, 2.6, 4.0):
        k = kh / H
        for axis, pol, c in ((0, [1, 0, 0], VP), (0, [0, 1, 0], VS), (2, [1, 0, 0], VS), (1, [0, 1, 0], VP)):
            kvec = np.zeros(3); kvec[axis] = k
            w = main_branch(Dp.plane_wave_branches(n, H, K, m, kvec, [pol])[0])
            np.testing.assert_allclose(w, indep.sem1d_bloch_omega(n, H, c, k), rtol=1e-11)


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_spectral_convergence_axis(elem, n):
    """Error ratio between 9 and 18 points per wavelength: 2^{2N}."""
    K, m = elem(n)
    N = n - 1
    for wave in "PS":
        e9 = Dp.dispersion_error(n, H, LAM, MU, RHO, [1, 0, 0], 9.0, wave, K, m)["error"]
        e18 = Dp.dispersion_error(n, H, LAM, MU, RHO, [1, 0, 0], 18.0, wave, K, m)["error"]
        assert e9 < 0 and e18 < 0  # lumped GLL mass: axis waves are slow
        assert abs(np.log2(e9 / e18) - 2 * N) <= 0.25


@pytest.mark.parametrize("n", [3, 4])
def test_spectral_convergence_oblique(elem, n):
    """Off-axis the P and S error terms mix before the asymptotic range, so
    the ratio is taken between 18 and 36 points per wavelength (at higher
    orders the error there is at the eigen-solver's rounding level)."""
    K, m = elem(n)
    N = n - 1
    for d in ([1, 2, 0], [1, 1, 1], [1, 2, 3]):
        for wave in "PS":
            e18 = Dp.dispersion_error(n, H, LAM, MU, RHO, d, 18.0, wave, K, m)["error"]
            e36 = Dp.dispersion_error(n, H, LAM, MU, RHO, d, 36.0, wave, K, m)["error"]
            assert abs(np.log2(abs(e18 / e36)) - 2 * N) <= 0.25


@pytest.mark.parametrize("n", [3, 5])
def test_long_wave_isotropic_speeds(elem, n):
    K, m = elem(n)
    for d in ([1, 0, 0], [0, 1, 1], [1, 1, 1], [1, 2, 3], [-3, 1, 2]):
        for wave in "PS":
            r = Dp.dispersion_error(n, H, LAM, MU, RHO, d, 60.0, wave, K, m)
            assert not r["boundary"] and r["captured"] > 0.9999
            assert max(abs(e) for e in r["branches"]) <= 1e-5


def test_cubic_symmetry(elem):
    K, m = elem(4)
    for wave in "PS":
        ref = Dp.dispersion_error(4, H, LAM, MU, RHO, [1, 0, 0], 5.0, wave, K, m)["error"]
        for d in ([0, 1, 0], [0, 0, 1], [-1, 0, 0]):
            e = Dp.dispersion_error(4, H, LAM, MU, RHO, d, 5.0, wave, K, m)["error"]
            assert abs(e - ref) <= 1e-12
        ref = Dp.dispersion_error(4, H, LAM, MU, RHO, [1, 1, 1], 5.0, wave, K, m)["error"]
        for d in ([-1, 1, 1], [1, -1, 1], [1, 1, -1]):
            e = Dp.dispersion_error(4, H, LAM, MU, RHO, d, 5.0, wave, K, m)["error"]
            assert abs(e - ref) <= 1e-12


@pytest.mark.parametrize("n", [3, 5])
def test_rigid_translations(elem, n):
    K, m = elem(n)
    w, V, Mr = Dp.bloch_modes(n, H, K, m, [0.0, 0.0, 0.0])
    assert np.all(w[:3] <= 1e-6 * w[-1])
    assert w[3] >= 1e-2 * w[-1]


def test_zone_boundary_split(elem):
    """At k h = 2 pi (N = 5, 5 points per wavelength) k and -k coincide as
    Bloch vectors: the wave is carried by two standing modes, both close to
    c k; at 5.5 points per wavelength by one travelling mode."""
    K, m = elem(6)
    r = Dp.dispersion_error(6, H, LAM, MU, RHO, [1, 0, 0], 5.0, "P", K, m)
    assert r["boundary"] and len(r["branches"]) == 2 and r["captured"] > 0.999
    e0, e1 = r["branches"]
    assert e0 < e1 and abs(e0) < 0.02 and abs(e1) < 0.02
    r = Dp.dispersion_error(6, H, LAM, MU, RHO, [1, 0, 0], 5.5, "P", K, m)
    assert not r["boundary"] and len(r["branches"]) == 1 and r["captured"] > 0.999


def test_shear_branches(elem):
    """Along [100] and [111] the two S polarisations are degenerate by
    symmetry (one eigenspace); along [1,2,3] the discrete lattice splits
    them into two quasi-S branches."""
    K, m = elem(4)
    for d in ([1, 0, 0], [1, 1, 1]):
        r = Dp.dispersion_error(4, H, LAM, MU, RHO, d, 5.0, "S", K, m)
        assert len(r["branches"]) == 1 and r["captured"] > 0.99
    r = Dp.dispersion_error(4, H, LAM, MU, RHO, [1, 2, 3], 5.0, "S", K, m)
    assert len(r["branches"]) == 2 and r["captured"] > 0.98
    assert abs(r["branches"][0] - r["branches"][1]) > 1e-6


def test_mode_on_lattice_is_bloch_periodic():
    n, N = 4, 3
    k = np.array([2 * np.pi / (5 * H), 0.0, 4 * np.pi / (5 * H)])
    v = np.arange(3 * N ** 3) + 1j
    g = np.arange(5 * N)
    phi = Dp.mode_on_lattice(n, H, v, k, g, np.zeros_like(g), np.zeros_like(g))
    # one element to the right multiplies by exp(i k_x h)
    np.testing.assert_allclose(phi[N:], phi[:-N] * np.exp(1j * k[0] * H), rtol=1e-13)
    x = Dp.lattice_coordinates(n, H, g, g, g)
    assert np.all(np.diff(x[:, 0]) > 0) and abs(x[N, 0] - H) < 1e-12


@pytest.mark.parametrize("n,m,wave", [(4, (3, 0, 0), "P"), (4, (2, 2, 2), "S"), (5, (1, 2, 0), "S")])
def test_periodic_mesh_time_loop_recovers_bloch_frequency(n, m, wave):
    """The assembled operator of a periodic 5^3-element box (wrap-around
    numbering), stepped in FP64 from a sampled plane wave, projected on the
    Bloch mode and fitted, gives the one-element Bloch frequency: pins the
    Bloch reduction against the assembled operator, and the projection and
    fit that the GPU dispersion test uses."""
    import workloads as W
    mesh = W.box_mesh(5, n, 5 * H, periodic=True)
    pw = Dp.periodic_plane_wave(mesh, LAM, MU, RHO, m, wave)
    assert pw["captured"] > 0.99
    dt = 0.3 * 0.17 * H / VP
    s = Dp.newmark_free(mesh, LAM, MU, RHO, pw["u0"], dt, 60, pw["w"])
    omega_h, omega_run = Dp.fit_frequency(s, dt)
    assert abs(omega_h / pw["omega_h"] - 1.0) <= 1e-10
    # the run's frequency is the central-difference image of omega_h
    assert abs(omega_run - 2.0 / dt * np.arcsin(pw["omega_h"] * dt / 2.0)) <= 1e-9 * omega_run


# --- axis (1-D) Bloch analysis and the equal-accuracy table --------------------

@pytest.mark.parametrize("n", [3, 5, 8, 12, 16])
def test_axis_omega_equals_independent_1d(n):
    for kh in (0.7, 1.9, 4.0, 9.0):
        if kh > 0.9 * np.pi * (n - 1):
            continue
        assert abs(Dp.axis_omega(n, kh) / indep.sem1d_bloch_omega(n, 1.0, 1.0, kh) - 1.0) <= 1e-11


@pytest.mark.parametrize("n", [3, 4, 6])
def test_axis_omega_equals_3d_operator(elem, n):
    """The cheap 1-D routine is the 3-D operator's frequency along an axis
    (assembled from the oracle force), for both wave speeds."""
    K, m = elem(n)
    for kh in (0.9, 2.3):
        for pol, c in (([1, 0, 0], VP), ([0, 0, 1], VS)):
            w3 = main_branch(Dp.plane_wave_branches(n, H, K, m, [kh / H, 0, 0], [pol])[0])
            assert abs(w3 * H / c / Dp.axis_omega(n, kh) - 1.0) <= 1e-11


def test_axis_linear_closed_form_and_crossing():
    for kh in (0.2, 1.0, 2.5):
        assert abs(Dp.axis_omega(2, kh) - 2.0 * np.sin(kh / 2.0)) <= 1e-13
    # linear elements: error(ppw) = sin(pi/ppw) ppw/pi - 1; its eps-crossing by a root finder
    from scipy.optimize import brentq
    for eps in (1e-3, 1e-4):
        ref = brentq(lambda p: 1.0 - np.sin(np.pi / p) * p / np.pi - eps, 3.0, 3000.0, xtol=1e-12)
        assert abs(Dp.iso_accuracy_ppw(2, eps) / ref - 1.0) <= 1e-8


@pytest.mark.parametrize("n", [4, 8, 16])
def test_iso_accuracy_ppw_is_the_last_crossing(n):
    for eps in (1e-3, 1e-5):
        p = Dp.iso_accuracy_ppw(n, eps)
        assert abs(abs(Dp.axis_error(n, p)) / eps - 1.0) <= 1e-3
        for q in np.geomspace(p * 1.001, 3 * p, 25):
            assert abs(Dp.axis_error(n, q)) <= eps


def test_iso_accuracy_table_reproducible():
    """tests/golden/iso_accuracy.json is what its generator writes from the
    oracle (values rounded to 6 decimals)."""
    import json
    import os
    import importlib.util
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_iso_accuracy", os.path.join(here, "make_iso_accuracy.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with open(os.path.join(here, "iso_accuracy.json")) as fh:
        stored = json.load(fh)
    fresh = mod.table()
    assert stored["eps"] == fresh["eps"] and stored["ngll"] == fresh["ngll"]
    np.testing.assert_allclose(stored["ppw"], fresh["ppw"], rtol=0, atol=2e-6)
    # fewer points per wavelength are needed as the order grows (asymptotic range)
    for row in stored["ppw"]:
        assert row[0] > row[3] > row[6] > row[14]


@pytest.mark.parametrize("n,m,wave", [(4, 4, "P"), (6, 3, "S")])
def test_periodic_axis_wave_from_1d_mode(n, m, wave):
    """The 1-D Bloch mode, extended uniformly across the axis, is an exact
    mode of the assembled periodic 3-D operator: the FP64 time loop projected
    on it recovers the 1-D frequency, which is also the 3-D Bloch one."""
    import workloads as W
    mesh = W.box_mesh(5, n, 5 * H, periodic=True)
    pw = Dp.periodic_axis_wave(mesh, LAM, MU, RHO, m, wave)
    dt = 0.03 * H / VP
    s = Dp.newmark_free(mesh, LAM, MU, RHO, pw["u0"], dt, 60, pw["w"])
    omega_h, _ = Dp.fit_frequency(s, dt)
    assert abs(omega_h / pw["omega_h"] - 1.0) <= 1e-10
    pw3 = Dp.periodic_plane_wave(mesh, LAM, MU, RHO, (m, 0, 0), wave)
    assert abs(pw3["omega_h"] / pw["omega_h"] - 1.0) <= 1e-11
