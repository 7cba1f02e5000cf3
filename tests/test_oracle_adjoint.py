"""Pin of the oracle's discrete adjoint: its gradients must equal central
finite differences of the same FP64 misfit (the exact gradient of the
discrete chi), on small jittered heterogeneous meshes, for random
directions in lambda, mu and rho."""
import numpy as np
import pytest

import workloads as W


def _problem(orc, n=4, ne=(2, 2, 2), nt=40, seed=0):
    m = W.box_mesh(ne, n, 2000.0, jitter=0.12, seed=seed)
    lam, mu, rho = W.layered_model(m, vp_layers=(3000.0, 2500.0), grf_amp=0.05, grf_seed=seed,
                                   grf_corr_elems=1.0)
    gam, jac, _ = orc.geometry(n, m.elem_vert, m.vert)
    dt = 2e-3
    se = np.array([0], np.int32); sx = np.array([[0.3, -0.2, 0.4]]); sd = np.array([[0.3, 0.2, 1.0]])
    stf = W.ricker(25.0, 0.04, dt, nt + 1)[None, :]
    re = np.array([m.nspec - 1, 1], np.int32); rx = np.array([[0.1, 0.5, 1.0], [-0.4, 0.2, 0.9]])
    return m, lam, mu, rho, gam, jac, dt, nt, se, sx, sd, stf, re, rx


def _chi(orc, P, lam, mu, rho, data):
    m, _, _, _, gam, jac, dt, nt, se, sx, sd, stf, re, rx = P
    s = orc.forward(m.n, m.ibool, gam, jac, lam, mu, rho, m.nglob, dt, nt, se, sx, sd, stf, re, rx)["seis"]
    return orc.misfit(s, data, dt), s


@pytest.mark.parametrize("n,seed", [(3, 1), (4, 2)])
def test_adjoint_matches_central_differences(orc, n, seed):
    P = _problem(orc, n=n, seed=seed)
    m, lam, mu, rho, gam, jac, dt, nt, se, sx, sd, stf, re, rx = P
    rng = np.random.default_rng(seed)
    # observed data: the same run in a slightly different model
    _, data = _chi(orc, P, lam * 1.02, mu * 0.97, rho, np.zeros((len(re), 3, nt)))
    chi0, s0 = _chi(orc, P, lam, mu, rho, data)
    gseis = dt * (s0 - data)
    gl, gm, gr = orc.adjoint(m.n, m.ibool, gam, jac, lam, mu, rho, m.nglob, dt, nt, se, sx, sd, stf, re, rx, gseis)
    for k in range(4):
        dl = lam * rng.standard_normal(lam.shape)
        dm = mu * rng.standard_normal(mu.shape)
        dr = rho * rng.standard_normal(rho.shape)
        if k == 1:
            dm[:] = 0; dr[:] = 0
        elif k == 2:
            dl[:] = 0; dr[:] = 0
        elif k == 3:
            dl[:] = 0; dm[:] = 0
        eps = 1e-6
        cp, _ = _chi(orc, P, lam + eps * dl, mu + eps * dm, rho + eps * dr, data)
        cm, _ = _chi(orc, P, lam - eps * dl, mu - eps * dm, rho - eps * dr, data)
        fd = (cp - cm) / (2 * eps)
        ad = np.sum(gl * dl) + np.sum(gm * dm) + np.sum(gr * dr)
        assert abs(ad - fd) <= 1e-7 * abs(fd) + 1e-12 * chi0, (k, ad, fd)


def test_adjoint_of_linear_functional_is_reciprocal(orc):
    """For chi = <w, seis> the lambda-gradient must not depend on w's scale
    other than linearly (a plausible bookkeeping slip -- a missing factor on
    the adjoint source -- breaks this)."""
    P = _problem(orc, n=3, seed=3)
    m, lam, mu, rho, gam, jac, dt, nt, se, sx, sd, stf, re, rx = P
    w = np.random.default_rng(5).standard_normal((len(re), 3, nt))
    g1 = orc.adjoint(m.n, m.ibool, gam, jac, lam, mu, rho, m.nglob, dt, nt, se, sx, sd, stf, re, rx, w)
    g2 = orc.adjoint(m.n, m.ibool, gam, jac, lam, mu, rho, m.nglob, dt, nt, se, sx, sd, stf, re, rx, 3.0 * w)
    for a, b in zip(g1, g2):
        np.testing.assert_allclose(b, 3.0 * a, rtol=1e-12, atol=1e-30)
