"""Pins of the oracle's vector-Jacobian product of L = sum w.a + sum c.phi
with respect to positions and masses (lists and tree frozen): central finite
differences of the oracle's own forward pass with frozen lists, and at theta = 0
the analytic gradient of the direct soft sum."""
import numpy as np
import pytest

from inputs import plummer
from oracle import direct


def _loss(t, w, c):
    a, ph = t.force()
    return float((w * a).sum() + (c * ph).sum())


@pytest.mark.parametrize("quad,theta", [(1, 0.5), (0, 0.6), (1, 0.0)])
def test_vjp_vs_central_fd_frozen_lists(oracle_lib, quad, theta):
    n = 600
    c = plummer(n, 31)
    mass = np.random.default_rng(7).uniform(0.5, 2.0, n)
    mass /= mass.sum()
    # r_out large enough that many pairs sit inside the changeover band
    p = dict(eps=4.0 / n, r_in=0.02, r_out=0.2, theta=theta, r_search=0.22, n_crit=32, n_leaf=8,
             use_quadrupole=quad)
    rng = np.random.default_rng(8)
    w = rng.normal(size=(n, 3))
    cw = rng.normal(size=n)
    t = oracle_lib.Tree(c.pos, mass, p)
    if theta > 0:
        assert t.counts()["n_cells"] > 0
    gp, gm = t.vjp(w, cw)
    hstep = 1e-6
    for k in rng.choice(n, 10, replace=False):
        for a in range(3):
            pp = c.pos.copy(); pp[k, a] += hstep
            t.refresh(pp, mass); lp = _loss(t, w, cw)
            pm = c.pos.copy(); pm[k, a] -= hstep
            t.refresh(pm, mass); lm = _loss(t, w, cw)
            fd = (lp - lm) / (2 * hstep)
            assert abs(gp[k, a] - fd) <= 1e-6 * (abs(fd) + 1e-3 * np.abs(gp).max()), (k, a, gp[k, a], fd)
        # L is linear in m_j through particle terms; a relative step of 1e-4 keeps
        # the cancellation error of the difference small
        hm = 1e-4 * mass[k]
        mp = mass.copy(); mp[k] += hm
        t.refresh(c.pos, mp); lp = _loss(t, w, cw)
        mm = mass.copy(); mm[k] -= hm
        t.refresh(c.pos, mm); lm = _loss(t, w, cw)
        fd = (lp - lm) / (2 * hm)
        assert abs(gm[k] - fd) <= 1e-6 * (abs(fd) + 1e-3 * np.abs(gm).max()), (k, gm[k], fd)
    t.refresh(c.pos, mass)


@pytest.mark.parametrize("r_out", [0.05, 0.3])
def test_vjp_theta0_equals_direct_gradient(oracle_lib, r_out):
    n = 800
    c = plummer(n, 32)
    p = dict(eps=4.0 / n, r_in=0.1 * r_out, r_out=r_out, theta=0.0, r_search=1.1 * r_out,
             n_crit=64, n_leaf=8)
    rng = np.random.default_rng(9)
    w = rng.normal(size=(n, 3))
    cw = rng.normal(size=n)
    gp, gm = oracle_lib.Tree(c.pos, c.mass, p).vjp(w, cw)
    gpd, gmd = direct.soft_direct_grad(c.pos, c.mass, p["eps"], p["r_in"], p["r_out"], w, cw)
    np.testing.assert_allclose(gp, gpd, rtol=0, atol=1e-11 * np.abs(gpd).max())
    np.testing.assert_allclose(gm, gmd, rtol=0, atol=1e-11 * np.abs(gmd).max())
