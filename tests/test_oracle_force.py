"""Pins of the oracle's tree force and potential (Section 2.1 force split,
Section 2.2 tree).

theta = 0 opens every cell, so the tree result must equal the direct soft sum
(with W taken from K by quadrature); limits of the cutoffs reduce it to closed
forms; the Plummer model's potential is textbook; the quadrupole must improve
on the monopole at fixed theta.
"""
import math

import numpy as np
import pytest

from inputs import plummer
from oracle import direct


def _rel_rms(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def _p(n, **kw):
    d = dict(eps=4.0 / n, r_in=0.005, r_out=0.05, theta=0.0, r_search=0.055, n_crit=64, n_leaf=8)
    d.update(kw)
    return d


@pytest.mark.parametrize("quad", [0, 1])
@pytest.mark.parametrize("r_out", [0.02, 0.08, 0.3])
def test_theta0_equals_direct_sum(oracle_lib, quad, r_out):
    c = plummer(1200, 11)
    mass = np.random.default_rng(5).uniform(0.2, 3.0, 1200)
    mass /= mass.sum()
    p = _p(1200, r_out=r_out, r_in=0.1 * r_out, r_search=1.1 * r_out, use_quadrupole=quad)
    t = oracle_lib.Tree(c.pos, mass, p)
    a, ph = t.force()
    ad, pd = direct.soft_direct(c.pos, mass, p["eps"], p["r_in"], p["r_out"])
    assert _rel_rms(a, ad) < 1e-13
    assert _rel_rms(ph, pd) < 1e-13


def test_outer_cutoff_below_softening_is_newton(oracle_lib):
    c = plummer(1000, 12)
    eps = 0.05
    p = dict(eps=eps, r_in=0.001, r_out=0.01, theta=0.0, r_search=0.011, n_crit=64, n_leaf=8)
    a, ph = oracle_lib.Tree(c.pos, c.mass, p).force()
    an, pn = direct.newton_direct(c.pos, c.mass, eps)
    assert _rel_rms(a, an) < 1e-13 and _rel_rms(ph, pn) < 1e-13


@pytest.mark.parametrize("theta", [0.0, 0.5])
def test_inner_cutoff_beyond_all_pairs(oracle_lib, theta):
    """r_in larger than every softened pair distance: K = 0, W = C(gamma) y."""
    c = plummer(700, 13)
    ext = np.sqrt(((c.pos.max(0) - c.pos.min(0)) ** 2).sum()) * 1.01 + 1.0
    g = 0.1
    p = dict(eps=0.01, r_in=ext, r_out=ext / g, theta=theta, r_search=1.1 * ext / g,
             n_crit=32, n_leaf=8)
    t = oracle_lib.Tree(c.pos, c.mass, p)
    a, ph = t.force()
    assert np.all(a == 0.0)
    Cg = oracle_lib.C_gamma(g)
    exp = -Cg * (c.mass.sum() - c.mass) / p["r_out"]
    np.testing.assert_allclose(ph, exp, rtol=1e-13)
    assert t.counts()["n_cells"] == 0


def test_momentum_balance_theta0(oracle_lib):
    c = plummer(1500, 14)
    mass = np.random.default_rng(6).uniform(0.1, 5.0, 1500)
    mass /= mass.sum()
    a, _ = oracle_lib.Tree(c.pos, mass, _p(1500)).force()
    f = mass[:, None] * a
    assert np.abs(f.sum(0)).max() < 1e-14 * np.abs(f).sum()


def test_long_plus_short_is_newton(oracle_lib):
    """Soft part over the tree + hard part over the neighbour lists = full force."""
    c = plummer(2000, 15)
    p = _p(2000, r_out=0.1, r_in=0.01, r_search=0.11, theta=0.0)
    t = oracle_lib.Tree(c.pos, c.mass, p)
    a, ph = t.force()
    off, idx = t.neighbors()
    ah, phh = direct.hard_direct_pairs(c.pos, c.mass, p["eps"], p["r_in"], p["r_out"], off, idx)
    an, pn = direct.newton_direct(c.pos, c.mass, p["eps"])
    assert _rel_rms(a + ah, an) < 1e-12
    assert _rel_rms(ph + phh, pn) < 1e-12


def test_plummer_closed_form(oracle_lib):
    n = 20000
    c = plummer(n, 16)
    p = dict(eps=4.0 / n, r_in=0.0005, r_out=0.005, theta=0.5, r_search=0.0055, n_crit=128,
             n_leaf=16)
    t = oracle_lib.Tree(c.pos, c.mass, p)
    a, ph = t.force()
    off, idx = t.neighbors()
    ah, phh = direct.hard_direct_pairs(c.pos, c.mass, p["eps"], p["r_in"], p["r_out"], off, idx)
    phi = ph + phh
    acc = a + ah
    r = np.sqrt((c.pos ** 2).sum(1))
    edges = np.quantile(r, np.linspace(0.02, 0.9, 12))
    for lo_, hi_ in zip(edges[:-1], edges[1:]):
        sel = (r >= lo_) & (r < hi_)
        rm = r[sel].mean()
        assert abs(phi[sel].mean() - direct.plummer_potential(rm)) < 0.02 * abs(direct.plummer_potential(rm))
        ar = -(acc[sel] * c.pos[sel]).sum(1) / r[sel]
        assert abs(ar.mean() - direct.plummer_accel(rm)) < 0.06 * direct.plummer_accel(rm) + 0.02
    # total potential energy of the virialised model: W = 1/2 sum m phi -> -1/2
    assert abs(0.5 * (c.mass * phi).sum() + 0.5) < 0.02


def test_quadrupole_beats_monopole_and_error_shrinks(oracle_lib):
    c = plummer(4000, 17)
    p = _p(4000)
    ad, pd = direct.soft_direct(c.pos, c.mass, p["eps"], p["r_in"], p["r_out"])
    errs = {}
    for quad in (0, 1):
        for th in (0.25, 0.5, 0.8):
            a, ph = oracle_lib.Tree(c.pos, c.mass, dict(p, theta=th, use_quadrupole=quad)).force()
            errs[quad, th] = (_rel_rms(a, ad), _rel_rms(ph, pd))
    for th in (0.25, 0.5):
        assert errs[1, th][0] < 0.5 * errs[0, th][0]
        assert errs[1, th][1] < 0.5 * errs[0, th][1]
    assert errs[1, 0.8][0] < errs[0, 0.8][0] and errs[1, 0.8][1] < errs[0, 0.8][1]
    for quad in (0, 1):
        assert errs[quad, 0.25][0] < errs[quad, 0.5][0] < errs[quad, 0.8][0]
    # expansion order: halving theta gains more with the quadrupole than without
    gain_mono = errs[0, 0.5][0] / errs[0, 0.25][0]
    gain_quad = errs[1, 0.5][0] / errs[1, 0.25][0]
    assert gain_quad > gain_mono


def test_single_far_cell_multipole_order(oracle_lib):
    """Two well-separated clumps: the quadrupole error falls faster with distance."""
    rng = np.random.default_rng(18)
    clump = rng.normal(0, 0.05, (64, 3))
    m = rng.uniform(0.5, 1.5, 64)
    errs = {0: [], 1: []}
    for dist in (2.0, 12.0):
        probe = np.array([[dist, 0.3, -0.2]])
        pos = np.concatenate([clump, probe])
        mass = np.concatenate([m, [1e-9]])
        for quad in (0, 1):
            # theta = 10 accepts every cell that does not contain the probe
            p = dict(eps=1e-4, r_in=1e-4, r_out=1e-3, theta=10.0, r_search=1.1e-3, n_crit=1,
                     n_leaf=64, use_quadrupole=quad)
            t = oracle_lib.Tree(pos, mass, p)
            a, ph = t.force()
            assert t.counts()["n_cells"] >= 1
            an, pn = direct.newton_direct(pos, mass, 1e-4)
            errs[quad].append(np.abs(a[-1] - an[-1]).max() / np.abs(an[-1]).max())
    # relative force error: monopole ~ dist^-2 (ratio 36), quadrupole ~ dist^-3 (ratio 216)
    assert 20.0 < errs[0][0] / errs[0][1] < 60.0
    assert errs[1][0] / errs[1][1] > 120.0
    assert errs[1][0] < 0.2 * errs[0][0]
