"""Pins of the oracle's particle kinds (Section 3.2.2, the SMBH runs: a cutoff
radius and a softening per kind of pair; between SMBHs no split and no
softening; a timestep accuracy per kind).

* with no special particle the kinds change nothing, bit for bit;
* soft + hard = plain Newton with each pair's own softening, when every pair
  is listed (the soft sum of normal pairs from the plain numpy definition);
* two special particles whose pair is not split follow the unsoftened Kepler
  circle with fourth-order convergence in their own eta, and their step
  counts follow the block-step rules under that eta;
* a split special pair inside its r_in integrates exactly like an unsplit one
  (K = 0 there);
* neighbour sets: symmetric, special pairs always present when not split.
"""
import math

import numpy as np

from oracle import direct

KINDS = dict(n_special=2, r_in_ns=0.003, r_out_ns=0.03, eps_ns=2e-3, split_ss=0, r_in_ss=0.0,
             r_out_ss=1.0, eps_ss=0.0, eta_sp=0.03, eta_s_sp=0.003)


def _system(seed, n_normal=40, scale=0.02):
    rng = np.random.default_rng(seed)
    pos = np.concatenate([rng.normal(scale=scale, size=(n_normal, 3)),
                          np.array([[-0.01, 0.0, 0.0], [0.01, 0.0, 0.0]])])
    vel = rng.normal(scale=0.1, size=(n_normal + 2, 3))
    mass = np.concatenate([np.full(n_normal, 1e-4), [0.01, 0.01]])
    return pos, vel, mass


def _all_pairs(n):
    off = np.arange(n + 1, dtype=np.int64) * (n - 1)
    idx = np.array([j for i in range(n) for j in range(n) if j != i], np.int64)
    return off, idx


def test_no_special_particle_changes_nothing(oracle_lib):
    pos, vel, mass = _system(1)
    off, idx = direct.brute_neighbors(pos, 0.02)
    none = dict(KINDS, n_special=0)
    a0, j0, p0 = oracle_lib.hard_force(pos, vel, mass, off, idx, 1e-3, 0.001, 0.01)
    a1, j1, p1 = oracle_lib.hard_force(pos, vel, mass, off, idx, 1e-3, 0.001, 0.01, kinds=none)
    assert np.array_equal(a0, a1) and np.array_equal(j0, j1) and np.array_equal(p0, p1)
    kw = dict(dt_soft=2.0 ** -8, dt_max=2.0 ** -10, eta=0.1, eta_s=0.01, a0=1.0)
    x0 = oracle_lib.hermite(pos, vel, mass, off, idx, 1e-3, 0.001, 0.01, **kw)
    x1 = oracle_lib.hermite(pos, vel, mass, off, idx, 1e-3, 0.001, 0.01, **kw, kinds=none)
    assert all(np.array_equal(u, v) for u, v in zip(x0[:3], x1[:3]))


def test_soft_plus_hard_is_newton_with_pair_softening(oracle_lib):
    pos, vel, mass = _system(2)
    n = len(mass)
    ns = KINDS["n_special"]
    eps, r_in, r_out = 1e-3, 0.002, 0.02
    off, idx = _all_pairs(n)
    ah, _, ph = oracle_lib.hard_force(pos, vel, mass, off, idx, eps, r_in, r_out, kinds=KINDS)
    # soft: normal pairs by the plain soft sum over the normal particles, the rest by kinds
    asn, psn = direct.soft_direct(pos[:n - ns], mass[:n - ns], eps, r_in, r_out)
    ak, pk = direct.kinds_soft(pos, mass, eps, r_in, r_out, KINDS)
    asoft = ak.copy()
    psoft = pk.copy()
    asoft[:n - ns] += asn
    psoft[:n - ns] += psn
    # Newton with the softening of each pair's kind, written out
    an = np.zeros((n, 3))
    pn = np.zeros(n)
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            si, sj = i >= n - ns, j >= n - ns
            e = KINDS["eps_ss"] if si and sj else KINDS["eps_ns"] if si or sj else eps
            d = pos[j] - pos[i]
            s = math.sqrt(float(d @ d) + e * e)
            an[i] += mass[j] * d / s ** 3
            pn[i] -= mass[j] / s
    assert np.abs(ah + asoft - an).max() <= 1e-13 * np.abs(an).max()
    assert np.abs(ph + psoft - pn).max() <= 1e-13 * np.abs(pn).max()


def _special_binary(r0=0.5, m=0.5):
    omega = math.sqrt(2 * m / r0 ** 3)
    pos = np.array([[10.0, 0, 0], [-r0 / 2, 0, 0], [r0 / 2, 0, 0]])
    vel = np.array([[0.0, 0, 0], [0, -omega * r0 / 2, 0], [0, omega * r0 / 2, 0]])
    mass = np.array([1e-6, m, m])
    off = np.array([0, 0, 1, 2], np.int64)          # the two special particles list each other
    idx = np.array([2, 1], np.int32)
    return pos, vel, mass, off, idx, omega


def _circle(r0, omega, t):
    c, s = math.cos(omega * t), math.sin(omega * t)
    rel = r0 * np.array([c, s, 0.0])
    return np.array([-rel / 2, rel / 2])


def test_unsplit_special_pair_is_a_kepler_circle(oracle_lib):
    r0 = 0.5
    pos, vel, mass, off, idx, omega = _special_binary(r0)
    dt_soft = 2.0 ** math.floor(math.log2(2 * math.pi / omega))
    errs = []
    for eta in (0.2, 0.1, 0.05):
        kinds = dict(KINDS, eta_sp=eta, eta_s_sp=eta / 10)
        # the normal particles' eta is far smaller: only the special eta may act
        x, v, ns, _ = oracle_lib.hermite(pos, vel, mass, off, idx, 1e-3, 0.01, 0.1, dt_soft,
                                         dt_soft, 1e-6, 1e-7, 0.0, kinds=kinds)
        errs.append(np.abs(x[1:] - _circle(r0, omega, dt_soft)).max() / r0)
        assert ns[0] == 0 and ns[1] == ns[2] > 0
        assert np.array_equal(x[0], pos[0])          # isolated: drifts with v = 0
    for a, b in zip(errs, errs[1:]):
        assert 10.0 < a / b < 24.0, errs


def test_special_eta_sets_the_steps(oracle_lib):
    pos, vel, mass, off, idx, omega = _special_binary()
    dt_max = 2.0 ** -4
    eta = 0.75 * (dt_max / 8) * omega
    kinds = dict(KINDS, eta_sp=eta, eta_s_sp=eta / 10)
    _, _, ns, _ = oracle_lib.hermite(pos, vel, mass, off, idx, 1e-3, 0.01, 0.1, 4 * dt_max,
                                     dt_max, 1e-6, 1e-7, 0.0, kinds=kinds)
    d = dt_max
    while d > eta / 10 / omega:
        d /= 2
    t, exp = 0.0, 0
    while t < 4 * dt_max:
        t += d
        exp += 1
        if 2 * d <= eta / omega and 2 * d <= dt_max and math.fmod(t, 2 * d) == 0.0:
            d *= 2
        else:
            while d > eta / omega:
                d /= 2
    assert ns[1] == ns[2] == exp


def test_split_pair_inside_r_in_matches_unsplit(oracle_lib):
    pos, vel, mass, off, idx, omega = _special_binary(r0=0.5)
    kw = dict(dt_soft=2.0 ** -3, dt_max=2.0 ** -5, eta=0.1, eta_s=0.01, a0=0.0)
    unsplit = dict(KINDS, eps_ss=1e-3)
    split = dict(unsplit, split_ss=1, r_in_ss=2.0, r_out_ss=20.0)   # separation < r_in
    a = oracle_lib.hermite(pos, vel, mass, off, idx, 1e-3, 0.01, 0.1, **kw, kinds=unsplit)
    b = oracle_lib.hermite(pos, vel, mass, off, idx, 1e-3, 0.01, 0.1, **kw, kinds=split)
    assert all(np.array_equal(u, v) for u, v in zip(a[:3], b[:3]))


def test_kinds_neighbors():
    pos, _, _ = _system(3)
    n = len(pos)
    off, idx = direct.kinds_neighbors(pos, 2, 0.01, 0.03, 0, 0.0)
    pairs = {(i, int(j)) for i in range(n) for j in idx[off[i]:off[i + 1]]}
    assert all((j, i) in pairs for i, j in pairs)
    assert (n - 2, n - 1) in pairs
    for i, j in pairs:
        r = np.linalg.norm(pos[i] - pos[j])
        if i < n - 2 and j < n - 2:
            assert r < 0.01
        elif not (i >= n - 2 and j >= n - 2):
            assert r < 0.03
