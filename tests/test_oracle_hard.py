"""Pins of the oracle's hard part (Section 2.1: F_hard with (1 - K), the hard
potential with (1 - W), fourth-order Hermite integration with block timesteps).

* hard + soft = plain softened Newton, force and potential, when every pair is
  listed (the soft sum and W come from the independent numpy definitions);
* the jerk is the time derivative of the hard force along straight-line motion
  (central differences);
* a circular binary inside r_in (K = 0) follows the Kepler circle, with
  fourth-order convergence in eta, and its timesteps follow the block-step
  rules applied to the exact derivatives of circular motion;
* the energy of H_hard is conserved to the integration error when pairs cross
  the changeover region, with the error falling as eta falls;
* isolated particles drift; separate clusters evolve bit for bit as if alone.
"""
import math

import numpy as np
import pytest

from oracle import direct


def _all_pairs_csr(n):
    rows = [np.array([j for j in range(n) if j != i], np.int64) for i in range(n)]
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    return off, np.concatenate(rows)


def _rel(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


@pytest.mark.parametrize("r_out", [0.05, 0.2, 0.6])
def test_hard_plus_soft_is_newton(oracle_lib, r_out):
    rng = np.random.default_rng(3)
    n = 150
    pos = rng.normal(scale=0.2, size=(n, 3))
    vel = rng.normal(size=(n, 3))
    mass = rng.uniform(0.5, 2.0, n) / n
    eps, r_in = 1e-3, 0.1 * r_out
    off, idx = _all_pairs_csr(n)
    ah, _, ph = oracle_lib.hard_force(pos, vel, mass, off, idx, eps, r_in, r_out)
    as_, ps = direct.soft_direct(pos, mass, eps, r_in, r_out)
    an, pn = direct.newton_direct(pos, mass, eps)
    assert _rel(ah + as_, an) < 1e-13
    assert _rel(ph + ps, pn) < 1e-13
    # and against the numpy hard sum over the same lists
    ad, pd = direct.hard_direct_pairs(pos, mass, eps, r_in, r_out, off, idx)
    assert _rel(ah, ad) < 1e-13 and _rel(ph, pd) < 1e-13


def test_jerk_is_time_derivative(oracle_lib):
    """Pairs spread over all three regions of K (inside r_in, changeover, beyond r_out)."""
    rng = np.random.default_rng(4)
    n = 60
    pos = rng.uniform(-0.06, 0.06, size=(n, 3))
    vel = rng.normal(size=(n, 3))
    mass = rng.uniform(0.5, 2.0, n) / n
    eps, r_in, r_out = 1e-3, 0.01, 0.1
    off, idx = _all_pairs_csr(n)
    _, jk, _ = oracle_lib.hard_force(pos, vel, mass, off, idx, eps, r_in, r_out)
    h = 1e-7
    ap, _, _ = oracle_lib.hard_force(pos + h * vel, vel, mass, off, idx, eps, r_in, r_out)
    am, _, _ = oracle_lib.hard_force(pos - h * vel, vel, mass, off, idx, eps, r_in, r_out)
    fd = (ap - am) / (2 * h)
    assert _rel(jk, fd) < 1e-7
    # the K'(s) term matters here: dropping it would fail the comparison
    s = np.linalg.norm(pos[:, None] - pos[None], axis=-1)
    assert ((s > r_in) & (s < r_out)).sum() > 100


def _binary(r0, m=0.5):
    omega = math.sqrt(2 * m / r0 ** 3)
    pos = np.array([[-r0 / 2, 0, 0], [r0 / 2, 0, 0]], float)
    vel = np.array([[0, -omega * r0 / 2, 0], [0, omega * r0 / 2, 0]], float)
    return pos, vel, np.array([m, m]), omega


def _circle(r0, omega, t):
    c, s = math.cos(omega * t), math.sin(omega * t)
    rel = r0 * np.array([c, s, 0.0])
    return np.array([-rel / 2, rel / 2])


def _binary_run(oracle_lib, eta, dt_soft, dt_max, r0=1e-3):
    pos, vel, mass, omega = _binary(r0)
    off, idx = np.array([0, 1, 2], np.int64), np.array([1, 0], np.int64)
    # r_in = 0.01 > r0: K = 0 on the whole orbit, plain Newton with eps = 0
    x, v, ns, nb = oracle_lib.hermite(pos, vel, mass, off, idx, 0.0, 0.01, 0.1, dt_soft, dt_max,
                                      eta, eta / 10, 0.0)
    return x, v, ns, nb, omega


def test_circular_binary_fourth_order(oracle_lib):
    r0 = 1e-3
    period = 2 * math.pi / math.sqrt(1.0 / r0 ** 3)
    dt_soft = 2.0 ** math.floor(math.log2(period))     # about half an orbit
    errs = []
    for eta in (0.2, 0.1, 0.05):
        x, v, ns, nb, omega = _binary_run(oracle_lib, eta, dt_soft, dt_soft)
        errs.append(np.abs(x - _circle(r0, omega, dt_soft)).max() / r0)
        assert ns[0] == ns[1] > 0
    assert errs[-1] < 1e-6
    for a, b in zip(errs, errs[1:]):
        assert 10.0 < a / b < 24.0, errs          # 2^4 per halving of eta


def _expected_steps(omega, eta, eta_s, dt_soft, dt_max):
    """Block-step rules with the exact circular-motion derivatives:
    first criterion eta_s / omega, later eta / omega."""
    d = dt_max
    while d > eta_s / omega:
        d /= 2
    t, n = 0.0, 0
    while t < dt_soft:
        t += d
        n += 1
        c = eta / omega
        if 2 * d <= c and 2 * d <= dt_max and math.fmod(t, 2 * d) == 0.0:
            d *= 2
        else:
            while d > c:
                d /= 2
    return n


def test_binary_timestep_rules(oracle_lib):
    r0 = 1e-3
    omega = math.sqrt(1.0 / r0 ** 3)
    dt_max = 2.0 ** -16
    # eta / omega sits well inside a power-of-two bracket of dt_max / 2^k
    eta = 0.75 * (dt_max / 8) * omega
    dt_soft = 4 * dt_max
    x, v, ns, nb, _ = _binary_run(oracle_lib, eta, dt_soft, dt_max, r0)
    exp = _expected_steps(omega, eta, eta / 10, dt_soft, dt_max)
    assert ns[0] == ns[1] == exp == nb


def _cluster(seed, centre, n=5, scale=0.02, m=1e-3):
    rng = np.random.default_rng(seed)
    pos = centre + rng.uniform(-scale, scale, size=(n, 3))
    vel = rng.normal(scale=0.3 * math.sqrt(n * m / scale), size=(n, 3))
    vel -= vel.mean(0)
    return pos, vel, np.full(n, m)


def _energy(oracle_lib, pos, vel, mass, off, idx, eps, r_in, r_out):
    _, _, ph = oracle_lib.hard_force(pos, vel, mass, off, idx, eps, r_in, r_out)
    return 0.5 * (mass * (vel ** 2).sum(1)).sum() + 0.5 * (mass * ph).sum()


def test_hard_energy_conservation(oracle_lib):
    pos, vel, mass = _cluster(7, np.zeros(3))
    n = len(mass)
    off, idx = _all_pairs_csr(n)
    eps, r_in, r_out = 1e-3, 0.004, 0.04
    s = np.linalg.norm(pos[:, None] - pos[None], axis=-1)[np.triu_indices(n, 1)]
    assert ((s > r_in) & (s < r_out)).any()
    e0 = _energy(oracle_lib, pos, vel, mass, off, idx, eps, r_in, r_out)
    kin = 0.5 * (mass * (vel ** 2).sum(1)).sum()
    dt_soft = 2.0 ** -3
    errs = []
    for eta in (0.4, 0.2, 0.1):
        x, v, ns, _ = oracle_lib.hermite(pos, vel, mass, off, idx, eps, r_in, r_out, dt_soft,
                                         dt_soft / 4, eta, eta / 10, 0.1 * mass[0] / r_out ** 2)
        errs.append(abs(_energy(oracle_lib, x, v, mass, off, idx, eps, r_in, r_out) - e0) / kin)
        assert (ns > 0).all()
    assert errs[-1] < 1e-6, errs
    assert errs[0] > errs[1] > errs[2], errs


def test_isolated_drift_and_cluster_independence(oracle_lib):
    pa, va, ma = _cluster(8, np.zeros(3))
    pb, vb, mb = _cluster(9, np.array([1.0, 0.0, 0.0]))
    pi, vi = np.array([[5.0, 5.0, 5.0]]), np.array([[0.1, -0.2, 0.3]])
    eps, r_in, r_out, h = 1e-3, 0.004, 0.04, 0.1
    kw = dict(dt_soft=2.0 ** -4, dt_max=2.0 ** -6, eta=0.2, eta_s=0.02, a0=0.1 * 1e-3 / r_out ** 2)

    def run(pos, vel, mass):
        off, idx = direct.brute_neighbors(pos, h)
        return oracle_lib.hermite(pos, vel, mass, off, idx, eps, r_in, r_out, **kw)

    xa, vxa, na, _ = run(pa, va, ma)
    xb, vxb, nb, _ = run(pb, vb, mb)
    pos = np.concatenate([pa, pi, pb])
    vel = np.concatenate([va, vi, vb])
    mass = np.concatenate([ma, [1e-3], mb])
    x, v, ns, _ = run(pos, vel, mass)
    k = len(ma)
    assert np.array_equal(x[:k], xa) and np.array_equal(v[:k], vxa) and np.array_equal(ns[:k], na)
    assert np.array_equal(x[k + 1:], xb) and np.array_equal(v[k + 1:], vxb)
    assert np.array_equal(ns[k + 1:], nb)
    assert np.array_equal(x[k], pi[0] + kw["dt_soft"] * vi[0]) and np.array_equal(v[k], vi[0])
    assert ns[k] == 0


def p3t_energy_errors(oracle_lib, dts, n=1024, seed=91, r_out=0.1, eta=0.01, t_end=0.125,
                      first_kick=0.5):
    """|dE/E| after t_end of the P3T step composed from oracle pieces (Section
    2.1: half kick by the soft force, the hard part over the neighbour lists
    by block-step Hermite, half kick), for each soft step in dts.  theta = 0
    makes the soft force exact; eta is small enough that the Hermite error
    sits far below the splitting error; the buffer is 3 sigma dt_soft with
    sigma = 1/sqrt(2) (Section 3.1.1).  first_kick is the fraction of the
    soft step given to the first kick (0.5 for the scheme)."""
    from inputs import plummer
    c = plummer(n, seed)
    m = c.mass
    eps = 1.0 / 256
    out = []
    for dt in dts:
        p = dict(eps=eps, r_in=0.1 * r_out, r_out=r_out, theta=0.0,
                 r_search=r_out + 3.0 / math.sqrt(2.0) * dt, n_crit=64, n_leaf=16)
        a0 = 0.1 * float(m.mean()) / r_out ** 2
        x, v = c.pos.copy(), c.vel.copy()

        def energy(x_, v_):
            _, ph = direct.newton_direct(x_, m, eps)
            return 0.5 * (m * (v_ * v_).sum(1)).sum() + 0.5 * (m * ph).sum()

        e0 = energy(x, v)
        t = oracle_lib.Tree(x, m, p)
        a, _ = t.force()
        for _ in range(int(round(t_end / dt))):
            v = v + first_kick * dt * a
            off, idx = t.neighbors()
            x, v, _, _ = oracle_lib.hermite(x, v, m, off, idx, eps, p["r_in"], r_out, dt, dt / 4,
                                            eta, eta / 10, a0)
            t = oracle_lib.Tree(x, m, p)
            a, _ = t.force()
            v = v + (1.0 - first_kick) * dt * a
        out.append(abs(energy(x, v) - e0) / abs(e0))
    return out


def test_p3t_splitting_is_second_order(oracle_lib):
    """The kick - Hermite - kick step is a symmetric (Strang) splitting of
    H_soft and H_hard, so its energy error falls four-fold per halving of the
    soft step once dt_soft sigma / r_cut is small (here 0.03 - 0.11); measured
    ratios 0.25 and 0.25.  The same composition with the whole kick before the
    hard part (a first-order splitting) halves its error per halving
    (measured 0.50 and 0.50)."""
    dts = (2.0 ** -6, 2.0 ** -7, 2.0 ** -8)
    errs = p3t_energy_errors(oracle_lib, dts, n=512)
    assert errs[0] < 1e-4, errs
    assert errs[1] < 0.35 * errs[0] and errs[2] < 0.35 * errs[1], errs
    first = p3t_energy_errors(oracle_lib, dts, n=512, first_kick=1.0)
    assert first[1] > 0.4 * first[0] and first[2] > 0.4 * first[1], first
