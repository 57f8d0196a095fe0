"""GPU O(N^2) direct sums (Newton, soft with K and W, hard with 1 - K and
1 - W; Section 2.1) against the numpy definitions, on ragged sizes, at 2^18
particles on sampled rows, and against the FP64 tree at theta = 0 (which opens
every cell, so it sums the same pairs)."""
import numpy as np
import pytest

from inputs import WORKLOADS, make_cluster, plummer
from oracle import direct
from tests.gpu_cases import log, rel_rms

pytestmark = pytest.mark.gpu

TOL = 1e-12   # FP64: same terms, different summation order and rsqrt rounding


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1506_04553_amd import P3T
    assert torch.cuda.is_available()
    c = P3T(0)
    yield c
    c.close()


def _p(n, r_out=0.05):
    return dict(eps=4.0 / max(n, 64), r_in=0.1 * r_out, r_out=r_out, theta=0.5,
                r_search=1.1 * r_out, n_crit=64, n_leaf=16)


def _all_pairs(n):
    off = np.arange(n + 1, dtype=np.int64) * (n - 1)
    idx = np.array([j for i in range(n) for j in range(n) if j != i], np.int64)
    return off, idx


def _oracle(mode, pos, mass, p):
    if mode == "newton":
        return direct.newton_direct(pos, mass, p["eps"])
    if mode == "soft":
        return direct.soft_direct(pos, mass, p["eps"], p["r_in"], p["r_out"])
    off, idx = _all_pairs(len(mass))
    return direct.hard_direct_pairs(pos, mass, p["eps"], p["r_in"], p["r_out"], off, idx)


def _err(got, ref, scale):
    """RMS error relative to the RMS of the Newton sum (the summands' scale;
    the hard sum can vanish)."""
    return float(np.sqrt(((got - ref) ** 2).sum() / (scale ** 2).sum()))


def _gpu(ctx, mode, pos, mass, p):
    import torch
    a, ph = ctx.direct(torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda(), mode, **p)
    return a.cpu().numpy(), ph.cpu().numpy()


@pytest.mark.parametrize("mode", ["newton", "soft", "hard"])
@pytest.mark.parametrize("n", [2, 255, 257, 1500, 3000])
def test_direct_matches_definition(ctx, mode, n):
    c = plummer(max(n, 4), 100 + n)
    pos, mass = c.pos[:n].copy(), c.mass[:n].copy()
    p = _p(n, r_out=0.3)        # a wide changeover band: many pairs inside r_out
    a, ph = _gpu(ctx, mode, pos, mass, p)
    oa, oph = _oracle(mode, pos, mass, p)
    na, nph = direct.newton_direct(pos, mass, p["eps"])
    ea, ep = _err(a, oa, na), _err(ph, oph, nph)
    log(f"direct {mode} n={n}: acc {ea:.1e} pot {ep:.1e}")
    assert ea < TOL and ep < TOL


def test_direct_single_particle_and_split_identity(ctx):
    a, ph = _gpu(ctx, "newton", np.zeros((1, 3)), np.ones(1), _p(1))
    assert not a.any() and not ph.any()
    # hard + soft = Newton on the GPU itself (each already checked against its definition)
    n = 600
    c = plummer(n, 7)
    p = _p(n, r_out=0.5)
    ah, ph_h = _gpu(ctx, "hard", c.pos, c.mass, p)
    as_, ph_s = _gpu(ctx, "soft", c.pos, c.mass, p)
    an, ph_n = _gpu(ctx, "newton", c.pos, c.mass, p)
    assert rel_rms(ah + as_, an) < TOL and rel_rms(ph_h + ph_s, ph_n) < TOL


def test_direct_plummer256k_sampled_rows(ctx):
    """The 2^18 Plummer workload (its r_out and softening): soft sums on 64
    sampled particles against the definition evaluated row by row."""
    w = WORKLOADS["plummer256k"]
    c = make_cluster(w, seed=1)
    p = w.params()
    a, ph = _gpu(ctx, "soft", c.pos, c.mass, p)
    rng = np.random.default_rng(8)
    rows = rng.choice(w.n, 64, replace=False)
    gamma = p["r_in"] / p["r_out"]
    ea, ep = [], []
    for i in rows:
        d = c.pos - c.pos[i]
        s2 = (d * d).sum(1) + p["eps"] ** 2
        s = np.sqrt(s2)
        y = s / p["r_out"]
        K = direct.K_np(y, gamma)
        W = direct.W_over_y_np(y, gamma) * y
        f = c.mass * K / (s2 * s)
        f[i] = 0.0
        ph_i = -(c.mass * W / s)
        ph_i[i] = 0.0
        ra = (f[:, None] * d).sum(0)
        # relative to the summands' magnitude (the net force of a row can nearly cancel)
        ea.append(np.linalg.norm(a[i] - ra) / np.abs(f[:, None] * d).sum())
        ep.append(abs(ph[i] - ph_i.sum()) / abs(ph_i.sum()))
    log(f"direct soft 2^18 sampled rows: max rel acc {max(ea):.1e} pot {max(ep):.1e}")
    assert max(ea) < 1e-13 and max(ep) < 1e-12


def test_tree_theta0_equals_direct_soft(ctx):
    """FP64 tree at theta = 0 against the direct soft sum, 2^16 particles: two
    independent GPU paths over the same pairs."""
    import torch
    n = 1 << 16
    c = plummer(n, 12)
    p = dict(eps=4.0 / n, r_in=0.0004, r_out=0.004, theta=0.0, r_search=0.0044, n_crit=128,
             n_leaf=16, precision="fp64")
    pos, mass = torch.from_numpy(c.pos).cuda(), torch.from_numpy(c.mass).cuda()
    ctx.build_tree(pos, mass, **p)
    at, pt = ctx.long_force()
    ad, pd = ctx.direct(pos, mass, "soft", **p)
    ea = rel_rms(at.cpu().numpy(), ad.cpu().numpy())
    ep = rel_rms(pt.cpu().numpy(), pd.cpu().numpy())
    log(f"tree theta=0 vs direct soft n={n}: acc {ea:.1e} pot {ep:.1e}")
    assert ea < TOL and ep < TOL
