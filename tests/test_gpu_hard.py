"""GPU hard part (Section 2.1 H_hard, Section 2.2 GPU procedure) against the
oracle: the (1 - K) force and jerk over neighbour lists, the block-timestep
Hermite integration of one soft step, and the whole P3T step.

The force and jerk of a list are the same IEEE operation sequence on both
sides (no contraction, correctly rounded division and square root), so they
must agree bit for bit, and so must the Hermite trajectories and step counts
built from them.  The potential uses the device logarithm in the changeover
region and is compared to 1e-14 relative.
"""
import math

import numpy as np
import pytest

import oracle
from inputs import plummer
from oracle import direct
from tests.gpu_cases import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1506_04553_amd import P3T
    assert torch.cuda.is_available()
    c = P3T(0)
    yield c
    c.close()


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _clumpy(n, seed, scale, vscale):
    """A Plummer sphere shrunk by `scale` (velocities by `vscale`), so that its
    neighbour pairs sample the changeover region of K (and, for the densest
    case, the region inside r_in)."""
    c = plummer(n, seed)
    return c.pos * scale, c.vel * vscale, c.mass


CASES = [(2048, 61, 0.004, 0.1, 3.0), (5000, 62, 0.01, 0.2, 2.0), (3000, 63, 0.02, 0.1, 3.0)]


def _params(r_out, eps=1e-4):
    return dict(eps=eps, r_in=0.1 * r_out, r_out=r_out, theta=0.5, r_search=1.1 * r_out,
                n_crit=64, n_leaf=16)


def _run_hard(ctx, pos, vel, mass, off, idx, p):
    import torch
    a, j, ph = ctx.hard_force(_dev(pos), _dev(vel), _dev(mass), _dev(off, torch.int64),
                              _dev(idx, torch.int32), **p)
    return a.cpu().numpy(), j.cpu().numpy(), ph.cpu().numpy()


@pytest.mark.parametrize("n,seed,r_out,sc,vs", CASES)
def test_hard_force_bit_exact(ctx, n, seed, r_out, sc, vs):
    pos, vel, mass = _clumpy(n, seed, sc, vs)
    p = _params(r_out)
    off, idx = direct.brute_neighbors(pos, p["r_search"])
    log(f"hard force n={n} pairs={len(idx)} isolated={(np.diff(off) == 0).sum()}")
    assert len(idx) > 300
    a, j, ph = _run_hard(ctx, pos, vel, mass, off, idx, p)
    oa, oj, oph = oracle.hard_force(pos, vel, mass, off, idx, p["eps"], p["r_in"], p["r_out"])
    assert np.array_equal(a, oa) and np.array_equal(j, oj)
    assert np.max(np.abs(ph - oph)) <= 1e-14 * np.max(np.abs(oph))
    assert not a[np.diff(off) == 0].any()


def _hermite_kw(r_out, mass, dt_soft=2.0 ** -7, eta=0.1):
    # the block-step bound is far above what these cases need (< 10^4)
    return dict(dt_soft=dt_soft, dt_max=dt_soft / 4, eta=eta, eta_s=eta / 10,
                a0=0.1 * float(np.mean(mass)) / r_out ** 2, max_block_steps=200000)


def _okw(hk):
    return {k: hk[k] for k in ("dt_soft", "dt_max", "eta", "eta_s", "a0")}


def _run_hermite(ctx, pos, vel, mass, off, idx, p, hk):
    import torch
    x, v = _dev(pos), _dev(vel)
    ns, st = ctx.hermite_hard(x, v, _dev(mass), _dev(off, torch.int64), _dev(idx, torch.int32),
                              hk, **p)
    return x.cpu().numpy(), v.cpu().numpy(), ns.cpu().numpy(), st


@pytest.mark.parametrize("n,seed,r_out,sc,vs", CASES)
def test_hermite_matches_oracle(ctx, n, seed, r_out, sc, vs):
    pos, vel, mass = _clumpy(n, seed, sc, vs)
    p = _params(r_out)
    off, idx = direct.brute_neighbors(pos, p["r_search"])
    hk = _hermite_kw(r_out, mass)
    x, v, ns, st = _run_hermite(ctx, pos, vel, mass, off, idx, p, hk)
    ox, ov, ons, _ = oracle.hermite(pos, vel, mass, off, idx, p["eps"], p["r_in"], p["r_out"],
                                    **_okw(hk))
    log(f"hermite n={n}: {st}")
    assert np.array_equal(ns, ons)
    assert np.array_equal(x, ox) and np.array_equal(v, ov)
    assert st["n_hard"] == int((np.diff(off) > 0).sum())
    assert st["steps"] == int(ons.sum())


def test_hermite_edge_cases(ctx):
    import torch
    from paper_1506_04553_amd.p3t import P3TError
    rng = np.random.default_rng(70)
    pos = rng.uniform(-1, 1, (64, 3))
    vel = rng.normal(size=(64, 3))
    mass = np.full(64, 1.0 / 64)
    p = _params(0.01)
    hk = _hermite_kw(0.01, mass)
    # every particle isolated: pure drift, no steps
    off = np.zeros(65, np.int64)
    idx = np.zeros(1, np.int32)
    x, v, ns, st = _run_hermite(ctx, pos, vel, mass, off, idx, p, hk)
    assert np.array_equal(x, pos + hk["dt_soft"] * vel) and np.array_equal(v, vel)
    assert not ns.any() and st["n_hard"] == 0 and st["n_clusters"] == 0
    # one pair
    pos2 = pos.copy()
    pos2[1] = pos2[0] + np.array([0.003, 0.0, 0.0])
    off2 = np.zeros(65, np.int64)
    off2[1:] = 2
    off2[1] = 1
    idx2 = np.array([1, 0], np.int32)
    x, v, ns, st = _run_hermite(ctx, pos2, vel, mass, off2, idx2, p, hk)
    ox, ov, ons, _ = oracle.hermite(pos2, vel, mass, off2, idx2, p["eps"], p["r_in"], p["r_out"],
                                    **_okw(hk))
    assert np.array_equal(x, ox) and np.array_equal(ns, ons) and st["n_clusters"] == 1
    # malformed lists are rejected before any integration
    for bad in (np.array([0, 1], np.int32), np.array([1, 64], np.int32)):
        with pytest.raises(P3TError) as e:
            _run_hermite(ctx, pos2, vel, mass, off2, bad, p, hk)
        assert e.value.status == -1
    asym = np.zeros(65, np.int64)
    asym[1:] = 1                           # 0 lists 1, 1 lists nothing
    with pytest.raises(P3TError) as e:
        _run_hermite(ctx, pos2, vel, mass, asym, np.array([1], np.int32), p, hk)
    assert e.value.status == -1
    # a block-step limit set from the host ends the call with ELIMIT
    with pytest.raises(P3TError) as e:
        _run_hermite(ctx, pos2, vel, mass, off2, idx2, p, dict(hk, max_block_steps=2))
    assert e.value.status == -6
    # dt_soft must be a whole multiple of dt_max
    with pytest.raises(P3TError) as e:
        _run_hermite(ctx, pos2, vel, mass, off2, idx2, p, dict(hk, dt_max=hk["dt_soft"] / 3))
    assert e.value.status == -1


def test_hermite_dense_clusters_global_index_path(ctx):
    """Components whose lists outgrow the LDS index areas of their size class
    (every pair within h: 60 members, 3540 entries; 200 members, 39800
    entries) read their indices from the global copy; a 7-member component
    fills its packed lane group.  All bit for bit against the oracle."""
    rng = np.random.default_rng(90)
    parts = []
    for k, (m, rad) in enumerate(((60, 0.004), (200, 0.004), (7, 0.004))):
        centre = np.array([k * 1.0, 0.0, 0.0])
        d = rng.normal(size=(m, 3))
        d *= (rad * rng.uniform(0, 1, m) ** (1 / 3) / np.linalg.norm(d, axis=1))[:, None]
        parts.append(centre + d)
    pos = np.concatenate(parts)
    n = len(pos)
    vel = rng.normal(scale=0.05, size=(n, 3))
    mass = np.full(n, 1e-6)
    p = dict(eps=1e-4, r_in=0.001, r_out=0.01, theta=0.5, r_search=0.011, n_crit=64, n_leaf=16)
    off, idx = direct.brute_neighbors(pos, p["r_search"])
    assert len(idx) == 60 * 59 + 200 * 199 + 7 * 6
    hk = _hermite_kw(p["r_out"], mass, dt_soft=2.0 ** -10)
    x, v, ns, st = _run_hermite(ctx, pos, vel, mass, off, idx, p, hk)
    ox, ov, ons, _ = oracle.hermite(pos, vel, mass, off, idx, p["eps"], p["r_in"], p["r_out"],
                                    **_okw(hk))
    log(f"dense clusters: {st}")
    assert st["n_clusters"] == 3 and st["max_cluster"] == 200
    assert np.array_equal(ns, ons)
    assert np.array_equal(x, ox) and np.array_equal(v, ov)


def test_hermite_king_1m_sampled_clusters(ctx):
    """The King W0=9, N=2^20 workload's own neighbour lists (h = 1.1 r_out):
    the whole GPU integration, checked bit for bit on the particles of sampled
    clusters (the largest ones and random ones) integrated alone by the oracle
    -- clusters evolve independently (pinned on the oracle)."""
    import torch
    from inputs import WORKLOADS, make_cluster
    w_ = WORKLOADS["king9_1m"]
    c = make_cluster(w_, seed=1)
    p = w_.params(precision="fp64")
    pos, vel, mass = _dev(c.pos), _dev(c.vel), _dev(c.mass)
    ctx.build_tree(pos, mass, **p)
    off, idx = ctx.neighbors()
    hk = _hermite_kw(p["r_out"], c.mass, dt_soft=w_.extra["dt"])
    x, v = pos.clone(), vel.clone()
    ns, st = ctx.hermite_hard(x, v, mass, off, idx, hk, **p)
    log(f"king9_1m hermite: {st}")
    off, idx = off.cpu().numpy(), idx.cpu().numpy()
    x, v, ns = x.cpu().numpy(), v.cpu().numpy(), ns.cpu().numpy()
    hard = np.diff(off) > 0
    iso = ~hard
    assert np.array_equal(x[iso], c.pos[iso] + hk["dt_soft"] * c.vel[iso])
    # components on the host
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    g = sp.csr_matrix((np.ones(len(idx)), idx, off), shape=(len(off) - 1,) * 2)
    ncomp, lab = connected_components(g, directed=False)
    sizes = np.bincount(lab[hard])
    comps = [k for k in np.argsort(-sizes)[:3] if sizes[k] > 0]
    rng = np.random.default_rng(5)
    cand = np.unique(lab[hard])
    comps += list(rng.choice(cand, size=min(20, len(cand)), replace=False))
    sel = np.nonzero(np.isin(lab, comps) & hard)[0]
    remap = -np.ones(len(off) - 1, np.int64)
    remap[sel] = np.arange(len(sel))
    rows = [remap[idx[off[i]:off[i + 1]]] for i in sel]
    soff = np.zeros(len(sel) + 1, np.int64)
    soff[1:] = np.cumsum([len(r) for r in rows])
    sidx = np.concatenate(rows).astype(np.int32)
    assert (sidx >= 0).all()
    ox, ov, ons, _ = oracle.hermite(c.pos[sel], c.vel[sel], c.mass[sel], soff, sidx, p["eps"],
                                    p["r_in"], p["r_out"],
                                    **_okw(hk))
    log(f"  checked {len(sel)} particles in {len(comps)} clusters (largest {sizes.max()})")
    assert np.array_equal(ns[sel], ons)
    assert np.array_equal(x[sel], ox) and np.array_equal(v[sel], ov)
    assert st["n_hard"] == int(hard.sum()) and st["max_cluster"] == int(sizes.max())


def test_p3t_step_matches_oracle_composition(ctx):
    """One P3T step (kick, hard part over the lists of the build, rebuild,
    force, kick) against the same sequence composed from oracle pieces, FP64."""
    import torch
    n = 4096
    c = plummer(n, 81)
    p = dict(eps=4.0 / n, r_in=0.003, r_out=0.03, theta=0.5, r_search=0.04, n_crit=64,
             n_leaf=16, precision="fp64")
    hk = _hermite_kw(p["r_out"], c.mass, dt_soft=2.0 ** -6)
    pos, vel, mass = _dev(c.pos), _dev(c.vel), _dev(c.mass)
    ctx.build_tree(pos, mass, **p)
    acc, _ = ctx.long_force()
    st = ctx.step(pos, vel, mass, acc, hk, **p)
    log(f"p3t step n={n}: {st}")
    # oracle composition
    t0 = oracle.Tree(c.pos, c.mass, p)
    a0, _ = t0.force()
    off, idx = t0.neighbors()
    v1 = c.vel + 0.5 * hk["dt_soft"] * a0
    x2, v2, ns, _ = oracle.hermite(c.pos, v1, c.mass, off, idx, p["eps"], p["r_in"], p["r_out"],
                                   **_okw(hk))
    a2, _ = oracle.Tree(x2, c.mass, p).force()
    v3 = v2 + 0.5 * hk["dt_soft"] * a2
    gx, gv, ga = pos.cpu().numpy(), vel.cpu().numpy(), acc.cpu().numpy()
    ex = np.abs(gx - x2).max() / np.abs(x2).max()
    ev = np.sqrt(((gv - v3) ** 2).sum() / (v3 ** 2).sum())
    ea = np.sqrt(((ga - a2) ** 2).sum() / (a2 ** 2).sum())
    log(f"  pos max rel {ex:.2e}  vel rel-RMS {ev:.2e}  acc rel-RMS {ea:.2e}")
    assert st["n_hard"] == int((np.diff(off) > 0).sum()) and st["n_hard"] > 0
    assert ex < 1e-12 and ev < 1e-12 and ea < 1e-12


def test_p3t_energy_conservation(ctx):
    """Whole P3T steps of a Plummer cluster (N = 512) over 1/8 time unit: the
    total energy (kinetic plus the softened Newton potential of the direct
    sum) is conserved to the splitting error of the scheme, which is second
    order (Section 2.1: half kick, Hermite, half kick), so each halving of
    the soft step cuts the error four-fold.  theta = 0 makes the soft force
    exact, eta = 0.01 puts the Hermite error far below the splitting error,
    r_out = 0.1 keeps dt_soft sigma / r_cut small (0.03 - 0.11) and the buffer
    is 3 sigma dt_soft (Section 3.1.1).  The errors match those of the same
    steps composed from oracle pieces."""
    from tests.test_oracle_hard import p3t_energy_errors
    n = 512
    c = plummer(n, 91)
    r_out, eta = 0.1, 0.01
    mass = _dev(c.mass)
    dts = (2.0 ** -6, 2.0 ** -7, 2.0 ** -8)

    def energy(pos, vel, p):
        _, ph = ctx.direct(pos, mass, "newton", **p)
        return float(0.5 * (mass * (vel * vel).sum(1)).sum() + 0.5 * (mass * ph).sum())

    errs = []
    for dt in dts:
        p = dict(eps=1.0 / 256, r_in=0.1 * r_out, r_out=r_out, theta=0.0,
                 r_search=r_out + 3.0 / math.sqrt(2.0) * dt, n_crit=64, n_leaf=16,
                 precision="fp64")
        pos, vel = _dev(c.pos), _dev(c.vel)
        e0 = energy(pos, vel, p)
        ctx.build_tree(pos, mass, **p)
        acc, _ = ctx.long_force(want_pot=False)
        hk = dict(dt_soft=dt, dt_max=dt / 4, eta=eta, eta_s=eta / 10,
                  a0=0.1 * float(c.mass.mean()) / r_out ** 2, max_block_steps=200000)
        steps = int(round(0.125 / dt))
        n_hard = 0
        for _ in range(steps):
            st = ctx.step(pos, vel, mass, acc, hk, **p)
            n_hard = max(n_hard, st["n_hard"])
        errs.append(abs(energy(pos, vel, p) - e0) / abs(e0))
        log(f"p3t energy: dt_soft {dt:g}, {steps} steps, up to {n_hard} hard particles, "
            f"|dE/E| {errs[-1]:.3e}")
        assert n_hard > 0
    ref = p3t_energy_errors(oracle, dts, n=n, r_out=r_out, eta=eta)
    log(f"  oracle composition: {['%.3e' % e for e in ref]}; ratios "
        f"{errs[1] / errs[0]:.3f} {errs[2] / errs[1]:.3f}")
    assert errs[0] < 1e-4
    assert errs[1] < 0.35 * errs[0] and errs[2] < 0.35 * errs[1], errs
    for g, o in zip(errs, ref):
        assert abs(g - o) <= 0.01 * o, (errs, ref)


def test_null_index_array_through_the_abi(ctx):
    """idx may be NULL only when every row is empty: then the hard force is zero
    and the Hermite call drifts every particle; with a non-empty row the call is
    rejected by the offsets-only check, before any kernel reads an entry.  The
    kinds neighbour lists check the caller's normal lists the same way."""
    import ctypes as C
    import torch
    from paper_1506_04553_amd.p3t import (HermiteParams, HermiteStats, Kinds, P3T_EINVAL, P3T_OK,
                                          make_params)
    L, h = ctx._L, ctx._h
    rng = np.random.default_rng(71)
    n = 40
    pos, vel = _dev(rng.uniform(-1, 1, (n, 3))), _dev(rng.normal(size=(n, 3)))
    mass = _dev(np.full(n, 1.0 / n))
    p = make_params(**_params(0.01))
    empty = _dev(np.zeros(n + 1, np.int64))
    one = np.zeros(n + 1, np.int64)
    one[1:] = 1
    one = _dev(one)
    acc = torch.full((n, 3), 7.0, dtype=torch.float64, device="cuda")
    jerk = torch.full((n, 3), 7.0, dtype=torch.float64, device="cuda")
    args = lambda off: (h, n, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), off.data_ptr(), None,
                        C.byref(p), None, acc.data_ptr(), jerk.data_ptr(), None)
    assert L.p3t_hard_force(*args(empty)) == P3T_OK
    torch.cuda.synchronize()
    assert not acc.any() and not jerk.any()
    assert L.p3t_hard_force(*args(one)) == P3T_EINVAL
    log(f"  NULL idx with an entry: {L.p3t_last_error(h).decode()}")
    hp = HermiteParams(2.0 ** -7, 2.0 ** -9, 0.1, 0.01, 0.0, 0)
    st = HermiteStats()
    x0 = pos.clone()
    assert L.p3t_hermite_hard(h, n, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(),
                              empty.data_ptr(), None, C.byref(p), None, C.byref(hp), None,
                              C.byref(st)) == P3T_OK
    torch.cuda.synchronize()
    assert torch.equal(pos, x0 + 2.0 ** -7 * vel) and st.n_hard == 0
    assert L.p3t_hermite_hard(h, n, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(),
                              one.data_ptr(), None, C.byref(p), None, C.byref(hp), None,
                              C.byref(st)) == P3T_EINVAL
    # kinds: the normal lists (first n - 2 rows) must be well formed
    kd = Kinds(n_special=2, r_in_ns=0.001, r_out_ns=0.01, r_search_ns=0.011, eps_ns=1e-4,
               split_ss=0, eta_sp=0.03, eta_s_sp=0.003)
    out_off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    out_idx = torch.empty(64, dtype=torch.int32, device="cuda")
    nnz = C.c_int64(0)
    nn_empty = _dev(np.zeros(n - 1, np.int64))
    assert L.p3t_kinds_neighbors(h, n, pos.data_ptr(), C.byref(kd), nn_empty.data_ptr(), None,
                                 out_off.data_ptr(), out_idx.data_ptr(), 64, C.byref(nnz)) == P3T_OK
    asym = np.zeros(n - 1, np.int64)
    asym[1:] = 1                             # 0 lists 1, 1 lists nothing
    asym, bad = _dev(asym), _dev(np.array([1], np.int32))
    assert L.p3t_kinds_neighbors(h, n, pos.data_ptr(), C.byref(kd), asym.data_ptr(),
                                 bad.data_ptr(), out_off.data_ptr(), out_idx.data_ptr(), 64,
                                 C.byref(nnz)) == P3T_EINVAL


def test_hermite_every_packing(ctx):
    """Components of every packing of the small-component kernels, bit for bit
    against the oracle: about 40 members (one per 64 lanes, list in LDS, terms
    spread over the lanes), 20 (two per wavefront), 10 (four), 5 (eight) and 2
    (sixteen), with counts that leave the last wavefront of each packing partly
    empty, so that finished and idle lane groups step beside live ones."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    rng = np.random.default_rng(91)
    parts, k = [], 0
    for members, count, rad in ((40, 3, 0.012), (20, 5, 0.008), (10, 9, 0.006), (5, 17, 0.004),
                                (2, 33, 0.003)):
        for _ in range(count):
            d = rng.normal(size=(members, 3))
            d *= (rad * rng.uniform(0, 1, members) ** (1 / 3) / np.linalg.norm(d, axis=1))[:, None]
            parts.append(np.array([k * 0.5, 0.0, 0.0]) + d)
            k += 1
    pos = np.concatenate(parts)
    n = len(pos)
    vel = rng.normal(scale=0.05, size=(n, 3))
    mass = np.full(n, 1e-6)
    p = dict(eps=1e-4, r_in=0.001, r_out=0.01, theta=0.5, r_search=0.011, n_crit=64, n_leaf=16)
    off, idx = direct.brute_neighbors(pos, p["r_search"])
    hard = np.diff(off) > 0
    _, lab = connected_components(csr_matrix((np.ones(len(idx)), idx, off), shape=(n, n)),
                                  directed=False)
    sizes = np.bincount(lab[hard])
    sizes = sizes[sizes > 0]
    for lo, hi in ((2, 4), (4, 8), (8, 16), (16, 32), (32, 64)):
        assert ((sizes >= lo) & (sizes < hi)).any(), (lo, hi)
    hk = _hermite_kw(p["r_out"], mass, dt_soft=2.0 ** -6)
    x, v, ns, st = _run_hermite(ctx, pos, vel, mass, off, idx, p, hk)
    ox, ov, ons, _ = oracle.hermite(pos, vel, mass, off, idx, p["eps"], p["r_in"], p["r_out"],
                                    **_okw(hk))
    log(f"every packing: {st}; sizes {np.bincount(np.minimum(sizes, 64))[1:].tolist()}")
    assert np.array_equal(ns, ons)
    assert np.array_equal(x, ox) and np.array_equal(v, ov)


def test_asymmetric_lists_are_rejected(ctx):
    """Every row non-empty but the lists not symmetric (2 lists 0, 0 does not
    list 2): the hard force, the Hermite integration and the kinds neighbour
    merge must reject them with EINVAL before any kernel uses them, and leave
    the outputs untouched."""
    import ctypes as C
    import torch
    from paper_1506_04553_amd.p3t import (HermiteParams, HermiteStats, Kinds, P3T_EINVAL, P3T_OK,
                                          make_params)
    L, h = ctx._L, ctx._h
    rng = np.random.default_rng(72)
    n = 4
    pos, vel = _dev(rng.uniform(-0.002, 0.002, (n, 3))), _dev(rng.normal(size=(n, 3)))
    mass = _dev(np.full(n, 1.0 / n))
    p = make_params(**_params(0.01))
    # rows: 0 -> {1}, 1 -> {0, 3}, 2 -> {0}, 3 -> {1}
    off = _dev(np.array([0, 1, 3, 4, 5], np.int64))
    idx = _dev(np.array([1, 0, 3, 0, 1], np.int32))
    acc = torch.full((n, 3), 7.0, dtype=torch.float64, device="cuda")
    jerk = torch.full((n, 3), 7.0, dtype=torch.float64, device="cuda")
    rc = L.p3t_hard_force(h, n, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), off.data_ptr(),
                          idx.data_ptr(), C.byref(p), None, acc.data_ptr(), jerk.data_ptr(), None)
    assert rc == P3T_EINVAL, rc
    log(f"  asymmetric lists: {L.p3t_last_error(h).decode()}")
    torch.cuda.synchronize()
    assert bool((acc == 7.0).all()) and bool((jerk == 7.0).all())
    hp = HermiteParams(2.0 ** -7, 2.0 ** -9, 0.1, 0.01, 0.0, 0)
    st = HermiteStats()
    x0 = pos.clone()
    assert L.p3t_hermite_hard(h, n, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(),
                              off.data_ptr(), idx.data_ptr(), C.byref(p), None, C.byref(hp), None,
                              C.byref(st)) == P3T_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(pos, x0)
    # the same lists made symmetric (0 also lists 2) are accepted
    off_s = _dev(np.array([0, 2, 4, 5, 6], np.int64))
    idx_s = _dev(np.array([1, 2, 0, 3, 0, 1], np.int32))
    rc = L.p3t_hard_force(h, n, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(),
                          off_s.data_ptr(), idx_s.data_ptr(), C.byref(p), None, acc.data_ptr(),
                          jerk.data_ptr(), None)
    assert rc == P3T_OK, rc
    # kinds: the same asymmetric rows as the normal particles' lists of six
    # particles, the last two special
    kd = Kinds(n_special=2, r_in_ns=0.001, r_out_ns=0.01, r_search_ns=0.011, eps_ns=1e-4,
               split_ss=0, eta_sp=0.03, eta_s_sp=0.003)
    pos6 = _dev(rng.uniform(-0.002, 0.002, (6, 3)))
    out_off = torch.full((7,), -7, dtype=torch.int64, device="cuda")
    out_idx = torch.empty(64, dtype=torch.int32, device="cuda")
    nnz = C.c_int64(0)
    assert L.p3t_kinds_neighbors(h, 6, pos6.data_ptr(), C.byref(kd), off.data_ptr(),
                                 idx.data_ptr(), out_off.data_ptr(), out_idx.data_ptr(), 64,
                                 C.byref(nnz)) == P3T_EINVAL
    torch.cuda.synchronize()
    assert bool((out_off == -7).all())
    assert L.p3t_kinds_neighbors(h, 6, pos6.data_ptr(), C.byref(kd), off_s.data_ptr(),
                                 idx_s.data_ptr(), out_off.data_ptr(), out_idx.data_ptr(), 64,
                                 C.byref(nnz)) == P3T_OK


def test_step_after_released_lists(ctx):
    """p3t_step reads the build's near lists for its neighbour search: after
    p3t_release_lists it must walk the tree again first, and give bit for bit
    the step it gives without the release."""
    n = 4096
    c = plummer(n, 82)
    p = dict(eps=4.0 / n, r_in=0.003, r_out=0.03, theta=0.5, r_search=0.04, n_crit=64,
             n_leaf=16, precision="mixed")
    hk = _hermite_kw(p["r_out"], c.mass, dt_soft=2.0 ** -6)
    out = []
    for release in (False, True):
        pos, vel, mass = _dev(c.pos), _dev(c.vel), _dev(c.mass)
        ctx.build_tree(pos, mass, **p)
        acc, _ = ctx.long_force()
        if release:
            ctx.release_lists()
        st = ctx.step(pos, vel, mass, acc, hk, **p)
        out.append([t.cpu().numpy() for t in (pos, vel, acc)] + [st["n_hard"], st["steps"]])
    a, b = out
    assert all(np.array_equal(u, v) for u, v in zip(a[:3], b[:3]))
    assert a[3:] == b[3:] and a[3] > 0
    log(f"  step after release: identical ({a[3]} hard particles, {a[4]} Hermite steps)")


def test_step_rejects_search_radius_below_r_out(ctx):
    """The step's lists must hold every pair inside r_out (h = r_cut + a buffer,
    Section 2.2): r_search < r_out is EINVAL, positions untouched."""
    from paper_1506_04553_amd import P3TError
    from paper_1506_04553_amd.p3t import P3T_EINVAL
    n = 1024
    c = plummer(n, 83)
    p = dict(eps=4.0 / n, r_in=0.003, r_out=0.03, theta=0.5, r_search=0.02, n_crit=64,
             n_leaf=16, precision="fp64")
    hk = _hermite_kw(p["r_out"], c.mass, dt_soft=2.0 ** -6)
    pos, vel, mass = _dev(c.pos), _dev(c.vel), _dev(c.mass)
    ctx.build_tree(pos, mass, **p)
    acc, _ = ctx.long_force()
    with pytest.raises(P3TError) as e:
        ctx.step(pos, vel, mass, acc, hk, **p)
    assert e.value.status == P3T_EINVAL
    assert np.array_equal(pos.cpu().numpy(), c.pos) and np.array_equal(vel.cpu().numpy(), c.vel)
