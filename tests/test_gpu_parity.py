"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Keys, order, topology, centres of mass, boxes, groups, interaction lists and
neighbour lists must match bit for bit.  Forces: the FP64 path within 1e-12
relative RMS (the terms are the same; only rsqrt rounding and summation order
differ, ~1e-16 per term), the mixed path within the 1e-4 relative RMS bar;
and every row (acceleration and potential) within 1e-11 (FP64) or 1e-3
(mixed) of its own magnitude, floored at 1e-3 of the RMS magnitude.
"""
import numpy as np
import pytest

import oracle
from inputs import WORKLOADS, make_cluster, plummer
from tests.gpu_cases import (ROW_TOL, compare_neighbors, compare_tree, gpu_run, log, rel_rms,
                             row_errors)

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-4


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1506_04553_amd import P3T
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    c = P3T(0)
    yield c
    c.close()


def _params(w, **over):
    p = w.params(**over)
    return p


def _check_forces(g, acc, pot, tol, label, rows=None):
    """Relative RMS over all rows within tol, and every row within the per-row
    bound of its precision."""
    ga, gp = g["acc"], g["pot"]
    if rows is not None:
        ga, gp, acc, pot = ga[rows], gp[rows], acc[rows], pot[rows]
    ea, ep = rel_rms(ga, acc), rel_rms(gp, pot)
    ra, rp = row_errors(ga, acc), row_errors(gp, pot)
    rtol = ROW_TOL["fp64" if tol <= FP64_TOL else "mixed"]
    log(f"{label}: acc rel-RMS {ea:.3e} max row {ra:.3e}  pot rel-RMS {ep:.3e} max row {rp:.3e}")
    assert ea <= tol and ep <= tol, (ea, ep)
    assert ra <= rtol and rp <= rtol, (ra, rp)
    return ea, ep


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_plummer4k(ctx, prec):
    w = WORKLOADS["plummer4k"]
    c = make_cluster(w, seed=1)
    p = _params(w, precision=prec)
    log(f"case plummer4k {prec}")
    g = gpu_run(ctx, c.pos, c.mass, p)
    t = oracle.Tree(c.pos, c.mass, p)
    compare_tree(g, t)
    acc, pot = t.force()
    _check_forces(g, acc, pot, FP64_TOL if prec == "fp64" else MIXED_TOL, f"plummer4k {prec}")
    compare_neighbors(g, t)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_plummer64k_salpeter(ctx, prec):
    w = WORKLOADS["plummer64k_salpeter"]
    c = make_cluster(w, seed=1)
    p = _params(w, precision=prec)
    log(f"case plummer64k_salpeter {prec}")
    g = gpu_run(ctx, c.pos, c.mass, p)
    t = oracle.Tree(c.pos, c.mass, p)
    compare_tree(g, t)
    acc, pot = t.force()
    _check_forces(g, acc, pot, FP64_TOL if prec == "fp64" else MIXED_TOL, f"plummer64k {prec}")
    compare_neighbors(g, t)


def _sampled_neighbors(pos, h, rows):
    """Exact neighbour rows for a sample of particles: KD-tree candidates, then the
    FP64 test dx*dx + dy*dy + dz*dz < h*h."""
    from scipy.spatial import cKDTree
    kd = cKDTree(pos)
    out = {}
    for i in rows:
        cand = np.array(sorted(kd.query_ball_point(pos[i], h * (1 + 1e-9))), dtype=np.int64)
        d = pos[cand] - pos[i]
        r2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
        out[i] = cand[(r2 < h * h) & (cand != i)]
    return out


@pytest.mark.parametrize("name,prec", [("plummer256k", "mixed"), ("king9_1m", "mixed"),
                                       ("king9_1m", "fp64")])
def test_large_sampled(ctx, name, prec):
    w = WORKLOADS[name]
    c = make_cluster(w, seed=1)
    p = _params(w, precision=prec)
    log(f"case {name} {prec} n={w.n}")
    g = gpu_run(ctx, c.pos, c.mass, p)
    t = oracle.Tree(c.pos, c.mass, p)
    rng = np.random.default_rng(5)
    G = t.n_groups
    sample = np.unique(np.concatenate([[0, G - 1], rng.choice(G, min(G, 48), replace=False)]))
    compare_tree(g, t, groups_sample=sample)
    acc, pot = t.force_groups(sample)
    rows = np.nonzero(~np.isnan(pot))[0]
    _check_forces(g, acc, pot, FP64_TOL if prec == "fp64" else MIXED_TOL, f"{name} {prec}", rows)
    # neighbour rows of particles in the sampled groups against an independent search
    off, idx = g["nbr_off"], g["nbr_idx"]
    check = rows[:: max(1, len(rows) // 3000)]
    ref = _sampled_neighbors(c.pos, p["r_search"], check)
    for i in check:
        np.testing.assert_array_equal(idx[off[i]:off[i + 1]], ref[i])
    # symmetry of the whole CSR
    rws = np.repeat(np.arange(len(c.mass)), np.diff(off))
    a = np.sort(rws * len(c.mass) + idx)
    b = np.sort(idx * len(c.mass) + rws)
    np.testing.assert_array_equal(a, b)


_P4M = {}


def _plummer4m():
    if "c" not in _P4M:
        _P4M["c"] = make_cluster(WORKLOADS["plummer4m_salpeter"], seed=1)
    return _P4M["c"]


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.7])
@pytest.mark.parametrize("n_crit", [64, 128, 256, 512])
def test_plummer4m_sampled(ctx, theta, n_crit):
    """The 2^22-particle Salpeter workload at every theta x n_crit setting of
    its sweep: whole tree bit-exact, lists of every 997th group (the oracle
    walks only those), forces of 96 of them in both precisions."""
    w = WORKLOADS["plummer4m_salpeter"]
    c = _plummer4m()
    log(f"case plummer4m theta={theta} n_crit={n_crit}")
    for prec in ("mixed", "fp64"):
        p = _params(w, theta=theta, n_crit=n_crit, precision=prec)
        g = gpu_run(ctx, c.pos, c.mass, p, want_neighbors=(prec == "mixed"),
                    want_arrays=(prec == "mixed"))
        if prec == "mixed":
            t = oracle.Tree(c.pos, c.mass, p, walk_stride=997)
            compare_tree(g, t)
            rng = np.random.default_rng(9)
            walked = np.arange(0, t.n_groups, 997)
            sample = rng.choice(walked, min(96, len(walked)), replace=False)
            acc, pot = t.force_groups(sample)
            rows = np.nonzero(~np.isnan(pot))[0]
            del t
        _check_forces(g, acc, pot, FP64_TOL if prec == "fp64" else MIXED_TOL,
                      f"plummer4m theta={theta} n_crit={n_crit} {prec}", rows)


def _edge_cases():
    rng = np.random.default_rng(11)
    base = dict(eps=1e-3, r_in=0.002, r_out=0.02, theta=0.5, r_search=0.022, n_crit=64, n_leaf=16)
    cases = {}
    cases["n1"] = (np.array([[0.3, -0.2, 0.1]]), np.array([1.0]), base)
    cases["n2"] = (np.array([[0.0, 0.0, 0.0], [0.01, 0.0, 0.0]]), np.array([0.5, 0.5]), base)
    cases["coincident"] = (np.full((50, 3), 0.125), np.full(50, 0.02), base)
    dup = np.repeat(rng.uniform(-1, 1, (40, 3)), 9, axis=0)
    cases["duplicates"] = (dup, np.full(len(dup), 1.0 / len(dup)), base)
    big_leaf = np.concatenate([np.full((600, 3), 0.3), rng.normal(0, 0.5, (400, 3))])
    cases["leaf_over_block"] = (big_leaf, np.full(1000, 1e-3), dict(base, n_crit=32, n_leaf=8))
    line = np.stack([np.linspace(0, 1, 3000) ** 2, np.zeros(3000), np.zeros(3000)], 1)
    cases["collinear"] = (line, np.full(3000, 1 / 3000), base)
    pc = plummer(4097, 12)
    cases["ragged_4097"] = (pc.pos, pc.mass, dict(base, n_crit=100))
    cases["leaf1_group1"] = (plummer(700, 13).pos, np.full(700, 1 / 700),
                             dict(base, n_crit=1, n_leaf=1))
    cases["theta0"] = (plummer(1500, 14).pos, np.full(1500, 1 / 1500), dict(base, theta=0.0))
    cases["one_group"] = (plummer(900, 15).pos, np.full(900, 1 / 900), dict(base, n_crit=5000))
    cases["monopole_rin0"] = (plummer(2500, 16).pos, np.full(2500, 1 / 2500),
                              dict(base, use_quadrupole=0, r_in=0.0))
    cases["big_h"] = (plummer(2000, 17).pos, np.full(2000, 1 / 2000),
                      dict(base, r_out=0.2, r_in=0.02, r_search=0.3, theta=0.7))
    cases["large_theta"] = (plummer(3000, 18).pos, np.full(3000, 1 / 3000), dict(base, theta=1.5))
    # zero softening: every pair distance is positive except a particle's own
    cases["eps0"] = (plummer(2000, 19).pos, np.full(2000, 1 / 2000), dict(base, eps=0.0))
    # softening beyond r_out: no pair reaches inside r_out, the own pair (s = eps)
    # must still be left out of the potential
    cases["eps_beyond_rout"] = (plummer(1500, 20).pos, np.full(1500, 1 / 1500),
                                dict(base, eps=0.03))
    # leaves of more than 64 particles: the topology searches the sorted keys
    # instead of reading a window of them
    cases["leaf100"] = (plummer(3000, 21).pos, np.full(3000, 1 / 3000),
                        dict(base, n_crit=256, n_leaf=100))
    cases["duplicates_leaf80"] = (dup, np.full(len(dup), 1.0 / len(dup)),
                                  dict(base, n_crit=128, n_leaf=80))
    return cases


EDGE = _edge_cases()


@pytest.mark.parametrize("name", list(EDGE))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_edge_cases(ctx, name, prec):
    pos, mass, p = EDGE[name]
    p = dict(p, precision=prec)
    log(f"edge case {name} {prec} n={len(mass)}")
    g = gpu_run(ctx, pos, mass, p)
    t = oracle.Tree(pos, mass, p)
    compare_tree(g, t)
    acc, pot = t.force()
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    if np.all(acc == 0) and np.all(pot == 0):
        assert np.all(g["acc"] == 0) and np.all(g["pot"] == 0)
    else:
        _check_forces(g, acc, pot, tol, f"{name} {prec}")
    compare_neighbors(g, t)


def _band_cases():
    """Neighbour radius below r_out, so that accepted cells lie inside the
    changeover band and their K(y_c), W(y_c) differ from 1: eight particles
    whose accepted cells are single particles (the tree sum is then the direct
    sum), a Plummer sphere with the band across the cluster, and the 2^16
    Salpeter workload with r_out = 0.1 and h = r_out / 2 (at the workload's own
    r_out = 0.005 no accepted cell lies within r_out of a member: cells that
    close are far smaller than the particle spacing; at 0.1 about 8 000
    (member, cell) pairs do)."""
    from tests.test_oracle_cells_in_band import CORNER_CASES, _band_tree, _corner_setup
    cases = {}
    for name in CORNER_CASES:
        cases["corners_" + name] = _corner_setup(name)
    cases["corners_band_monopole"] = _corner_setup("band", quad=0)
    cases["plummer3000_band"] = _band_tree(0.5)
    w = WORKLOADS["plummer64k_salpeter"]
    c = make_cluster(w, seed=3)
    cases["plummer64k_h_half_rout"] = (c.pos, c.mass, w.params(r_out=0.1, r_in=0.01,
                                                                r_search=0.05))
    return cases


BAND = _band_cases()


@pytest.mark.parametrize("name", list(BAND))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cells_in_band(ctx, name, prec):
    """Accepted cells inside r_out (h < r_out): the kernels' cell-term
    changeover path against the oracle, lists and neighbours bit-exact."""
    from tests.test_oracle_cells_in_band import band_pairs
    pos, mass, p = BAND[name]
    p = dict(p, precision=prec)
    log(f"band case {name} {prec} n={len(mass)}")
    g = gpu_run(ctx, pos, mass, p)
    t = oracle.Tree(pos, mass, p)
    nb = band_pairs(t, pos, p)
    log(f"  {nb} (member, cell) pairs inside r_out")
    assert nb > 0
    compare_tree(g, t)
    acc, pot = t.force()
    _check_forces(g, acc, pot, FP64_TOL if prec == "fp64" else MIXED_TOL, f"{name} {prec}")
    compare_neighbors(g, t)


def test_neighbor_rows_longer_than_slots(ctx):
    """A fresh context reserves 32 entries per neighbour row: 80 coincident
    particles (79 neighbours each) overflow it, so the rows are written straight
    into the CSR; the next call reserves room for the longest row and packs the
    rows from their slots.  Both must equal the oracle's lists."""
    from paper_1506_04553_amd import P3T
    rng = np.random.default_rng(21)
    pos = np.concatenate([np.full((80, 3), 0.25), rng.normal(0, 0.3, (3000, 3))])
    mass = np.full(len(pos), 1.0 / len(pos))
    p = dict(eps=1e-3, r_in=0.002, r_out=0.02, theta=0.5, r_search=0.022, n_crit=64, n_leaf=16)
    t = oracle.Tree(pos, mass, p)
    fresh = P3T(0)
    for _ in range(2):
        g = gpu_run(fresh, pos, mass, p, want_arrays=False)
        compare_neighbors(g, t)
    fresh.close()


def test_walk_global_stack_path(monkeypatch):
    """With the walk's LDS stack capped at 64 entries most groups move to the
    global-memory stack; lists, forces and neighbours must still match the oracle,
    in both the two-pass and the fixed-stride walk."""
    from paper_1506_04553_amd import P3T
    w = WORKLOADS["plummer64k_salpeter"]
    c = make_cluster(w, seed=6)
    p = _params(w, precision="fp64")
    t = oracle.Tree(c.pos, c.mass, p)
    acc, pot = t.force()
    monkeypatch.setenv("P3T_WALK_LDS_STACK", "64")
    small = P3T(0)
    monkeypatch.delenv("P3T_WALK_LDS_STACK")
    for k in range(2):
        g = gpu_run(small, c.pos, c.mass, p)
        assert g["stats"]["walk_global_stack"] == 1
        assert g["stats"]["walk_fixed_stride"] == k
        compare_tree(g, t)
        compare_neighbors(g, t)
        _check_forces(g, acc, pot, FP64_TOL, f"global stack walk {k}")
    small.close()


def test_groups_generic_path(monkeypatch):
    """The group compaction of the largest inputs (a plain scan of the group
    flags, then the records), forced at a small size: groups, lists and forces
    must still match the oracle, in both the two-pass and the fixed-stride walk."""
    from paper_1506_04553_amd import P3T
    w = WORKLOADS["plummer64k_salpeter"]
    c = make_cluster(w, seed=7)
    p = _params(w, precision="fp64")
    t = oracle.Tree(c.pos, c.mass, p)
    acc, pot = t.force()
    monkeypatch.setenv("P3T_GROUPS_GENERIC", "1")
    gen = P3T(0)
    monkeypatch.delenv("P3T_GROUPS_GENERIC")
    for k in range(2):
        g = gpu_run(gen, c.pos, c.mass, p)
        assert g["stats"]["walk_fixed_stride"] == k
        compare_tree(g, t)
        compare_neighbors(g, t)
        _check_forces(g, acc, pot, FP64_TOL, f"generic group compaction {k}")
    gen.close()


def test_neighbors_beside_force():
    """The neighbour search runs on the context's second stream while the
    interaction kernel is still running on its first: neighbours called right
    after the force launch (no synchronisation in between), on a fresh context
    (whose first search allocates its workspaces) and on rebuilds, must match
    the oracle's lists, and the forces those of a serial run, bit for bit."""
    import torch
    from paper_1506_04553_amd import P3T
    w = WORKLOADS["plummer64k_salpeter"]
    c = make_cluster(w, seed=9)
    dev = torch.device("cuda", 0)
    tp = torch.from_numpy(c.pos).to(dev)
    tm = torch.from_numpy(c.mass).to(dev)
    for prec in ("fp64", "mixed"):
        p = _params(w, precision=prec)
        if prec == "fp64":
            t = oracle.Tree(c.pos, c.mass, p)
        serial = P3T(0)
        ref = gpu_run(serial, c.pos, c.mass, p, want_arrays=False)
        serial.close()
        compare_neighbors(ref, t)
        ctx = P3T(0)
        for rep in range(3):
            log(f"neighbours beside the force: {prec} rep {rep}")
            ctx.build_tree(tp, tm, **p)
            acc, pot = ctx.long_force()
            off, idx = ctx.neighbors()
            # work queued on the caller's stream after the call sees the rows
            total = int(off[-1].item())
            g = {"nbr_off": off.cpu().numpy(), "nbr_idx": idx.cpu().numpy().astype(np.int64)}
            assert total == len(g["nbr_idx"])
            compare_neighbors(g, t)
            assert np.array_equal(acc.cpu().numpy(), ref["acc"])
            assert np.array_equal(pot.cpu().numpy(), ref["pot"])
        ctx.close()


def test_forward_is_deterministic(ctx):
    w = WORKLOADS["plummer64k_salpeter"]
    c = make_cluster(w, seed=2)
    for prec in ("fp64", "mixed"):
        p = _params(w, precision=prec)
        a = gpu_run(ctx, c.pos, c.mass, p, want_arrays=False)
        b = gpu_run(ctx, c.pos, c.mass, p, want_arrays=False)
        assert np.array_equal(a["acc"], b["acc"]) and np.array_equal(a["pot"], b["pot"])
        assert np.array_equal(a["nbr_idx"], b["nbr_idx"])


def _same_lists(a, b):
    for lst in ("cell", "part", "near"):
        assert len(a["group_node"]) == len(b["group_node"])
        for k in range(len(a["group_node"])):
            np.testing.assert_array_equal(
                a[lst + "_idx"][a[lst + "_beg"][k]:a[lst + "_end"][k]],
                b[lst + "_idx"][b[lst + "_beg"][k]:b[lst + "_end"][k]])


def test_fixed_stride_walk_matches_two_pass(ctx):
    """The first build of a context walks twice (count, then emit at exact offsets);
    a repeated build writes the lists in one walk into segments reserved from the
    first build's sizes.  Lists (per group, in order), forces and neighbours must
    be identical."""
    from paper_1506_04553_amd import P3T
    w = WORKLOADS["plummer64k_salpeter"]
    c = make_cluster(w, seed=3)
    for prec in ("mixed", "fp64"):
        fresh = P3T(0)
        p = _params(w, precision=prec)
        a = gpu_run(fresh, c.pos, c.mass, p)
        b = gpu_run(fresh, c.pos, c.mass, p)
        fresh.close()
        assert a["stats"]["walk_fixed_stride"] == 0 and b["stats"]["walk_fixed_stride"] == 1
        _same_lists(a, b)
        assert np.array_equal(a["acc"], b["acc"]) and np.array_equal(a["pot"], b["pot"])
        assert np.array_equal(a["nbr_idx"], b["nbr_idx"])
        for k in ("n_cell_entries", "n_part_entries", "n_near_entries", "n_pc", "n_pp",
                  "n_pp_near", "n_leaves", "n_groups"):
            assert a["stats"][k] == b["stats"][k]


def test_fixed_stride_overflow_falls_back(ctx):
    """Lists longer than the reserved segments (a smaller opening angle after a
    larger one) make the build fall back to the two-pass walk with the same
    result as a fresh context."""
    from paper_1506_04553_amd import P3T
    w = WORKLOADS["plummer64k_salpeter"]
    c = make_cluster(w, seed=5)
    used = P3T(0)
    gpu_run(used, c.pos, c.mass, _params(w, theta=0.8), want_arrays=False)
    p = _params(w, theta=0.3)
    b = gpu_run(used, c.pos, c.mass, p)
    used.close()
    assert b["stats"]["walk_fixed_stride"] == 0
    fresh = P3T(0)
    a = gpu_run(fresh, c.pos, c.mass, p)
    fresh.close()
    _same_lists(a, b)
    assert np.array_equal(a["acc"], b["acc"]) and np.array_equal(a["pot"], b["pot"])


def test_more_groups_than_reserved(ctx):
    """A build with many more groups than the last one reserved room for: the
    walk into fixed-stride segments flags the groups past the room and the
    build walks again in two passes; lists, forces and neighbours equal those
    of a fresh context."""
    from paper_1506_04553_amd import P3T
    w = WORKLOADS["plummer64k_salpeter"]
    c = make_cluster(w, seed=6)
    small = plummer(8192, 7)
    for prec in ("fp64", "mixed"):
        p = _params(w, precision=prec)
        used = P3T(0)
        gpu_run(used, small.pos, small.mass, p, want_arrays=False)
        log(f"more groups than reserved: {prec}")
        b = gpu_run(used, c.pos, c.mass, p)
        used.close()
        assert b["stats"]["walk_fixed_stride"] == 0
        fresh = P3T(0)
        a = gpu_run(fresh, c.pos, c.mass, p)
        fresh.close()
        _same_lists(a, b)
        assert np.array_equal(a["acc"], b["acc"]) and np.array_equal(a["pot"], b["pot"])
        assert np.array_equal(a["nbr_idx"], b["nbr_idx"])


def test_reused_context_matches_fresh_context(ctx):
    """Workspaces left by a larger problem must not leak into a smaller one: a
    context that has just built a bigger tree gives the same lists (as per-group
    sequences), forces and neighbours as a fresh context."""
    from paper_1506_04553_amd import P3T
    w = WORKLOADS["plummer64k_salpeter"]
    c = make_cluster(w, seed=3)
    big = make_cluster(WORKLOADS["plummer256k"], seed=4)
    used = P3T(0)
    gpu_run(used, big.pos, big.mass, _params(WORKLOADS["plummer256k"]), want_arrays=False)
    for prec in ("mixed", "fp64"):
        p = _params(w, precision=prec)
        fresh = P3T(0)
        a = gpu_run(fresh, c.pos, c.mass, p)
        fresh.close()
        b = gpu_run(used, c.pos, c.mass, p)
        for lst in ("cell", "part", "near"):
            for k in range(len(a["group_node"])):
                np.testing.assert_array_equal(
                    a[lst + "_idx"][a[lst + "_beg"][k]:a[lst + "_end"][k]],
                    b[lst + "_idx"][b[lst + "_beg"][k]:b[lst + "_end"][k]])
        assert np.array_equal(a["acc"], b["acc"]) and np.array_equal(a["pot"], b["pot"])
        assert np.array_equal(a["nbr_idx"], b["nbr_idx"])
    used.close()


def test_errors_and_capacity(ctx):
    import torch
    from paper_1506_04553_amd import P3T, P3TError
    from paper_1506_04553_amd.p3t import P3T_ECAPACITY, P3T_EINVAL, P3T_ESTATE
    fresh = P3T(0)
    with pytest.raises(P3TError) as e:
        fresh.long_force(torch.empty((0, 3), dtype=torch.float64, device="cuda"))
    assert e.value.status in (P3T_ESTATE, P3T_EINVAL)
    fresh.n = 0
    import ctypes as C
    rc = fresh._L.p3t_long_force(fresh._h, None, None)
    assert rc == P3T_ESTATE
    c = plummer(3000, 19)
    pos = torch.from_numpy(c.pos).cuda()
    mass = torch.from_numpy(c.mass).cuda()
    p = dict(eps=1e-3, r_in=0.005, r_out=0.05, theta=0.5, r_search=0.055, n_crit=64, n_leaf=16)
    fresh.build_tree(pos, mass, **p)
    off, idx = fresh.neighbors()
    nnz = len(idx)
    assert nnz > 10
    o2 = torch.full((3001,), -7, dtype=torch.int64, device="cuda")
    i2 = torch.empty((5,), dtype=torch.int32, device="cuda")
    got = C.c_int64(0)
    rc = fresh._L.p3t_neighbors(fresh._h, C.c_void_p(o2.data_ptr()), C.c_void_p(i2.data_ptr()), 5,
                                C.byref(got))
    assert rc == P3T_ECAPACITY and got.value == nnz
    assert torch.all(o2 == -7)             # untouched on error
    bad = pos.clone()
    bad[17, 1] = float("nan")
    with pytest.raises(P3TError) as e:
        fresh.build_tree(bad, mass, **p)
    assert e.value.status == P3T_EINVAL
    badm = mass.clone()
    badm[3] = 0.0
    with pytest.raises(P3TError):
        fresh.build_tree(pos, badm, **p)
    with pytest.raises(P3TError):
        fresh.build_tree(pos, mass, **dict(p, r_in=0.06))
    # the context stays usable after errors
    fresh.build_tree(pos, mass, **p)
    a, _ = fresh.long_force()
    assert torch.isfinite(a).all()
    fresh.close()


def test_kick_drift(ctx):
    import torch
    rng = np.random.default_rng(3)
    x, v, a = (rng.normal(size=(1001, 3)) for _ in range(3))
    tx, tv, ta = (torch.from_numpy(q.copy()).cuda() for q in (x, v, a))
    ctx.kick_drift(tx, tv, ta, 0.125, 0.25)
    v2 = v + 0.125 * a
    x2 = x + 0.25 * v2
    assert np.array_equal(tv.cpu().numpy(), v2) and np.array_equal(tx.cpu().numpy(), x2)


def test_allocator_failure_is_enomem():
    """Every device workspace of a build, force, neighbour search and VJP comes
    from the context's allocator.  When its k-th allocation fails (for every k
    that the sequence reaches), the call returns P3T_ENOMEM and leaves the
    caller's outputs untouched; with the allocator working again the same
    context gives the same forces, lists and VJP as an unfailing context."""
    import ctypes as C
    import torch
    from paper_1506_04553_amd import P3T
    from paper_1506_04553_amd.p3t import (ALLOC_FN, FREE_FN, P3T_ENOMEM, P3T_OK, P3TError,
                                          load_library)
    L = load_library()
    c = plummer(3000, 23)
    p = dict(eps=1e-3, r_in=0.005, r_out=0.05, theta=0.5, r_search=0.055, n_crit=64, n_leaf=16,
             precision="mixed")
    st = torch.cuda.current_stream(0)
    state = {"count": 0, "fail_at": 0}

    def _alloc(nbytes, _user):
        state["count"] += 1
        if state["count"] == state["fail_at"]:
            return None
        return torch.cuda.caching_allocator_alloc(int(nbytes), 0, st)

    def _free(ptr, _user):
        torch.cuda.caching_allocator_delete(int(ptr))

    acb, fcb = ALLOC_FN(_alloc), FREE_FN(_free)

    def new_ctx():
        obj = P3T.__new__(P3T)
        obj._L, obj.device, obj.stream, obj._allocs = L, 0, st, {}
        obj._alloc_cb, obj._free_cb = acb, fcb
        h = C.c_void_p()
        assert L.p3t_create(C.byref(h), 0, C.c_void_p(st.cuda_stream), acb, fcb, None) == P3T_OK
        obj._h, obj.n, obj.params, obj.build_id = h, 0, None, 0
        return obj

    n = len(c.mass)
    pos, mass = torch.from_numpy(c.pos).cuda(), torch.from_numpy(c.mass).cuda()
    rng = np.random.default_rng(24)
    w = torch.from_numpy(rng.normal(size=(n, 3))).cuda()
    cw = torch.from_numpy(rng.normal(size=n)).cuda()
    SENT = -7.0

    def sequence(ctx_):
        """Build, force, neighbours, VJP; returns (results, status of the
        failing call or OK, whether that call left its outputs untouched)."""
        try:
            ctx_.build_tree(pos, mass, **p)
        except P3TError as e:
            return None, e.status, True
        acc = torch.full((n, 3), SENT, dtype=torch.float64, device="cuda")
        pot = torch.full((n,), SENT, dtype=torch.float64, device="cuda")
        rc = L.p3t_long_force(ctx_._h, C.c_void_p(acc.data_ptr()), C.c_void_p(pot.data_ptr()))
        torch.cuda.synchronize()
        if rc != P3T_OK:
            return None, rc, bool((acc == SENT).all() and (pot == SENT).all())
        off = torch.full((n + 1,), -7, dtype=torch.int64, device="cuda")
        idx = torch.full((n * 8,), -7, dtype=torch.int32, device="cuda")
        nnz = C.c_int64(0)
        rc = L.p3t_neighbors(ctx_._h, C.c_void_p(off.data_ptr()), C.c_void_p(idx.data_ptr()),
                             n * 8, C.byref(nnz))
        torch.cuda.synchronize()
        if rc != P3T_OK:
            return None, rc, bool((off == -7).all() and (idx == -7).all())
        gp = torch.full((n, 3), SENT, dtype=torch.float64, device="cuda")
        gm = torch.full((n,), SENT, dtype=torch.float64, device="cuda")
        rc = L.p3t_long_force_vjp(ctx_._h, C.c_void_p(w.data_ptr()), C.c_void_p(cw.data_ptr()),
                                  C.c_void_p(gp.data_ptr()), C.c_void_p(gm.data_ptr()))
        torch.cuda.synchronize()
        if rc != P3T_OK:
            return None, rc, bool((gp == SENT).all() and (gm == SENT).all())
        res = [t.cpu().numpy() for t in (acc, pot, off, idx[:nnz.value], gp, gm)]
        return res, P3T_OK, True

    ref_ctx = new_ctx()
    ref, rc, _ = sequence(ref_ctx)
    assert rc == P3T_OK
    total = state["count"]
    ref_ctx.close()
    log(f"  {total} allocations in build, force, neighbours and VJP")
    assert total > 10
    for k in range(1, total + 1):
        state["count"], state["fail_at"] = 0, k
        ctx_ = new_ctx()
        res, rc, untouched = sequence(ctx_)
        assert rc == P3T_ENOMEM, (k, rc)
        assert untouched, k
        state["fail_at"] = 0
        res, rc, _ = sequence(ctx_)
        assert rc == P3T_OK, (k, rc)
        for u, v in zip(res[:4], ref[:4]):
            assert np.array_equal(u, v), k
        assert rel_rms(res[4], ref[4]) < 1e-13 and rel_rms(res[5], ref[5]) < 1e-13, k
        ctx_.close()
