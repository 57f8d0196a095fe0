"""Pins of the oracle's tree steps: keys, topology, moments, groups and walk.

Each step is checked against an independent brute-force construction written
from its definition (geometric subdivision of the root cube, direct sums over
member sets, exhaustive per-(group, cell) acceptance tests).
"""
import os

import numpy as np
import pytest

from inputs import plummer

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "morton_keys.txt")


def _params(**kw):
    d = dict(eps=1e-3, r_in=0.001, r_out=0.01, theta=0.5, r_search=0.011, n_crit=32, n_leaf=4)
    d.update(kw)
    return d


def test_morton_golden(oracle_lib):
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    pos = np.array([[float(v) for v in r[:3]] for r in rows])
    keys = np.array([int(r[3]) for r in rows], dtype=np.uint64)
    t = oracle_lib.Tree(pos, np.ones(len(pos)), _params())
    lo, L = t.root()
    assert L == 1.0 and np.all(lo == 0.0)
    k, perm = t.keys()
    np.testing.assert_array_equal(k, keys)
    # sorted by key, ties by index
    assert np.all(np.diff(k[perm].astype(object)) >= 0)


def test_root_cube_rule(oracle_lib):
    rng = np.random.default_rng(0)
    for ext in (0.3, 1.0, 1.7, 4.0, 5.5, 1e-3):
        pos = rng.uniform(0, 1, (50, 3)) * ext + 7.0
        t = oracle_lib.Tree(pos, np.ones(50), _params())
        lo, L = t.root()
        e = (pos.max(0) - pos.min(0)).max()
        np.testing.assert_array_equal(lo, pos.min(0))
        assert L >= e and L / 2 < e and np.log2(L) == round(np.log2(L))


def _grid(pos, lo, L):
    return np.minimum(np.floor((pos - lo) * (2.0 ** 21 / L)), 2 ** 21 - 1).astype(np.int64)


def _brute_tree(pos, n_leaf, lo, L):
    """Recursive geometric subdivision: {(level, ix, iy, iz): set(original indices)}."""
    q = _grid(pos, lo, L)
    nodes = {}

    def rec(level, cell, members):
        nodes[(level, *cell)] = frozenset(members.tolist())
        if len(members) > n_leaf and level < 21:
            sh = 21 - (level + 1)
            sub = q[members] >> sh
            for c in sorted(set(map(tuple, sub.tolist()))):
                m = members[np.all(sub == np.array(c), axis=1)]
                rec(level + 1, c, m)

    rec(0, (0, 0, 0), np.arange(len(pos)))
    return nodes


def _decode(prefix, level):
    ix = iy = iz = 0
    for b in range(level):
        trip = (int(prefix) >> (3 * b)) & 7
        ix |= ((trip >> 2) & 1) << b
        iy |= ((trip >> 1) & 1) << b
        iz |= (trip & 1) << b
    return ix, iy, iz


def _oracle_node_sets(t):
    nd = t.nodes()
    _, perm = t.keys()
    out = {}
    for i in range(t.n_nodes):
        lev = int(nd["level"][i])
        f, c = int(nd["first"][i]), int(nd["count"][i])
        out[(lev, *_decode(nd["prefix"][i], lev))] = frozenset(perm[f:f + c].tolist())
    return out, nd


CASES = {
    "plummer": lambda: plummer(600, 5).pos,
    "clumped": lambda: np.concatenate([np.random.default_rng(1).normal(0, 1e-4, (200, 3)),
                                       np.random.default_rng(2).uniform(-1, 1, (200, 3))]),
    "collinear": lambda: np.stack([np.linspace(0, 1, 300) ** 3, np.zeros(300), np.zeros(300)], 1),
    "duplicates": lambda: np.repeat(np.random.default_rng(3).uniform(0, 1, (20, 3)), 7, axis=0),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("n_leaf", [1, 4, 16])
def test_topology_vs_subdivision(oracle_lib, case, n_leaf):
    pos = CASES[case]()
    t = oracle_lib.Tree(pos, np.ones(len(pos)), _params(n_leaf=n_leaf))
    lo, L = t.root()
    ref = _brute_tree(pos, n_leaf, lo, L)
    got, nd = _oracle_node_sets(t)
    assert got == ref
    # BFS numbering: levels non-decreasing, prefixes increasing inside a level
    lev = nd["level"]
    assert np.all(np.diff(lev) >= 0)
    for l in np.unique(lev):
        p = nd["prefix"][lev == l].astype(object)
        assert all(a < b for a, b in zip(p[:-1], p[1:]))
    # children contiguous and point back to their parent
    for i in range(t.n_nodes):
        cf, nc = nd["child_first"][i], nd["n_child"][i]
        for c in range(cf, cf + nc):
            assert nd["parent"][c] == i
        if nc:
            assert nd["count"][cf:cf + nc].sum() == nd["count"][i]


def test_all_coincident_and_single(oracle_lib):
    pos = np.full((40, 3), 0.25)
    t = oracle_lib.Tree(pos, np.ones(40), _params(n_leaf=4))
    nd = t.nodes()
    # chain of single-child nodes down to the depth limit
    assert t.n_nodes == 22 and nd["level"][-1] == 21 and nd["count"][-1] == 40
    lo, L = t.root()
    assert L == 1.0
    t1 = oracle_lib.Tree(np.array([[0.1, 0.2, 0.3]]), np.array([1.0]), _params())
    assert t1.n_nodes == 1 and t1.n_groups == 1
    a, p = t1.force()
    assert np.all(a == 0.0) and p[0] == 0.0


def test_moments_from_members(oracle_lib):
    c = plummer(800, 7)
    mass = np.random.default_rng(4).uniform(0.5, 2.0, 800) / 800
    t = oracle_lib.Tree(c.pos, mass, _params(n_leaf=8))
    nd, mo = t.nodes(), t.moments()
    _, perm = t.keys()
    lo, L = t.root()
    for i in range(t.n_nodes):
        mem = perm[nd["first"][i]:nd["first"][i] + nd["count"][i]]
        m, x = mass[mem], c.pos[mem]
        M = m.sum()
        com = (m[:, None] * x).sum(0) / M
        d = x - com
        r2 = (d * d).sum(1)
        Q = np.einsum("k,ka,kb->ab", m, 3 * d, d) - np.eye(3) * (m * r2).sum()
        assert abs(mo["M"][i] - M) <= 1e-14 * M
        np.testing.assert_allclose(mo["com"][i], com, rtol=0, atol=1e-13 * (1 + np.abs(com).max()))
        q6 = np.array([Q[0, 0], Q[1, 1], Q[2, 2], Q[0, 1], Q[0, 2], Q[1, 2]])
        np.testing.assert_allclose(mo["Q"][i], q6, atol=1e-13 * (1 + np.abs(q6).max()))
        np.testing.assert_array_equal(mo["blo"][i], x.min(0))
        np.testing.assert_array_equal(mo["bhi"][i], x.max(0))
        assert mo["side"][i] == L * 2.0 ** -nd["level"][i]
        assert abs(q6[0] + q6[1] + q6[2]) < 1e-12 * (1 + np.abs(q6).max())


def _is_leaf(nd, i):
    return nd["n_child"][i] == 0


def test_groups_partition_and_rule(oracle_lib):
    c = plummer(3000, 8)
    for n_crit in (8, 40, 200, 5000):
        t = oracle_lib.Tree(c.pos, c.mass, _params(n_crit=n_crit, n_leaf=6))
        nd = t.nodes()
        g = t.groups()
        firsts = nd["first"][g]
        assert np.all(np.diff(firsts) > 0)
        cov = np.zeros(len(c.mass), int)
        for gi in g:
            cov[nd["first"][gi]:nd["first"][gi] + nd["count"][gi]] += 1
            assert nd["count"][gi] <= n_crit or _is_leaf(nd, gi)
            p = nd["parent"][gi]
            while p >= 0:        # no ancestor qualifies
                assert nd["count"][p] > n_crit
                p = nd["parent"][p]
        assert np.all(cov == 1)


def _expected_lists(t, pos_sorted_fn=None):
    """Exhaustive: cell c is in C_g iff accepted and every ancestor rejected."""
    p = t.params
    nd, mo = t.nodes(), t.moments()
    g = t.groups()
    th2 = p.theta * p.theta
    h2 = p.r_search * p.r_search
    nn = t.n_nodes
    out = []
    for gi in g:
        glo, ghi = mo["blo"][gi], mo["bhi"][gi]
        com = mo["com"]
        t1 = np.maximum(np.maximum(glo[None] - com, 0.0), com - ghi[None])
        D2 = t1[:, 0] * t1[:, 0] + t1[:, 1] * t1[:, 1] + t1[:, 2] * t1[:, 2]
        t2 = np.maximum(np.maximum(mo["blo"] - ghi[None], 0.0), glo[None] - mo["bhi"])
        B2 = t2[:, 0] * t2[:, 0] + t2[:, 1] * t2[:, 1] + t2[:, 2] * t2[:, 2]
        acc = (th2 * D2 > mo["side"] * mo["side"]) & (B2 >= h2)
        visited = np.zeros(nn, bool)
        visited[0] = True
        for i in range(nn):                      # BFS order: parents before children
            if visited[i] and not acc[i] and not _is_leaf(nd, i):
                cf, nc = nd["child_first"][i], nd["n_child"][i]
                visited[cf:cf + nc] = True
        C = np.nonzero(visited & acc)[0]
        leaves = np.nonzero(visited & ~acc & (nd["n_child"] == 0))[0]
        P = np.sort(np.concatenate([np.arange(nd["first"][l], nd["first"][l] + nd["count"][l])
                                    for l in leaves])) if len(leaves) else np.zeros(0, np.int64)
        out.append((C, P))
    return out


@pytest.mark.parametrize("theta", [0.0, 0.3, 0.6, 1.0])
@pytest.mark.parametrize("r_search", [0.011, 0.2])
def test_walk_lists_exhaustive(oracle_lib, theta, r_search):
    c = plummer(1500, 9)
    t = oracle_lib.Tree(c.pos, c.mass, _params(theta=theta, r_search=r_search, n_crit=48, n_leaf=8))
    from oracle import group_lists
    got = group_lists(t)
    exp = _expected_lists(t)
    nd = t.nodes()
    for (gnode, P, Cl), (Ce, Pe) in zip(got, exp):
        np.testing.assert_array_equal(Cl, Ce)
        np.testing.assert_array_equal(P, Pe)
        # partition: particles of P plus members of accepted cells = everything, disjoint
        cov = np.zeros(t.n, int)
        cov[P] += 1
        for cc in Cl:
            cov[nd["first"][cc]:nd["first"][cc] + nd["count"][cc]] += 1
        assert np.all(cov == 1)
        # own members are always in P
        f, n = nd["first"][gnode], nd["count"][gnode]
        assert np.isin(np.arange(f, f + n), P).all()
    if theta == 0.0:
        assert t.counts()["n_cells"] == 0
