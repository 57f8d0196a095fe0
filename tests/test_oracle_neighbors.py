"""Pins of the oracle's neighbour lists: the particles within distance h
(Section 2.2), tested against every pair with the identical FP64 expression."""
import numpy as np
import pytest

from inputs import king, plummer
from oracle import direct


@pytest.mark.parametrize("h,theta", [(0.011, 0.5), (0.06, 0.4), (0.2, 0.8), (0.02, 0.0)])
def test_neighbors_match_brute_force(oracle_lib, h, theta):
    c = plummer(3000, 21)
    p = dict(eps=4 / 3000, r_in=0.1 * h / 1.1, r_out=h / 1.1, theta=theta, r_search=h,
             n_crit=64, n_leaf=16)
    off, idx = oracle_lib.Tree(c.pos, c.mass, p).neighbors()
    off_b, idx_b = direct.brute_neighbors(c.pos, h)
    np.testing.assert_array_equal(off, off_b)
    np.testing.assert_array_equal(idx, idx_b)


def test_neighbors_dense_core_symmetric(oracle_lib):
    c = king(4000, 9.0, 22)
    h = 0.01
    p = dict(eps=1e-3, r_in=0.1 * h / 1.1, r_out=h / 1.1, theta=0.5, r_search=h, n_crit=128, n_leaf=16)
    off, idx = oracle_lib.Tree(c.pos, c.mass, p).neighbors()
    off_b, idx_b = direct.brute_neighbors(c.pos, h)
    np.testing.assert_array_equal(off, off_b)
    np.testing.assert_array_equal(idx, idx_b)
    assert len(idx) > 0
    rows = np.repeat(np.arange(len(c.mass)), np.diff(off))
    fwd = set(zip(rows.tolist(), idx.tolist()))
    assert fwd == set((j, i) for i, j in fwd)
    assert not any(i == j for i, j in fwd)
    for i in range(len(c.mass)):
        assert np.all(np.diff(idx[off[i]:off[i + 1]]) > 0)


def test_exact_boundary_is_excluded(oracle_lib):
    # pair at distance exactly h (representable): strict "<" excludes it
    pos = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.0, 0.25, 0.0]])
    p = dict(eps=1e-3, r_in=0.01, r_out=0.1, theta=0.5, r_search=0.5, n_crit=4, n_leaf=1)
    off, idx = oracle_lib.Tree(pos, np.ones(3) / 3, p).neighbors()
    assert off.tolist() == [0, 1, 1, 2]
    assert idx.tolist() == [2, 0]
