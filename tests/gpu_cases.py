"""Shared helpers for the GPU parity tests: run the HIP path through the C ABI
and compare every stage with the oracle on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

import oracle


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = float((b ** 2).sum())
    return float(np.sqrt(((a - b) ** 2).sum() / den)) if den > 0 else float(np.abs(a - b).max())


# Per-row bounds: the error of a particle's acceleration (vector norm) or
# potential, over the larger of its own magnitude and 1e-3 of the RMS
# magnitude (rows whose terms nearly cancel are held to the RMS scale).  The
# FP64 path sums the same terms as the oracle in another order (about 1e-16
# per term); the mixed path rounds each term to FP32 (about 6e-8) on offsets
# from the group's centre.
ROW_TOL = {"fp64": 1e-11, "mixed": 1e-3}


def row_errors(a, ref):
    """Largest per-row relative error of a [n,3] or [n] array against ref."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.ndim == 1:
        a, ref = a[:, None], ref[:, None]
    if len(ref) == 0:
        return 0.0
    mag = np.sqrt((ref ** 2).sum(1))
    floor = 1e-3 * float(np.sqrt((mag ** 2).mean()))
    if floor == 0.0:
        return float(np.abs(a - ref).max())
    err = np.sqrt(((a - ref) ** 2).sum(1))
    return float((err / np.maximum(mag, floor)).max())


def gpu_run(ctx, pos, mass, params, want_neighbors=True, want_arrays=True):
    """Build + force (+ neighbours) on the GPU; returns host numpy results."""
    import torch
    dev = torch.device("cuda", ctx.device)
    tp = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
    tm = torch.from_numpy(np.ascontiguousarray(mass)).to(dev)
    ctx.build_tree(tp, tm, **params)
    acc, pot = ctx.long_force()
    out = {"acc": acc.cpu().numpy(), "pot": pot.cpu().numpy(), "stats": ctx.stats()}
    if want_neighbors:
        off, idx = ctx.neighbors()
        out["nbr_off"] = off.cpu().numpy()
        out["nbr_idx"] = idx.cpu().numpy().astype(np.int64)
    if want_arrays:
        for k in ("sorted_keys", "perm", "node_level", "node_first", "node_count", "node_child",
                  "node_nchild", "node_parent", "node_prefix", "node_mass", "node_com",
                  "node_quad", "node_box", "group_node", "cell_beg", "cell_end", "cell_idx",
                  "part_beg", "part_end", "part_idx", "near_beg", "near_end", "near_idx", "root"):
            out[k] = ctx.copy_array(k)
    return out


def compare_tree(g, t: oracle.Tree, groups_sample=None):
    """Keys, order, topology, moments, groups and lists must match bit for bit.
    With an oracle that walked only every k-th group, lists are compared for those."""
    key, perm = t.keys()
    lo, L = t.root()
    assert np.array_equal(g["root"][:3], lo) and g["root"][3] == L
    np.testing.assert_array_equal(g["perm"].astype(np.int64), perm)
    np.testing.assert_array_equal(g["sorted_keys"], key[perm])
    nd = t.nodes()
    assert len(g["node_level"]) == t.n_nodes, (len(g["node_level"]), t.n_nodes)
    np.testing.assert_array_equal(g["node_level"], nd["level"])
    np.testing.assert_array_equal(g["node_first"], nd["first"])
    np.testing.assert_array_equal(g["node_count"], nd["count"])
    np.testing.assert_array_equal(g["node_nchild"], nd["n_child"])
    internal = nd["n_child"] > 0
    np.testing.assert_array_equal(g["node_child"][internal], nd["child_first"][internal])
    np.testing.assert_array_equal(g["node_parent"], nd["parent"])
    np.testing.assert_array_equal(g["node_prefix"], nd["prefix"])
    mo = t.moments()
    np.testing.assert_array_equal(g["node_mass"], mo["M"])          # decision-feeding: exact
    np.testing.assert_array_equal(g["node_com"], mo["com"])
    np.testing.assert_array_equal(g["node_box"][:, :3], mo["blo"])
    np.testing.assert_array_equal(g["node_box"][:, 3:], mo["bhi"])
    qs = np.abs(mo["Q"]).max(axis=1, keepdims=True) + 1e-300
    assert np.all(np.abs(g["node_quad"] - mo["Q"]) <= 1e-11 * qs + 1e-300)
    np.testing.assert_array_equal(g["group_node"].astype(np.int64), t.groups())
    ol = t.lists()
    G = t.n_groups
    gs = range(G) if groups_sample is None else groups_sample
    st = g["stats"]
    stride = getattr(t, "walk_stride", 1)
    # segments: disjoint, inside the index array, summing to the list total; the
    # two-pass layout tiles the array exactly (no gap, no overlap)
    for lst in ("cell", "part", "near"):
        tot = st[f"n_{lst}_entries"]
        ext = st[f"{lst}_extent"]
        b, e = g[lst + "_beg"], g[lst + "_end"]
        assert np.all(e >= b) and np.all(b >= 0) and np.all(e <= ext)
        assert int((e - b).sum()) == tot and len(g[lst + "_idx"]) == ext
        o = np.argsort(b, kind="stable")
        nz = (e - b)[o] > 0
        bb, ee = b[o][nz], e[o][nz]
        assert np.all(bb[1:] >= ee[:-1])
        if not st["walk_fixed_stride"]:
            assert ext == tot
            assert (len(bb) == 0 and tot == 0) or (bb[0] == 0 and ee[-1] == tot
                                                   and np.all(bb[1:] == ee[:-1]))
    if stride == 1:
        assert st["n_cell_entries"] == ol["c_off"][-1]
        assert st["n_part_entries"] + st["n_near_entries"] == ol["p_off"][-1]
        np.testing.assert_array_equal(g["cell_end"] - g["cell_beg"], np.diff(ol["c_off"]))
        np.testing.assert_array_equal(g["part_end"] - g["part_beg"] + g["near_end"] - g["near_beg"],
                                      np.diff(ol["p_off"]))
    else:
        gs = [k for k in gs if k % stride == 0]
    for k in gs:
        a, b = ol["c_off"][k], ol["c_off"][k + 1]
        np.testing.assert_array_equal(np.sort(g["cell_idx"][g["cell_beg"][k]:g["cell_end"][k]]),
                                      ol["c_idx"][a:b])
        # the walk's particle list P_g is the union of the far and near parts
        far = g["part_idx"][g["part_beg"][k]:g["part_end"][k]]
        near = g["near_idx"][g["near_beg"][k]:g["near_end"][k]]
        a, b = ol["p_off"][k], ol["p_off"][k + 1]
        np.testing.assert_array_equal(np.sort(np.concatenate([far, near])), ol["p_idx"][a:b])
    if stride == 1:
        cnt = t.counts()
        assert st["n_pc"] == cnt["n_pc"] and st["n_pp"] == cnt["n_pp"]


def compare_neighbors(g, t: oracle.Tree):
    off, idx = t.neighbors()
    np.testing.assert_array_equal(g["nbr_off"], off)
    np.testing.assert_array_equal(g["nbr_idx"], idx)
