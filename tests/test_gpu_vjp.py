"""GPU VJP of the long-range force and potential (lists frozen).

Checked against: the oracle's VJP (same tree, same lists) to 1e-10 in FP64
and 1e-4 relative RMS in mixed precision (FP32 terms on group-centred
offsets, FP64 sums); at theta = 0 the analytic gradient of the direct soft
sum; central finite differences of the GPU FP64 forward (h = 1e-6) on sampled
coordinates whose perturbation leaves the lists unchanged; a direct-summation
FP64 reference gradient at the tree-error level; and torch.autograd.gradcheck
on a tiny case.
"""
import numpy as np
import pytest

import oracle
from inputs import WORKLOADS, make_cluster, plummer
from oracle import direct
from tests.gpu_cases import log, rel_rms, row_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1506_04553_amd import P3T
    assert torch.cuda.is_available()
    c = P3T(0)
    yield c
    c.close()


def _gpu_vjp(ctx, pos, mass, params, w, cw):
    import torch
    dev = torch.device("cuda", ctx.device)
    ctx.build_tree(torch.from_numpy(pos).to(dev), torch.from_numpy(mass).to(dev), **params)
    gp, gm = ctx.long_force_vjp(torch.from_numpy(w).to(dev),
                                None if cw is None else torch.from_numpy(cw).to(dev))
    return gp.cpu().numpy(), gm.cpu().numpy()


VJP_TOL = {"fp64": 1e-10, "mixed": 1e-4}
# per particle (gradient vector, and the mass gradient), relative to the larger
# of its own magnitude and 1e-3 of the RMS magnitude: the FP64 adjoint sums
# about 10^4 terms in another order than the oracle (1e-16 each), the mixed one
# rounds each term to FP32 (6e-8) before FP64 sums; the floor allows a
# thousand-fold cancellation in a row
VJP_ROW_TOL = {"fp64": 1e-9, "mixed": 1e-2}


def _check_vjp(gp, gm, op, om, precision, label):
    ep, em = rel_rms(gp, op), rel_rms(gm, om)
    rp, rm = row_errors(gp, op), row_errors(gm, om)
    log(f"  {label}: gpos rel-RMS {ep:.2e} max row {rp:.2e}  gmass rel-RMS {em:.2e} "
        f"max row {rm:.2e}")
    assert ep < VJP_TOL[precision] and em < VJP_TOL[precision]
    assert rp < VJP_ROW_TOL[precision] and rm < VJP_ROW_TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("quad,theta,r_out,with_c", [(1, 0.5, 0.05, True), (0, 0.6, 0.05, True),
                                                     (1, 0.4, 0.3, True), (1, 0.7, 0.01, False)])
def test_vjp_matches_oracle(ctx, quad, theta, r_out, with_c, precision):
    n = 4096
    c = plummer(n, 41)
    mass = np.random.default_rng(42).uniform(0.5, 2.0, n)
    mass /= mass.sum()
    p = dict(eps=4.0 / n, r_in=0.1 * r_out, r_out=r_out, theta=theta, r_search=1.1 * r_out,
             n_crit=64, n_leaf=16, use_quadrupole=quad, precision=precision)
    rng = np.random.default_rng(43)
    w = rng.normal(size=(n, 3))
    cw = rng.normal(size=n) if with_c else None
    log(f"vjp vs oracle {precision} quad={quad} theta={theta} r_out={r_out}")
    gp, gm = _gpu_vjp(ctx, c.pos, mass, p, w, cw)
    op, om = oracle.Tree(c.pos, mass, p).vjp(w, cw)
    _check_vjp(gp, gm, op, om, precision, "vs oracle")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["corners_band", "corners_inner", "corners_mixed",
                                  "plummer3000_band", "plummer64k_h_half_rout"])
def test_vjp_cells_in_band(ctx, name, precision):
    """Neighbour radius below r_out: the adjoint of K(y_c) and W(y_c) on cells
    inside the changeover band (the kernels' cell-changeover variant) against
    the oracle's VJP; with one-member cells also against the analytic gradient
    of the direct soft sum."""
    from tests.test_gpu_parity import BAND
    pos, mass, p = BAND[name]
    p = dict(p, precision=precision)
    n = len(mass)
    rng = np.random.default_rng(48)
    w, cw = rng.normal(size=(n, 3)), rng.normal(size=n)
    log(f"vjp band case {name} {precision} n={n}")
    gp, gm = _gpu_vjp(ctx, pos, mass, p, w, cw)
    op, om = oracle.Tree(pos, mass, p).vjp(w, cw)
    _check_vjp(gp, gm, op, om, precision, "vs oracle")
    if name.startswith("corners"):
        dp, dm = direct.soft_direct_grad(pos, mass, p["eps"], p["r_in"], p["r_out"], w, cw)
        _check_vjp(gp, gm, dp, dm, precision, "vs direct gradient")


def test_vjp_theta0_direct(ctx):
    n = 1500
    c = plummer(n, 44)
    p = dict(eps=4.0 / n, r_in=0.02, r_out=0.2, theta=0.0, r_search=0.22, n_crit=64, n_leaf=16)
    rng = np.random.default_rng(45)
    w, cw = rng.normal(size=(n, 3)), rng.normal(size=n)
    gp, gm = _gpu_vjp(ctx, c.pos, c.mass, p, w, cw)
    dp, dm = direct.soft_direct_grad(c.pos, c.mass, p["eps"], p["r_in"], p["r_out"], w, cw)
    assert rel_rms(gp, dp) < 1e-11 and rel_rms(gm, dm) < 1e-11


def _lists_signature(ctx):
    """Groups and every group's lists, concatenated in group order (segment
    placement in the list arrays may differ between builds)."""
    out = [ctx.copy_array("group_node")]
    for lst in ("cell", "part", "near"):
        b, e, idx = (ctx.copy_array(lst + s) for s in ("_beg", "_end", "_idx"))
        out.append(np.concatenate([idx[x:y] for x, y in zip(b, e)]) if len(b) else idx)
        out.append(e - b)
    return out


def _direct_grad_coords(pos, mass, p, w, cw, coords):
    """dL/dx_{k,a} of the direct soft sum for sampled (k, a), O(N) each."""
    gamma = p["r_in"] / p["r_out"]
    out = []
    for k, a in coords:
        d = pos - pos[k]                       # x_j - x_k
        s2 = (d * d).sum(1) + p["eps"] ** 2
        s = np.sqrt(s2)
        y = s / p["r_out"]
        K = direct.K_np(y, gamma)
        dK = direct.dKdy_np(y, gamma) / p["r_out"]
        W = direct.W_over_y_np(y, gamma) * y
        g = K / (s2 * s)
        gpd = dK / (s2 * s) - 3 * K / (s2 * s2)
        mask = np.ones(len(mass), bool)
        mask[k] = False
        # k as the i-particle: l_kj, d = x_j - x_k, dl/dx_k = -dl/dd
        wk = w[k]
        wd = d @ wk
        gd_k = mass[:, None] * (g[:, None] * wk[None] + (gpd * wd / s)[:, None] * d
                                + (cw[k] * K / (s2 * s))[:, None] * d)
        term1 = -(gd_k[mask, a]).sum()
        # k as the j-particle of every i: d = x_k - x_i = -d
        wi = w
        wdi = -(d * wi).sum(1)
        gd_i = mass[k] * (g[:, None] * wi + (gpd * wdi / s)[:, None] * (-d)
                          + (cw * K / (s2 * s))[:, None] * (-d))
        term2 = gd_i[mask, a].sum()
        out.append(term1 + term2)
    return np.array(out)


def test_vjp_plummer256k_fd_and_direct(ctx):
    """The 2^18-particle workload.  FP64 build: the VJP against FD with h = 1e-6
    of the FP64 forward on 64 sampled coordinates (those whose perturbation
    leaves the lists unchanged), and the direct-summation reference gradient
    on the same coordinates.  Mixed build (same lists): the mixed VJP against the FP64 VJP
    over every particle, and against the same FD values."""
    import torch
    w_ = WORKLOADS["plummer256k"]
    c = make_cluster(w_, seed=1)
    n = w_.n
    rng = np.random.default_rng(46)
    w = rng.normal(size=(n, 3))
    cw = rng.normal(size=n)
    dev = torch.device("cuda", ctx.device)
    tw, tc = torch.from_numpy(w).to(dev), torch.from_numpy(cw).to(dev)
    p32 = w_.params(precision="mixed")
    p64 = w_.params(precision="fp64")
    pos = torch.from_numpy(c.pos).to(dev)
    mass = torch.from_numpy(c.mass).to(dev)
    ctx.build_tree(pos, mass, **p32)
    ctx.long_force()
    g32, m32 = (t.cpu().numpy() for t in ctx.long_force_vjp(tw, tc))
    sig32 = _lists_signature(ctx)
    ctx.build_tree(pos, mass, **p64)
    g64, m64 = (t.cpu().numpy() for t in ctx.long_force_vjp(tw, tc))
    base = _lists_signature(ctx)
    assert all(np.array_equal(u, v) for u, v in zip(sig32, base))
    e32p, e32m = rel_rms(g32, g64), rel_rms(m32, m64)
    log(f"plummer256k mixed VJP vs FP64 VJP: gpos rel-RMS {e32p:.2e}  gmass rel-RMS {e32m:.2e}")
    assert e32p < 1e-4 and e32m < 1e-4

    def loss(pp):
        ctx.build_tree(pp, mass, **p64)
        a, ph = ctx.long_force()
        return float((tw * a).sum() + (tc * ph).sum()), _lists_signature(ctx)

    h = 1e-6
    coords, fds = [], []
    for k in rng.permutation(n):
        if len(coords) == 64:
            break
        a = int(rng.integers(3))
        pp = pos.clone(); pp[k, a] += h
        lp, sp = loss(pp)
        pm = pos.clone(); pm[k, a] -= h
        lm, sm = loss(pm)
        if not all(np.array_equal(u, v) for u, v in zip(sp, base)) or \
           not all(np.array_equal(u, v) for u, v in zip(sm, base)):
            continue
        coords.append((int(k), a))
        fds.append((lp - lm) / (2 * h))
    fds = np.array(fds)
    assert len(coords) == 64
    scale = np.abs(fds) + 1e-3 * np.abs(fds).max()
    for name, g, tol in (("FP64", g64, 2e-4), ("mixed", g32, 1e-3)):
        got = np.array([g[k, a] for k, a in coords])
        err = np.abs(got - fds)
        log(f"plummer256k {name} VJP vs FD: max rel err {np.max(err / scale):.2e} "
            f"over {len(coords)} coords")
        assert np.all(err <= tol * scale)
    got = np.array([g64[k, a] for k, a in coords])
    ref = _direct_grad_coords(c.pos, c.mass, p64, w, cw, coords)
    e_dir = rel_rms(got, ref)
    log(f"plummer256k VJP vs direct-summation gradient: rel-RMS {e_dir:.2e} (tree error level)")
    # the tree's own error at theta = 0.5 with the quadrupole (1.95e-4 measured)
    assert e_dir < 1e-3


def test_autograd_function_and_gradcheck(ctx):
    import torch
    from paper_1506_04553_amd import long_force
    n = 96
    c = plummer(n, 47)
    p = dict(eps=0.01, r_in=0.02, r_out=0.2, theta=0.8, r_search=0.22, n_crit=8, n_leaf=2,
             precision="fp64")
    pos = torch.from_numpy(c.pos).cuda().requires_grad_(True)
    mass = torch.from_numpy(c.mass).cuda().requires_grad_(True)
    acc, pot = long_force(pos, mass, ctx, **p)
    assert ctx.stats()["n_cell_entries"] > 0
    w = torch.randn_like(acc)
    cw = torch.randn_like(pot)
    L = (w * acc).sum() + (cw * pot).sum()
    L.backward()
    gp, gm = ctx.long_force_vjp(w, cw)
    assert torch.allclose(pos.grad, gp) and torch.allclose(mass.grad, gm)

    def f(x, m):
        return long_force(x, m, ctx, **p)
    torch.autograd.gradcheck(f, (pos.detach().clone().requires_grad_(True),
                                 mass.detach().clone().requires_grad_(True)),
                             eps=1e-7, atol=1e-6, rtol=1e-5, nondet_tol=1e-12)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_released_lists_are_recomputed(ctx, precision):
    """p3t_release_lists frees the interaction lists; the next force, neighbour
    or VJP call walks the tree again.  The walk is deterministic, so forces and
    neighbour lists are bit-identical and the VJP equal to rounding (its cell
    adjoints are summed with atomics); the autograd function with
    recompute_lists=True gives the same gradients."""
    import torch
    from paper_1506_04553_amd import long_force
    c = make_cluster(WORKLOADS["plummer64k_salpeter"], seed=2, n=20000)
    p = dict(WORKLOADS["plummer64k_salpeter"].params(precision=precision))
    dev = torch.device("cuda", ctx.device)
    pos, mass = torch.from_numpy(c.pos).to(dev), torch.from_numpy(c.mass).to(dev)
    rng = np.random.default_rng(5)
    w = torch.from_numpy(rng.normal(size=(len(c.mass), 3))).to(dev)
    cw = torch.from_numpy(rng.normal(size=len(c.mass))).to(dev)
    out = []
    for release in (False, True):
        ctx.build_tree(pos, mass, **p)
        st0 = ctx.stats()
        if release:
            ctx.release_lists()
            ctx.release_lists()   # twice is harmless
        acc, pot = ctx.long_force()
        if release:
            ctx.release_lists()
        off, idx = ctx.neighbors()
        if release:
            ctx.release_lists()
        gp, gm = ctx.long_force_vjp(w, cw)
        st1 = ctx.stats()
        for k in ("n_cell_entries", "n_part_entries", "n_near_entries", "n_pc", "n_pp", "n_groups"):
            assert st0[k] == st1[k], k
        out.append([t.cpu().numpy() for t in (acc, pot, off, idx, gp, gm)])
    a, b = out
    for u, v in zip(a[:4], b[:4]):
        assert np.array_equal(u, v)
    assert rel_rms(b[4], a[4]) < 1e-13 and rel_rms(b[5], a[5]) < 1e-13
    log(f"  recomputed lists ({precision}): forces and lists identical, "
        f"VJP {rel_rms(b[4], a[4]):.1e}")
    # the autograd function, with and without recomputation
    grads = []
    for rec in (False, True):
        x = pos.clone().requires_grad_(True)
        m = mass.clone().requires_grad_(True)
        acc, pot = long_force(x, m, ctx, recompute_lists=rec, **p)
        ((w * acc).sum() + (cw * pot).sum()).backward()
        grads.append((x.grad.cpu().numpy(), m.grad.cpu().numpy()))
    assert rel_rms(grads[1][0], grads[0][0]) < 1e-13 and rel_rms(grads[1][1], grads[0][1]) < 1e-13
