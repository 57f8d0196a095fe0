"""Plain O(N^2) definitions the tree method reduces to -- TEST INFRASTRUCTURE ONLY.

Everything here is written directly from the definitions, in numpy FP64:

* soft force and potential (Section 2.1): a_i = sum_{j!=i} m_j K(s_ij) d_ij / s_ij^3,
  phi_i = -sum_{j!=i} m_j W(s_ij) / s_ij, with s_ij the softened distance;
* the hard (short-range) part with (1 - K) and (1 - W), and plain softened Newton;
* W is obtained from K alone: the paper defines K = W - s dW/ds, which gives
  d(W/y)/dy = -K(y)/y^2, and W = 1 beyond the outer cutoff, so
  W(y)/y = 1 + integral_y^1 K(t)/t^2 dt  (y < 1), evaluated by Gauss-Legendre
  quadrature -- independent of the closed form the tree oracle uses;
* neighbour sets "within distance h" (Section 2.2) by testing every pair with
  dx*dx + dy*dy + dz*dz < h*h;
* the gradient of L = sum w.a + sum c.phi of the direct soft sum;
* particle kinds (Section 3.2.2, the SMBH runs): the soft sum of the pairs that
  involve a special particle, each pair with its own parameters, and the
  neighbour sets with a radius per kind of pair.
"""
from __future__ import annotations

import math

import numpy as np

_GL_X, _GL_W = np.polynomial.legendre.leggauss(48)

# K(x) = -20x^7 + 70x^6 - 84x^5 + 35x^4 on 0 <= x < 1 (Section 2.1), as a
# coefficient vector (highest power first) for numpy's polynomial helpers.
_KPOLY = np.array([-20.0, 70.0, -84.0, 35.0, 0.0, 0.0, 0.0, 0.0])
_DKPOLY = np.polyder(_KPOLY)


def K_np(y, gamma):
    y = np.asarray(y, dtype=np.float64)
    x = np.clip((y - gamma) / (1.0 - gamma), 0.0, 1.0)
    out = np.polyval(_KPOLY, x)
    out = np.where(y < gamma, 0.0, out)
    return np.where(y >= 1.0, 1.0, out)


def dKdy_np(y, gamma):
    y = np.asarray(y, dtype=np.float64)
    x = (y - gamma) / (1.0 - gamma)
    out = np.polyval(_DKPOLY, np.clip(x, 0.0, 1.0)) / (1.0 - gamma)
    return np.where((y < gamma) | (y >= 1.0), 0.0, out)


def W_over_y_np(y, gamma):
    """W(y)/y from K by quadrature; flat (= value at gamma) below gamma."""
    y = np.asarray(y, dtype=np.float64)
    out = np.empty_like(y)
    far = y >= 1.0
    out[far] = 1.0 / y[far]
    near = ~far
    if near.any():
        a = np.maximum(y[near], gamma)[:, None]
        t = 0.5 * (1.0 - a) * _GL_X[None, :] + 0.5 * (1.0 + a)
        integ = 0.5 * (1.0 - a[:, 0]) * (K_np(t, gamma) / (t * t) @ _GL_W)
        out[near] = 1.0 + integ
    return out


def C_np(gamma):
    return float(W_over_y_np(np.array([0.0]), gamma)[0])


def _pairs(pos, i0, i1, eps):
    d = pos[None, :, :] - pos[i0:i1, None, :]          # d[i, j] = x_j - x_i
    s2 = (d * d).sum(-1) + eps * eps
    return d, s2


def soft_direct(pos, mass, eps, r_in, r_out, block=512):
    """Direct soft acceleration and potential (all j != i)."""
    n = len(mass)
    gamma = r_in / r_out
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        d, s2 = _pairs(pos, i0, i1, eps)
        s = np.sqrt(s2)
        y = s / r_out
        k = K_np(y, gamma)
        wy = W_over_y_np(y.ravel(), gamma).reshape(y.shape)
        f = mass[None, :] * k / (s2 * s)
        ph = mass[None, :] * wy / r_out
        ii = np.arange(i0, i1)
        f[ii - i0, ii] = 0.0
        ph[ii - i0, ii] = 0.0
        acc[i0:i1] = (f[:, :, None] * d).sum(1)
        pot[i0:i1] = -ph.sum(1)
    return acc, pot


def hard_direct_pairs(pos, mass, eps, r_in, r_out, offsets, idx):
    """Hard part (1-K, 1-W) summed over given neighbour lists (CSR, original order)."""
    n = len(mass)
    gamma = r_in / r_out
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    rows = np.repeat(np.arange(n), np.diff(offsets))
    if len(idx):
        d = pos[idx] - pos[rows]
        s2 = (d * d).sum(-1) + eps * eps
        s = np.sqrt(s2)
        y = s / r_out
        k = K_np(y, gamma)
        w = W_over_y_np(y, gamma) * y
        f = mass[idx] * (1.0 - k) / (s2 * s)
        np.add.at(acc, rows, f[:, None] * d)
        np.add.at(pot, rows, -mass[idx] * (1.0 - w) / s)
    return acc, pot


def newton_direct(pos, mass, eps, block=512):
    """Plain softened Newtonian acceleration and potential."""
    n = len(mass)
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        d, s2 = _pairs(pos, i0, i1, eps)
        s = np.sqrt(s2)
        f = mass[None, :] / (s2 * s)
        ph = mass[None, :] / s
        ii = np.arange(i0, i1)
        f[ii - i0, ii] = 0.0
        ph[ii - i0, ii] = 0.0
        acc[i0:i1] = (f[:, :, None] * d).sum(1)
        pot[i0:i1] = -ph.sum(1)
    return acc, pot


def brute_neighbors(pos, h, block=1024):
    """CSR (offsets, idx) of j != i with dx*dx + dy*dy + dz*dz < h*h."""
    n = pos.shape[0]
    h2 = h * h
    rows = []
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        dx = pos[None, :, 0] - pos[i0:i1, None, 0]
        dy = pos[None, :, 1] - pos[i0:i1, None, 1]
        dz = pos[None, :, 2] - pos[i0:i1, None, 2]
        r2 = dx * dx + dy * dy + dz * dz
        hit = r2 < h2
        ii = np.arange(i0, i1)
        hit[ii - i0, ii] = False
        for r in range(i1 - i0):
            rows.append(np.nonzero(hit[r])[0])
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    idx = np.concatenate(rows).astype(np.int64) if rows else np.zeros(0, np.int64)
    return off, idx


def soft_direct_grad(pos, mass, eps, r_in, r_out, w, c=None, block=256):
    """Gradient of L = sum_i w_i.a_i + c_i phi_i (direct soft sum) wrt pos and mass."""
    n = len(mass)
    gamma = r_in / r_out
    c = np.zeros(n) if c is None else c
    gpos = np.zeros((n, 3))
    gmass = np.zeros(n)
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        d, s2 = _pairs(pos, i0, i1, eps)
        s = np.sqrt(s2)
        y = s / r_out
        k = K_np(y, gamma)
        dk = dKdy_np(y, gamma) / r_out
        wv = W_over_y_np(y.ravel(), gamma).reshape(y.shape) * y
        g = k / (s2 * s)
        dg = dk / (s2 * s) - 3.0 * k / (s2 * s2)
        wi = w[i0:i1]
        ci = c[i0:i1]
        wd = (wi[:, None, :] * d).sum(-1)
        ii = np.arange(i0, i1)
        mask = np.ones_like(g)
        mask[ii - i0, ii] = 0.0
        mj = mass[None, :] * mask
        gd = mj[:, :, None] * (g[:, :, None] * wi[:, None, :]
                               + (dg * wd / s)[:, :, None] * d
                               + (ci[:, None] * k / (s2 * s))[:, :, None] * d)
        gpos += gd.sum(0)                 # d/dx_j
        gpos[i0:i1] -= gd.sum(1)          # d/dx_i
        gmass += ((g * wd - ci[:, None] * wv / s) * mask).sum(0)
    return gpos, gmass


def plummer_potential(r, a=3.0 * math.pi / 16.0):
    """Potential of a unit-mass Plummer sphere with scale a (G = 1)."""
    return -1.0 / np.sqrt(r * r + a * a)


def plummer_accel(r, a=3.0 * math.pi / 16.0):
    """Magnitude of the inward acceleration of a unit-mass Plummer sphere."""
    return r / (r * r + a * a) ** 1.5


def _kind_pair(n_total, n_special, i, j, eps, r_in, r_out, kinds):
    """(eps, r_in, r_out, split) of the pair (i, j) by kinds: the last
    n_special particles are special (Section 3.2.2)."""
    first = n_total - n_special
    si, sj = i >= first, j >= first
    if si and sj:
        return kinds["eps_ss"], kinds["r_in_ss"], kinds["r_out_ss"], bool(kinds["split_ss"])
    if si or sj:
        return kinds["eps_ns"], kinds["r_in_ns"], kinds["r_out_ns"], True
    return eps, r_in, r_out, True


def kinds_soft(pos, mass, eps, r_in, r_out, kinds):
    """Soft acceleration and potential of every pair that involves a special
    particle, with that pair's own parameters (a special-special pair that is
    not split has no soft part).  Pairs of two normal particles are left out:
    the tree sums them."""
    n = len(mass)
    ns = int(kinds["n_special"])
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    for b in range(n - ns, n):
        for i in range(n):
            if i == b:
                continue
            e, ri, ro, split = _kind_pair(n, ns, i, b, eps, r_in, r_out, kinds)
            if not split:
                continue
            d = pos[b] - pos[i]
            s = math.sqrt(float(d @ d) + e * e)
            y = np.array([s / ro])
            g = ri / ro
            K = float(K_np(y, g)[0])
            W = float(W_over_y_np(y, g)[0] * y[0])
            if i < n - ns or i > b:
                # i gets b's pull; for two special particles each pair is visited once
                acc[i] += mass[b] * K * d / s ** 3
                pot[i] -= mass[b] * W / s
                acc[b] -= mass[i] * K * d / s ** 3
                pot[b] -= mass[i] * W / s
    return acc, pot


def kinds_neighbors(pos, n_special, h_nn, h_ns, split_ss, h_ss):
    """CSR of j != i within the pair's radius: h_nn for two normal particles,
    h_ns for a normal and a special one; two special particles are always
    neighbours when their pair is not split, else within h_ss.  Same FP64 test
    as brute_neighbors."""
    n = pos.shape[0]
    first = n - n_special
    rows = []
    for i in range(n):
        dx = pos[:, 0] - pos[i, 0]
        dy = pos[:, 1] - pos[i, 1]
        dz = pos[:, 2] - pos[i, 2]
        r2 = dx * dx + dy * dy + dz * dz
        sp = np.arange(n) >= first
        if i >= first:
            h = np.where(sp, h_ss, h_ns)
        else:
            h = np.where(sp, h_ns, h_nn)
        hit = r2 < h * h
        if i >= first and not split_ss:
            hit |= sp
        hit[i] = False
        rows.append(np.nonzero(hit)[0])
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    idx = np.concatenate(rows).astype(np.int64) if rows else np.zeros(0, np.int64)
    return off, idx
