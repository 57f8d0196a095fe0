"""Seeded synthetic star-cluster initial conditions (Plummer, King, Salpeter).

These generators are shared by the tests, the benchmark and the smoke check.
They hold none of the tree-force arithmetic: they only draw positions,
velocities and masses from textbook cluster models with numpy's PCG64.

Units are the N-body (Heggie) units the paper works in: G = M = 1 and total
energy E = -1/4 (Section 3.1).  Scaling to those units is analytic, from the
model's own energy integrals, followed by a centre-of-mass shift; there is no
empirical re-virialisation.

Conventions
-----------
* Every generator takes ``seed`` and uses ``numpy.random.Generator(PCG64(seed))``.
* Positions/velocities are float64 arrays of shape ``[N, 3]`` (row = particle),
  masses float64 ``[N]`` summing to 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.integrate import solve_ivp
from scipy.special import erf

# Plummer model: virial-unit scale length a = 3*pi/16 (E = -1/4 with G = M = 1).
PLUMMER_A_NBODY = 3.0 * math.pi / 16.0


@dataclass
class Cluster:
    pos: np.ndarray   # [N,3] float64
    vel: np.ndarray   # [N,3] float64
    mass: np.ndarray  # [N]   float64
    name: str = ""


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors uniform on the sphere: cos(theta) uniform in [-1,1], phi uniform."""
    ct = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    return np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)


def _com_shift(pos: np.ndarray, vel: np.ndarray, mass: np.ndarray):
    mtot = mass.sum()
    pos = pos - (mass[:, None] * pos).sum(0) / mtot
    vel = vel - (mass[:, None] * vel).sum(0) / mtot
    return pos, vel


def salpeter_masses(n: int, seed: int, slope: float = 2.35, m_lo: float = 0.1,
                    m_hi: float = 100.0) -> np.ndarray:
    """Power-law IMF dN/dm ~ m^-slope on [m_lo, m_hi] by inverse CDF, rescaled to sum 1."""
    rng = _rng(seed)
    u = rng.uniform(0.0, 1.0, n)
    e = 1.0 - slope
    m = (m_lo ** e + u * (m_hi ** e - m_lo ** e)) ** (1.0 / e)
    return m / m.sum()


def plummer(n: int, seed: int = 1, r_cut_nbody: float = 22.8,
            masses: np.ndarray | None = None) -> Cluster:
    """Plummer sphere, Aarseth-Henon-Wielen (1974) sampling, in N-body units.

    Radii come from the cumulative mass fraction X ~ U(0,1):
    r = (X^(-2/3) - 1)^(-1/2) in Plummer units (a = 1); radii beyond
    ``r_cut_nbody`` (N-body units) are redrawn.  Speeds are q * v_esc with q drawn
    by von Neumann rejection on g(q) = q^2 (1 - q^2)^(7/2) (bound 0.1).
    Positions are then scaled by 3*pi/16 and velocities by sqrt(16/(3*pi)).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = _rng(seed)
    r = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x = rng.uniform(0.0, 1.0, todo.size)
        x = np.clip(x, 1e-300, 1.0 - 1e-16)
        rr = 1.0 / np.sqrt(x ** (-2.0 / 3.0) - 1.0)
        ok = rr * PLUMMER_A_NBODY <= r_cut_nbody
        r[todo[ok]] = rr[ok]
        todo = todo[~ok]
    pos = _isotropic(rng, n) * r[:, None]
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        qq = rng.uniform(0.0, 1.0, todo.size)
        yy = rng.uniform(0.0, 0.1, todo.size)
        ok = yy < qq * qq * (1.0 - qq * qq) ** 3.5
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    vesc = math.sqrt(2.0) * (1.0 + r * r) ** -0.25
    vel = _isotropic(rng, n) * (q * vesc)[:, None]
    pos = pos * PLUMMER_A_NBODY
    vel = vel / math.sqrt(PLUMMER_A_NBODY)
    mass = np.full(n, 1.0 / n) if masses is None else np.asarray(masses, dtype=np.float64)
    if mass.shape != (n,):
        raise ValueError("masses must have shape [n]")
    pos, vel = _com_shift(pos, vel, mass)
    return Cluster(pos, vel, mass, f"plummer{n}")


# ---------------------------------------------------------------------------
# King (1966) model.  Dimensionless potential W = psi / sigma^2, radius in
# King radii r0 with r0^2 = 9 sigma^2 / (4 pi G rho0), G = sigma = 1.
# Density rho(W) ~ e^W erf(sqrt W) - sqrt(4W/pi) (1 + 2W/3);
# Poisson: W'' + 2 W'/r = -9 rho(W)/rho(W0); M(r) = -r^2 W'(r).
# ---------------------------------------------------------------------------

def _king_rho(w):
    w = np.maximum(w, 0.0)
    sw = np.sqrt(w)
    return np.exp(w) * erf(sw) - np.sqrt(4.0 * w / math.pi) * (1.0 + 2.0 * w / 3.0)


@dataclass
class KingProfile:
    r: np.ndarray      # radius grid (King radii)
    w: np.ndarray      # W(r)
    m: np.ndarray      # enclosed mass M(r) (model units)
    rt: float          # tidal radius
    mtot: float
    u_pot: float       # potential energy of the truncated model (model units)


def king_profile(w0: float, n_grid: int = 20000) -> KingProfile:
    """Integrate the King Poisson equation outward from W(0)=W0 until W=0."""
    rho0 = float(_king_rho(np.array(w0)))

    def rhs(r, s):
        w, dw, m, u = s
        rho = float(_king_rho(np.array(w))) / rho0
        d2w = -9.0 * rho - 2.0 * dw / r
        dm = 9.0 * r * r * rho
        du = -9.0 * m * r * rho
        return [dw, d2w, dm, du]

    r_start = 1e-6
    w_start = w0 - 1.5 * r_start ** 2
    s0 = [w_start, -3.0 * r_start, 3.0 * r_start ** 3, 0.0]

    def hit_zero(r, s):
        return s[0]
    hit_zero.terminal = True
    hit_zero.direction = -1
    sol = solve_ivp(rhs, (r_start, 1e6), s0, events=hit_zero, rtol=1e-10, atol=1e-12,
                    dense_output=True, method="RK45")
    if sol.status != 1:
        raise RuntimeError("King ODE did not reach W = 0")
    rt = float(sol.t_events[0][0])
    rr = np.concatenate([[0.0], np.geomspace(r_start, rt, n_grid)])
    st = sol.sol(rr[1:])
    w = np.concatenate([[w0], st[0]])
    m = np.concatenate([[0.0], st[2]])
    w[-1] = 0.0
    send = sol.sol(rt)
    return KingProfile(rr, w, m, rt, float(send[2]), float(send[3]))


def king(n: int, w0: float = 9.0, seed: int = 1) -> Cluster:
    """Equal-mass King model sampled from its distribution function, N-body units.

    Radii by inverse interpolation of M(r); speeds (units of sigma) by rejection
    on p(v) ~ v^2 (exp(W - v^2/2) - 1), 0 <= v < sqrt(2W).  Scaling to G=M=1,
    E=-1/4 uses the model's own potential energy U and the virial K = -U/2.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    prof = king_profile(w0)
    rng = _rng(seed)
    u = rng.uniform(0.0, 1.0, n) * prof.mtot
    r = np.interp(u, prof.m, prof.r)
    w = np.interp(r, prof.r, prof.w)
    w = np.maximum(w, 0.0)
    vmax = np.sqrt(2.0 * w)
    bound = np.minimum(2.0 * np.exp(w - 1.0), 2.0 * w * np.expm1(w)) * 1.0001 + 1e-300
    v = np.zeros(n)
    todo = np.nonzero(vmax > 0)[0]
    while todo.size:
        vv = rng.uniform(0.0, 1.0, todo.size) * vmax[todo]
        yy = rng.uniform(0.0, 1.0, todo.size) * bound[todo]
        ok = yy < vv * vv * np.expm1(w[todo] - 0.5 * vv * vv)
        v[todo[ok]] = vv[ok]
        todo = todo[~ok]
    pos = _isotropic(rng, n) * r[:, None]
    vel = _isotropic(rng, n) * v[:, None]
    # N-body scaling: masses / M, lengths * lam, velocities * mu.
    # U' = U / (M^2 lam) = -1/2  ->  lam = -2 U / M^2 ;  K' = 1/4 with K = -U/2.
    lam = -2.0 * prof.u_pot / prof.mtot ** 2
    kin_model = -0.5 * prof.u_pot
    mu = math.sqrt(0.25 * prof.mtot / kin_model)
    pos = pos * lam
    vel = vel * mu
    mass = np.full(n, 1.0 / n)
    pos, vel = _com_shift(pos, vel, mass)
    return Cluster(pos, vel, mass, f"king{w0:g}_{n}")


def king_scale(w0: float = 9.0):
    """(King radius, tidal radius) of the model in N-body units."""
    prof = king_profile(w0)
    lam = -2.0 * prof.u_pot / prof.mtot ** 2
    return lam, prof.rt * lam
