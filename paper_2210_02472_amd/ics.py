"""Seeded synthetic star-cluster inputs (positions, velocities, masses, active sets, levels).

These stand in for the paper's SCIC initial conditions (Appendix A), which are not
available: Plummer spheres sampled as described there (inversion sampling of the
cumulative mass profile; velocities by von Neumann rejection on the f(E) ~ E^(7/2)
distribution function), Kroupa (2001) IMF masses, a King (1966) W0 model for the
million-body case, binaries carried as centre-of-mass particles, and black holes.

All models are returned in Henon units (G = M = 1, E = -1/4) using the *model's*
energy (analytic for Plummer, integrated from the King profile), so this module
holds no pairwise arithmetic of the integrator itself.  Randomness comes from
numpy's PCG64 generator seeded per configuration.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 2210_02472


def rng_for(config_index: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([SEED_BASE + config_index, sub]))


def _isotropic(rng: np.random.Generator, r: np.ndarray) -> np.ndarray:
    """Vectors of length r with uniformly random directions on the unit sphere."""
    cost = rng.uniform(-1.0, 1.0, r.size)
    phi = rng.uniform(0.0, 2.0 * math.pi, r.size)
    sint = np.sqrt(1.0 - cost * cost)
    return np.stack([r * sint * np.cos(phi), r * sint * np.sin(phi), r * cost], axis=1)


def kroupa_masses(rng: np.random.Generator, n: int, mmin: float = 0.08, mmax: float = 100.0) -> np.ndarray:
    """Masses (solar units) from the two-segment Kroupa (2001) IMF:
    dN/dm ~ m^-1.3 on [mmin, 0.5), ~ m^-2.3 on [0.5, mmax], continuous at 0.5."""
    mb = 0.5
    a1, a2 = 1.3, 2.3
    # segment weights (continuity: k1 mb^-a1 = k2 mb^-a2 -> k1 = k2 mb^(a1-a2))
    k2 = 1.0
    k1 = k2 * mb ** (a1 - a2)
    w1 = k1 * (mb ** (1 - a1) - mmin ** (1 - a1)) / (1 - a1)
    w2 = k2 * (mmax ** (1 - a2) - mb ** (1 - a2)) / (1 - a2)
    u = rng.uniform(0.0, 1.0, n)
    seg1 = rng.uniform(0.0, 1.0, n) < w1 / (w1 + w2)

    def inv(u, lo, hi, a):
        e = 1.0 - a
        return (lo ** e + u * (hi ** e - lo ** e)) ** (1.0 / e)

    return np.where(seg1, inv(u, mmin, mb, a1), inv(u, mb, mmax, a2))


def plummer(rng: np.random.Generator, n: int, rmax_over_a: float = 20.0):
    """Plummer sphere with G = M = 1 and scale radius a = 3 pi / 16 (model energy -1/4).

    Radii by inverting M(<r) = r^3 / (r^2 + a^2)^(3/2) (re-drawn beyond rmax_over_a * a);
    speeds q * v_esc(r) with q from rejection on q^2 (1 - q^2)^(7/2)."""
    a = 3.0 * math.pi / 16.0
    r = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        X = rng.uniform(0.0, 1.0, todo.size)
        X = np.clip(X, 1e-300, None)
        rr = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
        ok = rr <= rmax_over_a * a
        r[todo[ok]] = rr[ok]
        todo = todo[~ok]
    pos = _isotropic(rng, r)
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x = rng.uniform(0.0, 1.0, todo.size)
        y = rng.uniform(0.0, 0.1, todo.size)
        ok = y < x * x * (1.0 - x * x) ** 3.5
        q[todo[ok]] = x[ok]
        todo = todo[~ok]
    vesc = math.sqrt(2.0 / a) * (1.0 + (r / a) ** 2) ** -0.25
    vel = _isotropic(rng, q * vesc)
    return pos, vel


# ---------------------------------------------------------------------------------------------
# King (1966) model
# ---------------------------------------------------------------------------------------------

def _king_rho(W):
    """Dimensionless King density for potential depth W >= 0 (sigma = 1)."""
    W = np.maximum(W, 0.0)
    from scipy.special import erf
    return np.exp(W) * erf(np.sqrt(W)) - np.sqrt(4.0 * W / math.pi) * (1.0 + 2.0 * W / 3.0)


def king_profile(W0: float, npts: int = 20000):
    """Integrate the King Poisson equation W'' + 2 W'/r = -9 rho(W)/rho(W0) (radius in King
    core radii, sigma = 1) from the centre out to the tidal radius where W = 0.
    Returns (r, W, M(<r)) on a grid with G = 1 (so 4 pi G rho0 = 9)."""
    from scipy.integrate import solve_ivp
    rho0 = _king_rho(np.array(W0))

    def rhs(r, y):
        W, dW = y
        rho = _king_rho(np.array(W)) / rho0
        if r == 0.0:
            return [dW, -3.0 * rho]
        return [dW, -9.0 * rho - 2.0 * dW / r]

    def hit(r, y):
        return y[0]
    hit.terminal = True
    hit.direction = -1
    r0 = 1e-6
    y0 = [W0 - 1.5 * r0 * r0, -3.0 * r0]  # series start: W ~ W0 - (3/2) r^2
    sol = solve_ivp(rhs, (r0, 1e4), y0, events=hit, rtol=1e-10, atol=1e-12, dense_output=True,
                    max_step=0.05)
    rt = float(sol.t_events[0][0]) if sol.t_events[0].size else float(sol.t[-1])
    r = np.concatenate([[0.0], np.geomspace(r0, rt, npts)])
    W = np.concatenate([[W0], sol.sol(r[1:])[0]])
    W = np.maximum(W, 0.0)
    W[-1] = 0.0
    rho = (9.0 / (4.0 * math.pi)) * _king_rho(W) / rho0
    # cumulative mass by trapezoid on 4 pi r^2 rho
    f = 4.0 * math.pi * r * r * rho
    M = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(r))])
    return r, W, M


def king(rng: np.random.Generator, n: int, W0: float = 6.0):
    """King W0 model sampled in Henon units.  Radii by inverting the tabulated M(<r);
    speeds by rejection from f ~ exp(W - v^2/2) - 1 with v < sqrt(2 W).  The length and
    velocity scales come from the model's own potential energy U = -int G M(r)/r dM
    (virial equilibrium, E = U/2), scaled to M = 1, E = -1/4."""
    r_t, W_t, M_t = king_profile(W0)
    Mtot = M_t[-1]
    u = rng.uniform(0.0, 1.0, n) * Mtot
    r = np.interp(u, M_t, r_t)
    W = np.interp(r, r_t, W_t)
    # speeds: g(q) = q^2 (exp(W (1 - q^2)) - 1), v = q sqrt(2W)
    qgrid = np.linspace(0.0, 1.0, 257)[None, :]
    v = np.zeros(n)
    todo = np.nonzero(W > 0)[0]
    gmax = (qgrid ** 2 * (np.exp(W[todo, None] * (1.0 - qgrid ** 2)) - 1.0)).max(axis=1) * 1.05 + 1e-300
    while todo.size:
        q = rng.uniform(0.0, 1.0, todo.size)
        y = rng.uniform(0.0, 1.0, todo.size) * gmax
        ok = y < q * q * (np.exp(W[todo] * (1.0 - q * q)) - 1.0)
        v[todo[ok]] = q[ok] * np.sqrt(2.0 * W[todo[ok]])
        todo, gmax = todo[~ok], gmax[~ok]
    # model potential energy (G = 1): U = -int M(r)/r dM
    dM = np.diff(M_t)
    rm = 0.5 * (r_t[1:] + r_t[:-1])
    Mm = 0.5 * (M_t[1:] + M_t[:-1])
    U = -np.sum(Mm / np.maximum(rm, 1e-300) * dM)
    E = 0.5 * U
    mu = 1.0 / Mtot
    lam = -4.0 * E * mu * mu
    nu = math.sqrt(mu / lam)
    pos = _isotropic(rng, r * lam)
    vel = _isotropic(rng, v * nu)
    return pos, vel


# ---------------------------------------------------------------------------------------------
# assembling particle sets
# ---------------------------------------------------------------------------------------------

def _to_com(pos, vel, m):
    M = m.sum()
    pos = pos - (m[:, None] * pos).sum(axis=0) / M
    vel = vel - (m[:, None] * vel).sum(axis=0) / M
    return pos, vel


def _pack(pos, vel, m):
    return {"x": np.ascontiguousarray(pos[:, 0]), "y": np.ascontiguousarray(pos[:, 1]),
            "z": np.ascontiguousarray(pos[:, 2]), "vx": np.ascontiguousarray(vel[:, 0]),
            "vy": np.ascontiguousarray(vel[:, 1]), "vz": np.ascontiguousarray(vel[:, 2]),
            "m": np.ascontiguousarray(m, dtype=np.float64)}


def plummer_cluster(rng, n: int, masses: str = "equal", rmax_over_a: float = 20.0):
    """Plummer sphere of n particles (equal masses or Kroupa masses), total mass 1, COM frame."""
    pos, vel = plummer(rng, n, rmax_over_a)
    if masses == "equal":
        m = np.full(n, 1.0 / n)
    else:
        m = kroupa_masses(rng, n)
        m = m / m.sum()
    pos, vel = _to_com(pos, vel, m)
    return _pack(pos, vel, m)


def king_cluster(rng, n: int, W0: float = 6.0, binary_fraction: float = 0.01):
    """King W0 cluster with Kroupa masses; a fraction of particles are binary centres of
    mass carrying the summed mass of two independent draws.  Total mass 1, COM frame."""
    pos, vel = king(rng, n, W0)
    m = kroupa_masses(rng, n)
    nb = int(round(binary_fraction * n))
    if nb:
        pick = rng.choice(n, size=nb, replace=False)
        m[pick] += kroupa_masses(rng, nb)
    m = m / m.sum()
    pos, vel = _to_com(pos, vel, m)
    return _pack(pos, vel, m)


def random_subset(rng, n: int, fraction: float) -> np.ndarray:
    """Sorted random subset (at least one element) of range(n), int32."""
    k = max(1, int(round(fraction * n)))
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)


# ---------------------------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------------------------

def config1_plummer1k(n: int = 1024):
    """Equal-mass Plummer sphere, N = 1024, Henon units, eps = 0, all active."""
    return plummer_cluster(rng_for(0), n, "equal")


def config2_plummer64k(n: int = 65536, active_fraction: float = 0.1):
    """Kroupa-mass Plummer sphere N = 65,536 with a random 10% active level."""
    rng = rng_for(1)
    P = plummer_cluster(rng, n, "kroupa")
    return P, random_subset(rng, n, active_fraction)


def config3_king1m(n: int = 1 << 20):
    """King W0 = 6, Kroupa masses, 1% binaries as centre-of-mass particles, N = 2^20."""
    return king_cluster(rng_for(2), n, 6.0, 0.01)


def config4_ensemble(n_clusters: int = 256, nmin: int = 1024, nmax: int = 65536, kmax: int = 6,
                     total_cap: int | None = None):
    """Ensemble of independent equal-mass Plummer clusters with log-uniform sizes and active
    fractions 2^-k, k uniform on {0..kmax}.  Returns the concatenated particle dict, the
    cluster offsets (int64, length n_clusters + 1), the concatenated global active indices
    (int32) and their per-cluster offsets (int64)."""
    rng = rng_for(3)
    sizes = np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax), n_clusters))).astype(np.int64)
    if total_cap is not None:
        sizes = np.minimum(sizes, max(nmin, total_cap // n_clusters))
    ks = rng.integers(0, kmax + 1, n_clusters)
    parts, act = [], []
    off = np.zeros(n_clusters + 1, dtype=np.int64)
    aoff = np.zeros(n_clusters + 1, dtype=np.int64)
    for c in range(n_clusters):
        sub = rng_for(3, 1 + c)
        parts.append(plummer_cluster(sub, int(sizes[c]), "equal"))
        off[c + 1] = off[c] + sizes[c]
        a = random_subset(sub, int(sizes[c]), 2.0 ** -int(ks[c])).astype(np.int64) + off[c]
        act.append(a)
        aoff[c + 1] = aoff[c] + a.size
    P = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    return P, off, np.concatenate(act).astype(np.int32), aoff


def config5_bh_cluster(n: int = 262144, n_bh: int = 16, levels: int = 7):
    """Kroupa Plummer cluster with n_bh stellar BHs (10-100 Msun, log-uniform) and one
    1000 Msun IMBH at rest at the centre, total mass 1.  Per-particle time-step levels
    0..levels with the fraction at level >= k equal to 2^-k; the IMBH and BHs sit at the
    deepest level.  Returns (particles, bh indices int32, levels int8)."""
    rng = rng_for(4)
    pos, vel = plummer(rng, n)
    m = kroupa_masses(rng, n)
    bh = np.sort(rng.choice(np.arange(1, n), size=n_bh, replace=False))
    m[bh] = np.exp(rng.uniform(math.log(10.0), math.log(100.0), n_bh))
    m[0] = 1000.0
    pos[0] = 0.0
    vel[0] = 0.0
    m = m / m.sum()
    pos, vel = _to_com(pos, vel, m)
    lv = np.zeros(n, dtype=np.int8)
    u = rng.uniform(0.0, 1.0, n)
    for k in range(1, levels + 1):
        lv[u < 2.0 ** -k] = k
    bh_all = np.concatenate([[0], bh]).astype(np.int32)
    lv[bh_all] = levels
    return _pack(pos, vel, m), bh_all, lv
