"""FP64 CPU oracle for the HHS-FSI direct-summation pass (BIFROST, arXiv 2210.02472).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this package; the product path (the HIP library and
its Python binding) never imports it and shares no code with it.

The pairwise sums live in ``bf_oracle.c`` (plain loops, one target at a time);
this module marshals numpy arrays into them and writes the integrator steps
(kick, drift, gradient kick; the FSI cycle of Sec. 2.1 and the HHS-FSI recursion
of Sec. 2.2) in numpy, in the paper's order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bf_oracle.c")
_SO = os.path.join(_HERE, "libbf_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle into ``oracle/libbf_oracle.so`` (gcc, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", _SO + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        lib.oracle_forces.argtypes = [P, P, P, P, I64, P, I64, P, P, D, D, P, P, P, P, P]
        lib.oracle_gradient.argtypes = [P, P, P, P, P, P, P, I64, P, I64, P, P, D, D, P, P, P, P, P]
        lib.oracle_dt_min.argtypes = [P, P, P, P, P, P, P, I64, P, I64, P, P, D, D, D, P, P, P]
        lib.oracle_neighbours.argtypes = [P, P, P, P, P, P, P, I64, P, I64, P, D, D, D, D, D, P]
        lib.oracle_pn1.argtypes = [P, P, P, P, P, P, P, P, I64, P, I64, P, D, D, P, P, P, P]
        lib.oracle_energy.argtypes = [P, P, P, P, P, P, P, I64, P, D, D, P, P, P]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


@dataclass
class Particles:
    """Structure-of-arrays FP64 particle state (positions, velocities, masses)."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    m: np.ndarray

    @property
    def n(self) -> int:
        return int(self.m.shape[0])

    def copy(self) -> "Particles":
        return Particles(*(np.array(a, dtype=np.float64, copy=True) for a in
                           (self.x, self.y, self.z, self.vx, self.vy, self.vz, self.m)))

    @staticmethod
    def from_dict(d) -> "Particles":
        """Copy of a dict of arrays keyed x, y, z, vx, vy, vz, m."""
        return Particles(*(np.array(d[k], dtype=np.float64, copy=True, order="C") for k in
                           ("x", "y", "z", "vx", "vy", "vz", "m")))

    def pos(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)

    def vel(self) -> np.ndarray:
        return np.stack([self.vx, self.vy, self.vz], axis=1)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _idx(sel, n: int) -> np.ndarray:
    if sel is None:
        return np.arange(n, dtype=np.int64)
    a = np.ascontiguousarray(sel, dtype=np.int64)
    if a.size and (a.min() < 0 or a.max() >= n):
        raise IndexError("particle index out of range")
    return a


def _check(p: Particles):
    for a in (p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m):
        assert a.dtype == np.float64 and a.flags.c_contiguous and a.shape == (p.n,)


def _sub(sub, n: int):
    """Particle-indexed subsystem labels as int64 (or None: no exclusion)."""
    if sub is None:
        return None
    a = np.ascontiguousarray(sub, dtype=np.int64)
    assert a.shape == (n,)
    return a


def forces(p: Particles, targets=None, sources=None, G: float = 1.0, eps2: float = 0.0,
           return_mag: bool = False, sub=None):
    """Newtonian accelerations of `targets` from `sources` (Sec. 2.1, Eq. new-newton-acc).

    Returns an (nt, 3) array indexed by target slot (and optionally the per-target
    sum of term magnitudes and the count of coincident distinct pairs).  With `sub`
    (particle-indexed subsystem labels) pairs inside one subsystem are left out (Alg. 1)."""
    _check(p)
    t, s = _idx(targets, p.n), _idx(sources, p.n)
    sb = _sub(sub, p.n)
    nt = t.size
    ax, ay, az, mag = (np.zeros(nt) for _ in range(4))
    nco = ctypes.c_int64(0)
    _load().oracle_forces(_ptr(p.x), _ptr(p.y), _ptr(p.z), _ptr(p.m), nt, _ptr(t), s.size, _ptr(s),
                          _ptr(sb) if sb is not None else None,
                          float(G), float(eps2), _ptr(ax), _ptr(ay), _ptr(az), _ptr(mag),
                          ctypes.byref(nco))
    a = np.stack([ax, ay, az], axis=1)
    return (a, mag, int(nco.value)) if return_mag else a


def gradient(p: Particles, acc_full: np.ndarray, targets=None, sources=None, G: float = 1.0,
             eps2: float = 0.0, return_mag: bool = False, sub=None):
    """Force-gradient sum Gsum (Sec. 2.1, Eq. new-grad-acc; inter-level form Sec. 2.2).

    `acc_full` is an (n, 3) particle-indexed array of the accelerations that enter
    a_ji.  The gradient acceleration of a kick of length eps is a + eps^2/24 Gsum."""
    _check(p)
    t, s = _idx(targets, p.n), _idx(sources, p.n)
    af = np.ascontiguousarray(acc_full, dtype=np.float64)
    assert af.shape == (p.n, 3)
    axf, ayf, azf = (np.ascontiguousarray(af[:, k]) for k in range(3))
    nt = t.size
    gx, gy, gz, mag = (np.zeros(nt) for _ in range(4))
    nco = ctypes.c_int64(0)
    sb = _sub(sub, p.n)
    _load().oracle_gradient(_ptr(p.x), _ptr(p.y), _ptr(p.z), _ptr(p.m), _ptr(axf), _ptr(ayf), _ptr(azf),
                            nt, _ptr(t), s.size, _ptr(s), _ptr(sb) if sb is not None else None,
                            float(G), float(eps2),
                            _ptr(gx), _ptr(gy), _ptr(gz), _ptr(mag), ctypes.byref(nco))
    g = np.stack([gx, gy, gz], axis=1)
    return (g, mag, int(nco.value)) if return_mag else g


def dt_min(p: Particles, targets=None, sources=None, G: float = 1.0, eta_ff: float = 0.2,
           eta_fb: float = 0.2, sub=None):
    """Free-fall and fly-by time-steps (Sec. 3.5.3, Eqs. dt-freefall, dt-flyby); returns (dt_ff, dt_fb)."""
    _check(p)
    t, s = _idx(targets, p.n), _idx(sources, p.n)
    nt = t.size
    ff, fb = np.zeros(nt), np.zeros(nt)
    nco = ctypes.c_int64(0)
    sb = _sub(sub, p.n)
    _load().oracle_dt_min(_ptr(p.x), _ptr(p.y), _ptr(p.z), _ptr(p.vx), _ptr(p.vy), _ptr(p.vz), _ptr(p.m),
                          nt, _ptr(t), s.size, _ptr(s), _ptr(sb) if sb is not None else None,
                          float(G), float(eta_ff), float(eta_fb),
                          _ptr(ff), _ptr(fb), ctypes.byref(nco))
    return ff, fb


def pn1(p: Particles, bh, targets=None, sources=None, G: float = 1.0, c: float = 1e4):
    """Global PN1.0 acceleration over pairs with a flagged massive particle (Sec. 3.8,
    Eqs. subsyspn, subsyspn-mass).  `bh` is a list of particle indices."""
    _check(p)
    t, s = _idx(targets, p.n), _idx(sources, p.n)
    flag = np.zeros(p.n, dtype=np.uint8)
    flag[_idx(bh, p.n)] = 1
    nt = t.size
    px, py, pz = (np.zeros(nt) for _ in range(3))
    nco = ctypes.c_int64(0)
    _load().oracle_pn1(_ptr(p.x), _ptr(p.y), _ptr(p.z), _ptr(p.vx), _ptr(p.vy), _ptr(p.vz), _ptr(p.m),
                       _ptr(flag), nt, _ptr(t), s.size, _ptr(s), float(G), float(c),
                       _ptr(px), _ptr(py), _ptr(pz), ctypes.byref(nco))
    return np.stack([px, py, pz], axis=1)


def jerk(p: Particles, targets=None, sources=None, G: float = 1.0, eps2: float = 0.0):
    """Jerk j_i = sum_j G m_j / s^5 (s^2 v_ji - 3 (r_ji . v_ji) r_ji) (Sec. 3.5.5).  It is the
    tidal tensor contracted with v_ji, i.e. the force-gradient sum of the C routine evaluated
    with the velocities in place of the accelerations."""
    return gradient(p, p.vel(), targets, sources, G, eps2)


def timestep_criteria(p: Particles, idx, dt_ff, dt_fb, acc, gsum=None, jrk=None, eta_grad: float = 0.1,
                      eta_jerk: float = 0.1):
    """Per-particle time-step: the minimum of the pairwise criteria (Sec. 3.5.3) and of
    eta_grad (|v|/|g'|)^(1/3), eta_grad (|a|/|g'|)^(1/2) with g' = Gsum/24 (Sec. 3.5.4, Eqs.
    dt-nabla1, dt-nabla2) and eta_jerk |a|/|j| (Sec. 3.5.5).  All arrays are per listed particle
    (row k belongs to particle idx[k]); a criterion with a zero denominator or eta <= 0 is skipped."""
    idx = np.asarray(idx)
    dt = np.minimum(np.asarray(dt_ff, float), np.asarray(dt_fb, float)).copy()
    v = np.linalg.norm(p.vel()[idx], axis=1)
    a = np.linalg.norm(np.asarray(acc), axis=1)
    for k in range(idx.size):
        if gsum is not None and eta_grad > 0:
            g = np.linalg.norm(gsum[k]) / 24.0
            if g > 0:
                dt[k] = min(dt[k], eta_grad * np.cbrt(v[k] / g), eta_grad * np.sqrt(a[k] / g))
        if jrk is not None and eta_jerk > 0:
            jn = np.linalg.norm(jrk[k])
            if jn > 0:
                dt[k] = min(dt[k], eta_jerk * a[k] / jn)
    return dt


def levels_from_dt(dt, tau: float, kmax: int):
    """Level of the power-of-two hierarchy: the smallest k in [0, kmax] with dt >= tau / 2^k
    (a particle is slow on the level whose pivot its time-step reaches, Sec. 2.2)."""
    out = np.full(np.shape(dt), kmax, dtype=np.int32)
    for i, d in enumerate(np.asarray(dt)):
        for k in range(kmax + 1):
            if d >= tau / 2.0 ** k:
                out[i] = k
                break
    return out


def energy(p: Particles, subset=None, G: float = 1.0, eps2: float = 0.0):
    """(kinetic, potential) of a particle set (Sec. 2.1, the N-body Hamiltonian)."""
    _check(p)
    s = _idx(subset, p.n)
    kin, pot = ctypes.c_double(0.0), ctypes.c_double(0.0)
    row = np.zeros(max(s.size, 1))
    _load().oracle_energy(_ptr(p.x), _ptr(p.y), _ptr(p.z), _ptr(p.vx), _ptr(p.vy), _ptr(p.vz), _ptr(p.m),
                          s.size, _ptr(s), float(G), float(eps2), ctypes.byref(kin), ctypes.byref(pot),
                          _ptr(row))
    return kin.value, pot.value


# ---------------------------------------------------------------------------------------------
# Integrator steps (numpy, FP64), in the paper's notation.
# ---------------------------------------------------------------------------------------------

def _kick(p: Particles, idx: np.ndarray, a: np.ndarray, h: float):
    """v_i <- v_i + h a_i for i in idx (Sec. 2.1, Eq. kick-new with h = eps/6 etc.)."""
    p.vx[idx] += h * a[:, 0]
    p.vy[idx] += h * a[:, 1]
    p.vz[idx] += h * a[:, 2]


def _drift(p: Particles, idx: np.ndarray, h: float):
    """r_i <- r_i + h v_i for i in idx (Sec. 2.1, Eq. drift-new with h = eps/2)."""
    p.x[idx] += h * p.vx[idx]
    p.y[idx] += h * p.vy[idx]
    p.z[idx] += h * p.vz[idx]


def fsi_step(p: Particles, dt: float, subset=None, G: float = 1.0, eps2: float = 0.0,
             bh=None, c: float = 1e4, sub=None) -> Particles:
    """One FSI cycle over `subset` in place (Sec. 2.1, Eq. fsi-cycle):
    kick eps/6, drift eps/2, gradient kick 2eps/3, drift eps/2, kick eps/6.
    With `bh` given, the cycle is wrapped in two PN1.0 half-kicks evaluated at the
    current state (Sec. 3.8, the e^{eps/2 U_PN} e^{eps H_FSI} e^{eps/2 U_PN} composition).
    With `sub` (subsystem labels) the accelerations and gradient sums leave out intra-subsystem
    pairs (Alg. 1); every particle still drifts (the subsystems' own integration, which would
    replace their drift, is outside this oracle)."""
    idx = _idx(subset, p.n)
    if bh is not None and len(bh):
        _kick(p, idx, pn1(p, bh, idx, idx, G, c), dt / 2)
    a = forces(p, idx, idx, G, eps2, sub=sub)
    _kick(p, idx, a, dt / 6)
    _drift(p, idx, dt / 2)
    a = forces(p, idx, idx, G, eps2, sub=sub)
    full = np.zeros((p.n, 3))
    full[idx] = a
    g = gradient(p, full, idx, idx, G, eps2, sub=sub)
    _kick(p, idx, a + (dt * dt / 24.0) * g, 2.0 * dt / 3.0)
    _drift(p, idx, dt / 2)
    a = forces(p, idx, idx, G, eps2, sub=sub)
    _kick(p, idx, a, dt / 6)
    if bh is not None and len(bh):
        _kick(p, idx, pn1(p, bh, idx, idx, G, c), dt / 2)
    return p


def _interlevel_acc(p: Particles, S: np.ndarray, F: np.ndarray, G: float, eps2: float):
    """Inter-level accelerations (Sec. 2.2): slow particles feel the fast set and
    fast particles feel the slow set.  Returns a particle-indexed (n, 3) array that
    is zero outside S and F."""
    full = np.zeros((p.n, 3))
    full[S] = forces(p, S, F, G, eps2)
    full[F] = forces(p, F, S, G, eps2)
    return full


def _interlevel_pn(p: Particles, S: np.ndarray, F: np.ndarray, bh, G: float, c: float):
    """PN1.0 accelerations over inter-level pairs with a flagged particle: slow targets from
    fast sources and fast targets from slow sources (particle-indexed, zero elsewhere)."""
    full = np.zeros((p.n, 3))
    full[S] = pn1(p, bh, S, F, G, c)
    full[F] = pn1(p, bh, F, S, G, c)
    return full


def hhs_interval(p: Particles, levels: np.ndarray, tau: float, subset=None, level: int = 0,
                 G: float = 1.0, eps2: float = 0.0, bh=None, c: float = 1e4) -> Particles:
    """One HHS-FSI interval of length tau over `subset`, with per-particle levels given
    (Sec. 2.2, Eq. hhsfsi-cycle).  Slow set S = particles at `level`, fast set F =
    particles at deeper levels.  Readings for cases the paper leaves open: with F
    empty the slow set takes one plain FSI cycle; with S empty the fast set takes two
    half intervals at the next level.  With `bh` given (PN1.0 for pairs with a flagged
    particle, Sec. 3.8), every plain FSI cycle is wrapped in PN half-kicks over its own pairs
    and every level's cycle in PN half-kicks over its inter-level pairs (a reading: the paper
    does not place the PN terms in the hierarchy)."""
    idx = _idx(subset, p.n)
    lv = np.asarray(levels)[idx]
    S = idx[lv == level]
    F = idx[lv > level]
    pn = bh is not None and len(bh) > 0
    sub = dict(G=G, eps2=eps2, bh=bh, c=c)
    if F.size == 0:
        if S.size:
            fsi_step(p, tau, S, G, eps2, bh=bh, c=c)
        return p
    if S.size == 0:
        hhs_interval(p, levels, tau / 2, F, level + 1, **sub)
        hhs_interval(p, levels, tau / 2, F, level + 1, **sub)
        return p
    both = np.concatenate([S, F])
    if pn:
        _kick(p, both, _interlevel_pn(p, S, F, bh, G, c)[both], tau / 2)
    a = _interlevel_acc(p, S, F, G, eps2)
    _kick(p, both, a[both], tau / 6)
    fsi_step(p, tau / 2, S, G, eps2, bh=bh, c=c)
    hhs_interval(p, levels, tau / 2, F, level + 1, **sub)
    a = _interlevel_acc(p, S, F, G, eps2)
    g = np.zeros((p.n, 3))
    g[S] = gradient(p, a, S, F, G, eps2)
    g[F] = gradient(p, a, F, S, G, eps2)
    _kick(p, both, a[both] + (tau * tau / 24.0) * g[both], 2.0 * tau / 3.0)
    hhs_interval(p, levels, tau / 2, F, level + 1, **sub)
    fsi_step(p, tau / 2, S, G, eps2, bh=bh, c=c)
    a = _interlevel_acc(p, S, F, G, eps2)
    _kick(p, both, a[both], tau / 6)
    if pn:
        _kick(p, both, _interlevel_pn(p, S, F, bh, G, c)[both], tau / 2)
    return p


def level_timesteps(p: Particles, idx, G: float = 1.0, eps2: float = 0.0, eta_ff: float = 0.2,
                    eta_fb: float = 0.2, eta_grad: float = 0.1, eta_jerk: float = 0.1):
    """Time-steps of the particles `idx` from the particles of `idx` alone, as a level of the
    hierarchy assigns them (Sec. 2.2): the pairwise free-fall and fly-by criteria (Sec. 3.5.3)
    and the per-particle gradient (Sec. 3.5.4, Eqs. dt-nabla1, dt-nabla2) and jerk (Sec. 3.5.5)
    criteria, with the acceleration, its gradient sum and the jerk all summed over the level's
    particles (softened with eps2; the pairwise criteria are unsoftened).  A criterion with
    eta <= 0 is left out.  Returns one time-step per entry of idx."""
    idx = np.asarray(idx)
    ff, fb = dt_min(p, idx, idx, G, max(eta_ff, 0.0), max(eta_fb, 0.0))
    if eta_ff <= 0:
        ff = np.full(idx.size, np.inf)
    if eta_fb <= 0:
        fb = np.full(idx.size, np.inf)
    a = forces(p, idx, idx, G, eps2)
    full = np.zeros((p.n, 3))
    full[idx] = a
    gs = gradient(p, full, idx, idx, G, eps2) if eta_grad > 0 else None
    jr = jerk(p, idx, idx, G, eps2) if eta_jerk > 0 else None
    return timestep_criteria(p, idx, ff, fb, a, gs, jr, eta_grad, eta_jerk)


def hhs_interval_adaptive(p: Particles, dt0: np.ndarray, tau: float, kmax: int, eta_ff: float = 0.2,
                          eta_fb: float = 0.2, eta_grad: float = 0.1, eta_jerk: float = 0.1,
                          subset=None, level: int = 0, G: float = 1.0, eps2: float = 0.0,
                          trace=None) -> Particles:
    """One HHS-FSI interval of length tau over `subset` in which every hierarchy level begins by
    assigning time-steps to its particles and dividing them into slow (dt >= pivot) and fast
    (dt < pivot) sets (Sec. 2.2).  `dt0` (particle-indexed) holds the time-steps assigned at the
    start of the interval from all particles; they are level 0's.  On a deeper level every
    criterion is evaluated again over the particles of that level alone (`level_timesteps`:
    free-fall, fly-by, both gradient criteria and the jerk criterion) and the result is capped
    by dt0, so that a time-step cannot grow within the interval (Sec. 3.5.1, the level-0
    minimum).  Particles on level kmax are all slow.  `trace`, if a list, receives (level,
    pivot, slow count, fast count, smallest distance of a time-step to the pivot relative to
    the pivot, slow particles, fast particles) per visited level, in visiting order."""
    idx = _idx(subset, p.n)
    if level == 0:
        dt = np.asarray(dt0, float)[idx]
    else:
        dt = level_timesteps(p, idx, G, eps2, eta_ff, eta_fb, eta_grad, eta_jerk)
        dt = np.minimum(dt, np.asarray(dt0, float)[idx])
    if level >= kmax:
        slow = np.ones(idx.size, dtype=bool)
    else:
        slow = dt >= tau
    S, F = idx[slow], idx[~slow]
    if trace is not None:
        gap = float(np.min(np.abs(dt / tau - 1.0))) if idx.size else np.inf
        trace.append((level, tau, S.size, F.size, gap, S.copy(), F.copy()))
    sub = dict(eta_ff=eta_ff, eta_fb=eta_fb, eta_grad=eta_grad, eta_jerk=eta_jerk, G=G, eps2=eps2,
               trace=trace)
    if F.size == 0:
        if S.size:
            fsi_step(p, tau, S, G, eps2)
        return p
    if S.size == 0:
        hhs_interval_adaptive(p, dt0, tau / 2, kmax, subset=F, level=level + 1, **sub)
        hhs_interval_adaptive(p, dt0, tau / 2, kmax, subset=F, level=level + 1, **sub)
        return p
    both = np.concatenate([S, F])
    a = _interlevel_acc(p, S, F, G, eps2)
    _kick(p, both, a[both], tau / 6)
    fsi_step(p, tau / 2, S, G, eps2)
    hhs_interval_adaptive(p, dt0, tau / 2, kmax, subset=F, level=level + 1, **sub)
    a = _interlevel_acc(p, S, F, G, eps2)
    g = np.zeros((p.n, 3))
    g[S] = gradient(p, a, S, F, G, eps2)
    g[F] = gradient(p, a, F, S, G, eps2)
    _kick(p, both, a[both] + (tau * tau / 24.0) * g[both], 2.0 * tau / 3.0)
    hhs_interval_adaptive(p, dt0, tau / 2, kmax, subset=F, level=level + 1, **sub)
    fsi_step(p, tau / 2, S, G, eps2)
    a = _interlevel_acc(p, S, F, G, eps2)
    _kick(p, both, a[both], tau / 6)
    return p


# ---------------------------------------------------------------------------------------------
# Subsystems (Sec. 3.3): neighbour search and connected components.
# ---------------------------------------------------------------------------------------------

def neighbours(p: Particles, targets=None, sources=None, G: float = 1.0, r_ngb: float = 1e-3,
               r_max: float = 0.1, C: float = 0.5, tau: float = 1e-3) -> np.ndarray:
    """Neighbour pairs (Sec. 3.3, Eqs. ngb-bound, ngb-unbound): an (m, 2) int64 array of
    (target particle, source particle) rows, sorted, for every pair closer than r_max that
    meets the bound or unbound criterion."""
    _check(p)
    t, s = _idx(targets, p.n), _idx(sources, p.n)
    out = np.zeros(t.size * s.size, dtype=np.uint8)
    _load().oracle_neighbours(_ptr(p.x), _ptr(p.y), _ptr(p.z), _ptr(p.vx), _ptr(p.vy), _ptr(p.vz), _ptr(p.m),
                              t.size, _ptr(t), s.size, _ptr(s), float(G), float(r_ngb), float(r_max), float(C),
                              float(tau), out.ctypes.data_as(ctypes.c_void_p))
    k, q = np.nonzero(out.reshape(t.size, s.size))
    e = np.stack([t[k], s[q]], axis=1)
    return e[np.lexsort((e[:, 1], e[:, 0]))] if e.size else e.reshape(0, 2)


def subsystems(n: int, edges: np.ndarray) -> np.ndarray:
    """Subsystem label of every particle: the components of the neighbour graph, found by
    depth-first search from each particle not yet visited (Sec. 3.3).  A component's label is
    its smallest particle index, so a particle without neighbours is labelled by itself."""
    adj = [[] for _ in range(n)]
    for i, j in np.asarray(edges, dtype=np.int64):
        adj[i].append(j)
        adj[j].append(i)
    label = np.full(n, -1, dtype=np.int64)
    for start in range(n):
        if label[start] >= 0:
            continue
        comp, stack = [], [start]
        label[start] = start
        while stack:
            v = stack.pop()
            comp.append(v)
            for w in adj[v]:
                if label[w] < 0:
                    label[w] = start
                    stack.append(w)
        label[comp] = min(comp)
    return label
