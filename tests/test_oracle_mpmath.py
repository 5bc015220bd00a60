"""The FP64 oracle against 50-digit brute force (mpmath) on small sets.

The sums are evaluated in 50-digit arithmetic from the definitions of the pair terms
(Sec. 2.1, Eqs. new-newton-acc and new-grad-acc; Sec. 3.5.3, Eqs. dt-freefall and dt-flyby;
Sec. 3.5.5, the jerk; the N-body Hamiltonian of Sec. 2.1; the harmonic-gauge two-body PN1.0
acceleration used for Sec. 3.8) on the FP64 inputs the oracle receives, and the oracle's
FP64 results must agree to a few units of FP64 rounding of the summed magnitudes.  This
checks the C loops' indexing, signs and accumulation, not the formulas themselves (those are
pinned by closed forms and invariants in test_oracle_pins.py)."""
import numpy as np
import pytest

import oracle
from oracle import Particles

mpmath = pytest.importorskip("mpmath")
mp = mpmath.mp


def _cluster(n, seed):
    rng = np.random.default_rng(seed)
    d = {"x": rng.normal(0, 1, n), "y": rng.normal(0, 1, n), "z": rng.normal(0, 1, n),
         "vx": rng.normal(0, 0.5, n), "vy": rng.normal(0, 0.5, n), "vz": rng.normal(0, 0.5, n),
         "m": rng.uniform(0.2, 3.0, n) / n}
    return Particles.from_dict(d)


def _mp_state(P):
    f = mpmath.mpf
    pos = [[f(float(P.x[i])), f(float(P.y[i])), f(float(P.z[i]))] for i in range(P.n)]
    vel = [[f(float(P.vx[i])), f(float(P.vy[i])), f(float(P.vz[i]))] for i in range(P.n)]
    m = [f(float(v)) for v in P.m]
    return pos, vel, m


def _sub(a, b):
    return [a[0] - b[0], a[1] - b[1], a[2] - b[2]]


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _close(got, ref, scale, tol):
    for c in range(3):
        assert abs(mpmath.mpf(float(got[c])) - ref[c]) <= tol * scale, (c, float(got[c]), float(ref[c]), float(scale))


@pytest.mark.parametrize("eps2", [0.0, 1e-2])
def test_forces_gradient_jerk_against_50_digits(eps2):
    mp.dps = 50
    P = _cluster(32, 11)
    pos, vel, m = _mp_state(P)
    G, e2 = mpmath.mpf(1), mpmath.mpf(eps2)
    a_or, mag = oracle.forces(P, eps2=eps2, return_mag=True)[:2]
    # gradient on FP64 accelerations that differ from the true ones (any a enters linearly)
    a_in = a_or * (1 + 0.1 * np.random.default_rng(3).standard_normal(a_or.shape))
    g_or, gmag = oracle.gradient(P, a_in, eps2=eps2, return_mag=True)[:2]
    j_or = oracle.jerk(P, eps2=eps2)
    a_mp_in = [[mpmath.mpf(float(a_in[i, c])) for c in range(3)] for i in range(P.n)]
    for i in range(P.n):
        acc, grd, jrk = [mpmath.mpf(0)] * 3, [mpmath.mpf(0)] * 3, [mpmath.mpf(0)] * 3
        jmag = mpmath.mpf(0)
        for j in range(P.n):
            if j == i:
                continue
            r = _sub(pos[j], pos[i])
            s2 = _dot(r, r) + e2
            s = mpmath.sqrt(s2)
            w3 = G * m[j] / (s2 * s)
            acc = [acc[c] + w3 * r[c] for c in range(3)]
            da = _sub(a_mp_in[j], a_mp_in[i])
            dv = _sub(vel[j], vel[i])
            w5 = w3 / s2
            ar, vr = _dot(da, r), _dot(dv, r)
            grd = [grd[c] + w5 * (s2 * da[c] - 3 * ar * r[c]) for c in range(3)]
            tj = [w5 * (s2 * dv[c] - 3 * vr * r[c]) for c in range(3)]
            jrk = [jrk[c] + tj[c] for c in range(3)]
            jmag += mpmath.sqrt(_dot(tj, tj))
        _close(a_or[i], acc, mpmath.mpf(float(mag[i])), 1e-14)
        _close(g_or[i], grd, mpmath.mpf(float(gmag[i])), 1e-14)
        _close(j_or[i], jrk, jmag, 1e-14)


def test_dt_min_against_50_digits():
    """eta_ff and eta_fb different from 1 and from each other, so their scaling is checked."""
    mp.dps = 50
    P = _cluster(29, 12)
    P.vx[5], P.vy[5], P.vz[5] = P.vx[9], P.vy[9], P.vz[9]  # one pair with v_ij = 0
    pos, vel, m = _mp_state(P)
    eff, efb = 0.23, 0.061
    ff, fb = oracle.dt_min(P, eta_ff=eff, eta_fb=efb)
    for i in range(P.n):
        tff, tfb = mpmath.inf, mpmath.inf
        for j in range(P.n):
            if j == i:
                continue
            r = mpmath.sqrt(_dot(_sub(pos[j], pos[i]), _sub(pos[j], pos[i])))
            u = mpmath.sqrt(_dot(_sub(vel[j], vel[i]), _sub(vel[j], vel[i])))
            tff = min(tff, mpmath.sqrt(r ** 3 / (m[i] + m[j])))
            if u > 0:
                tfb = min(tfb, r / u)
        assert abs(ff[i] / float(mpmath.mpf(eff) * tff) - 1) < 1e-14
        assert abs(fb[i] / float(mpmath.mpf(efb) * tfb) - 1) < 1e-14


def test_pn1_against_50_digits():
    """Two flagged particles among 24: pairs with a flagged member only."""
    mp.dps = 50
    P = _cluster(24, 13)
    P.m[[3, 17]] *= 40.0
    bh = [3, 17]
    c = 30.0
    pos, vel, m = _mp_state(P)
    got = oracle.pn1(P, bh, G=1.0, c=c)
    cc = mpmath.mpf(c) ** 2
    for i in range(P.n):
        tot, scale = [mpmath.mpf(0)] * 3, mpmath.mpf(0)
        for j in range(P.n):
            if j == i or not (i in bh or j in bh):
                continue
            d = _sub(pos[i], pos[j])
            r = mpmath.sqrt(_dot(d, d))
            nvec = [d[k] / r for k in range(3)]
            vi, vj = vel[i], vel[j]
            radial = (5 * m[i] + 4 * m[j]) / r + mpmath.mpf(3) / 2 * _dot(nvec, vj) ** 2 - _dot(vi, vi) \
                + 4 * _dot(vi, vj) - 2 * _dot(vj, vj)
            along = 4 * _dot(nvec, vi) - 3 * _dot(nvec, vj)
            pre = m[j] / (cc * r * r)
            t = [pre * (radial * nvec[k] + along * (vi[k] - vj[k])) for k in range(3)]
            tot = [tot[k] + t[k] for k in range(3)]
            scale += mpmath.sqrt(_dot(t, t))
        if scale == 0:
            assert np.all(got[i] == 0)
        else:
            _close(got[i], tot, scale, 1e-13)


@pytest.mark.parametrize("eps2", [0.0, 1e-2])
def test_energy_against_50_digits(eps2):
    mp.dps = 50
    P = _cluster(32, 14)
    pos, vel, m = _mp_state(P)
    kin, pot = oracle.energy(P, eps2=eps2)
    T = sum(m[i] * _dot(vel[i], vel[i]) / 2 for i in range(P.n))
    U, Umag = mpmath.mpf(0), mpmath.mpf(0)
    for i in range(P.n):
        for j in range(i + 1, P.n):
            d = _sub(pos[j], pos[i])
            u = m[i] * m[j] / mpmath.sqrt(_dot(d, d) + mpmath.mpf(eps2))
            U -= u
            Umag += u
    assert abs(mpmath.mpf(kin) - T) <= 1e-15 * T
    assert abs(mpmath.mpf(pot) - U) <= 1e-15 * Umag
