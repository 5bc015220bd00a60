"""Two-body (Kepler) closed form used to pin the integrator oracle.

Elliptic orbits only.  Kepler's equation M = E - e sin E (the form the paper
solves for its secular binaries and Kepler solver, Secs. 3.10-3.11) is solved by Newton iteration started
at E = M + e sin M and safeguarded by bisection on [M - e, M + e].  Nothing here
uses the force routines: the state at any time follows from the orbital
elements of the initial relative state.
"""
import math

import numpy as np


def solve_kepler(M: float, e: float, tol: float = 1e-15) -> float:
    M = math.fmod(M, 2 * math.pi)
    lo, hi = M - e - 1e-12, M + e + 1e-12  # E - M = e sin E lies in [-e, e]
    E = M + e * math.sin(M)
    for _ in range(100):
        f = E - e * math.sin(E) - M
        if f > 0:
            hi = min(hi, E)
        else:
            lo = max(lo, E)
        fp = 1.0 - e * math.cos(E)
        En = E - f / fp
        if not (lo <= En <= hi):
            En = 0.5 * (lo + hi)
        if abs(En - E) < tol:
            return En
        E = En
    return E


def elements(r0, v0, GM):
    """(a, e, P-hat, Q-hat, E0) of the relative orbit."""
    r0 = np.asarray(r0, float)
    v0 = np.asarray(v0, float)
    r = np.linalg.norm(r0)
    v2 = v0 @ v0
    a = 1.0 / (2.0 / r - v2 / GM)
    h = np.cross(r0, v0)
    evec = np.cross(v0, h) / GM - r0 / r
    e = np.linalg.norm(evec)
    P = evec / e
    Q = np.cross(h / np.linalg.norm(h), P)
    cosE = (1.0 - r / a) / e
    sinE = (r0 @ v0) / (e * math.sqrt(GM * a))
    E0 = math.atan2(sinE, cosE)
    return a, e, P, Q, E0


def propagate(r0, v0, GM, t):
    """Relative position and velocity after time t on the Kepler orbit through (r0, v0)."""
    a, e, P, Q, E0 = elements(r0, v0, GM)
    n = math.sqrt(GM / a ** 3)
    M = E0 - e * math.sin(E0) + n * t
    E = solve_kepler(M, e)
    b = a * math.sqrt(1 - e * e)
    pos = a * (math.cos(E) - e) * P + b * math.sin(E) * Q
    rr = a * (1 - e * math.cos(E))
    vel = (math.sqrt(GM * a) / rr) * (-math.sin(E) * P + math.sqrt(1 - e * e) * math.cos(E) * Q)
    return pos, vel


def binary_state(m1, m2, a, e, G=1.0, phase_E=0.0):
    """Particle dict of a bound binary in its centre-of-mass frame with the given elements,
    started at eccentric anomaly phase_E, orbit in the x-y plane tilted about x by 0.3 rad."""
    M = m1 + m2
    GM = G * M
    b = a * math.sqrt(1 - e * e)
    E = phase_E
    rel = np.array([a * (math.cos(E) - e), b * math.sin(E), 0.0])
    rr = a * (1 - e * math.cos(E))
    vrel = (math.sqrt(GM * a) / rr) * np.array([-math.sin(E), math.sqrt(1 - e * e) * math.cos(E), 0.0])
    c, s = math.cos(0.3), math.sin(0.3)
    R = np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    rel, vrel = R @ rel, R @ vrel
    x1, x2 = -m2 / M * rel, m1 / M * rel
    v1, v2 = -m2 / M * vrel, m1 / M * vrel
    return {"x": np.array([x1[0], x2[0]]), "y": np.array([x1[1], x2[1]]), "z": np.array([x1[2], x2[2]]),
            "vx": np.array([v1[0], v2[0]]), "vy": np.array([v1[1], v2[1]]), "vz": np.array([v1[2], v2[2]]),
            "m": np.array([m1, m2], dtype=float)}
