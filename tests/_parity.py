"""Shared helpers of the GPU parity tests: moving seeded inputs to the device and error metrics."""
import numpy as np

import oracle


def rel_errors(gpu: np.ndarray, ref: np.ndarray):
    """Per-target relative error of a vector result: |y_gpu - y_ref| / |y_ref| (2-norms)."""
    d = np.linalg.norm(gpu - ref, axis=1)
    r = np.linalg.norm(ref, axis=1)
    return d / np.where(r > 0, r, 1.0)


def stats(err: np.ndarray):
    return float(np.sqrt(np.mean(err ** 2))), float(err.max())


def gather(ts, idx):
    """Stack particle-indexed torch outputs (k tensors) into an (len(idx), k) numpy array."""
    return np.stack([t.cpu().numpy()[idx] for t in ts], axis=1)


def oracle_particles(d):
    return oracle.Particles.from_dict(d)


def smooth_acc_field(d):
    """A smooth input acceleration field for gradient parity at sizes where the oracle cannot
    produce every particle's acceleration in test time (any field is a valid input: the
    gradient pass contracts the tidal tensor with whatever accelerations it is given)."""
    x, y, z = d["x"], d["y"], d["z"]
    s = (x * x + y * y + z * z + 0.1) ** -1.5
    return np.stack([-x * s, -y * s, -z * s], axis=1)


def assert_state_close(got, ref, ref0, tol: float, floor: float = 1e-3):
    """Mixed-precision state check, per particle: the position and the velocity vectors of every
    particle lie within tol x (the particle's own change |ref - ref0| + floor x the largest
    change) of the oracle's.  got, ref, ref0: objects with x, y, z, vx, vy, vz (numpy arrays or
    device tensors for got)."""
    def arr(o, k):
        v = getattr(o, k)
        return v.cpu().numpy() if hasattr(v, "cpu") else np.asarray(v)
    for group in (("x", "y", "z"), ("vx", "vy", "vz")):
        g = np.stack([arr(got, k) for k in group], axis=1)
        r = np.stack([arr(ref, k) for k in group], axis=1)
        r0 = np.stack([arr(ref0, k) for k in group], axis=1)
        change = np.linalg.norm(r - r0, axis=1)
        bound = tol * (change + floor * change.max())
        err = np.linalg.norm(g - r, axis=1)
        worst = int(np.argmax(err / bound))
        assert np.all(err <= bound), (group[0], worst, float(err[worst]), float(change[worst]))
