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
