"""ctypes binding of libbifrost_hip.so (the C ABI declared in include/bifrost.h).

Argument marshalling only: tensors are passed as device pointers, torch supplies device
memory and the current stream, and every numerical step runs in the library's kernels.
There is no fallback: if the library or a GPU is missing the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbifrost_hip.so")

BF_OK = 0
BF_PREC_FP64 = 0
BF_PREC_MIXED = 1
BF_FLAG_NONFINITE = 0x1
BF_FLAG_COINCIDENT = 0x2
BF_FLAG_BADINDEX = 0x4
BF_A_VALID = 0x1
BF_ERR_NOMEM = -5
BF_SORT_ANY_SIZE = 0x100
BF_SORT_DIRECTED = 0x200
BF_OP_FORCES, BF_OP_GRADIENT, BF_OP_DTMIN = 0, 1, 2

PRECISIONS = {"fp64": BF_PREC_FP64, "mixed": BF_PREC_MIXED}

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_d = ctypes.c_double
_int = ctypes.c_int


class _Particles(ctypes.Structure):
    _fields_ = [("x", _vp), ("y", _vp), ("z", _vp), ("vx", _vp), ("vy", _vp), ("vz", _vp), ("m", _vp), ("n", _i64)]


class _State(ctypes.Structure):
    _fields_ = [("x", _vp), ("y", _vp), ("z", _vp), ("vx", _vp), ("vy", _vp), ("vz", _vp), ("m", _vp), ("n", _i64)]


class _Set(ctypes.Structure):
    _fields_ = [("idx", _vp), ("count", _i32), ("begin", _i32)]


class _FsiParams(ctypes.Structure):
    _fields_ = [("G", _d), ("eps2", _d), ("prec", _int), ("r_fb", _d), ("bh_idx", _vp), ("n_bh", _i32), ("c", _d)]


class BifrostError(RuntimeError):
    def __init__(self, func: str, code: int, msg: str):
        super().__init__(f"{func} failed with status {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libbifrost_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python paper_2210_02472_amd/build.py`")
    lib = ctypes.CDLL(path)
    P, S, ST, FP = ctypes.POINTER(_Particles), ctypes.POINTER(_Set), ctypes.POINTER(_State), ctypes.POINTER(_FsiParams)
    sig = {
        "bf_create": [ctypes.POINTER(_vp), _int, _vp],
        "bf_destroy": [_vp],
        "bf_set_stream": [_vp, _vp],
        "bf_read_flags": [_vp, ctypes.POINTER(ctypes.c_uint32), _int],
        "bf_validate_set": [_vp, S, _i64],
        "bf_forces": [_vp, P, S, S, _d, _d, _int, _d, _vp, _vp, _vp],
        "bf_forces_noalloc": [_vp, P, S, S, _d, _d, _int, _d, _vp, _vp, _vp],
        "bf_force_gradient": [_vp, P, S, S, _vp, _vp, _vp, _d, _d, _int, _d, _vp, _vp, _vp],
        "bf_dt_min": [_vp, P, S, S, _d, _d, _d, _int, _d, _vp, _vp],
        "bf_pn1_bh": [_vp, P, S, S, _vp, _i32, _d, _d, _vp, _vp, _vp],
        "bf_energy": [_vp, P, S, _d, _d, ctypes.POINTER(_d), ctypes.POINTER(_d)],
        "bf_fsi_step": [_vp, ST, S, _d, FP, _vp, _vp, _vp, _int],
        "bf_kick": [_vp, ST, S, _d, _vp, _vp, _vp, _d, _vp, _vp, _vp],
        "bf_jerk": [_vp, P, S, S, _d, _d, _int, _vp, _vp, _vp],
        "bf_timestep_assign": [_vp, P, S, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _d, _d, _d, _int,
                               _vp, _vp],
        "bf_level_partition": [_vp, S, _i64, _vp, _int, _vp, ctypes.POINTER(_i64)],
        "bf_hhs_interval": [_vp, ST, S, _vp, _int, _d, FP],
        "bf_graph_capture_hhs_interval": [_vp, ST, S, _vp, _int, _d, FP, ctypes.POINTER(_vp)],
        "bf_hhs_interval_adaptive": [_vp, ST, S, _vp, _int, _d, _d, _d, _d, _d, FP, ctypes.POINTER(_int),
                                     ctypes.POINTER(_i64)],
        "bf_drift": [_vp, ST, S, _d],
        "bf_forces_batched": [_vp, P, _i32, _vp, _vp, _vp, _i64, _i64, _d, _d, _int, _d, _vp, _vp, _vp],
        "bf_force_gradient_batched": [_vp, P, _i32, _vp, _vp, _vp, _i64, _i64, _vp, _vp, _vp, _d, _d, _int, _d,
                                      _vp, _vp, _vp],
        "bf_fsi_step_batched": [_vp, ST, _i32, _vp, _vp, _vp, _i64, _i64, _d, _d, _int, _d, _d, _vp, _vp, _vp],
        "bf_graph_capture_batched_fsi": [_vp, ST, _i32, _vp, _vp, _vp, _i64, _i64, _d, _d, _int, _d, _d, _vp, _vp,
                                         _vp, ctypes.POINTER(_vp)],
        "bf_graph_launch": [_vp, _vp],
        "bf_graph_destroy": [_vp],
        "bf_autotune": [_vp, _int, _int, _i64, _i64, ctypes.c_char_p],
        "bf_autotune_load": [_vp, ctypes.c_char_p],
        "bf_query_config": [_vp, _int, _int, _i64, _i64, ctypes.POINTER(_int), ctypes.POINTER(_int),
                            ctypes.POINTER(_int)],
        "bf_set_config": [_vp, _int, _int, _int, _int, _int],
        "bf_enable_timing": [_vp, _int],
        "bf_set_spatial_sort": [_vp, _int, ctypes.c_double],
        "bf_pair_credit": [_vp, _int, ctypes.POINTER(_i64), _int],
        "bf_autotune_pass": [_vp, _int, _int, P, S, S, _vp, _vp, _vp, ctypes.c_char_p],
        "bf_autotune_batched": [_vp, _int, _int, P, _i32, _vp, _vp, _vp, _i64, _i64, _vp, _vp, _vp, ctypes.c_char_p],
        "bf_set_symmetric_config": [_vp, _int, _int, _int, _int],
        "bf_set_symmetric_scratch_limit": [_vp, ctypes.c_size_t],
        "bf_last_symmetric_passes": [_vp, ctypes.POINTER(_int)],
        "bf_query_batched_config": [_vp, _int, _int, _i64, _i64, ctypes.POINTER(_int), ctypes.POINTER(_int),
                                    ctypes.POINTER(_int)],
        "bf_set_batched_config": [_vp, _int, _int, _int, _int, _int],
        "bf_set_hhs_reuse": [_vp, _int],
        "bf_neighbours": [_vp, P, S, S, _d, _d, _d, _d, _d, _vp, _i64, ctypes.POINTER(_i64)],
        "bf_subsystems": [_vp, _i64, _vp, _i64, _vp, ctypes.POINTER(_i64)],
        "bf_set_subsystems": [_vp, _vp, _i64],
        "bf_last_pass_stats": [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)],
        "bf_forces_between": [_vp, P, S, S, _d, _d, _int, _d, _vp, _vp, _vp],
        "bf_force_gradient_between": [_vp, P, S, S, _vp, _vp, _vp, _d, _d, _int, _d, _vp, _vp, _vp],
        "bf_release_scratch": [_vp, ctypes.POINTER(ctypes.c_size_t)],
        "bf_last_pass_config": [_vp, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_int),
                                ctypes.POINTER(_int)],
        "bf_kernel_times": [_vp, _int, ctypes.POINTER(ctypes.c_float), _int, ctypes.POINTER(_int)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = _int
    lib.bf_status_string.argtypes = [_int]
    lib.bf_status_string.restype = ctypes.c_char_p
    lib.bf_last_error.argtypes = []
    lib.bf_last_error.restype = ctypes.c_char_p
    lib.bf_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(name: str, rc: int):
    if rc != BF_OK:
        msg = _lib.bf_last_error().decode() or _lib.bf_status_string(rc).decode()
        raise BifrostError(name, rc, msg)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, dtype, n: Optional[int] = None, name: str = "tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements")
    return t


@dataclass
class ParticleSet:
    """A set of particles: an int32 device index list, or the range [begin, begin + count)."""
    idx: Optional[torch.Tensor] = None
    begin: int = 0
    count: int = 0

    @staticmethod
    def range(begin: int, count: int) -> "ParticleSet":
        return ParticleSet(None, int(begin), int(count))

    @staticmethod
    def of(sel, n: int, device=None) -> "ParticleSet":
        """None -> all n particles; a ParticleSet as is; a tensor/array/list -> index list."""
        if sel is None:
            return ParticleSet(None, 0, n)
        if isinstance(sel, ParticleSet):
            return sel
        t = sel if isinstance(sel, torch.Tensor) else torch.as_tensor(sel)
        t = t.to(device=device or "cuda", dtype=torch.int32).contiguous()
        return ParticleSet(t, 0, int(t.numel()))

    def _c(self) -> _Set:
        return _Set(_ptr(self.idx), int(self.count), int(self.begin))


class Particles:
    """FP64 structure-of-arrays particle state on the device (x, y, z, vx, vy, vz, m)."""
    KEYS = ("x", "y", "z", "vx", "vy", "vz", "m")

    def __init__(self, **arrays: torch.Tensor):
        n = int(arrays["m"].numel())
        for k in self.KEYS:
            setattr(self, k, _need(arrays[k], torch.float64, n, k))
        self.n = n

    @staticmethod
    def from_numpy(d: dict, device="cuda") -> "Particles":
        return Particles(**{k: torch.as_tensor(d[k], dtype=torch.float64, device=device).contiguous()
                            for k in Particles.KEYS})

    def to_numpy(self) -> dict:
        return {k: getattr(self, k).cpu().numpy() for k in self.KEYS}

    def _c(self) -> _Particles:
        return _Particles(*(_ptr(getattr(self, k)) for k in self.KEYS), self.n)

    def _state(self) -> _State:
        return _State(*(_ptr(getattr(self, k)) for k in self.KEYS), self.n)


class Context:
    """A bf_ctx bound to a device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None):
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU available for libbifrost_hip")
        self.device = device
        st = stream if stream is not None else torch.cuda.current_stream(device)
        self._stream = st
        h = _vp()
        _check("bf_create", lib.bf_create(ctypes.byref(h), device, _vp(st.cuda_stream)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.bf_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def set_stream(self, stream: torch.cuda.Stream):
        self._stream = stream
        _check("bf_set_stream", _lib.bf_set_stream(self._h, _vp(stream.cuda_stream)))

    def read_flags(self, clear: bool = True) -> int:
        f = ctypes.c_uint32(0)
        _check("bf_read_flags", _lib.bf_read_flags(self._h, ctypes.byref(f), int(clear)))
        return int(f.value)

    def validate_set(self, s: ParticleSet, n: int):
        _check("bf_validate_set", _lib.bf_validate_set(self._h, ctypes.byref(s._c()), int(n)))

    # ---- the pass ----------------------------------------------------------------------------

    def _outs(self, P: Particles, out, k: int):
        if out is None:
            return [torch.zeros(P.n, dtype=torch.float64, device=P.m.device) for _ in range(k)]
        for t in out:
            _need(t, torch.float64, P.n, "output")
        return list(out)

    def forces(self, P: Particles, targets=None, sources=None, G=1.0, eps2=0.0, prec="mixed", r_fb=0.0,
               out: Optional[Sequence[torch.Tensor]] = None):
        """Accelerations (particle-indexed ax, ay, az; only target entries written).  r_fb > 0 re-evaluates
        in FP64 the 64-source slices holding a pair closer than r_fb; the default 0 relies on the mixed
        path's FP64 pair differences alone (and allows the spatially sorted sweeps)."""
        t, s = ParticleSet.of(targets, P.n), ParticleSet.of(sources, P.n)
        o = self._outs(P, out, 3)
        _check("bf_forces", _lib.bf_forces(self._h, ctypes.byref(P._c()), ctypes.byref(t._c()), ctypes.byref(s._c()),
                                           float(G), float(eps2), PRECISIONS[prec], float(r_fb), *map(_ptr, o)))
        return o

    def forces_noalloc(self, P: Particles, targets=None, sources=None, G=1.0, eps2=0.0, prec="mixed", r_fb=0.0,
                       out: Optional[Sequence[torch.Tensor]] = None):
        """The accelerations of `forces` through bf_forces_noalloc: the library allocates nothing
        (its pass runs in a static 64 MiB device array).  Pass `out` to allocate nothing here either."""
        t, s = ParticleSet.of(targets, P.n), ParticleSet.of(sources, P.n)
        o = self._outs(P, out, 3)
        _check("bf_forces_noalloc", _lib.bf_forces_noalloc(
            self._h, ctypes.byref(P._c()), ctypes.byref(t._c()), ctypes.byref(s._c()), float(G), float(eps2),
            PRECISIONS[prec], float(r_fb), *map(_ptr, o)))
        return o

    def force_gradient(self, P: Particles, acc: Sequence[torch.Tensor], targets=None, sources=None, G=1.0, eps2=0.0,
                       prec="mixed", r_fb=0.0, out: Optional[Sequence[torch.Tensor]] = None):
        """Force-gradient sums Gsum (particle-indexed gx, gy, gz)."""
        t, s = ParticleSet.of(targets, P.n), ParticleSet.of(sources, P.n)
        for a in acc:
            _need(a, torch.float64, P.n, "acceleration")
        o = self._outs(P, out, 3)
        _check("bf_force_gradient", _lib.bf_force_gradient(
            self._h, ctypes.byref(P._c()), ctypes.byref(t._c()), ctypes.byref(s._c()), *map(_ptr, acc), float(G),
            float(eps2), PRECISIONS[prec], float(r_fb), *map(_ptr, o)))
        return o

    def forces_between(self, P: Particles, a, b, G=1.0, eps2=0.0, prec="mixed", r_fb=0.0,
                       out: Optional[Sequence[torch.Tensor]] = None):
        """Accelerations of a's particles due to b and of b's due to a (disjoint sets), one output."""
        sa, sb = ParticleSet.of(a, P.n), ParticleSet.of(b, P.n)
        o = self._outs(P, out, 3)
        _check("bf_forces_between", _lib.bf_forces_between(self._h, ctypes.byref(P._c()), ctypes.byref(sa._c()),
                                                           ctypes.byref(sb._c()), float(G), float(eps2),
                                                           PRECISIONS[prec], float(r_fb), *map(_ptr, o)))
        return o

    def force_gradient_between(self, P: Particles, acc: Sequence[torch.Tensor], a, b, G=1.0, eps2=0.0, prec="mixed",
                               r_fb=0.0, out: Optional[Sequence[torch.Tensor]] = None):
        """Force-gradient sums of a's particles over b and of b's over a (disjoint sets)."""
        sa, sb = ParticleSet.of(a, P.n), ParticleSet.of(b, P.n)
        for x in acc:
            _need(x, torch.float64, P.n, "acceleration")
        o = self._outs(P, out, 3)
        _check("bf_force_gradient_between", _lib.bf_force_gradient_between(
            self._h, ctypes.byref(P._c()), ctypes.byref(sa._c()), ctypes.byref(sb._c()), *map(_ptr, acc), float(G),
            float(eps2), PRECISIONS[prec], float(r_fb), *map(_ptr, o)))
        return o

    def dt_min(self, P: Particles, targets=None, sources=None, G=1.0, eta_ff=0.2, eta_fb=0.2, prec="mixed", r_fb=0.0,
               out: Optional[Sequence[torch.Tensor]] = None):
        """Free-fall and fly-by time-steps (particle-indexed dt_ff, dt_fb); r_fb > 0 re-evaluates
        the tiles with a pair closer than r_fb in FP64 (mixed)."""
        t, s = ParticleSet.of(targets, P.n), ParticleSet.of(sources, P.n)
        o = self._outs(P, out, 2)
        _check("bf_dt_min", _lib.bf_dt_min(self._h, ctypes.byref(P._c()), ctypes.byref(t._c()), ctypes.byref(s._c()),
                                           float(G), float(eta_ff), float(eta_fb), PRECISIONS[prec], float(r_fb),
                                           *map(_ptr, o)))
        return o

    def pn1_bh(self, P: Particles, bh, targets=None, sources=None, G=1.0, c=1e4,
               out: Optional[Sequence[torch.Tensor]] = None):
        """PN1.0 accelerations over pairs that involve a listed black hole."""
        t, s = ParticleSet.of(targets, P.n), ParticleSet.of(sources, P.n)
        b = ParticleSet.of(bh, P.n)
        o = self._outs(P, out, 3)
        _check("bf_pn1_bh", _lib.bf_pn1_bh(self._h, ctypes.byref(P._c()), ctypes.byref(t._c()), ctypes.byref(s._c()),
                                           _ptr(b.idx), int(b.count), float(G), float(c), *map(_ptr, o)))
        return o

    def energy(self, P: Particles, subset=None, G=1.0, eps2=0.0):
        s = ParticleSet.of(subset, P.n)
        k, u = _d(0.0), _d(0.0)
        _check("bf_energy", _lib.bf_energy(self._h, ctypes.byref(P._c()), ctypes.byref(s._c()), float(G), float(eps2),
                                           ctypes.byref(k), ctypes.byref(u)))
        return k.value, u.value

    def fsi_step(self, P: Particles, dt: float, subset=None, G=1.0, eps2=0.0, prec="mixed", r_fb=0.0, bh=None,
                 c=1e4, acc: Optional[Sequence[torch.Tensor]] = None, acc_valid: bool = False):
        """One FSI cycle in place over `subset`; returns the accelerations of the final state."""
        s = ParticleSet.of(subset, P.n)
        b = ParticleSet.of(bh, P.n) if bh is not None else ParticleSet(None, 0, 0)
        a = self._outs(P, acc, 3)
        prm = _FsiParams(float(G), float(eps2), PRECISIONS[prec], float(r_fb), _ptr(b.idx), int(b.count), float(c))
        _check("bf_fsi_step", _lib.bf_fsi_step(self._h, ctypes.byref(P._state()), ctypes.byref(s._c()), float(dt),
                                               ctypes.byref(prm), *map(_ptr, a), BF_A_VALID if acc_valid else 0))
        return a

    def jerk(self, P: Particles, targets=None, sources=None, G=1.0, eps2=0.0, prec="mixed",
             out: Optional[Sequence[torch.Tensor]] = None):
        """Jerks (particle-indexed jx, jy, jz)."""
        t, s = ParticleSet.of(targets, P.n), ParticleSet.of(sources, P.n)
        o = self._outs(P, out, 3)
        _check("bf_jerk", _lib.bf_jerk(self._h, ctypes.byref(P._c()), ctypes.byref(t._c()), ctypes.byref(s._c()),
                                       float(G), float(eps2), PRECISIONS[prec], *map(_ptr, o)))
        return o

    def timestep_assign(self, P: Particles, subset, dt_ff, dt_fb, acc, grad=None, jerk=None, eta_grad=0.1,
                        eta_jerk=0.1, tau=1.0, kmax=0, with_levels=True):
        """Per-particle time-steps (minimum of the criteria) and levels; returns (dt, level)."""
        s = ParticleSet.of(subset, P.n)
        dt = torch.full((P.n,), float("nan"), dtype=torch.float64, device=P.m.device)
        lv = torch.full((P.n,), -1, dtype=torch.int32, device=P.m.device) if with_levels else None
        g = grad if grad is not None else (None, None, None)
        j = jerk if jerk is not None else (None, None, None)
        _check("bf_timestep_assign", _lib.bf_timestep_assign(
            self._h, ctypes.byref(P._c()), ctypes.byref(s._c()), _ptr(dt_ff), _ptr(dt_fb), *map(_ptr, acc),
            *map(_ptr, g), *map(_ptr, j), float(eta_grad), float(eta_jerk), float(tau), int(kmax), _ptr(dt), _ptr(lv)))
        return dt, lv

    def level_partition(self, subset, n: int, level: torch.Tensor, kmax: int):
        """Stable partition by level: (order int32 tensor, counts list)."""
        s = ParticleSet.of(subset, n)
        _need(level, torch.int32, n, "level")
        order = torch.empty(max(s.count, 1), dtype=torch.int32, device=level.device)
        counts = (_i64 * (kmax + 1))()
        _check("bf_level_partition", _lib.bf_level_partition(self._h, ctypes.byref(s._c()), int(n), _ptr(level),
                                                             int(kmax), _ptr(order), counts))
        return order[:s.count], [int(counts[k]) for k in range(kmax + 1)]

    def hhs_interval(self, P: Particles, level: torch.Tensor, kmax: int, tau: float, subset=None, G=1.0, eps2=0.0,
                     prec="mixed", r_fb=0.0, bh=None, c=1e4):
        """One HHS-FSI interval with fixed levels, in place (PN1.0 half-kicks when bh is given)."""
        s = ParticleSet.of(subset, P.n)
        _need(level, torch.int32, P.n, "level")
        b = ParticleSet.of(bh, P.n) if bh is not None else ParticleSet(None, 0, 0)
        prm = _FsiParams(float(G), float(eps2), PRECISIONS[prec], float(r_fb), _ptr(b.idx), int(b.count), float(c))
        _check("bf_hhs_interval", _lib.bf_hhs_interval(self._h, ctypes.byref(P._state()), ctypes.byref(s._c()),
                                                       _ptr(level), int(kmax), float(tau), ctypes.byref(prm)))

    def capture_hhs_interval(self, P: Particles, level: torch.Tensor, kmax: int, tau: float, subset=None, G=1.0,
                             eps2=0.0, prec="mixed", r_fb=0.0, bh=None, c=1e4) -> "Graph":
        """Capture one fixed-level HHS-FSI interval into a HIP graph (launch to advance P), with
        the PN1.0 half-kicks of the black holes in bh if given."""
        s = ParticleSet.of(subset, P.n)
        _need(level, torch.int32, P.n, "level")
        b = ParticleSet.of(bh, P.n) if bh is not None else ParticleSet(None, 0, 0)
        prm = _FsiParams(float(G), float(eps2), PRECISIONS[prec], float(r_fb), _ptr(b.idx), int(b.count), float(c))
        h = _vp()
        _check("bf_graph_capture_hhs_interval",
               _lib.bf_graph_capture_hhs_interval(self._h, ctypes.byref(P._state()), ctypes.byref(s._c()), _ptr(level),
                                                  int(kmax), float(tau), ctypes.byref(prm), ctypes.byref(h)))
        return Graph(self, h, keep=(P, level, s, b))

    def hhs_interval_adaptive(self, P: Particles, dt0: torch.Tensor, kmax: int, tau: float, eta_ff=0.2, eta_fb=0.2,
                              eta_grad=0.1, eta_jerk=0.1, subset=None, G=1.0, eps2=0.0, prec="fp64", r_fb=0.0):
        """One HHS-FSI interval with time-steps assigned on every level from all criteria over
        the level's particles (capped by dt0), in place.  Returns (deepest level reached, number
        of levels visited)."""
        s = ParticleSet.of(subset, P.n)
        _need(dt0, torch.float64, P.n, "dt0")
        prm = _FsiParams(float(G), float(eps2), PRECISIONS[prec], float(r_fb), None, 0, 1.0)
        ml, nl = _int(0), _i64(0)
        _check("bf_hhs_interval_adaptive",
               _lib.bf_hhs_interval_adaptive(self._h, ctypes.byref(P._state()), ctypes.byref(s._c()), _ptr(dt0),
                                             int(kmax), float(tau), float(eta_ff), float(eta_fb), float(eta_grad),
                                             float(eta_jerk), ctypes.byref(prm), ctypes.byref(ml), ctypes.byref(nl)))
        return ml.value, nl.value

    def set_hhs_reuse(self, on: bool = True) -> None:
        """Keep (True, the default) or recompute every acceleration between visits of an HHS level."""
        _check("bf_set_hhs_reuse", _lib.bf_set_hhs_reuse(self._h, 1 if on else 0))

    def kick(self, P: Particles, subset, h, acc, h2=0.0, grad=None):
        s = ParticleSet.of(subset, P.n)
        g = grad if grad is not None else (None, None, None)
        _check("bf_kick", _lib.bf_kick(self._h, ctypes.byref(P._state()), ctypes.byref(s._c()), float(h),
                                       *map(_ptr, acc), float(h2), *map(_ptr, g)))

    def drift(self, P: Particles, subset, h):
        s = ParticleSet.of(subset, P.n)
        _check("bf_drift", _lib.bf_drift(self._h, ctypes.byref(P._state()), ctypes.byref(s._c()), float(h)))

    # ---- batched ensembles -------------------------------------------------------------------

    def forces_batched(self, P: Particles, cluster_off: torch.Tensor, active_idx: torch.Tensor,
                       active_off: torch.Tensor, max_active_total: int, max_cluster_n: int, G=1.0, eps2=0.0,
                       prec="mixed", r_fb=0.0, out=None):
        _need(cluster_off, torch.int64, None, "cluster_off")
        _need(active_off, torch.int64, None, "active_off")
        _need(active_idx, torch.int32, None, "active_idx")
        o = self._outs(P, out, 3)
        nc = int(cluster_off.numel()) - 1
        _check("bf_forces_batched", _lib.bf_forces_batched(
            self._h, ctypes.byref(P._c()), nc, _ptr(cluster_off), _ptr(active_idx), _ptr(active_off),
            int(max_active_total), int(max_cluster_n), float(G), float(eps2), PRECISIONS[prec], float(r_fb),
            *map(_ptr, o)))
        return o

    def force_gradient_batched(self, P: Particles, cluster_off, active_idx, active_off, max_active_total: int,
                               max_cluster_n: int, acc, G=1.0, eps2=0.0, prec="mixed", r_fb=0.0, out=None):
        o = self._outs(P, out, 3)
        nc = int(cluster_off.numel()) - 1
        _check("bf_force_gradient_batched", _lib.bf_force_gradient_batched(
            self._h, ctypes.byref(P._c()), nc, _ptr(cluster_off), _ptr(active_idx), _ptr(active_off),
            int(max_active_total), int(max_cluster_n), *map(_ptr, acc), float(G), float(eps2), PRECISIONS[prec],
            float(r_fb), *map(_ptr, o)))
        return o

    def fsi_step_batched(self, P: Particles, cluster_off, active_idx, active_off, max_active_total, max_cluster_n,
                         dt, acc, G=1.0, eps2=0.0, prec="mixed", r_fb=0.0):
        """One FSI cycle of every cluster's active particles (see bf_fsi_step_batched)."""
        nc = int(cluster_off.numel()) - 1
        _check("bf_fsi_step_batched", _lib.bf_fsi_step_batched(
            self._h, ctypes.byref(P._state()), nc, _ptr(cluster_off), _ptr(active_idx), _ptr(active_off),
            int(max_active_total), int(max_cluster_n), float(G), float(eps2), PRECISIONS[prec], float(r_fb),
            float(dt), *map(_ptr, acc)))

    def capture_batched_fsi(self, P: Particles, cluster_off, active_idx, active_off, max_active_total,
                            max_cluster_n, dt, acc, G=1.0, eps2=0.0, prec="mixed", r_fb=0.0):
        """Capture one batched FSI cycle into a HIP graph (see bf_graph_capture_batched_fsi)."""
        g = _vp()
        nc = int(cluster_off.numel()) - 1
        _check("bf_graph_capture_batched_fsi", _lib.bf_graph_capture_batched_fsi(
            self._h, ctypes.byref(P._state()), nc, _ptr(cluster_off), _ptr(active_idx), _ptr(active_off),
            int(max_active_total), int(max_cluster_n), float(G), float(eps2), PRECISIONS[prec], float(r_fb),
            float(dt), *map(_ptr, acc), ctypes.byref(g)))
        return Graph(self, g, keep=(P, cluster_off, active_idx, active_off, tuple(acc)))

    # ---- configuration -----------------------------------------------------------------------

    def autotune(self, op: int, prec: str, n_targets: int, n_sources: int, cache_path: Optional[str] = None):
        _check("bf_autotune", _lib.bf_autotune(self._h, op, PRECISIONS[prec], int(n_targets), int(n_sources),
                                               cache_path.encode() if cache_path else None))

    def autotune_pass(self, op: int, prec: str, P: Particles, targets=None, sources=None, acc=None,
                      cache_path: Optional[str] = None):
        """Tune the launch shape of pass op on the caller's own particles and sets (the
        pair-symmetric sweep's shapes when the pass takes it, the directed variants otherwise)."""
        t, s = ParticleSet.of(targets, P.n), ParticleSet.of(sources, P.n)
        a = list(acc) if acc is not None else [None, None, None]
        for x in a:
            if x is not None:
                _need(x, torch.float64, P.n, "acc")
        _check("bf_autotune_pass", _lib.bf_autotune_pass(self._h, int(op), PRECISIONS[prec], ctypes.byref(P._c()),
                                                         ctypes.byref(t._c()), ctypes.byref(s._c()), *map(_ptr, a),
                                                         cache_path.encode() if cache_path else None))

    def autotune_batched(self, op: int, prec: str, P: Particles, cluster_off, active_idx, active_off,
                         max_active_total: int, max_cluster_n: int, acc=None, cache_path: Optional[str] = None):
        """Tune the batched pass op (targets per lane, waves, sources per work item) on the caller's
        ensemble."""
        a = list(acc) if acc is not None else [None, None, None]
        nc = int(cluster_off.numel()) - 1
        _check("bf_autotune_batched", _lib.bf_autotune_batched(
            self._h, int(op), PRECISIONS[prec], ctypes.byref(P._c()), nc, _ptr(cluster_off), _ptr(active_idx),
            _ptr(active_off), int(max_active_total), int(max_cluster_n), *map(_ptr, a),
            cache_path.encode() if cache_path else None))

    def set_symmetric_config(self, op: int, rows: int = 0, waves: int = 0, rounds: int = 0):
        """Force the pair-symmetric sweep's shape (rows = 0: the tuned or default choice)."""
        _check("bf_set_symmetric_config", _lib.bf_set_symmetric_config(self._h, int(op), int(rows), int(waves),
                                                                       int(rounds)))

    def set_symmetric_scratch_limit(self, nbytes: int = 0):
        """Scratch limit of a pair-symmetric pass (0: the default); above it the sweep runs its
        distance shares in several passes, with bitwise the same results."""
        _check("bf_set_symmetric_scratch_limit", _lib.bf_set_symmetric_scratch_limit(self._h, int(nbytes)))

    def last_symmetric_passes(self) -> int:
        """Sweeps over the distance shares of the most recent pass (1: one, or not symmetric)."""
        v = _int(0)
        _check("bf_last_symmetric_passes", _lib.bf_last_symmetric_passes(self._h, ctypes.byref(v)))
        return v.value

    def query_batched_config(self, op: int, prec: str, max_active_total: int, max_cluster_n: int):
        """(targets per lane, waves, sources per work item) a batched pass of these bounds runs."""
        k, w, ch = _int(0), _int(0), _int(0)
        _check("bf_query_batched_config", _lib.bf_query_batched_config(
            self._h, int(op), PRECISIONS[prec], int(max_active_total), int(max_cluster_n), ctypes.byref(k),
            ctypes.byref(w), ctypes.byref(ch)))
        return k.value, w.value, ch.value

    def set_batched_config(self, op: int, prec: str, k: int = 0, waves: int = 0, chunk: int = 0):
        """Force the batched pass's shape (k = 0: the tuned or default choice)."""
        _check("bf_set_batched_config", _lib.bf_set_batched_config(self._h, int(op), PRECISIONS[prec], int(k),
                                                                   int(waves), int(chunk)))

    def autotune_load(self, cache_path: str):
        _check("bf_autotune_load", _lib.bf_autotune_load(self._h, cache_path.encode()))

    def query_config(self, op: int, prec: str, n_targets: int, n_sources: int):
        k, w, s = _int(0), _int(0), _int(0)
        _check("bf_query_config", _lib.bf_query_config(self._h, op, PRECISIONS[prec], int(n_targets), int(n_sources),
                                                       ctypes.byref(k), ctypes.byref(w), ctypes.byref(s)))
        return k.value, w.value, s.value

    def last_pass_stats(self):
        """(fix-ups, near tile visits, far tile visits) of the most recent pass."""
        f, nn, nf = _i64(0), _i64(0), _i64(0)
        _check("bf_last_pass_stats", _lib.bf_last_pass_stats(self._h, ctypes.byref(f), ctypes.byref(nn),
                                                             ctypes.byref(nf)))
        return f.value, nn.value, nf.value

    def release_scratch(self) -> int:
        """Free the context's scratch buffers; returns the bytes freed."""
        freed = ctypes.c_size_t(0)
        _check("bf_release_scratch", _lib.bf_release_scratch(self._h, ctypes.byref(freed)))
        return freed.value

    def pair_credit(self, op: int, reset: bool = False) -> int:
        """Pair interactions credited by the passes of op since creation or the last reset."""
        v = _i64(0)
        _check("bf_pair_credit", _lib.bf_pair_credit(self._h, int(op), ctypes.byref(v), int(bool(reset))))
        return v.value

    def last_pass_config(self):
        """(kind, k_per_lane, waves, split) of the most recent pass; kind is "unsorted", "sorted"
        (directed sweep), "symmetric" (each unordered pair once) or "between" (the two-set sweep)."""
        v = [_int(0) for _ in range(4)]
        _check("bf_last_pass_config", _lib.bf_last_pass_config(self._h, *(ctypes.byref(x) for x in v)))
        return ("unsorted", "sorted", "symmetric", "between")[v[0].value], v[1].value, v[2].value, v[3].value

    def set_spatial_sort(self, forces: bool = True, gradient: bool = True, kappa: float = 0.0,
                         any_size: bool = False, symmetric: bool = True, timestep: bool = True):
        """Select the passes that use the spatially sorted mixed kernels (default: both); kappa = 0
        keeps the near-tile threshold (default 1); any_size lifts the minimum pass size;
        symmetric = False keeps the directed sweep where targets and sources are one set;
        timestep selects the pair-symmetric mixed time-step pass over one set (set order)."""
        mask = (int(bool(forces)) << BF_OP_FORCES) | (int(bool(gradient)) << BF_OP_GRADIENT)
        mask |= int(bool(timestep)) << BF_OP_DTMIN
        mask |= BF_SORT_ANY_SIZE if any_size else 0
        mask |= 0 if symmetric else BF_SORT_DIRECTED
        _check("bf_set_spatial_sort", _lib.bf_set_spatial_sort(self._h, mask, float(kappa)))

    # ---- subsystems --------------------------------------------------------------------------

    def neighbours(self, P: Particles, targets=None, sources=None, G=1.0, r_ngb=1e-3, r_max=0.1, C=0.5, tau=1e-3,
                   cap: int = 1 << 16) -> torch.Tensor:
        """Neighbour pairs (i, j) as an (m, 2) int32 device tensor, sorted (Sec. 3.3)."""
        t, s = ParticleSet.of(targets, P.n), ParticleSet.of(sources, P.n)
        while True:
            edges = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=P.m.device)
            m = _i64(0)
            rc = _lib.bf_neighbours(self._h, ctypes.byref(P._c()), ctypes.byref(t._c()),
                                    ctypes.byref(s._c()), float(G), float(r_ngb), float(r_max), float(C),
                                    float(tau), _ptr(edges), int(cap), ctypes.byref(m))
            if rc == BF_ERR_NOMEM and m.value > cap:
                cap = m.value
                continue
            _check("bf_neighbours", rc)
            return edges[:m.value]

    def subsystems(self, n: int, edges: torch.Tensor):
        """(labels, number of subsystems): components of the neighbour graph, each labelled by
        its smallest particle index."""
        e = edges.contiguous()
        _need(e, torch.int32, None, "edges")
        label = torch.empty(n, dtype=torch.int32, device=e.device)
        ns = _i64(0)
        _check("bf_subsystems", _lib.bf_subsystems(self._h, int(n), _ptr(e) if e.numel() else None,
                                                   int(e.shape[0]) if e.numel() else 0, _ptr(label),
                                                   ctypes.byref(ns)))
        return label, ns.value

    def set_subsystems(self, label: Optional[torch.Tensor]):
        """Exclude pairs with equal labels from later acc / gradient / time-step passes (None clears).
        The context keeps a reference to the tensor until cleared."""
        if label is None:
            self._sub = None
            _check("bf_set_subsystems", _lib.bf_set_subsystems(self._h, None, 0))
            return
        _need(label, torch.int32, None, "label")
        self._sub = label
        _check("bf_set_subsystems", _lib.bf_set_subsystems(self._h, _ptr(label), int(label.numel())))

    def enable_timing(self, on: bool = True):
        _check("bf_enable_timing", _lib.bf_enable_timing(self._h, int(on)))

    def kernel_times(self, op: int, cap: int = 4096):
        """Durations (ms) of the pair-kernel launches of op recorded since the last call."""
        buf = (ctypes.c_float * cap)()
        cnt = _int(0)
        _check("bf_kernel_times", _lib.bf_kernel_times(self._h, op, buf, cap, ctypes.byref(cnt)))
        return [float(buf[i]) for i in range(min(cnt.value, cap))]

    def set_config(self, op: int, prec: str, k: int = 0, waves: int = 0, split: int = 0):
        _check("bf_set_config", _lib.bf_set_config(self._h, op, PRECISIONS[prec], int(k), int(waves), int(split)))


class Graph:
    """A captured HIP graph (opaque handle) replayed on the context's stream."""

    def __init__(self, ctx: Context, handle, keep=()):
        # the graph reads and writes the captured tensors: keep them alive as long as it exists
        self.ctx, self._g, self._keep = ctx, handle, keep

    def launch(self):
        _check("bf_graph_launch", _lib.bf_graph_launch(self.ctx.handle, self._g))

    def close(self):
        if self._g and self._g.value:
            _lib.bf_graph_destroy(self._g)
            self._g = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
