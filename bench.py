"""Benchmark: pair interactions/s of the acceleration + force-gradient sweep on one MI355X.

Workload: King W0 = 6 cluster, N = 2^20, Kroupa masses with 1% binaries carried as centre-of-mass
particles, Henon units, eps = 0, all particles active; one step = the acceleration pass followed by
the force-gradient pass on the fresh accelerations (the middle of an FSI cycle), in mixed precision
(FP64 position/acceleration differences rounded once to FP32, FP32 pair arithmetic, FP32 tile
sums merged in FP64, FP64 re-evaluation of targets whose sum cancels strongly).  The all-FP64 path is timed on the same input for the speedup.  Inputs are resident
in HBM before timing starts.

Prints one JSON line.  Rate = N (N - 1) / (t_acc + t_grad): each pair credited once per sweep.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_ACC = 20     # flops per pair, acceleration (FMA = 2, rsqrt = 1)
FLOPS_GRAD = 35    # flops per pair, force gradient
FLOPS_DT = 25      # flops per pair, free-fall / fly-by time-step
# MI355X vector peaks: FP32 157.3 TFLOP/s (256 CUs x 128 FP32 lanes x 2 flops x 2.4 GHz, which
# needs packed FP32 issue) and FP64 78.6 TFLOP/s (256 x 64 x 2 x 2.4 GHz).  The library is built
# with packed FP32 instruction selection off, so the FP32 figure is an upper bound it cannot reach.
PEAK_FP32_TFLOPS = 256 * 128 * 2 * 2.4e9 / 1e12  # 157.29
PEAK_FP64_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12   # 78.64


# HBM traffic of the dominant kernel, measured with rocprofv3 counters (FETCH_SIZE, WRITE_SIZE)
# and scaled by the same counters' reading for a copy kernel of known size.  The figure is used
# only while the sources that define the kernel and its tile packs hash to the value recorded
# with it and the pass runs the recorded launch shape (row tiles, waves, distance shares).
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pairs_sym_SymGrad_king1m_hbm_traffic.txt")
TRAFFIC_KIND = "symmetric"  # the pass kind whose kernel the counters were taken on
KERNEL_SOURCES = ["pair_ops.h", "spatial.hip", "symmetric.hip", "bf_internal.h"]

# gradient kernel of each pass kind (the library's launch of that kind at this size)
KERNEL_NAMES = {"unsorted": "k_pairs<GradMixed>", "sorted": "k_pairs_sorted<GradMixed>",
                "symmetric": "k_pairs_sym<SymGrad>", "between": "k_pairs_sym<SymGrad> (two sets)"}


def pass_desc(cfg):
    """Report of bf_last_pass_config: the sweep and its launch shape."""
    kind, k, waves, split = cfg
    if kind == "symmetric":
        return {"sweep": "pair-symmetric, spatially sorted", "row_tiles_per_wave": k, "waves": waves,
                "distance_shares": split}
    return {"sweep": "directed, " + ("spatially sorted" if kind == "sorted" else "unsorted"),
            "k_per_lane": k, "waves": waves, "split": split}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2210_02472_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(n, cfg):
    """Bytes per launch from the committed counter summary, or None if absent or stale (other
    kernel sources, size or launch shape)."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        shape = [int(x) for x in kv["shape"].split(",")]
        if (kv.get("source_sha256") != kernel_source_hash() or int(kv.get("n", -1)) != n or cfg[0] != TRAFFIC_KIND
                or list(cfg[1:4]) != shape):
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def synthetic_acc_field(d):
    """Smooth input accelerations for the gradient parity sample (any field is a valid input)."""
    x, y, z = d["x"], d["y"], d["z"]
    s = (x * x + y * y + z * z + 0.1) ** -1.5
    return np.stack([-x * s, -y * s, -z * s], axis=1)


def _pass_rate(ctx, bf, op, call, reps=3):
    """Average pair-kernel duration (ms) of `call` over reps, from the context's HIP events."""
    call()
    ctx.enable_timing(True)
    for _ in range(reps):
        call()
    t = ctx.kernel_times(op)
    ctx.enable_timing(False)
    return float(np.mean(t)) if t else float("nan")


def _roofline(kernel, flops, kernel_ms, n_launches, peak, prec_note):
    """ALU roofline of a kernel class: credited flops per launch over its average HIP-event
    duration (launches of different sizes: their total flops over their total time)."""
    achieved = flops / (kernel_ms * 1e-3) / 1e12 if kernel_ms > 0 else float("nan")
    return {"bound": "alu", "kernel": kernel, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": None, "launches": n_launches,
            "flops_per_launch": flops / max(n_launches, 1), "avg_kernel_ms": kernel_ms / max(n_launches, 1),
            "peak_note": prec_note}


def _timed_ops(ctx, bf, fn, reps):
    """Run fn reps times with kernel timing on: (wall s per rep, {op: (kernel ms per rep,
    launches per rep)}, {op: credited pairs per rep})."""
    import torch
    fn()
    torch.cuda.synchronize()
    for op in (bf.BF_OP_FORCES, bf.BF_OP_GRADIENT, bf.BF_OP_DTMIN):
        ctx.pair_credit(op, reset=True)
    ctx.enable_timing(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / reps
    kt = {op: ctx.kernel_times(op) for op in (bf.BF_OP_FORCES, bf.BF_OP_GRADIENT, bf.BF_OP_DTMIN)}
    ctx.enable_timing(False)
    credit = {op: ctx.pair_credit(op, reset=True) / reps for op in kt}
    return wall, {op: (float(np.sum(v)) / reps, len(v) / reps) for op, v in kt.items()}, credit


def _dominant(bf, times, credit, names, peak, prec_note, flops_of=None):
    """Roofline of the op whose kernels took the most time; times and credit per step."""
    flops_of = flops_of or {bf.BF_OP_FORCES: FLOPS_ACC, bf.BF_OP_GRADIENT: FLOPS_GRAD, bf.BF_OP_DTMIN: FLOPS_DT}
    op = max(times, key=lambda o: times[o][0])
    ms, nl = times[op]
    return _roofline(names[op], flops_of[op] * credit[op], ms, nl, peak, prec_note)


def _cpu_rate(oracle, fn, pairs_of_call, seconds):
    """Oracle pairs/s: repeat fn until `seconds` of CPU work (at least once)."""
    k, tc, pairs = 0, 0.0, 0.0
    while tc < seconds or k == 0:
        t1 = time.perf_counter()
        fn(k)
        tc += time.perf_counter() - t1
        pairs += pairs_of_call(k)
        k += 1
    return pairs / tc, tc, k


def run_workload(name, args):
    """The other configurations: each prints one JSON line in the same form as the headline, its
    own metric, the roofline of its dominant kernel class and the oracle's rate beside it."""
    import torch

    import oracle
    import paper_2210_02472_amd as bf
    from paper_2210_02472_amd import ics

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    ctx = bf.Context(0)
    steps, warmup = args.steps, args.warmup
    nthreads = oracle.num_threads()
    names_mixed = {bf.BF_OP_FORCES: "k_pairs<AccMixed> (acceleration)", bf.BF_OP_GRADIENT: "k_pairs<GradMixed> (gradient)",
                   bf.BF_OP_DTMIN: "k_pairs<DtMixed> (free-fall / fly-by time-step)"}
    rec = {"n_gpus": 1, "steps": steps, "warmup": warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic"}
    if name == "plummer1k-fsi":
        # N = 1024 equal-mass Plummer, eps = 0, FP64: one acceleration + gradient evaluation, then
        # FSI steps with dt = 1e-3 (the first acceleration reused), energy logged every step.  A
        # step is one FSI cycle: two acceleration passes and one gradient pass (the third
        # acceleration pass is the next step's first).
        d = ics.config1_plummer1k()
        n = len(d["m"])
        dt = 1e-3
        P = bf.Particles.from_numpy(d)
        a = ctx.forces(P, prec="fp64")
        ctx.force_gradient(P, a, prec="fp64")
        e0 = sum(ctx.energy(P))
        energies = [e0]
        for s in range(10):  # the configured run: 10 steps, energy after each (untimed)
            a = ctx.fsi_step(P, dt, prec="fp64", acc=a, acc_valid=s > 0)
            energies.append(sum(ctx.energy(P)))
        Pt = bf.Particles.from_numpy(d)
        at = ctx.forces(Pt, prec="fp64")
        state = {"s": 0}

        def one():
            nonlocal at
            at = ctx.fsi_step(Pt, dt, prec="fp64", acc=at, acc_valid=state["s"] > 0)
            state["s"] += 1
        for _ in range(warmup):
            one()
        wall, times, credit = _timed_ops(ctx, bf, one, steps)
        pairs = sum(credit.values())
        names = {bf.BF_OP_FORCES: "k_pairs<Acc64> (acceleration)", bf.BF_OP_GRADIENT: "k_pairs<Grad64> (gradient)",
                 bf.BF_OP_DTMIN: "-"}
        roof = _dominant(bf, times, credit, names, PEAK_FP64_TFLOPS, "FP64 vector peak")
        # the same step replayed from a HIP graph: a one-level HHS interval of length dt (every
        # particle on level 0) is one FSI cycle whose first acceleration is computed afresh
        Pg = bf.Particles.from_numpy(d)
        lv0 = torch.zeros(n, dtype=torch.int32, device="cuda")
        ctx.hhs_interval(Pg, lv0, 0, dt, prec="fp64")
        torch.cuda.synchronize()
        for op in (bf.BF_OP_FORCES, bf.BF_OP_GRADIENT, bf.BF_OP_DTMIN):
            ctx.pair_credit(op, reset=True)
        ctx.hhs_interval(Pg, lv0, 0, dt, prec="fp64")
        torch.cuda.synchronize()
        g_pairs = sum(ctx.pair_credit(op, reset=True) for op in (bf.BF_OP_FORCES, bf.BF_OP_GRADIENT, bf.BF_OP_DTMIN))
        gr = ctx.capture_hhs_interval(Pg, lv0, 0, dt, prec="fp64")
        for _ in range(max(1, warmup)):
            gr.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            gr.launch()
        torch.cuda.synchronize()
        g_wall = (time.perf_counter() - t0) / steps
        gr.close()
        # oracle: the same FSI steps (acceleration of the first step included)
        Po = oracle.Particles.from_dict(d)
        rate, tc, k = _cpu_rate(oracle, lambda k: oracle.fsi_step(Po, dt), lambda k: 3.0 * n * (n - 1), 5.0)
        rec.update({"metric": "pair interactions/s (FSI steps, N=1024 Plummer, FP64)", "value": pairs / wall,
                    "unit": "pair interactions/s", "ms_per_step": wall * 1e3, "dtype": "f64",
                    "config": {"workload": "Plummer N=1024 equal mass, Henon units, eps=0, all active; one "
                                           "acceleration + gradient evaluation, then FSI steps dt=1e-3 in FP64 "
                                           "(a step: 2 acceleration passes + 1 gradient pass, FSAL)", "n": n,
                               "dt": dt},
                    "pairs_per_step": pairs, "energy_log": energies,
                    "rel_energy_drift_10_steps": abs(energies[-1] / energies[0] - 1),
                    "graph": {"ms_per_step": g_wall * 1e3, "pairs_per_step": g_pairs, "value": g_pairs / g_wall,
                              "note": "one-level HHS interval of length dt captured once and replayed; "
                                      "pairs as the library credits them for that interval"},
                    "roofline": roof,
                    "cpu_baseline": {"value": rate, "unit": "pair interactions/s", "cores": nthreads,
                                     "kind": "oracle", "sample": f"{k} full FSI steps of the same cluster, "
                                                                 f"3 N(N-1) pairs each (the oracle recomputes "
                                                                 f"every acceleration), {tc:.1f} s"}})
    elif name == "plummer64k-level":
        # N = 65,536 Kroupa Plummer, a random 10% level, eps = 1e-4: acc + grad + dt_min of the level
        # against all particles, mixed (and FP64 for the speedup)
        d, act = ics.config2_plummer64k()
        P = bf.Particles.from_numpy(d)
        T = torch.as_tensor(act, device="cuda")
        n, nt = len(d["m"]), len(act)
        eps2 = 1e-8
        a = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
        res = {}
        for prec in ("mixed", "fp64"):
            def step():
                ctx.forces(P, T, None, eps2=eps2, prec=prec, r_fb=0.0, out=a)
                ctx.force_gradient(P, a, T, None, eps2=eps2, prec=prec, r_fb=0.0)
                ctx.dt_min(P, T, None, prec=prec, r_fb=0.0)
            for _ in range(warmup):
                step()
            res[prec] = _timed_ops(ctx, bf, step, steps)
        wall, times, credit = res["mixed"]
        pairs = sum(credit.values())
        roof = _dominant(bf, times, credit, names_mixed, PEAK_FP32_TFLOPS, "FP32 vector peak (packed)")
        Po = oracle.Particles.from_dict(d)
        # mixed vs oracle on 256 sampled level particles (acceleration, gradient, time-steps)
        ctx.forces(P, T, None, eps2=eps2, prec="mixed", out=a)
        g = ctx.force_gradient(P, a, T, None, eps2=eps2, prec="mixed")
        dff, dfb = ctx.dt_min(P, T, None, prec="mixed")
        sample = np.sort(np.random.default_rng(1).choice(act, 256, replace=False))
        afull = np.stack([t.cpu().numpy() for t in a], axis=1)
        ref_a = oracle.forces(Po, sample, None, eps2=eps2)
        ref_g = oracle.gradient(Po, afull, sample, None, eps2=eps2)
        ref_dt = oracle.dt_min(Po, sample, None)
        def err(got, ref):
            e = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
            return float(np.sqrt(np.mean(e * e))), float(e.max())
        e_a = err(afull[sample], ref_a)
        e_g = err(np.stack([t.cpu().numpy()[sample] for t in g], axis=1), ref_g)
        got_dt = np.stack([dff.cpu().numpy()[sample], dfb.cpu().numpy()[sample]], axis=1)
        ref_dt = np.stack(ref_dt, axis=1) if isinstance(ref_dt, tuple) else np.asarray(ref_dt)
        e_dt = float(np.max(np.abs(got_dt - ref_dt) / np.abs(ref_dt)))
        # oracle: the whole level, acc + grad + dt_min
        def cpu_step(k):
            oracle.forces(Po, act, None, eps2=eps2)
            oracle.gradient(Po, afull, act, None, eps2=eps2)
            oracle.dt_min(Po, act, None)
        rate, tc, k = _cpu_rate(oracle, cpu_step, lambda k: 3.0 * nt * n, 1.0)
        w64, t64, c64 = res["fp64"]
        rec.update({"metric": "pair interactions/s (acc+grad+dt_min of a 10% level, N=65536, mixed)",
                    "value": pairs / wall, "unit": "pair interactions/s", "ms_per_step": wall * 1e3,
                    "dtype": "f32 pair arithmetic, f64 accumulate",
                    "config": {"workload": "Plummer N=65536, Kroupa IMF, Henon units, eps=1e-4; a random 10% "
                                           "level (6554 targets) against all particles: acceleration + "
                                           "force-gradient + free-fall/fly-by time-step passes, mixed", "n": n,
                               "n_active": nt, "eps2": eps2},
                    "pairs_per_step": pairs,
                    "kernel_ms": {k2: times[v][0] / max(times[v][1], 1e-9) for k2, v in
                                  (("acc", bf.BF_OP_FORCES), ("grad", bf.BF_OP_GRADIENT), ("dt_min", bf.BF_OP_DTMIN))},
                    "fp64": {"ms_per_step": w64 * 1e3, "value": sum(c64.values()) / w64,
                             "kernel_ms": {k2: t64[v][0] / max(t64[v][1], 1e-9) for k2, v in
                                           (("acc", bf.BF_OP_FORCES), ("grad", bf.BF_OP_GRADIENT),
                                            ("dt_min", bf.BF_OP_DTMIN))}},
                    "speedup_vs_fp64": w64 / wall,
                    "rel_err_vs_oracle": {"acc_rms": e_a[0], "acc_max": e_a[1], "grad_rms": e_g[0],
                                          "grad_max": e_g[1], "dt_max": e_dt, "sample_targets": 256},
                    "roofline": roof,
                    "cpu_baseline": {"value": rate, "unit": "pair interactions/s", "cores": nthreads,
                                     "kind": "oracle", "sample": f"{k} x the whole level: acceleration + gradient "
                                                                 f"+ time-step passes, 6554 x 65536 pairs each, "
                                                                 f"FP64, {tc:.1f} s"}})
    elif name == "ensemble256":
        # 256 equal-mass Plummer clusters, N log-uniform in [1024, 65536], active fractions 2^-k:
        # one persistent batched launch per pass; a step is the HIP-graph captured batched FSI cycle
        # (2 acceleration passes + 1 gradient pass over every cluster's active particles)
        d, off, act, aoff = ics.config4_ensemble()
        P = bf.Particles.from_numpy(d)
        co, ai, ao = (torch.as_tensor(x, device="cuda") for x in (off, act, aoff))
        sizes = np.diff(off)
        nact = np.diff(aoff)
        pairs_pass = float(np.sum(sizes.astype(np.float64) * nact))
        maxn, ntot, na = int(sizes.max()), int(off[-1]), int(aoff[-1])
        eps2 = 1e-8
        dt = 1e-4
        res = {}
        shapes = {}
        if args.autotune:
            t1 = time.time()
            af = synthetic_acc_field(d)
            acc_t = [torch.as_tensor(np.ascontiguousarray(af[:, k]), device="cuda") for k in range(3)]
            for prec in ("mixed", "fp64"):
                ctx.autotune_batched(bf.BF_OP_FORCES, prec, P, co, ai, ao, na, maxn)
                ctx.autotune_batched(bf.BF_OP_GRADIENT, prec, P, co, ai, ao, na, maxn, acc=acc_t)
            log(f"autotuned the batched passes in {time.time() - t1:.1f}s")
        for prec in ("mixed", "fp64"):
            shapes[prec] = {op_name: dict(zip(("k_per_lane", "waves", "sources_per_item"),
                                              ctx.query_batched_config(op, prec, na, maxn)))
                            for op_name, op in (("acc", bf.BF_OP_FORCES), ("grad", bf.BF_OP_GRADIENT))}
            a = ctx.forces_batched(P, co, ai, ao, na, maxn, eps2=eps2, prec=prec)
            g = ctx.capture_batched_fsi(P, co, ai, ao, na, maxn, dt, a, eps2=eps2, prec=prec)
            for _ in range(warmup):
                g.launch()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(steps):
                g.launch()
            torch.cuda.synchronize()
            tg = (time.perf_counter() - t) / steps
            g.close()
            # per-kernel durations from the eager cycle (events are not recorded inside graphs)
            wall_e, times, _ = _timed_ops(ctx, bf, lambda: ctx.fsi_step_batched(P, co, ai, ao, na, maxn, dt, a,
                                                                                eps2=eps2, prec=prec), 2)
            res[prec] = (tg, wall_e, times)
        tg, wall_e, times = res["mixed"]
        credit = {bf.BF_OP_FORCES: 2 * pairs_pass, bf.BF_OP_GRADIENT: pairs_pass, bf.BF_OP_DTMIN: 0.0}
        names = {bf.BF_OP_FORCES: "k_batch_pairs<AccMixed> (acceleration)",
                 bf.BF_OP_GRADIENT: "k_batch_pairs<GradMixed> (gradient)", bf.BF_OP_DTMIN: "-"}
        roof = _dominant(bf, times, credit, names, PEAK_FP32_TFLOPS, "FP32 vector peak (packed)")
        # oracle on 16 sampled clusters: acceleration + gradient of the active particles
        Po = oracle.Particles.from_dict(d)
        pick = np.sort(np.random.default_rng(7).choice(len(sizes), 16, replace=False))
        sub = []
        for c in pick:
            rng_c = np.arange(off[c], off[c + 1])
            sub.append((rng_c, act[aoff[c]:aoff[c + 1]]))

        def cpu_clusters(k):
            for src, tg_ in sub:
                a_ = oracle.forces(Po, tg_, src, eps2=eps2)
                full = np.zeros((ntot, 3))
                full[tg_] = a_
                oracle.gradient(Po, full, tg_, src, eps2=eps2)
        cpu_pairs = 2.0 * sum(float(len(t_)) * len(s_) for s_, t_ in sub)
        rate, tc, k = _cpu_rate(oracle, cpu_clusters, lambda k: cpu_pairs, 2.0)
        t64 = res["fp64"][0]
        rec.update({"metric": "active pair interactions/s (batched FSI cycle, 256-cluster ensemble, mixed)",
                    "value": 3 * pairs_pass / tg, "unit": "pair interactions/s", "ms_per_step": tg * 1e3,
                    "dtype": "f32 pair arithmetic, f64 accumulate",
                    "config": {"workload": "256 equal-mass Plummer clusters, N log-uniform in [1024, 65536], "
                                           "active fractions 2^-k (k uniform in 0..6), eps=1e-4; one HIP-graph "
                                           "replay of the batched FSI cycle (persistent kernel per pass), mixed",
                               "clusters": len(sizes), "particles": ntot, "active": na,
                               "active_pairs_per_pass": pairs_pass, "dt": dt, "autotuned": bool(args.autotune),
                               "batched_shapes": shapes},
                    "eager_cycle_ms": wall_e * 1e3,
                    "kernel_ms": {"acc": times[bf.BF_OP_FORCES][0] / max(times[bf.BF_OP_FORCES][1], 1e-9),
                                  "grad": times[bf.BF_OP_GRADIENT][0] / max(times[bf.BF_OP_GRADIENT][1], 1e-9)},
                    "fp64": {"ms_per_step": t64 * 1e3, "value": 3 * pairs_pass / t64},
                    "speedup_vs_fp64": t64 / tg,
                    "roofline": roof,
                    "cpu_baseline": {"value": rate, "unit": "pair interactions/s", "cores": nthreads,
                                     "kind": "oracle", "sample": f"{k} x (acceleration + gradient of the active "
                                                                 f"particles of 16 sampled clusters), FP64, "
                                                                 f"{tc:.1f} s"}})
    elif name == "bh-levels":
        # N = 262,144 Kroupa Plummer with 16 BHs + 1000 Msun IMBH, levels 0..7 (2^-k at >= k):
        # per level, acceleration + gradient of the level's particles from all particles (mixed)
        # and PN1.0 for BH pairs (FP64, c = 1e4)
        d, bh, lv = ics.config5_bh_cluster()
        P = bf.Particles.from_numpy(d)
        n = len(d["m"])
        levels = []
        for k in range(int(lv.max()) + 1):
            idx = np.nonzero(lv >= k)[0].astype(np.int32)
            T = torch.as_tensor(idx, device="cuda")
            a = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
            ta = _pass_rate(ctx, bf, bf.BF_OP_FORCES, lambda: ctx.forces(P, T, None, prec="mixed", r_fb=0.0, out=a))
            tg = _pass_rate(ctx, bf, bf.BF_OP_GRADIENT, lambda: ctx.force_gradient(P, a, T, None, prec="mixed",
                                                                                   r_fb=0.0))
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.pn1_bh(P, bh, T, None, c=1e4)
            torch.cuda.synchronize()
            tp = time.perf_counter() - t
            levels.append({"level": k, "n_active": int(idx.size), "acc_ms": ta, "grad_ms": tg, "pn1_ms": tp * 1e3,
                           "acc_grad_pairs_per_s": idx.size * float(n) / ((ta + tg) * 1e-3)})
        rec.update({"workload": name, "n": n, "n_bh": int(len(bh)), "levels": levels})
    elif name == "bh-hhs":
        # One HHS-FSI interval over the same cluster and levels: Newtonian part mixed, PN1.0 for
        # every pair with a black hole (FP64, c = 1e4).  A step is one interval (fixed levels,
        # eager device driver); also: the same interval replayed from a HIP graph, the eager
        # interval with every pass unsorted, and the interval with time-steps reassigned on every
        # level (Newtonian only: the initial time-steps put each particle on its level; the
        # free-fall, fly-by, gradient and jerk time-steps over each level's particles may move it
        # deeper)
        d, bh, lv = ics.config5_bh_cluster()
        n = len(d["m"])
        kmax = int(lv.max())
        tau = 1.0 / 4096
        level = torch.as_tensor(lv.astype(np.int32), device="cuda")
        P = bf.Particles.from_numpy(d)
        clight = 1e4

        def wall(fn, reps):
            fn()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t) / reps * 1e3

        dt0 = torch.as_tensor(1.5 * tau / 2.0 ** lv.astype(np.float64), device="cuda")
        if args.hhs_adaptive_only:  # for a kernel trace of the reassigned interval alone
            seen = []
            adaptive = wall(lambda: seen.append(ctx.hhs_interval_adaptive(P, dt0, kmax, tau, 0.05, 0.05, 0.05, 0.05,
                                                                            prec="mixed")), 2)
            rec.update({"workload": name, "n": n, "kmax": kmax, "tau": tau, "interval_ms": {"adaptive": adaptive},
                        "adaptive_levels_visited": seen[-1][1]})
            ctx.close()
            print(json.dumps(rec), flush=True)
            return
        interval = lambda: ctx.hhs_interval(P, level, kmax, tau, prec="mixed", bh=bh, c=clight)  # noqa: E731
        if args.hhs_eager_only:  # for a kernel trace of the eager interval alone
            rec.update({"workload": name, "n": n, "kmax": kmax, "tau": tau,
                        "interval_ms": {"eager": wall(interval, steps)}})
            ctx.close()
            print(json.dumps(rec), flush=True)
            return
        for _ in range(warmup):
            interval()
        w, times, credit = _timed_ops(ctx, bf, interval, steps)
        pairs = sum(credit.values())
        names = {bf.BF_OP_FORCES: "k_pairs_sym<SymAcc> / two-set and directed acceleration kernels",
                 bf.BF_OP_GRADIENT: "k_pairs_sym<SymGrad> / two-set and directed gradient kernels",
                 bf.BF_OP_DTMIN: "-"}
        roof = _dominant(bf, times, credit, names, PEAK_FP32_TFLOPS, "FP32 vector peak (packed)")
        g = ctx.capture_hhs_interval(P, level, kmax, tau, prec="mixed", bh=bh, c=clight)
        graph = wall(g.launch, steps)
        g.close()
        ctx.set_spatial_sort(False, False)  # reference: every pass unsorted
        eager_unsorted = wall(interval, 2)
        ctx.set_spatial_sort(True, True)
        levels_seen = []
        adaptive = wall(lambda: levels_seen.append(ctx.hhs_interval_adaptive(P, dt0, kmax, tau, 0.05, 0.05, 0.05,
                                                                                0.05, prec="mixed")), 2)
        counts = np.bincount(lv, minlength=kmax + 1)
        # oracle: a bounded sample of the interval's largest passes, level 0 against all particles
        Po = oracle.Particles.from_dict(d)
        rng = np.random.default_rng(5)
        afield = synthetic_acc_field(d)

        def cpu_sample(k):
            Ts = np.sort(rng.choice(n, 512, replace=False))
            oracle.forces(Po, Ts, None)
            oracle.gradient(Po, afield, Ts, None)
        rate, tc, k = _cpu_rate(oracle, cpu_sample, lambda k: 2.0 * 512 * (n - 1), 10.0)
        rec.update({"metric": "pair interactions/s (one HHS-FSI interval, N=262144 with 17 BHs, PN1.0)",
                    "value": pairs / (w), "unit": "pair interactions/s", "ms_per_step": w * 1e3,
                    "dtype": "f32 pair arithmetic, f64 accumulate; PN1.0 f64",
                    "config": {"workload": "Plummer N=262144, Kroupa IMF, 16 BHs (10-100 Msun) + 1000 Msun IMBH "
                                           "at the centre, M=1, eps=0; fixed levels 0..7 (fraction 2^-k at "
                                           "level >= k, BHs deepest); one HHS-FSI interval tau=1/4096, "
                                           "Newtonian passes mixed, PN1.0 FP64 c=1e4", "n": n, "n_bh": int(len(bh)),
                               "kmax": kmax, "tau": tau, "particles_per_level": counts.tolist()},
                    "pairs_per_step": pairs,
                    "kernel_ms_per_step": {"acc": times[bf.BF_OP_FORCES][0], "grad": times[bf.BF_OP_GRADIENT][0],
                                           "acc_launches": times[bf.BF_OP_FORCES][1],
                                           "grad_launches": times[bf.BF_OP_GRADIENT][1]},
                    "interval_ms": {"eager": w * 1e3, "graph": graph, "eager_unsorted": eager_unsorted,
                                    "adaptive_newtonian": adaptive},
                    "adaptive_deepest_level": levels_seen[-1][0], "adaptive_levels_visited": levels_seen[-1][1],
                    "roofline": roof,
                    "cpu_baseline": {"value": rate, "unit": "pair interactions/s", "cores": nthreads,
                                     "kind": "oracle", "sample": f"{k} x 512 random targets x all {n} sources, "
                                                                 f"acceleration + gradient (the level-0 passes), "
                                                                 f"FP64, {tc:.1f} s"}})
    elif name == "bh-aux":
        # The same 262,144-body cluster, every particle a target and a source: the passes around
        # the force sweeps, each timed on its own (wall clock, synchronised, mean of 3 after one
        # untimed call). Time-step assignment: pairwise free-fall and fly-by time-steps, jerk,
        # criteria and levels, stable level partition; subsystems: neighbour search, labels, and
        # an acceleration pass with intra-subsystem pairs excluded; the FP64 energy.
        d, _, _ = ics.config5_bh_cluster()
        n = len(d["m"])
        kmax, tau = 7, 1.0 / 4096
        P = bf.Particles.from_numpy(d)

        def wall(fn, reps=3):
            fn()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t) / reps * 1e3

        out = {}
        out["forces_ms"] = wall(lambda: ctx.forces(P, prec="mixed"))
        a = ctx.forces(P, prec="mixed")
        g = ctx.force_gradient(P, a, prec="mixed")
        out["dt_min_ms"] = wall(lambda: ctx.dt_min(P, prec="mixed"))
        out["jerk_ms"] = wall(lambda: ctx.jerk(P, prec="mixed"))
        dff, dfb = ctx.dt_min(P, prec="mixed")
        j = ctx.jerk(P, prec="mixed")
        out["timestep_assign_ms"] = wall(lambda: ctx.timestep_assign(P, None, dff, dfb, a, g, j, tau=tau, kmax=kmax))
        _, lv = ctx.timestep_assign(P, None, dff, dfb, a, g, j, tau=tau, kmax=kmax)
        out["level_partition_ms"] = wall(lambda: ctx.level_partition(None, n, lv, kmax))
        _, counts = ctx.level_partition(None, n, lv, kmax)
        out["neighbours_ms"] = wall(lambda: ctx.neighbours(P, tau=tau))
        edges = ctx.neighbours(P, tau=tau)
        out["subsystems_ms"] = wall(lambda: ctx.subsystems(n, edges))
        label, nsub = ctx.subsystems(n, edges)
        ctx.set_subsystems(label)
        out["forces_excluded_ms"] = wall(lambda: ctx.forces(P, prec="mixed"))
        ctx.set_subsystems(None)
        out["energy_ms"] = wall(lambda: ctx.energy(P))
        rec.update({"workload": name, "n": n, "pairs_per_pass": float(n) * n, "level_counts": [int(c) for c in counts],
                    "neighbour_pairs": int(edges.shape[0]), "subsystems": int(nsub), "ms": out})
    ctx.close()
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--r-fb", type=float, default=0.0,
                    help="radius below which whole tiles are re-evaluated in FP64 (0: off; every pair's "
                         "separation is formed in FP64 in any case)")
    ap.add_argument("--rfb-variant", type=float, default=1e-3,
                    help="also time the sweep with this re-evaluation radius (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--cpu-single-seconds", type=float, default=5.0,
                    help="target time of a one-thread oracle sample (0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--hhs-eager-only", action="store_true",
                    help="bh-hhs workload: time only the eager interval (for kernel traces)")
    ap.add_argument("--hhs-adaptive-only", action="store_true",
                    help="bh-hhs workload: time only the interval with reassigned time-steps (for kernel traces)")
    ap.add_argument("--sample", type=int, default=256, help="targets sampled for the error check")
    ap.add_argument("--spatial-sort", default="default", choices=["default", "off", "acc", "grad", "both", "directed"],
                    help="passes that use the spatially sorted mixed kernels (default: the library's; directed: sorted without the pair-symmetric sweep)")
    ap.add_argument("--kappa", type=float, default=0.0, help="near-tile threshold (0: the library's)")
    ap.add_argument("--autotune", action="store_true",
                    help="run the library autotuner on the workload's own particles before timing")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 2 GiB device-to-device copy kernel first (HBM counter calibration)")
    ap.add_argument("--workload", default="king1m",
                    choices=["king1m", "plummer1k-fsi", "plummer64k-level", "ensemble256", "bh-levels", "bh-hhs",
                             "bh-aux"],
                    help="king1m (default): the headline sweep; the others measure the remaining "
                         "workloads and print their own JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is described, not built)", file=sys.stderr)
        sys.exit(2)
    if args.workload != "king1m":
        run_workload(args.workload, args)
        return

    import torch

    import paper_2210_02472_amd as bf
    from paper_2210_02472_amd import ics

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    t0 = time.time()
    d = ics.king_cluster(ics.rng_for(2), args.n, 6.0, 0.01) if args.n != (1 << 20) else ics.config3_king1m()
    n = args.n
    log(f"generated King W0=6 N={n} in {time.time() - t0:.1f}s")
    P = bf.Particles.from_numpy(d, "cuda:0")
    if args.calib_copy:
        # a plain elementwise copy of known size (2 GiB read, 2 GiB written; larger than the
        # 256 MB last-level cache): its FETCH_SIZE / WRITE_SIZE calibrate the HBM counters
        src = torch.ones(256 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    ctx = bf.Context(0)
    if args.spatial_sort != "default" or args.kappa:
        mode = {"default": (True, True), "off": (False, False), "acc": (True, False), "grad": (False, True),
                "both": (True, True), "directed": (True, True)}[args.spatial_sort]
        ctx.set_spatial_sort(forces=mode[0], gradient=mode[1], kappa=args.kappa,
                             symmetric=args.spatial_sort != "directed")
    out_a = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    if args.autotune:  # on this cluster: the pair-symmetric sweep's shapes
        t1 = time.time()
        ctx.autotune_pass(bf.BF_OP_FORCES, "mixed", P)
        ctx.forces(P, None, None, prec="mixed", out=out_a)
        ctx.autotune_pass(bf.BF_OP_GRADIENT, "mixed", P, acc=out_a)
        log(f"autotuned in {time.time() - t1:.1f}s")
    out_g = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]

    def sweep(prec, r_fb):
        ctx.forces(P, None, None, G=1.0, eps2=0.0, prec=prec, r_fb=r_fb, out=out_a)
        ctx.force_gradient(P, out_a, None, None, G=1.0, eps2=0.0, prec=prec, r_fb=r_fb, out=out_g)

    def timed(prec, steps, warmup, r_fb=args.r_fb):
        for _ in range(warmup):
            sweep(prec, r_fb)
        torch.cuda.synchronize()
        ctx.enable_timing(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            sweep(prec, r_fb)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        ka = ctx.kernel_times(bf.BF_OP_FORCES)
        kg = ctx.kernel_times(bf.BF_OP_GRADIENT)
        ctx.enable_timing(False)
        return wall, ka, kg

    pairs = float(n) * float(n - 1)
    log("mixed sweep ...")
    wall_m, ka_m, kg_m = timed("mixed", args.steps, args.warmup)
    ms_step = wall_m / args.steps * 1e3
    value = pairs / (wall_m / args.steps)
    acc_m = [t.clone() for t in out_a]
    grad_m = [t.clone() for t in out_g]
    log(f"mixed: {ms_step:.1f} ms/step, {value:.4e} pairs/s")
    stats_m = ctx.last_pass_stats()
    rfb_var = None
    if args.rfb_variant > 0:
        log(f"mixed sweep with r_fb = {args.rfb_variant} ...")
        wall_v, ka_v, kg_v = timed("mixed", 2, 1, r_fb=args.rfb_variant)
        rfb_var = {"r_fb": args.rfb_variant, "value": pairs / (wall_v / 2), "ms_per_step": wall_v / 2 * 1e3,
                   "acc_kernel_ms": float(np.mean(ka_v)), "grad_kernel_ms": float(np.mean(kg_v))}
    log("fp64 sweep ...")
    wall_d, ka_d, kg_d = timed("fp64", args.fp64_steps, 1)  # one untimed sweep sizes its scratch first
    ms_fp64 = wall_d / args.fp64_steps * 1e3
    log(f"fp64: {ms_fp64:.1f} ms/step")

    # mixed vs FP64 GPU, all 2^20 targets, per-target relative error.  The acceleration passes
    # see the same positions; the gradient is compared on the same input accelerations (the
    # mixed ones), and separately end to end (each precision on its own accelerations).
    def rel(a, b):
        da = torch.sqrt(sum((x - y) ** 2 for x, y in zip(a, b)))
        nb = torch.sqrt(sum(y ** 2 for y in b))
        e = (da / nb).cpu().numpy()
        return float(np.sqrt(np.mean(e * e))), float(e.max()), int(np.sum(e > 1e-5))
    acc_vs64 = rel(acc_m, out_a)
    grad_e2e = rel(grad_m, out_g)
    g64_same = ctx.force_gradient(P, acc_m, None, None, G=1.0, eps2=0.0, prec="fp64")
    grad_vs64 = rel(grad_m, g64_same)
    del g64_same

    # mixed vs the FP64 CPU oracle on sampled targets (same inputs on both sides)
    import oracle
    Po = oracle.Particles.from_dict(d)
    rng = np.random.default_rng(2210)
    T = np.sort(rng.choice(n, args.sample, replace=False))
    ref_a = oracle.forces(Po, T, None)
    got_a = np.stack([t.cpu().numpy()[T] for t in acc_m], axis=1)
    e_a = np.linalg.norm(got_a - ref_a, axis=1) / np.linalg.norm(ref_a, axis=1)
    af = synthetic_acc_field(d)
    acc_in = [torch.as_tensor(np.ascontiguousarray(af[:, k]), device="cuda") for k in range(3)]
    g = ctx.force_gradient(P, acc_in, None, None, prec="mixed", r_fb=args.r_fb)
    ref_g = oracle.gradient(Po, af, T, None)
    got_g = np.stack([t.cpu().numpy()[T] for t in g], axis=1)
    e_g = np.linalg.norm(got_g - ref_g, axis=1) / np.linalg.norm(ref_g, axis=1)
    flags = ctx.read_flags()

    ctx.force_gradient(P, acc_m, None, None, prec="mixed", r_fb=args.r_fb, out=out_g)
    cfg_g = ctx.last_pass_config()
    ctx.forces(P, None, None, prec="mixed", r_fb=args.r_fb, out=out_a)
    stats_a = ctx.last_pass_stats()
    cfg_a = ctx.last_pass_config()
    avg = lambda v: float(np.mean(v)) if v else float("nan")  # noqa: E731
    ka, kg = avg(ka_m), avg(kg_m)
    grad_tflops = pairs * FLOPS_GRAD / (kg * 1e-3) / 1e12
    acc_tflops = pairs * FLOPS_ACC / (ka * 1e-3) / 1e12

    cpu = None
    if not args.no_cpu_baseline:
        nthreads = oracle.num_threads()
        warm = np.sort(rng.choice(n, 16, replace=False))
        oracle.forces(Po, warm, None)  # thread pool start-up, not timed
        # batches of random targets against all sources until about cpu_seconds have passed
        log(f"cpu oracle sample: batches of 1024 targets x {n} sources on {nthreads} threads ...")
        k, tc = 0, 0.0
        while tc < args.cpu_seconds and k < 65536:
            Ts = np.sort(rng.choice(n, 1024, replace=False))
            t1 = time.perf_counter()
            oracle.forces(Po, Ts, None)
            oracle.gradient(Po, af, Ts, None)
            tc += time.perf_counter() - t1
            k += Ts.size
        cpu = {"value": k * (n - 1) / tc, "unit": "pair interactions/s", "cores": nthreads, "kind": "oracle",
               "sample": f"{k} random targets x all {n} sources, acceleration + force-gradient passes, FP64, "
                         f"{tc:.1f} s"}
        if args.cpu_single_seconds > 0 and nthreads > 1:
            # the same passes on one thread, in smaller batches, for a per-core figure
            log("cpu oracle sample: batches of 64 targets on 1 thread ...")
            oracle.set_num_threads(1)
            try:
                k1, t1c = 0, 0.0
                while t1c < args.cpu_single_seconds and k1 < 4096:
                    Ts = np.sort(rng.choice(n, 64, replace=False))
                    t1 = time.perf_counter()
                    oracle.forces(Po, Ts, None)
                    oracle.gradient(Po, af, Ts, None)
                    t1c += time.perf_counter() - t1
                    k1 += Ts.size
            finally:
                oracle.set_num_threads(nthreads)
            cpu["single_core"] = {"value": k1 * (n - 1) / t1c, "cores": 1,
                                  "sample": f"{k1} random targets x all {n} sources, {t1c:.1f} s"}

    rec = {
        "metric": "pair interactions/s (acc+force-gradient) at N=2^20, mixed vs FP64; rel. err",
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic, f64 accumulate",
        "data": "synthetic",
        "config": {"workload": f"King W0=6 cluster N={n}, Kroupa IMF + 1% binaries as COM particles, Henon units, "
                               f"eps=0, all active; acceleration + force-gradient sweep, mixed precision (pair "
                               f"separations of near tiles formed in FP64 and rounded once, of far tiles from FP32 "
                               f"offsets to the tile centre; FP32 pair arithmetic, FP64 merge and cancellation "
                               f"fix-up)",
                   "n": n, "eps": 0.0, "r_fb": args.r_fb,
                   "fp64_differences": "near tiles (gap to the wavefront's rows below kappa x tile half-extent, "
                                       "kappa = 1, and the diagonal tiles); far-tile separations come from FP32 "
                                       "offsets to the tile centre, relative error <= u (1 + 2 sqrt(3) / kappa) "
                                       "= 4.5 u at every separation, pairs at r < 1e-3 included",
                   "autotuned": bool(args.autotune),
                   "acc_pass": pass_desc(cfg_a), "grad_pass": pass_desc(cfg_g)},
        "roofline": {"bound": "alu",
                     "kernel": KERNEL_NAMES[cfg_g[0]] + " (force-gradient pass)",
                     "achieved": grad_tflops, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": grad_tflops / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic(n, cfg_g),
                     "flops_per_pair": FLOPS_GRAD, "pairs_per_launch": pairs,
                     "pair_evaluations_per_launch": pairs // 2 if cfg_g[0] == "symmetric" else pairs,
                     "avg_kernel_ms": kg},
        "acc_pass": {"avg_kernel_ms": ka, "tflops": acc_tflops, "frac": acc_tflops / PEAK_FP32_TFLOPS,
                     "pairs_per_s": pairs / (ka * 1e-3)},
        "fp64": {"ms_per_step": ms_fp64, "value": pairs / (wall_d / args.fp64_steps),
                 "acc_kernel_ms": avg(ka_d), "grad_kernel_ms": avg(kg_d),
                 "frac_fp64_peak": pairs * (FLOPS_ACC + FLOPS_GRAD) / ((avg(ka_d) + avg(kg_d)) * 1e-3) / 1e12 / PEAK_FP64_TFLOPS},
        "sweep_frac_fp32_peak": pairs * (FLOPS_ACC + FLOPS_GRAD) / (wall_m / args.steps) / 1e12 / PEAK_FP32_TFLOPS,
        "speedup_vs_fp64": ms_fp64 / ms_step,
        "rel_err": {"acc_vs_oracle_rms": float(np.sqrt(np.mean(e_a ** 2))), "acc_vs_oracle_max": float(e_a.max()),
                    "grad_vs_oracle_rms": float(np.sqrt(np.mean(e_g ** 2))), "grad_vs_oracle_max": float(e_g.max()),
                    "oracle_sample_targets": int(args.sample),
                    "acc_vs_fp64_gpu_rms": acc_vs64[0], "acc_vs_fp64_gpu_max": acc_vs64[1],
                    "acc_vs_fp64_gpu_n_above_1e-5": acc_vs64[2],
                    "grad_vs_fp64_gpu_rms": grad_vs64[0], "grad_vs_fp64_gpu_max": grad_vs64[1],
                    "grad_vs_fp64_gpu_n_above_1e-5": grad_vs64[2],
                    "grad_end_to_end_vs_fp64_gpu_rms": grad_e2e[0], "grad_end_to_end_vs_fp64_gpu_max": grad_e2e[1]},
        "fixups": {"acc": stats_a[0], "grad": stats_m[0]},
        "rfb_variant": rfb_var,
        "device_flags": flags,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
