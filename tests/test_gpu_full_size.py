"""Parity at the full sizes of the measured workloads, in the launch configuration bench.py
times (library defaults: spatially sorted mixed passes), on sampled outputs the oracle computes
one by one:

  * King W0 = 6, N = 2^20, all active (the headline sweep): acceleration and gradient on
    sampled targets against the oracle; every target against the all-FP64 GPU path, and the 64
    targets farthest from it against the oracle;
  * Kroupa Plummer N = 65,536 with a random 10% level, eps = 1e-4: acceleration, gradient and
    time-steps of every active particle;
  * 256-cluster ensemble (about 3.9 million particles): batched accelerations and gradient sums
    of sampled clusters, and one graph-captured batched FSI cycle against the oracle's cycle on
    16 sampled clusters;
  * N = 262,144 cluster with 16 BHs and an IMBH: the deepest level's accelerations and PN1.0; the
    inter-level sums (both directions, accelerations and gradient) at the shapes of levels 0 and
    3; PN1.0 of sampled level-0 particles.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2210_02472_amd import ics
from tests._parity import assert_state_close, gather, rel_errors, smooth_acc_field, stats

bf = pytest.importorskip("paper_2210_02472_amd")

pytestmark = pytest.mark.gpu

RMS_TOL, MAX_TOL = 1e-6, 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = bf.Context(0)
    yield c
    c.close()


def _check_mixed(got, ref):
    rms, mx = stats(rel_errors(got, ref))
    assert rms <= RMS_TOL and mx <= MAX_TOL, (rms, mx)


def test_king_2e20_sweep_sampled(ctx):
    d = ics.config3_king1m()
    n = len(d["m"])
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    T = np.sort(np.random.default_rng(31).choice(n, 48, replace=False))
    a = ctx.forces(Pd, prec="mixed", r_fb=0.0)
    _check_mixed(gather(a, T), oracle.forces(P, T, None))
    af = smooth_acc_field(d)
    g = ctx.force_gradient(Pd, [torch.as_tensor(np.ascontiguousarray(af[:, k]), device="cuda") for k in range(3)],
                           prec="mixed", r_fb=0.0)
    _check_mixed(gather(g, T), oracle.gradient(P, af, T, None))
    # the time-step pass over the whole set (pair-symmetric), sampled
    ff, fb = ctx.dt_min(Pd, eta_ff=0.2, eta_fb=0.2, prec="mixed")
    assert ctx.last_pass_config()[0] == "symmetric"
    rff, rfb = oracle.dt_min(P, T, None, eta_ff=0.2, eta_fb=0.2)
    np.testing.assert_allclose(ff.cpu().numpy()[T], rff, rtol=1e-6)
    np.testing.assert_allclose(fb.cpu().numpy()[T], rfb, rtol=1e-6)
    # a 4 GiB scratch limit: the acceleration sweep's 16 shares of 33 block distances in passes
    try:
        ctx.set_symmetric_scratch_limit(4 << 30)
        a2 = ctx.forces(Pd, prec="mixed", r_fb=0.0)
        passes = ctx.last_symmetric_passes()
    finally:
        ctx.set_symmetric_scratch_limit(0)
    assert passes >= 2, passes
    assert all(torch.equal(x, y) for x, y in zip(a, a2))
    assert ctx.read_flags() == 0


def test_plummer_64k_level_all_active_targets(ctx):
    d, act = ics.config2_plummer64k()
    n = len(d["m"])
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    T = torch.as_tensor(act, device="cuda")
    eps2 = 1e-8
    a = ctx.forces(Pd, T, None, eps2=eps2, prec="mixed", r_fb=0.0)
    _check_mixed(gather(a, act), oracle.forces(P, act, None, eps2=eps2))
    af = smooth_acc_field(d)
    g = ctx.force_gradient(Pd, [torch.as_tensor(np.ascontiguousarray(af[:, k]), device="cuda") for k in range(3)],
                           T, None, eps2=eps2, prec="mixed", r_fb=0.0)
    _check_mixed(gather(g, act), oracle.gradient(P, af, act, None, eps2=eps2))
    ff, fb = ctx.dt_min(Pd, T, None, eta_ff=0.2, eta_fb=0.2, prec="mixed")
    rff, rfb = oracle.dt_min(P, act, None, eta_ff=0.2, eta_fb=0.2)
    np.testing.assert_allclose(ff.cpu().numpy()[act], rff, rtol=1e-6)
    np.testing.assert_allclose(fb.cpu().numpy()[act], rfb, rtol=1e-6)
    assert ctx.read_flags() == 0


def test_ensemble_256_sampled_clusters(ctx):
    d, off, act, aoff = ics.config4_ensemble()
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    co, ai, ao = (torch.as_tensor(x, device="cuda") for x in (off, act, aoff))
    sizes = np.diff(off)
    a = ctx.forces_batched(Pd, co, ai, ao, int(aoff[-1]), int(sizes.max()), eps2=1e-8, prec="mixed", r_fb=0.0)
    rng = np.random.default_rng(32)
    for c in rng.choice(len(sizes), 6, replace=False):
        T = act[aoff[c]:aoff[c + 1]].astype(np.int64)
        if T.size > 512:
            T = np.sort(rng.choice(T, 512, replace=False))
        src = np.arange(off[c], off[c + 1])
        _check_mixed(gather(a, T), oracle.forces(P, T, src, eps2=1e-8))
    assert ctx.read_flags() == 0


def test_bh_cluster_deepest_level(ctx):
    d, bh, lv = ics.config5_bh_cluster()
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    idx = np.nonzero(lv >= lv.max())[0]
    T = torch.as_tensor(idx.astype(np.int32), device="cuda")
    a = ctx.forces(Pd, T, None, prec="mixed", r_fb=0.0)
    _check_mixed(gather(a, idx), oracle.forces(P, idx, None))
    p = ctx.pn1_bh(Pd, torch.as_tensor(bh, device="cuda"), T, None, c=1e4)
    ref = oracle.pn1(P, bh, idx, None, c=1e4)
    got = gather(p, idx)
    scale = np.linalg.norm(ref, axis=1).max()
    assert np.abs(got - ref).max() <= 1e-12 * scale
    assert ctx.read_flags() == 0


def _dev_field(af):
    return [torch.as_tensor(np.ascontiguousarray(af[:, k]), device="cuda") for k in range(3)]


def test_king_2e20_all_targets_vs_fp64_gpu(ctx):
    """Every one of the 2^20 targets, mixed against the all-FP64 GPU path (itself within 1e-12 of
    the oracle wherever both are compared): relative RMS <= 1e-6 and max <= 1e-5 for the
    acceleration and the gradient (same input accelerations on both sides).  The 64 targets with
    the largest mixed-vs-FP64 error of each pass are then compared with the oracle itself."""
    d = ics.config3_king1m()
    n = len(d["m"])
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    am = ctx.forces(Pd, prec="mixed", r_fb=0.0)
    a64 = ctx.forces(Pd, prec="fp64")
    af = smooth_acc_field(d)
    acc_in = _dev_field(af)
    gm = ctx.force_gradient(Pd, acc_in, prec="mixed", r_fb=0.0)
    g64 = ctx.force_gradient(Pd, acc_in, prec="fp64")
    for got, ref, what in ((am, a64, "acc"), (gm, g64, "grad")):
        gn = np.stack([t.cpu().numpy() for t in got], axis=1)
        rn = np.stack([t.cpu().numpy() for t in ref], axis=1)
        e = rel_errors(gn, rn)
        rms, mx = stats(e)
        assert rms <= RMS_TOL and mx <= MAX_TOL, (what, rms, mx)
        worst = np.sort(np.argsort(e)[-64:])
        oref = oracle.forces(P, worst, None) if what == "acc" else oracle.gradient(P, af, worst, None)
        # the worst targets by construction: each within the max bound (the RMS bound is the
        # all-target one above)
        ew = rel_errors(gn[worst], oref)
        assert ew.max() <= MAX_TOL, (what, ew.max())
        # and the FP64 GPU path on the same targets against the oracle
        assert np.all(rel_errors(rn[worst], oref) <= 1e-12), what
    del am, a64, gm, g64
    assert ctx.read_flags() == 0


def test_ensemble_256_gradient_sampled_clusters(ctx):
    """Batched force-gradient sums over the 256-cluster ensemble (input accelerations: a smooth
    field, the same on both sides) against the oracle on sampled clusters."""
    d, off, act, aoff = ics.config4_ensemble()
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    co, ai, ao = (torch.as_tensor(x, device="cuda") for x in (off, act, aoff))
    sizes = np.diff(off)
    af = smooth_acc_field(d)
    g = ctx.force_gradient_batched(Pd, co, ai, ao, int(aoff[-1]), int(sizes.max()), _dev_field(af), eps2=1e-8,
                                   prec="mixed", r_fb=0.0)
    rng = np.random.default_rng(33)
    for c in rng.choice(len(sizes), 16, replace=False):
        T = act[aoff[c]:aoff[c + 1]].astype(np.int64)
        if T.size > 512:
            T = np.sort(rng.choice(T, 512, replace=False))
        src = np.arange(off[c], off[c + 1])
        _check_mixed(gather(g, T), oracle.gradient(P, af, T, src, eps2=1e-8))
    assert ctx.read_flags() == 0


class _State:
    """x, y, z, vx, vy, vz of the particles T of a state (device or host)."""

    def __init__(self, o, T):
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            v = getattr(o, k)
            setattr(self, k, (v.cpu().numpy() if hasattr(v, "cpu") else np.asarray(v))[T])


def _oracle_batched_cycle(P, acc, T, src, dt, eps2):
    """The FSI cycle that bf_fsi_step_batched documents, for one cluster, from oracle passes:
    active particles T, every particle of the cluster (src) a source, inactive ones frozen; acc
    (n x 3) holds the accelerations on entry (updated for T)."""
    def kick(a, h):
        P.vx[T] += h * a[:, 0]; P.vy[T] += h * a[:, 1]; P.vz[T] += h * a[:, 2]

    def drift(h):
        P.x[T] += h * P.vx[T]; P.y[T] += h * P.vy[T]; P.z[T] += h * P.vz[T]
    kick(acc[T], dt / 6.0)
    drift(0.5 * dt)
    acc[T] = oracle.forces(P, T, src, eps2=eps2)
    gs = oracle.gradient(P, acc, T, src, eps2=eps2)
    kick(acc[T] + (dt * dt / 24.0) * gs, 2.0 * dt / 3.0)
    drift(0.5 * dt)
    acc[T] = oracle.forces(P, T, src, eps2=eps2)
    kick(acc[T], dt / 6.0)


def test_ensemble_256_graph_fsi_cycle_sampled_clusters(ctx):
    """One replay of the graph-captured batched FSI cycle over the 256-cluster ensemble (mixed,
    eps = 1e-4) against the oracle's cycle on 16 sampled clusters (among those whose cycle the
    oracle runs in about a second): per particle, position and velocity within 1e-5 of the
    particle's own change, and the new accelerations of the active particles within the mixed
    tolerance.  Entry accelerations: a smooth field, the same on both sides."""
    d, off, act, aoff = ics.config4_ensemble()
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    P0 = P.copy()
    co, ai, ao = (torch.as_tensor(x, device="cuda") for x in (off, act, aoff))
    sizes, nact = np.diff(off), np.diff(aoff)
    af = smooth_acc_field(d)
    acc = _dev_field(af)
    dt, eps2 = 1e-3, 1e-8
    g = ctx.capture_batched_fsi(Pd, co, ai, ao, int(aoff[-1]), int(sizes.max()), dt, acc, eps2=eps2, prec="mixed")
    g.launch()
    torch.cuda.synchronize()
    g.close()
    assert ctx.read_flags() & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0
    rng = np.random.default_rng(34)
    cand = np.nonzero(sizes.astype(np.float64) * nact <= 2.5e8)[0]
    got_acc = np.stack([t.cpu().numpy() for t in acc], axis=1)
    ref_acc = af.copy()
    for c in np.sort(rng.choice(cand, 16, replace=False)):
        T = act[aoff[c]:aoff[c + 1]].astype(np.int64)
        src = np.arange(off[c], off[c + 1])
        _oracle_batched_cycle(P, ref_acc, T, src, dt, eps2)
        assert_state_close(_State(Pd, T), _State(P, T), _State(P0, T), MAX_TOL)
        _check_mixed(got_acc[T], ref_acc[T])


def test_bh_cluster_interlevel_sums_and_pn(ctx):
    """The 262,144-body cluster with its levels: the inter-level sums S <- F and F <- S that the
    hierarchy's kicks use (bf_forces_between, bf_force_gradient_between with a smooth input
    field), at the shapes of level 0 (S = level 0, F = deeper: both about 131,000 particles, the
    two-set symmetric sweep) and level 3 (about 16,000 each), on sampled particles of both sets
    against the oracle; and PN1.0 of sampled level-0 particles from all particles (FP64)."""
    d, bh, lv = ics.config5_bh_cluster()
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    af = smooth_acc_field(d)
    acc_in = _dev_field(af)
    rng = np.random.default_rng(35)
    for k in (0, 3):
        S = np.nonzero(lv == k)[0].astype(np.int32)
        F = np.nonzero(lv > k)[0].astype(np.int32)
        Sd, Fd = torch.as_tensor(S, device="cuda"), torch.as_tensor(F, device="cuda")
        a = ctx.forces_between(Pd, Sd, Fd, prec="mixed")
        gs = ctx.force_gradient_between(Pd, acc_in, Sd, Fd, prec="mixed")
        for A, B in ((S, F), (F, S)):
            T = np.sort(rng.choice(A, 128, replace=False))
            _check_mixed(gather(a, T), oracle.forces(P, T, B))
            _check_mixed(gather(gs, T), oracle.gradient(P, af, T, B))
    T = np.sort(rng.choice(np.nonzero(lv == 0)[0], 256, replace=False)).astype(np.int32)
    p = ctx.pn1_bh(Pd, torch.as_tensor(bh, device="cuda"), torch.as_tensor(T, device="cuda"), None, c=1e4)
    ref = oracle.pn1(P, bh, T, None, c=1e4)
    got = gather(p, T)
    assert np.all(np.linalg.norm(got - ref, axis=1) <= 1e-12 * np.linalg.norm(ref, axis=1))
    assert ctx.read_flags() == 0
