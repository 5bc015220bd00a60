"""GPU parity of the time-step assignment (jerk, gradient and pairwise criteria, levels), the
level partition and the device HHS-FSI interval driver against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2210_02472_amd import ics
from tests._parity import assert_state_close, gather, rel_errors, stats

bf = pytest.importorskip("paper_2210_02472_amd")

pytestmark = pytest.mark.gpu

RMS_TOL, MAX_TOL = 1e-6, 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = bf.Context(0)
    yield c
    c.close()


def _cluster(n, seed):
    return ics.plummer_cluster(ics.rng_for(300, seed), n, "kroupa")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_jerk_parity(ctx, prec):
    d = _cluster(2500, 1)
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    ref = oracle.jerk(P)
    got = gather(ctx.jerk(Pd, prec=prec), np.arange(2500))
    if prec == "fp64":
        _, mag, _ = oracle.gradient(P, P.vel(), return_mag=True)
        assert np.all(np.linalg.norm(got - ref, axis=1) <= 1e-12 * mag)
    else:
        rms, mx = stats(rel_errors(got, ref))
        assert rms <= RMS_TOL and mx <= MAX_TOL, (rms, mx)


def test_timestep_assign_parity(ctx):
    """The whole assignment in FP64: dt to 1e-12 relative; levels equal except where dt lies
    within that tolerance of a pivot (where both sides may round to different sides)."""
    n, kmax, tau = 3000, 7, 0.05
    d = _cluster(n, 2)
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    idx = np.arange(n)
    ff, fb = oracle.dt_min(P, eta_ff=0.2, eta_fb=0.2)
    a = oracle.forces(P)
    g = oracle.gradient(P, a)
    j = oracle.jerk(P)
    dt_ref = oracle.timestep_criteria(P, idx, ff, fb, a, g, j, eta_grad=0.1, eta_jerk=0.1)
    lv_ref = oracle.levels_from_dt(dt_ref, tau, kmax)

    dff, dfb = ctx.dt_min(Pd, eta_ff=0.2, eta_fb=0.2, prec="fp64")
    ad = ctx.forces(Pd, prec="fp64")
    gd = ctx.force_gradient(Pd, ad, prec="fp64")
    jd = ctx.jerk(Pd, prec="fp64")
    dt, lv = ctx.timestep_assign(Pd, None, dff, dfb, ad, gd, jd, eta_grad=0.1, eta_jerk=0.1, tau=tau, kmax=kmax)
    dt, lv = dt.cpu().numpy(), lv.cpu().numpy()
    np.testing.assert_allclose(dt, dt_ref, rtol=1e-12)
    pivots = tau / 2.0 ** np.arange(kmax + 1)
    near_pivot = np.min(np.abs(dt_ref[:, None] / pivots[None, :] - 1.0), axis=1) < 1e-11
    assert np.array_equal(lv[~near_pivot], lv_ref[~near_pivot])
    assert lv.min() >= 0 and lv.max() <= kmax


def test_timestep_assign_mixed_parity(ctx):
    """The assignment from mixed-precision passes (free-fall / fly-by time-steps, acceleration,
    gradient and jerk; the epilogue itself is FP64) against the FP64 oracle: time-steps within
    relative RMS 1e-6 and max 1e-5 (the criteria are powers 1/2 and 1/3 of the mixed results'
    ratios, whose errors stay below 1e-5); levels equal except where the oracle's time-step lies
    within 1e-5 of a pivot."""
    n, kmax, tau = 3000, 7, 0.05
    d = _cluster(n, 2)
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    idx = np.arange(n)
    ff, fb = oracle.dt_min(P, eta_ff=0.2, eta_fb=0.2)
    a = oracle.forces(P)
    g = oracle.gradient(P, a)
    j = oracle.jerk(P)
    dt_ref = oracle.timestep_criteria(P, idx, ff, fb, a, g, j, eta_grad=0.1, eta_jerk=0.1)
    lv_ref = oracle.levels_from_dt(dt_ref, tau, kmax)
    dff, dfb = ctx.dt_min(Pd, eta_ff=0.2, eta_fb=0.2, prec="mixed")
    ad = ctx.forces(Pd, prec="mixed")
    gd = ctx.force_gradient(Pd, ad, prec="mixed")
    jd = ctx.jerk(Pd, prec="mixed")
    dt, lv = ctx.timestep_assign(Pd, None, dff, dfb, ad, gd, jd, eta_grad=0.1, eta_jerk=0.1, tau=tau, kmax=kmax)
    dt, lv = dt.cpu().numpy(), lv.cpu().numpy()
    e = np.abs(dt / dt_ref - 1.0)
    assert np.sqrt(np.mean(e * e)) <= 1e-6 and e.max() <= 1e-5, (np.sqrt(np.mean(e * e)), e.max())
    pivots = tau / 2.0 ** np.arange(kmax + 1)
    near_pivot = np.min(np.abs(dt_ref[:, None] / pivots[None, :] - 1.0), axis=1) < 1e-5
    assert np.array_equal(lv[~near_pivot], lv_ref[~near_pivot])
    assert ctx.read_flags() & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0


def test_level_partition_is_stable_sort(ctx):
    n, kmax = 5000, 6
    rng = np.random.default_rng(4)
    level = rng.integers(0, kmax + 1, n).astype(np.int32)
    sub = np.sort(rng.choice(n, 3000, replace=False)).astype(np.int32)
    lv = torch.as_tensor(level, device="cuda")
    order, counts = ctx.level_partition(sub, n, lv, kmax)
    ref = sub[np.argsort(level[sub], kind="stable")]
    assert np.array_equal(order.cpu().numpy(), ref)
    assert counts == [int(np.sum(level[sub] == k)) for k in range(kmax + 1)]
    order, counts = ctx.level_partition(None, n, lv, kmax)
    assert np.array_equal(order.cpu().numpy(), np.argsort(level, kind="stable"))
    # many workgroups and a ragged tail, every level up to the largest kmax, most particles on
    # level 0 (the counts are gathered per workgroup, then added once per level)
    n, kmax = 300001, 63
    level = np.minimum(rng.geometric(0.7, n) - 1, kmax).astype(np.int32)
    level[rng.choice(n, kmax + 1, replace=False)] = np.arange(kmax + 1, dtype=np.int32)
    lv = torch.as_tensor(level, device="cuda")
    order, counts = ctx.level_partition(None, n, lv, kmax)
    assert counts == np.bincount(level, minlength=kmax + 1).tolist()
    assert np.array_equal(order.cpu().numpy(), np.argsort(level, kind="stable"))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_hhs_interval_parity(ctx, prec):
    """One HHS-FSI interval with four populated levels (and an empty one) on the device against the
    oracle recursion.  FP64: state to 1e-12 of its scale; mixed: per particle, position and
    velocity within 1e-5 of the particle's own change (floor: 1e-3 of the largest change)."""
    n = 900
    d = _cluster(n, 3)
    rng = np.random.default_rng(5)
    level = rng.choice([0, 1, 2, 4], size=n, p=[0.5, 0.25, 0.15, 0.10]).astype(np.int32)
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    P0 = P.copy()
    tau = 2e-3
    oracle.hhs_interval(P, level, tau)
    ctx.hhs_interval(Pd, torch.as_tensor(level, device="cuda"), 4, tau, prec=prec)
    if prec == "mixed":
        assert_state_close(Pd, P, P0, MAX_TOL)
    else:
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            ref = getattr(P, k)
            got = getattr(Pd, k).cpu().numpy()
            assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), k
    assert ctx.read_flags() & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0


def _hhs_composed(ctx, P, level, kmax, tau, prec):
    """The fixed-level interval (the cycle documented for bf_hhs_interval) composed from the
    public passes, every acceleration recomputed where the cycle needs it."""
    n = P.n
    order, counts = ctx.level_partition(None, n, level, kmax)
    begin = np.concatenate([[0], np.cumsum(counts)]).astype(int)
    total = int(begin[-1])
    z3 = lambda: [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    asf, gsf, afsi = z3(), z3(), z3()

    def rec(k, t):
        sb, fb = int(begin[k]), int(begin[k + 1]) if k < kmax else total
        S, F, B = order[sb:fb], order[fb:total], order[sb:total]
        if F.numel() == 0:
            if S.numel():
                ctx.fsi_step(P, t, S, prec=prec, acc=afsi)
            return
        if S.numel() == 0:
            rec(k + 1, 0.5 * t)
            rec(k + 1, 0.5 * t)
            return
        ctx.forces_between(P, S, F, prec=prec, out=asf)
        ctx.kick(P, B, t / 6.0, asf)
        ctx.fsi_step(P, 0.5 * t, S, prec=prec, acc=afsi)
        rec(k + 1, 0.5 * t)
        ctx.forces_between(P, S, F, prec=prec, out=asf)
        ctx.force_gradient_between(P, asf, S, F, prec=prec, out=gsf)
        ctx.kick(P, B, 2.0 * t / 3.0, asf, h2=t * t / 24.0, grad=gsf)
        rec(k + 1, 0.5 * t)
        ctx.fsi_step(P, 0.5 * t, S, prec=prec, acc=afsi)
        ctx.forces_between(P, S, F, prec=prec, out=asf)
        ctx.kick(P, B, t / 6.0, asf)

    rec(0, tau)


@pytest.mark.parametrize("prec,mode", [("fp64", "default"), ("mixed", "default"), ("mixed", "sorted-any-size")])
def test_hhs_interval_reuse_matches_composed_passes(ctx, prec, mode):
    """The driver keeps each level's own and inter-level accelerations between its visits
    instead of recomputing them; the interval must equal, bit for bit, the same cycle composed
    from the public passes with every acceleration recomputed (mixed with the sorted mode at
    every size: pair-symmetric and two-set sweeps on every level)."""
    n, kmax, tau = 1500, 5, 1e-3
    d = _cluster(n, 16)
    level = np.random.default_rng(17).choice([0, 1, 2, 3, 5], size=n, p=[0.4, 0.25, 0.15, 0.1, 0.1])
    lv = torch.as_tensor(level.astype(np.int32), device="cuda")
    A, B = bf.Particles.from_numpy(d), bf.Particles.from_numpy(d)
    try:
        if mode == "sorted-any-size":
            ctx.set_spatial_sort(forces=True, gradient=True, any_size=True)
        for _ in range(2):
            ctx.hhs_interval(A, lv, kmax, tau, prec=prec)
            _hhs_composed(ctx, B, lv, kmax, tau, prec)
            for k in ("x", "y", "z", "vx", "vy", "vz"):
                assert torch.equal(getattr(A, k), getattr(B, k)), k
    finally:
        ctx.set_spatial_sort(forces=True, gradient=True)
    assert ctx.read_flags() & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0


def test_hhs_single_level_matches_fsi(ctx):
    d = _cluster(700, 6)
    A, B = bf.Particles.from_numpy(d), bf.Particles.from_numpy(d)
    lv = torch.zeros(700, dtype=torch.int32, device="cuda")
    ctx.hhs_interval(A, lv, 3, 1e-3, prec="fp64")
    ctx.fsi_step(B, 1e-3, prec="fp64")
    for k in ("x", "vy"):
        assert torch.allclose(getattr(A, k), getattr(B, k), rtol=0, atol=1e-15)


def _stale_visits(trace):
    """Visits of a level whose slow and fast lists equal those of its previous visit although a
    shallower level changed its split or ran with an empty fast set in between (so particles of
    the level may have drifted): the visits at which keeping the level's accelerations would be
    wrong.  `trace` is the oracle's visiting-order trace with the lists."""
    last, dropped, hits = {}, set(), 0
    for k, _, _, nf, _, S, F in trace:
        prev = last.get(k)
        same = prev is not None and np.array_equal(prev[0], S) and np.array_equal(prev[1], F)
        hits += same and k in dropped
        dropped.discard(k)
        if not same or nf == 0:
            dropped.update(range(k + 1, 64))
        last[k] = (S, F)
    return hits


def _adaptive_case():
    """A softened Kroupa Plummer sphere whose adaptive interval reaches level 6, where the
    gradient and jerk criteria change the levels' splits and where level lists repeat after a
    shallower level changed (every time-step the oracle compares lies at least 4e-4 of the pivot
    away from it)."""
    n, kmax, tau, eta, eta_gj, eps2 = 700, 6, 1.0 / 64, 0.05, 0.1, 1e-6
    d = _cluster(n, 9)
    P = oracle.Particles.from_dict(d)
    ff, fb = oracle.dt_min(P, eta_ff=eta, eta_fb=eta)
    return d, np.minimum(ff, fb), dict(kmax=kmax, tau=tau, eta=eta, eta_gj=eta_gj, eps2=eps2)


def _oracle_adaptive(d, dt0, c, eta_gj=None):
    P = oracle.Particles.from_dict(d)
    trace = []
    e = c["eta_gj"] if eta_gj is None else eta_gj
    oracle.hhs_interval_adaptive(P, dt0, c["tau"], c["kmax"], c["eta"], c["eta"], eta_grad=e, eta_jerk=e,
                                 eps2=c["eps2"], trace=trace)
    return P, trace


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_hhs_adaptive_parity(ctx, prec):
    """The adaptive interval (every level assigns its particles' time-steps from the free-fall,
    fly-by, gradient and jerk criteria over its own particles, capped by the initial ones)
    against the oracle recursion.  Both sides must take the same slow / fast decisions, so the
    case is one where every time-step the oracle compares lies clear of its pivot (relative gap
    > 1e-9 in FP64, > 1e-4 in mixed precision).  The case is checked to be one where the
    gradient and jerk criteria decide splits and where lists repeat after a shallower level
    changed.  Mixed states are compared per particle against the particle's own change over
    the interval."""
    d, dt0, c = _adaptive_case()
    P, trace = _oracle_adaptive(d, dt0, c)
    _, trace_ff_fb = _oracle_adaptive(d, dt0, c, eta_gj=0.0)
    assert [t[:4] for t in trace] != [t[:4] for t in trace_ff_fb]
    assert _stale_visits(trace) > 0
    gap = min(t[4] for t in trace)
    assert gap > (1e-9 if prec == "fp64" else 1e-4), gap
    assert max(t[0] for t in trace) >= 3
    P0 = oracle.Particles.from_dict(d)
    Pd = bf.Particles.from_numpy(d)
    ml, nl = ctx.hhs_interval_adaptive(Pd, torch.as_tensor(dt0, device="cuda"), c["kmax"], c["tau"], c["eta"],
                                       c["eta"], c["eta_gj"], c["eta_gj"], eps2=c["eps2"], prec=prec)
    assert (ml, nl) == (max(t[0] for t in trace), len(trace))
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        ref = getattr(P, k)
        got = getattr(Pd, k).cpu().numpy()
        if prec == "fp64":
            assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), k
        else:
            change = np.abs(ref - getattr(P0, k))
            bound = MAX_TOL * (change + 1e-3 * change.max())
            worst = int(np.argmax(np.abs(got - ref) / bound))
            assert np.all(np.abs(got - ref) <= bound), (k, worst, got[worst] - ref[worst], change[worst])
    assert ctx.read_flags() & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_hhs_adaptive_reuse_matches_recompute(ctx, prec):
    """The adaptive driver keeps a level's accelerations between visits only while no
    shallower level changed its split or emptied its fast set; on a case where level lists
    repeat after such a change, the interval with kept accelerations equals, bit for bit, the
    one that recomputes every acceleration."""
    d, dt0, c = _adaptive_case()
    _, trace = _oracle_adaptive(d, dt0, c)
    assert _stale_visits(trace) > 0
    A, B = bf.Particles.from_numpy(d), bf.Particles.from_numpy(d)
    t0 = torch.as_tensor(dt0, device="cuda")
    args = (c["kmax"], c["tau"], c["eta"], c["eta"], c["eta_gj"], c["eta_gj"])
    try:
        ctx.set_hhs_reuse(True)
        ra = ctx.hhs_interval_adaptive(A, t0, *args, eps2=c["eps2"], prec=prec)
        ctx.set_hhs_reuse(False)
        rb = ctx.hhs_interval_adaptive(B, t0, *args, eps2=c["eps2"], prec=prec)
    finally:
        ctx.set_hhs_reuse(True)
    assert ra == rb
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert torch.equal(getattr(A, k), getattr(B, k)), k


def test_hhs_adaptive_fixed_level_equivalence(ctx):
    """With huge eta the level-0 cap decides every level, and the adaptive driver reproduces the
    fixed-level driver on the device (to FP64 rounding: the fast sets are held in a different
    order, so sums run in a different order)."""
    n, tau = 800, 2e-3
    d = _cluster(n, 10)
    lv = np.random.default_rng(12).choice([0, 1, 2, 3], size=n, p=[0.4, 0.3, 0.2, 0.1]).astype(np.int32)
    A, B = bf.Particles.from_numpy(d), bf.Particles.from_numpy(d)
    dt0 = torch.as_tensor(1.5 * tau / 2.0 ** lv, device="cuda")
    ml, _ = ctx.hhs_interval_adaptive(A, dt0, 5, tau, 1e9, 1e9, 1e9, 1e9, prec="fp64")
    ctx.hhs_interval(B, torch.as_tensor(lv, device="cuda"), 5, tau, prec="fp64")
    assert ml == 3
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        a, b = getattr(A, k), getattr(B, k)
        assert (a - b).abs().max().item() <= 1e-13 * b.abs().max().item(), k


@pytest.mark.parametrize("prec,mode", [("fp64", "unsorted"), ("mixed", "unsorted"), ("fp64", "any-size"),
                                       ("mixed", "any-size")])
def test_hhs_interval_graph_replays_match_eager(ctx, prec, mode):
    """One fixed-level interval captured into a HIP graph and replayed three times, with eager
    work and synchronisation between the replays, against three eager intervals on a copy of the
    state: equal bit for bit after every replay.  "unsorted": the sorted mode off on both sides;
    "any-size": the sorted mode at every size, so that the graph holds Morton sorts (a merge sort
    inside the graph, the radix sort eager), pair-symmetric sweeps (mixed and FP64) and two-set
    sweeps."""
    n, kmax, tau = 3000, 4, 1e-3
    d = _cluster(n, 11)
    level = np.random.default_rng(14).choice([0, 1, 2, 4], size=n, p=[0.4, 0.3, 0.2, 0.1]).astype(np.int32)
    lv = torch.as_tensor(level, device="cuda")
    A, B = bf.Particles.from_numpy(d), bf.Particles.from_numpy(d)
    try:
        if mode == "unsorted":
            ctx.set_spatial_sort(forces=False, gradient=False)
        else:
            ctx.set_spatial_sort(forces=True, gradient=True, any_size=True)
        g = ctx.capture_hhs_interval(A, lv, kmax, tau, prec=prec)
        for _ in range(3):
            g.launch()
            ctx.hhs_interval(B, lv, kmax, tau, prec=prec)
            ctx.forces(bf.Particles.from_numpy(d), prec=prec)  # unrelated eager work in between
            torch.cuda.synchronize()
            for k in ("x", "y", "z", "vx", "vy", "vz"):
                assert torch.equal(getattr(A, k), getattr(B, k)), k
        g.close()
    finally:
        ctx.set_spatial_sort(forces=True, gradient=True)
    assert ctx.read_flags() & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0


def test_hhs_interval_with_pn_parity(ctx):
    """A fixed-level interval with black holes on the deepest level and PN1.0 (FP64, c = 30):
    the device driver against the oracle recursion with the same placement of the PN kicks
    (each FSI cycle over its own pairs, each level's cycle over its inter-level pairs)."""
    n = 900
    d = _cluster(n, 13)
    bh = np.array([3, 100, 450], dtype=np.int32)
    d["m"][bh] *= 50.0
    rng = np.random.default_rng(15)
    level = rng.choice([0, 1, 2], size=n, p=[0.6, 0.3, 0.1]).astype(np.int32)
    level[bh] = 2
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    tau = 2e-3
    oracle.hhs_interval(P, level, tau, bh=bh, c=30.0)
    ctx.hhs_interval(Pd, torch.as_tensor(level, device="cuda"), 2, tau, prec="fp64", bh=bh, c=30.0)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        ref = getattr(P, k)
        got = getattr(Pd, k).cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), k


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_hhs_interval_with_pn_graph_replays_match_eager(ctx, prec):
    """A fixed-level interval with black holes and PN1.0 kicks captured into a HIP graph and
    replayed three times (eager work and synchronisation in between) against three eager
    intervals on a copy of the state: equal bit for bit after every replay; the first replay also
    against the oracle recursion (FP64)."""
    n = 900
    d = _cluster(n, 13)
    bh = np.array([3, 100, 450], dtype=np.int32)
    d["m"][bh] *= 50.0
    rng = np.random.default_rng(15)
    level = rng.choice([0, 1, 2], size=n, p=[0.6, 0.3, 0.1]).astype(np.int32)
    level[bh] = 2
    lv = torch.as_tensor(level, device="cuda")
    tau = 2e-3
    A, B = bf.Particles.from_numpy(d), bf.Particles.from_numpy(d)
    g = ctx.capture_hhs_interval(A, lv, 2, tau, prec=prec, bh=bh, c=30.0)
    for r in range(3):
        g.launch()
        ctx.hhs_interval(B, lv, 2, tau, prec=prec, bh=bh, c=30.0)
        ctx.forces(bf.Particles.from_numpy(d), prec=prec)  # unrelated eager work in between
        torch.cuda.synchronize()
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            assert torch.equal(getattr(A, k), getattr(B, k)), (r, k)
        if r == 0 and prec == "fp64":
            P = oracle.Particles.from_dict(d)
            oracle.hhs_interval(P, level, tau, bh=bh, c=30.0)
            for k in ("x", "y", "z", "vx", "vy", "vz"):
                ref = getattr(P, k)
                got = getattr(A, k).cpu().numpy()
                assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), k
    g.close()
    assert ctx.read_flags() & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0
