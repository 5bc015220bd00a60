"""GPU parity of the pair-symmetric sorted sweep (targets and sources one set) against the oracle.

The symmetric sweep evaluates each unordered pair once and keeps both terms (Sec. 2.1: the
acceleration and force-gradient terms of a pair are equal and opposite up to the mass factor).
The block sizes below cover one block, two blocks (the half-ring distance), an odd and an even
block count (the block pair at distance nb/2 visited from one side only) and ragged last tiles.
Tolerances are those of the mixed pass: relative error RMS <= 1e-6 and max <= 1e-5 per target.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2210_02472_amd import ics
from tests._parity import assert_state_close, gather, rel_errors, stats

bf = pytest.importorskip("paper_2210_02472_amd")

pytestmark = pytest.mark.gpu

RMS_TOL, MAX_TOL = 1e-6, 1e-5
BLOCK_TILES = 16  # row tiles of 64 per workgroup of the symmetric sweep
WALKS = {"forces": (8, 2), "gradient": (4, 4)}  # (wavefronts, row tiles per wavefront)


@pytest.fixture(scope="module")
def ctx():
    c = bf.Context(0)
    c.set_spatial_sort(forces=True, gradient=True, any_size=True)
    yield c
    c.close()


def _king(n, seed):
    return ics.king_cluster(ics.rng_for(200, seed), n, 6.0, 0.01)


def _tile_pairs(n, op="forces"):
    """Tile visits of the symmetric walk: every unordered pair of 64-particle tiles once; a
    wavefront's visit of a column tile covers its row tiles together."""
    WAVES, ROWS = WALKS[op]
    t = (n + 63) // 64
    bt = WAVES * ROWS
    nb = -(-t // bt)
    visits = 0
    for w in range(nb):
        for v in range(WAVES):
            rows = [w * bt + v * ROWS + r for r in range(ROWS) if w * bt + v * ROWS + r < t]
            if not rows:
                continue
            for d in range(nb // 2 + 1):
                if d > 0 and 2 * d == nb and w >= d:
                    break
                b = (w + d) % nb
                for ct in range(b * bt, min(b * bt + bt, t)):
                    visits += 1 if d > 0 or ct >= rows[0] else 0
    return visits


@pytest.mark.parametrize("n", [1000, 1100, 17000, 20000])
@pytest.mark.parametrize("op", ["forces", "gradient"])
def test_symmetric_sweep_parity(ctx, n, op):
    """All targets against the oracle; the sweep visits every unordered pair of 64-particle
    tiles exactly once (the near + far visit count of the walk)."""
    blocks = -(-((n + 63) // 64) // BLOCK_TILES)
    print(f"n={n} blocks={blocks} op={op}", flush=True)
    d = _king(n, n)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    if op == "forces":
        ref = oracle.forces(P)
        out = ctx.forces(Pd, prec="mixed", r_fb=0.0)
    else:
        a = oracle.forces(P)
        ref = oracle.gradient(P, a)
        acc = [torch.as_tensor(np.ascontiguousarray(a[:, k]), device="cuda") for k in range(3)]
        out = ctx.force_gradient(Pd, acc, prec="mixed", r_fb=0.0)
    fix, near, far = ctx.last_pass_stats()
    kind, rows, waves, _ = ctx.last_pass_config()
    assert (kind, waves, rows) == ("symmetric", *WALKS[op])
    assert near + far == _tile_pairs(n, op), (near, far, _tile_pairs(n, op))
    got = gather(out, np.arange(n))
    f = ctx.read_flags(clear=True)
    assert f & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0, f"device flags {f:#x}"
    rms, mx = stats(rel_errors(got, ref))
    assert rms <= RMS_TOL and mx <= MAX_TOL, (rms, mx, fix)


@pytest.mark.parametrize("op", ["forces", "gradient"])
def test_symmetric_softened_and_repeatable(ctx, op):
    """Softened pairs (eps^2 = 1e-6), bitwise repeatable results, and agreement with the directed
    sorted sweep (both within the mixed tolerance of the oracle)."""
    n = 9000
    d = _king(n, 5)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    eps2 = 1e-6
    a = oracle.forces(P, eps2=eps2)
    acc = [torch.as_tensor(np.ascontiguousarray(a[:, k]), device="cuda") for k in range(3)]

    def run():
        if op == "forces":
            return ctx.forces(Pd, eps2=eps2, prec="mixed", r_fb=0.0)
        return ctx.force_gradient(Pd, acc, eps2=eps2, prec="mixed", r_fb=0.0)

    ref = oracle.forces(P, eps2=eps2) if op == "forces" else oracle.gradient(P, a, eps2=eps2)
    x, y = run(), run()
    assert all(torch.equal(u, v) for u, v in zip(x, y))
    try:
        ctx.set_spatial_sort(forces=True, gradient=True, any_size=True, symmetric=False)
        z = run()
        assert ctx.last_pass_config()[0] == "sorted"  # the directed sweep ran
    finally:
        ctx.set_spatial_sort(forces=True, gradient=True, any_size=True)
    for out in (x, z):
        rms, mx = stats(rel_errors(gather(out, np.arange(n)), ref))
        assert rms <= RMS_TOL and mx <= MAX_TOL, (rms, mx)


def test_symmetric_momentum_balance(ctx):
    """Evaluating each pair once makes sum_i m_i a_i vanish up to the FP32 rounding of the terms."""
    n = 12000
    d = _king(n, 9)
    Pd = _dev(d)
    a = ctx.forces(Pd, prec="mixed", r_fb=0.0)
    m = Pd.m
    tot = torch.stack([(m * x).sum() for x in a]).abs()
    scale = (m * torch.sqrt(a[0] ** 2 + a[1] ** 2 + a[2] ** 2)).sum()
    assert torch.all(tot <= 1e-6 * scale), (tot, scale)


def test_symmetric_subset_runs_directed(ctx):
    """Target and source sets that differ (an index list against all) keep the directed sweep."""
    n = 5000
    d = _king(n, 3)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    T = np.sort(np.random.default_rng(4).choice(n, 3000, replace=False))
    got = gather(ctx.forces(Pd, T, None, prec="mixed", r_fb=0.0), T)
    assert ctx.last_pass_config()[0] == "sorted"
    rms, mx = stats(rel_errors(got, oracle.forces(P, T, None)))
    assert rms <= RMS_TOL and mx <= MAX_TOL


def _dev(d):
    return bf.Particles.from_numpy(d)


def test_symmetric_fsi_steps_parity(ctx):
    """Three FSI cycles (Sec. 2.1) of a King cluster whose acceleration and gradient passes take
    the symmetric sweep: per particle, position and velocity within 1e-5 of the particle's own
    change (floor: 1e-3 of the largest change)."""
    n = 4000
    d = _king(n, 21)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    P0 = P.copy()
    acc = None
    for s in range(3):
        oracle.fsi_step(P, 2e-4)
        acc = ctx.fsi_step(Pd, 2e-4, prec="mixed", acc=acc, acc_valid=s > 0)
    assert ctx.last_pass_config()[0] == "symmetric"
    assert_state_close(Pd, P, P0, MAX_TOL)


def test_symmetric_hhs_interval_parity(ctx):
    """One HHS-FSI interval (Sec. 2.2) with four populated levels: each level's own FSI passes take
    the symmetric sweep and the inter-level passes the directed one; per particle, position and
    velocity within 1e-5 of the particle's own change (floor: 1e-3 of the largest change)."""
    n = 3000
    d = _king(n, 23)
    level = np.random.default_rng(6).choice([0, 1, 2, 4], size=n, p=[0.5, 0.25, 0.15, 0.10]).astype(np.int32)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    P0 = P.copy()
    tau = 4e-4
    oracle.hhs_interval(P, level, tau)
    ctx.hhs_interval(Pd, torch.as_tensor(level, device="cuda"), 4, tau, prec="mixed")
    assert_state_close(Pd, P, P0, MAX_TOL)
    assert ctx.read_flags() & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0


@pytest.mark.parametrize("kind", ["list", "range"])
@pytest.mark.parametrize("op", ["forces", "gradient"])
def test_between_parity(ctx, kind, op):
    """bf_forces_between / bf_force_gradient_between: the sums of set a over set b and of b over a
    (Sec. 2.2, the inter-level terms) from one two-set symmetric sweep, against the oracle's two
    directed sums, on every particle of both sets."""
    n = 12000
    d = _king(n, 31)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    if kind == "list":
        rng = np.random.default_rng(32)
        A = np.sort(rng.choice(n, 7001, replace=False))
        B = np.setdiff1d(np.arange(n), A)
        Ag, Bg = A, B
    else:
        A, B = np.arange(0, 5003), np.arange(5003, n)
        Ag, Bg = bf.ParticleSet.range(0, 5003), bf.ParticleSet.range(5003, n - 5003)
    if op == "forces":
        out = ctx.forces_between(Pd, Ag, Bg, prec="mixed")
        ref_a, ref_b = oracle.forces(P, A, B), oracle.forces(P, B, A)
    else:
        a = oracle.forces(P)
        acc = [torch.as_tensor(np.ascontiguousarray(a[:, k]), device="cuda") for k in range(3)]
        out = ctx.force_gradient_between(Pd, acc, Ag, Bg, prec="mixed")
        ref_a, ref_b = oracle.gradient(P, a, A, B), oracle.gradient(P, a, B, A)
    assert ctx.last_pass_config()[0] == "between"
    f = ctx.read_flags(clear=True)
    assert f & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0, f"device flags {f:#x}"
    for idx, ref in ((A, ref_a), (B, ref_b)):
        rms, mx = stats(rel_errors(gather(out, idx), ref))
        assert rms <= RMS_TOL and mx <= MAX_TOL, (rms, mx)


def test_between_fallbacks_and_checks(ctx):
    """The two-set entry with the directed sweep forced, and with sets too small for the sorted
    mode (two directed passes either way), gives the same sums; overlapping ranges are refused."""
    n = 3000
    d = _king(n, 33)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    A, B = np.arange(0, 40), np.arange(40, n)
    out = ctx.forces_between(Pd, bf.ParticleSet.range(0, 40), bf.ParticleSet.range(40, n - 40), prec="mixed")
    assert ctx.last_pass_config()[0] != "between"
    for idx, ref in ((A, oracle.forces(P, A, B)), (B, oracle.forces(P, B, A))):
        rms, mx = stats(rel_errors(gather(out, idx), ref))
        assert rms <= RMS_TOL and mx <= MAX_TOL, (rms, mx)
    try:
        ctx.set_spatial_sort(forces=True, gradient=True, any_size=True, symmetric=False)
        A, B = np.arange(0, 1500), np.arange(1500, n)
        out = ctx.forces_between(Pd, bf.ParticleSet.range(0, 1500), bf.ParticleSet.range(1500, 1500), prec="mixed")
        assert ctx.last_pass_config()[0] == "sorted"
        for idx, ref in ((A, oracle.forces(P, A, B)), (B, oracle.forces(P, B, A))):
            rms, mx = stats(rel_errors(gather(out, idx), ref))
            assert rms <= RMS_TOL and mx <= MAX_TOL, (rms, mx)
    finally:
        ctx.set_spatial_sort(forces=True, gradient=True, any_size=True)
    with pytest.raises(bf.BifrostError):
        ctx.forces_between(Pd, bf.ParticleSet.range(0, 100), bf.ParticleSet.range(50, 100))


def test_release_scratch(ctx):
    """The symmetric sweep's scratch is freed on request and allocated again by the next pass,
    with the same results."""
    n = 6000
    d = _king(n, 41)
    Pd = _dev(d)
    a = ctx.forces(Pd, prec="mixed")
    assert ctx.release_scratch() > 0
    assert ctx.release_scratch() == 0
    b = ctx.forces(Pd, prec="mixed")
    assert ctx.last_pass_config()[0] == "symmetric"
    assert all(torch.equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("n", [1100, 17000, 20000])
@pytest.mark.parametrize("op", ["forces", "gradient"])
@pytest.mark.parametrize("eps2", [0.0, 1e-6])
def test_symmetric_fp64_parity(ctx, n, op, eps2):
    """FP64 passes over one set take the symmetric sweep in the set's own order: every target
    within 1e-12 of the oracle's magnitude sum (the FP64 tolerance), bitwise repeatable."""
    d = _king(n, 50 + n % 7)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    if op == "forces":
        ref, mag, _ = oracle.forces(P, eps2=eps2, return_mag=True)
        run = lambda: ctx.forces(Pd, eps2=eps2, prec="fp64")  # noqa: E731
    else:
        a = oracle.forces(P, eps2=eps2)
        ref, mag, _ = oracle.gradient(P, a, eps2=eps2, return_mag=True)
        acc = [torch.as_tensor(np.ascontiguousarray(a[:, k]), device="cuda") for k in range(3)]
        run = lambda: ctx.force_gradient(Pd, acc, eps2=eps2, prec="fp64")  # noqa: E731
    out = run()
    assert ctx.last_pass_config()[0] == "symmetric"
    again = run()
    assert all(torch.equal(x, y) for x, y in zip(out, again))
    got = gather(out, np.arange(n))
    assert np.all(np.linalg.norm(got - ref, axis=1) <= 1e-12 * mag)
    assert ctx.read_flags(clear=True) & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0


# --------------------------------------------------------------------------------------------
# the time-step pass over one set (each unordered pair once, the set's own order)
# --------------------------------------------------------------------------------------------

def _dt_both(ctx, Pd, **kw):
    """The mixed time-step pass twice with the symmetric sweep, then with the directed one."""
    s1 = ctx.dt_min(Pd, eta_ff=0.2, eta_fb=0.15, prec="mixed", **kw)
    cfg = ctx.last_pass_config()
    s2 = ctx.dt_min(Pd, eta_ff=0.2, eta_fb=0.15, prec="mixed", **kw)
    try:
        ctx.set_spatial_sort(forces=True, gradient=True, any_size=True, timestep=False)
        dr = ctx.dt_min(Pd, eta_ff=0.2, eta_fb=0.15, prec="mixed", **kw)
        assert ctx.last_pass_config()[0] == "unsorted"
    finally:
        ctx.set_spatial_sort(forces=True, gradient=True, any_size=True)
    return s1, s2, dr, cfg


@pytest.mark.parametrize("n", [64, 65, 1000, 1100, 17000, 20000])
def test_symmetric_dt_parity(ctx, n):
    """Both time-steps of every particle within relative 1e-6 of the oracle; bitwise repeatable
    and bitwise equal to the directed pass (a pair's FP32 rates do not depend on its orientation
    and a maximum is exact in any order).  Sizes: one tile (the diagonal only), a ragged second
    tile, one and two blocks, odd and even block counts with ragged last tiles."""
    print(f"dt n={n}", flush=True)
    d = _king(n, 60 + n % 11)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    ff, fb = oracle.dt_min(P, eta_ff=0.2, eta_fb=0.15)
    s1, s2, dr, cfg = _dt_both(ctx, Pd)
    assert cfg[:3] == ("symmetric", 2, 8), cfg
    for x, y, z in zip(s1, s2, dr):
        assert torch.equal(x, y) and torch.equal(x, z)
    np.testing.assert_allclose(s1[0].cpu().numpy(), ff, rtol=1e-6)
    np.testing.assert_allclose(s1[1].cpu().numpy(), fb, rtol=1e-6)
    assert ctx.read_flags(clear=True) == 0


def test_symmetric_dt_close_and_coincident(ctx):
    """A coincident pair is left out and flagged; a pair 3e-15 apart, whose FP32 free-fall rate
    overflows, and a pair one FP64 ulp apart send their tiles through the FP64 evaluation: every
    time-step within relative 1e-6 of the oracle (the close pairs' own time-steps included), in
    the symmetric and the directed pass; equal velocities give no fly-by bound."""
    n = 3000
    d = _king(n, 71)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        d[k][2500] = d[k][10]            # coincident, equal velocities
        d[k][1700] = d[k][40]
        d[k][2999] = d[k][900]
    d["x"][1700] = d["x"][40] + 3e-15    # r^2 = 9e-30: the FP32 free-fall rate overflows
    d["vx"][1700] += 1e-3
    d["y"][2999] = np.nextafter(d["y"][900], np.inf)  # one ulp: r^2 below the FP32 range
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    ff, fb = oracle.dt_min(P, eta_ff=0.2, eta_fb=0.15)
    ctx.read_flags(clear=True)
    s1, s2, dr, cfg = _dt_both(ctx, Pd)
    assert cfg[0] == "symmetric"
    assert ctx.read_flags(clear=True) & bf.BF_FLAG_COINCIDENT
    for x, y in zip(s1, s2):
        assert torch.equal(x, y)
    for out in (s1, dr):
        np.testing.assert_allclose(out[0].cpu().numpy(), ff, rtol=1e-6)
        np.testing.assert_allclose(out[1].cpu().numpy(), fb, rtol=1e-6)
    assert np.all(np.isfinite(ff[[40, 1700, 900, 2999]])) and ff[1700] < 1e-12


@pytest.mark.parametrize("shape", [(1, 16), (2, 8), (4, 4)])
@pytest.mark.parametrize("rounds", [1, 4, 32])
def test_symmetric_dt_shapes_bitwise(ctx, shape, rounds):
    """Every shape and share count of the time-step sweep gives bitwise the same maxima."""
    n = 9000
    d = _king(n, 73)
    Pd = _dev(d)
    ref = ctx.dt_min(Pd, eta_ff=0.2, eta_fb=0.15, prec="mixed")
    rows, waves = shape
    try:
        ctx.set_symmetric_config(bf.BF_OP_DTMIN, rows, waves, rounds)
        got = ctx.dt_min(Pd, eta_ff=0.2, eta_fb=0.15, prec="mixed")
        assert ctx.last_pass_config()[:3] == ("symmetric", rows, waves)
    finally:
        ctx.set_symmetric_config(bf.BF_OP_DTMIN, 0, 0, 0)
    assert all(torch.equal(x, y) for x, y in zip(ref, got))


def test_symmetric_dt_fly_by_radius_runs_directed(ctx):
    """A fly-by radius (r_fb > 0) keeps the directed pass, with its close-pair re-evaluation."""
    n = 2000
    d = _king(n, 75)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    ff, fb = oracle.dt_min(P, eta_ff=0.2, eta_fb=0.15)
    out = ctx.dt_min(Pd, eta_ff=0.2, eta_fb=0.15, prec="mixed", r_fb=0.05)
    assert ctx.last_pass_config()[0] == "unsorted"
    np.testing.assert_allclose(out[0].cpu().numpy(), ff, rtol=1e-6)
    np.testing.assert_allclose(out[1].cpu().numpy(), fb, rtol=1e-6)


# --------------------------------------------------------------------------------------------
# sweeps in several passes over the distance shares (a scratch limit below one pass)
# --------------------------------------------------------------------------------------------

@pytest.mark.parametrize("op", ["forces", "gradient", "fp64", "dt"])
def test_symmetric_passes_bitwise(ctx, op):
    """A scratch limit below one sweep's partials splits its distance shares over several
    passes, each adding onto running sums in the order of a single pass: bitwise the same
    results (20,000 bodies: 20 blocks, 11 block distances, one share each)."""
    n = 20000
    d = _king(n, 80)
    Pd = _dev(d)
    a = oracle.forces(oracle.Particles.from_dict(d))
    acc = [torch.as_tensor(np.ascontiguousarray(a[:, k]), device="cuda") for k in range(3)]
    run = {
        "forces": lambda: ctx.forces(Pd, prec="mixed"),
        "gradient": lambda: ctx.force_gradient(Pd, acc, prec="mixed"),
        "fp64": lambda: ctx.forces(Pd, prec="fp64"),
        "dt": lambda: ctx.dt_min(Pd, eta_ff=0.2, eta_fb=0.15, prec="mixed"),
    }[op]
    ref = run()
    assert ctx.last_pass_config()[0] == "symmetric" and ctx.last_symmetric_passes() == 1
    try:
        ctx.set_symmetric_scratch_limit(3 << 20)
        got = run()
        kind, passes = ctx.last_pass_config()[0], ctx.last_symmetric_passes()
    finally:
        ctx.set_symmetric_scratch_limit(0)
    print(f"{op}: {passes} passes", flush=True)
    assert kind == "symmetric" and passes >= 2, (kind, passes)
    assert all(torch.equal(x, y) for x, y in zip(ref, got))
    assert ctx.read_flags(clear=True) & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0


@pytest.mark.parametrize("n", [5000, 70000])
def test_symmetric_passes_limits(ctx, n):
    """Scratch limits from below one distance's partials up to one pass less than needed, on a
    small and a larger set (whose default shares hold several distances): results are bitwise
    repeatable at every limit; bitwise those of a single pass while the limit leaves the shares
    as they are (it only groups them into passes), and within 1e-13 of them when it has to cut
    the shares finer (the row sums are then grouped differently); the time-step maxima are
    bitwise the same at every limit."""
    d = _king(n, 90 + n % 13)
    Pd = _dev(d)
    a = ctx.forces(Pd, prec="mixed")
    runs = {
        "forces": lambda: ctx.forces(Pd, prec="mixed"),
        "gradient": lambda: ctx.force_gradient(Pd, a, prec="mixed"),
        "fp64": lambda: ctx.force_gradient(Pd, a, prec="fp64"),
        "dt": lambda: ctx.dt_min(Pd, eta_ff=0.2, eta_fb=0.15, prec="mixed"),
    }
    for name, run in runs.items():
        ref = run()
        ref_shares = ctx.last_pass_config()[3]
        assert ctx.last_symmetric_passes() == 1
        seen = set()
        for limit in (1, 1 << 20, 5 << 20, 40 << 20):
            try:
                ctx.set_symmetric_scratch_limit(limit)
                got = run()
                kind, shares = ctx.last_pass_config()[0], ctx.last_pass_config()[3]
                passes = ctx.last_symmetric_passes()
                again = run()
            finally:
                ctx.set_symmetric_scratch_limit(0)
            assert kind == "symmetric", (name, limit)
            seen.add((passes, shares))
            assert all(torch.equal(x, y) for x, y in zip(got, again)), (name, limit)
            if shares == ref_shares or name == "dt":
                assert all(torch.equal(x, y) for x, y in zip(ref, got)), (name, limit, passes, shares)
            else:
                for x, y in zip(ref, got):
                    assert torch.allclose(x, y, rtol=1e-13, atol=1e-13 * float(y.abs().max())), (name, limit)
        print(f"n={n} {name}: (passes, shares) {sorted(seen)}, one pass {ref_shares} shares", flush=True)
        assert max(p for p, _ in seen) > 1, (name, seen)
    assert ctx.read_flags(clear=True) & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0


def test_set_order_sweeps_on_an_index_list(ctx):
    """The set-order sweeps (time-step rates, FP64 acceleration) take a permuted index list that
    is both targets and sources (the same list): each unordered pair of the listed particles
    once; results at the listed particles against the oracle over the same list, the rest of
    the output untouched."""
    n, m = 40000, 33001
    d = _king(n, 97)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    rng = np.random.default_rng(98)
    lst = rng.permutation(n)[:m]
    S = bf.ParticleSet.of(torch.as_tensor(lst.astype(np.int32), device="cuda"), n)
    ff, fb = oracle.dt_min(P, lst, lst, eta_ff=0.2, eta_fb=0.15)
    out = [torch.full((n,), -1.0, dtype=torch.float64, device="cuda") for _ in range(2)]
    ctx.dt_min(Pd, S, S, eta_ff=0.2, eta_fb=0.15, prec="mixed", out=out)
    assert ctx.last_pass_config()[0] == "symmetric"
    np.testing.assert_allclose(out[0].cpu().numpy()[lst], ff, rtol=1e-6)
    np.testing.assert_allclose(out[1].cpu().numpy()[lst], fb, rtol=1e-6)
    rest = np.setdiff1d(np.arange(n), lst)
    assert np.all(out[0].cpu().numpy()[rest] == -1.0) and np.all(out[1].cpu().numpy()[rest] == -1.0)
    ref, mag, _ = oracle.forces(P, lst, lst, return_mag=True)
    acc = ctx.forces(Pd, S, S, prec="fp64")
    assert ctx.last_pass_config()[0] == "symmetric"
    got = gather(acc, lst)
    assert np.all(np.linalg.norm(got - ref, axis=1) <= 1e-12 * mag)
    assert ctx.read_flags(clear=True) & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0
