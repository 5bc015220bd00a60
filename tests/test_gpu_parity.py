"""GPU parity: every entry point of the C ABI against the FP64 oracle on the same seeded inputs.

Tolerances:
  * FP64 path: |y_gpu - y_ref| <= 1e-12 * sum_j |term_j| per target (the oracle's magnitude
    sum; summation order differs, so the bound is relative to the conditioning scale);
  * mixed path: per-target relative error |y_gpu - y_ref| / |y_ref| with RMS <= 1e-6 and
    max <= 1e-5 (the stated accuracy targets of the mixed-precision pass).
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


@pytest.fixture(scope="module")
def ctx():
    c = bf.Context(0)
    yield c
    c.close()


def _cluster(n, seed, masses="kroupa"):
    return ics.plummer_cluster(ics.rng_for(100, seed), n, masses)


def _dev(d):
    return bf.Particles.from_numpy(d)


def _flags_clean(ctx):
    f = ctx.read_flags(clear=True)
    assert f & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0, f"device flags {f:#x}"


# --------------------------------------------------------------------------------------------
# accelerations
# --------------------------------------------------------------------------------------------

@pytest.fixture(params=["sorted", "directed", "unsorted"])
def sort_mode(ctx, request):
    """Run a test with the spatially sorted mixed kernels on (the default: pair-symmetric where
    targets and sources are one set), on but directed, and off."""
    on = request.param != "unsorted"
    # test sets are below the size limits
    ctx.set_spatial_sort(forces=on, gradient=on, any_size=on, symmetric=request.param == "sorted")
    yield request.param
    ctx.set_spatial_sort(forces=True, gradient=True, kappa=1.0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("kind", ["all", "list", "range"])
@pytest.mark.parametrize("eps2", [0.0, 1e-6])
def test_forces_parity(ctx, sort_mode, prec, kind, eps2):
    n = 3001  # several 256-source tiles plus a ragged tail
    d = _cluster(n, 1)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    rng = np.random.default_rng(7)
    if kind == "all":
        T, S, Tg, Sg = None, None, None, None
    elif kind == "list":
        T = np.sort(rng.choice(n, 777, replace=False))
        S = np.sort(rng.choice(n, 2300, replace=False))
        Tg, Sg = T, S
    else:
        T, S = np.arange(100, 1400), np.arange(900, 3001)
        Tg, Sg = bf.ParticleSet.range(100, 1300), bf.ParticleSet.range(900, 2101)
    ref, mag, _ = oracle.forces(P, T, S, eps2=eps2, return_mag=True)
    out = ctx.forces(Pd, Tg, Sg, eps2=eps2, prec=prec, r_fb=0.0)
    ti = np.arange(n) if T is None else T
    got = gather(out, ti)
    _flags_clean(ctx)
    if prec == "fp64":
        assert np.all(np.linalg.norm(got - ref, axis=1) <= 1e-12 * mag)
    else:
        rms, mx = stats(rel_errors(got, ref))
        assert rms <= RMS_TOL and mx <= MAX_TOL, (rms, mx)
    # entries that are not targets are untouched
    if T is not None:
        mask = np.ones(n, bool)
        mask[ti] = False
        assert np.all(out[0].cpu().numpy()[mask] == 0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_forces_momentum_balance(ctx, prec):
    d = _cluster(2048, 2)
    Pd = _dev(d)
    ax, ay, az = ctx.forces(Pd, prec=prec)
    m = Pd.m
    tot = torch.stack([(m * ax).sum(), (m * ay).sum(), (m * az).sum()]).abs()
    scale = (m * torch.sqrt(ax * ax + ay * ay + az * az)).sum()
    tol = 1e-14 if prec == "fp64" else 1e-6
    assert torch.all(tot <= tol * scale)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 255, 256, 257, 513])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_forces_ragged_sizes(ctx, n, prec):
    d = _cluster(n, 3 + n)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    ref, mag, _ = oracle.forces(P, return_mag=True)
    got = gather(ctx.forces(Pd, prec=prec), np.arange(n))
    if n == 1:
        assert np.all(got == 0)
        return
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert np.all(np.linalg.norm(got - ref, axis=1) <= tol * mag + 1e-300)


def test_forces_empty_sets(ctx):
    d = _cluster(300, 4)
    Pd = _dev(d)
    out = [torch.full((300,), 7.0, dtype=torch.float64, device="cuda") for _ in range(3)]
    ctx.forces(Pd, bf.ParticleSet.range(0, 0), None, out=out)
    assert all(torch.all(o == 7.0) for o in out)
    ctx.forces(Pd, bf.ParticleSet.range(10, 20), bf.ParticleSet.range(0, 0), out=out)
    assert all(torch.all(o[10:30] == 0.0) and torch.all(o[:10] == 7.0) for o in out)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_forces_config_invariance_and_determinism(ctx, prec):
    """Every kernel shape gives the same result within tolerance; a shape is bitwise repeatable."""
    d = _cluster(5000, 5)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    ref, mag, _ = oracle.forces(P, return_mag=True)
    try:
        for k in (1, 2, 4):
            for w in (2, 4, 8):
                for split in (1, 3, 8):
                    ctx.set_config(bf.BF_OP_FORCES, prec, k, w, split)
                    a = ctx.forces(Pd, prec=prec)
                    b = ctx.forces(Pd, prec=prec)
                    assert all(torch.equal(x, y) for x, y in zip(a, b))
                    got = gather(a, np.arange(5000))
                    if prec == "fp64":
                        assert np.all(np.linalg.norm(got - ref, axis=1) <= 1e-12 * mag)
                    else:
                        rms, mx = stats(rel_errors(got, ref))
                        assert rms <= RMS_TOL and mx <= MAX_TOL, (k, w, split, rms, mx)
    finally:
        ctx.set_config(bf.BF_OP_FORCES, prec, 0)


@pytest.mark.parametrize("op", ["forces", "gradient"])
def test_sorted_mode_king_cluster(ctx, op):
    """A 20,000-body King W0 = 6 cluster with Kroupa masses and binaries: the spatially sorted
    mixed kernels (near tiles in FP64 differences, far tiles from FP32 tile offsets), at the
    default near threshold and at the smallest one accepted, and the unsorted ones all meet the
    mixed tolerance against the oracle, on all targets and on a list."""
    d = ics.king_cluster(ics.rng_for(102), 20000, 6.0, 0.01)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    T = np.sort(np.random.default_rng(11).choice(20000, 700, replace=False))
    if op == "forces":
        ref = oracle.forces(P, T, None)
    else:
        x, y, z = d["x"], d["y"], d["z"]
        s3 = (x * x + y * y + z * z + 0.1) ** -1.5
        af = np.stack([-x * s3, -y * s3, -z * s3], axis=1)
        ref = oracle.gradient(P, af, T, None)
        acc = [torch.as_tensor(np.ascontiguousarray(af[:, k]), device="cuda") for k in range(3)]
    try:
        for mode, kappa in ((True, 3.0), (True, 0.5), (True, 1.0), (False, 1.0)):
            ctx.set_spatial_sort(forces=mode, gradient=mode, kappa=kappa, any_size=mode)
            for targets in (None, T):
                if op == "forces":
                    out = ctx.forces(Pd, targets, None, prec="mixed", r_fb=0.0)
                else:
                    out = ctx.force_gradient(Pd, acc, targets, None, prec="mixed", r_fb=0.0)
                rms, mx = stats(rel_errors(gather(out, T), ref))
                assert rms <= RMS_TOL and mx <= MAX_TOL, (mode, kappa, targets is None, rms, mx)
        with pytest.raises(bf.BifrostError):
            ctx.set_spatial_sort(gradient=True, kappa=0.25)
    finally:
        ctx.set_spatial_sort(forces=True, gradient=True, kappa=1.0)
    _flags_clean(ctx)


def test_forces_close_pair_fallback(ctx):
    """A pair well inside r_fb: the FP64 re-evaluation keeps the mixed result at FP64 quality."""
    d = _cluster(1000, 6)
    d["x"][10] = d["x"][11] + 2e-6
    d["y"][10] = d["y"][11] - 1e-6
    d["z"][10] = d["z"][11]
    d["m"][10] *= 50
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    ref = oracle.forces(P)
    got = gather(ctx.forces(Pd, prec="mixed", r_fb=1e-3), np.arange(1000))
    err = rel_errors(got, ref)
    assert err[10] < 1e-9 and err[11] < 1e-9
    rms, mx = stats(err)
    assert rms <= RMS_TOL and mx <= MAX_TOL


def test_forces_coincident_flag(ctx):
    d = _cluster(400, 7)
    d["x"][5], d["y"][5], d["z"][5] = d["x"][9], d["y"][9], d["z"][9]
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    ctx.read_flags(clear=True)
    got = gather(ctx.forces(Pd, prec="mixed", r_fb=1e-3), np.arange(400))
    assert ctx.read_flags(clear=True) & bf.BF_FLAG_COINCIDENT
    ref = oracle.forces(P)  # coincident pair contributes nothing on both sides
    rms, mx = stats(rel_errors(got, ref))
    assert mx < MAX_TOL


def test_bad_index_is_flagged_not_faulted(ctx):
    d = _cluster(200, 8)
    Pd = _dev(d)
    T = torch.tensor([0, 5, 199, 250], dtype=torch.int32, device="cuda")  # 250 is out of range
    ctx.read_flags(clear=True)
    ctx.forces(Pd, bf.ParticleSet(T, 0, 4), None, prec="mixed")
    assert ctx.read_flags(clear=True) & bf.BF_FLAG_BADINDEX
    with pytest.raises(bf.BifrostError):
        ctx.validate_set(bf.ParticleSet(T, 0, 4), 200)
    with pytest.raises(bf.BifrostError):
        ctx.forces(Pd, bf.ParticleSet.range(150, 100), None)  # range past n, caught on the host
    with pytest.raises(bf.BifrostError):
        ctx.forces(Pd, None, None, eps2=-1.0)


# --------------------------------------------------------------------------------------------
# force gradient
# --------------------------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("kind", ["all", "list"])
@pytest.mark.parametrize("eps2", [0.0, 1e-6])
def test_gradient_parity(ctx, sort_mode, prec, kind, eps2):
    n = 2999
    d = _cluster(n, 11)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    a = oracle.forces(P, eps2=eps2)
    rng = np.random.default_rng(8)
    if kind == "all":
        T = S = None
    else:
        T = np.sort(rng.choice(n, 500, replace=False))
        S = np.sort(rng.choice(n, 2500, replace=False))
    ref, mag, _ = oracle.gradient(P, a, T, S, eps2=eps2, return_mag=True)
    acc = [torch.as_tensor(np.ascontiguousarray(a[:, k]), device="cuda") for k in range(3)]
    out = ctx.force_gradient(Pd, acc, T, S, eps2=eps2, prec=prec, r_fb=0.0)
    ti = np.arange(n) if T is None else T
    got = gather(out, ti)
    _flags_clean(ctx)
    if prec == "fp64":
        assert np.all(np.linalg.norm(got - ref, axis=1) <= 1e-12 * mag)
    else:
        rms, mx = stats(rel_errors(got, ref))
        assert rms <= RMS_TOL and mx <= MAX_TOL, (rms, mx)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_gradient_momentum_balance(ctx, prec):
    d = _cluster(2048, 12)
    Pd = _dev(d)
    a = ctx.forces(Pd, prec="fp64")
    g = ctx.force_gradient(Pd, a, prec=prec)
    m = Pd.m
    tot = torch.stack([(m * x).sum() for x in g]).abs()
    scale = (m * torch.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2)).sum()
    tol = 1e-13 if prec == "fp64" else 1e-6
    assert torch.all(tot <= tol * scale)


# --------------------------------------------------------------------------------------------
# time-steps, PN1.0, energy
# --------------------------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("kind", ["all", "list"])
def test_dt_min_parity(ctx, prec, kind):
    n = 2500
    d = _cluster(n, 21)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    rng = np.random.default_rng(9)
    T = None if kind == "all" else np.sort(rng.choice(n, 300, replace=False))
    ff, fb = oracle.dt_min(P, T, None, eta_ff=0.2, eta_fb=0.15)
    o = ctx.dt_min(Pd, T, None, eta_ff=0.2, eta_fb=0.15, prec=prec)
    ti = np.arange(n) if T is None else T
    gff, gfb = (x.cpu().numpy()[ti] for x in o)
    tol = 1e-13 if prec == "fp64" else 1e-6
    np.testing.assert_allclose(gff, ff, rtol=tol)
    np.testing.assert_allclose(gfb, fb, rtol=tol)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_dt_min_edge_cases(ctx, prec):
    d = _cluster(100, 22)
    d["vx"][:] = 0.3; d["vy"][:] = 0.0; d["vz"][:] = 0.0
    Pd = _dev(d)
    ff, fb = ctx.dt_min(Pd, prec=prec)
    assert torch.all(torch.isinf(fb)) and torch.all(torch.isfinite(ff))
    ff, fb = ctx.dt_min(Pd, bf.ParticleSet.range(3, 1), bf.ParticleSet.range(3, 1), prec=prec)
    assert torch.isinf(ff[3]) and torch.isinf(fb[3])


@pytest.mark.parametrize("kind", ["all", "list"])
def test_pn1_parity(ctx, kind):
    n = 3000
    d = _cluster(n, 31)
    bh = np.array([0, 17, 1500, 2999])
    d["m"][bh] *= 100
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    rng = np.random.default_rng(10)
    if kind == "all":
        T = S = None
    else:
        T = np.sort(np.concatenate([rng.choice(np.arange(1, 1500), 400, replace=False), [1500]]))
        S = np.sort(rng.choice(n, 2000, replace=False))
    ref = oracle.pn1(P, bh, T, S, c=50.0)
    out = ctx.pn1_bh(Pd, bh, T, S, c=50.0)
    ti = np.arange(n) if T is None else T
    got = gather(out, ti)
    scale = np.abs(ref).max()
    assert np.all(np.abs(got - ref) <= 1e-12 * scale + 1e-14 * np.abs(ref))
    _flags_clean(ctx)


@pytest.mark.parametrize("kind", ["range", "list"])
def test_pn1_many_bhs(ctx, kind):
    """A list of 5,000 BHs (more than the target kernel keeps in LDS: the BH-source flags come
    from their own kernels) and of 300 (the flags from the BH sums' records), sources a range or
    an index list that holds some of the BHs: against the oracle."""
    n = 9000
    d = _cluster(n, 33)
    rng = np.random.default_rng(11)
    for nbh in (5000, 300):
        bh = np.sort(rng.choice(n, nbh, replace=False))
        P, Pd = oracle.Particles.from_dict(d), _dev(d)
        if kind == "range":
            T, S = None, bf.ParticleSet.range(1000, 6000)
            So = np.arange(1000, 7000)
        else:
            T = np.sort(rng.choice(n, 2500, replace=False))
            So = np.sort(rng.choice(n, 5000, replace=False))
            S = So
        ref = oracle.pn1(P, bh, T, So, c=50.0)
        out = ctx.pn1_bh(Pd, bh, T, S, c=50.0)
        ti = np.arange(n) if T is None else T
        got = gather(out, ti)
        scale = np.abs(ref).max()
        assert np.all(np.abs(got - ref) <= 1e-12 * scale + 1e-14 * np.abs(ref)), (nbh, kind)
    _flags_clean(ctx)


def test_energy_parity(ctx):
    d = _cluster(4097, 41)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    k0, u0 = oracle.energy(P, eps2=1e-6)
    k1, u1 = ctx.energy(Pd, eps2=1e-6)
    assert abs(k1 / k0 - 1) < 1e-13 and abs(u1 / u0 - 1) < 1e-13
    sub = np.sort(np.random.default_rng(3).choice(4097, 1000, replace=False))
    k0, u0 = oracle.energy(P, sub)
    k1, u1 = ctx.energy(Pd, sub)
    assert abs(k1 / k0 - 1) < 1e-13 and abs(u1 / u0 - 1) < 1e-13


@pytest.mark.parametrize("eps2", [0.0, 1e-6])
def test_energy_chunks_ragged_and_coincident(ctx, eps2):
    """The energy's pair workgroups span several 8,192-column chunks with ragged last tiles
    (20,037 particles; a sampled list of 9,001 of them), every unordered pair once; at eps = 0 a
    coincident pair of distinct particles adds nothing, as in the oracle."""
    d = _cluster(20037, 42)
    d["x"][7], d["y"][7], d["z"][7] = d["x"][19000], d["y"][19000], d["z"][19000]
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    k0, u0 = oracle.energy(P, eps2=eps2)
    k1, u1 = ctx.energy(Pd, eps2=eps2)
    assert abs(k1 / k0 - 1) < 1e-13 and abs(u1 / u0 - 1) < 1e-13, (k1 / k0 - 1, u1 / u0 - 1)
    sub = np.sort(np.random.default_rng(4).choice(20037, 9001, replace=False))
    k0, u0 = oracle.energy(P, sub, eps2=eps2)
    k1, u1 = ctx.energy(Pd, sub, eps2=eps2)
    assert abs(k1 / k0 - 1) < 1e-13 and abs(u1 / u0 - 1) < 1e-13, (k1 / k0 - 1, u1 / u0 - 1)


# --------------------------------------------------------------------------------------------
# FSI cycle
# --------------------------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fsi_step_parity(ctx, prec):
    """Three FSI cycles of the N = 1024 Plummer sphere.  FP64: state within 1e-12 of its scale.
    Mixed: per particle, the position and velocity within the mixed tolerance (1e-5) of the
    particle's own change over the steps (the kicks carry the relative error of the
    accelerations), with a floor of 1e-3 of the largest change."""
    d = ics.config1_plummer1k()
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    P0 = P.copy()
    acc = None
    for s in range(3):
        oracle.fsi_step(P, 1e-3)
        acc = ctx.fsi_step(Pd, 1e-3, prec=prec, acc=acc, acc_valid=s > 0)
    if prec == "mixed":
        assert_state_close(Pd, P, P0, MAX_TOL)
        return
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        ref = getattr(P, k)
        got = getattr(Pd, k).cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), k


def test_fsi_step_with_pn_parity(ctx):
    d = ics.plummer_cluster(ics.rng_for(101), 512, "kroupa")
    bh = np.array([3, 100])
    d["m"][bh] *= 200
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    for _ in range(2):
        oracle.fsi_step(P, 1e-3, bh=bh, c=30.0)
        ctx.fsi_step(Pd, 1e-3, prec="fp64", bh=bh, c=30.0)
    for k in ("x", "vx", "vz"):
        ref = getattr(P, k)
        assert np.abs(getattr(Pd, k).cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


def test_fsi_subset_leaves_others(ctx):
    d = _cluster(600, 51)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    sub = np.arange(100, 400)
    oracle.fsi_step(P, 2e-3, sub)
    ctx.fsi_step(Pd, 2e-3, sub, prec="fp64")
    for k in ("x", "vy"):
        ref = getattr(P, k)
        got = getattr(Pd, k).cpu().numpy()
        assert np.array_equal(got[:100], ref[:100]) and np.array_equal(got[400:], ref[400:])
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("op", ["forces", "gradient"])
def test_fixups_are_rare(ctx, sort_mode, op):
    """The FP64 re-evaluation is for cancelling targets only: on a Kroupa Plummer sphere it
    touches a small fraction of the targets (a magnitude estimate that counted the self pair,
    for instance, would send every target there and still pass the parity tests)."""
    n = 8000
    d = _cluster(n, 21)
    Pd = _dev(d)
    a = ctx.forces(Pd, prec="mixed", r_fb=0.0)
    if op == "gradient":
        ctx.force_gradient(Pd, a, prec="mixed", r_fb=0.0)
    fixups = ctx.last_pass_stats()[0]
    assert fixups <= (0.01 if op == "forces" else 0.05) * n, fixups


@pytest.mark.parametrize("op,n_cancel,half", [("forces", 10, 10000), ("forces", 300, 10000), ("forces", 16, 3000),
                                              ("forces", 100, 3000), ("gradient", 10, 10000),
                                              ("gradient", 300, 10000)])
def test_fixup_of_cancelling_targets(ctx, n_cancel, half, op):
    """Targets near the centre of a mirror-symmetric source cloud (each point and its
    reflection through the origin) feel sums that cancel to about 1e-3 of their magnitude
    estimate, so every one is re-evaluated in FP64.  With 20,000 sources, 10 queued targets
    take the fix-up's workgroup-per-target split, 300 its thread-per-target tiles.  With 6,000
    sources the forces pass runs in the one-launch small kernel, whose failing targets (16:
    one full workgroup, and 100) go to the same fix-up queue.  (Gradients of that smaller cloud
    do not all cancel below the check's threshold.)  All must give the oracle's FP64 sums to
    1e-12 of the magnitude estimate."""
    rng = np.random.default_rng(60 + n_cancel)
    p = rng.normal(size=(half, 3))
    pos = np.concatenate([p, -p, 1e-3 * rng.normal(size=(n_cancel, 3))])
    n = pos.shape[0]
    m = np.concatenate([np.full(2 * half, 1.0 / (2 * half)), np.full(n_cancel, 1e-12)])
    vel = 0.1 * rng.normal(size=(n, 3))
    d = {"x": pos[:, 0], "y": pos[:, 1], "z": pos[:, 2], "vx": vel[:, 0], "vy": vel[:, 1], "vz": vel[:, 2], "m": m}
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    tg = np.arange(2 * half, n)
    if op == "forces":
        ref, mag, _ = oracle.forces(P, tg, return_mag=True)
        got = gather(ctx.forces(Pd, tg, prec="mixed"), tg)
    else:
        af = oracle.forces(P)
        ref, mag, _ = oracle.gradient(P, af, tg, return_mag=True)
        ad = [torch.as_tensor(af[:, k].copy(), device="cuda") for k in range(3)]
        got = gather(ctx.force_gradient(Pd, ad, tg, prec="mixed"), tg)
    fixups = ctx.last_pass_stats()[0]
    assert fixups >= 0.9 * n_cancel, fixups
    assert (ctx.last_pass_config()[2] == 16) == (n <= 6144)
    err = np.linalg.norm(got - ref, axis=1)
    assert np.all(err <= 1e-12 * mag), (err / mag).max()


@pytest.mark.parametrize("op", ["forces", "gradient"])
def test_small_pass_kernel_parity(ctx, op):
    """Mixed passes of up to 6,144 targets and sources run as one launch of the small kernel
    (16 wavefronts and 4 lane groups splitting the sources of 16 targets, the sums added in
    the workgroup): ragged and tiny shapes against the oracle, bitwise repeatable, and equal
    within tolerance to the split kernels that a forced configuration selects; larger passes
    keep the split kernels."""
    d = _cluster(20000, 71)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    rng = np.random.default_rng(72)
    af = oracle.forces(P)
    ad = [torch.as_tensor(af[:, k].copy(), device="cuda") for k in range(3)]
    opc = bf.BF_OP_FORCES if op == "forces" else bf.BF_OP_GRADIENT
    for nt, ns in ((1, 5), (17, 1000), (333, 4097), (6144, 6144), (6145, 100), (2000, 20000)):
        tg = np.sort(rng.choice(20000, nt, replace=False))
        sr = np.sort(rng.choice(20000, ns, replace=False))
        run = (lambda: ctx.forces(Pd, tg, sr, prec="mixed")) if op == "forces" else \
            (lambda: ctx.force_gradient(Pd, ad, tg, sr, prec="mixed"))
        a, b = run(), run()
        assert all(torch.equal(x, y) for x, y in zip(a, b))
        kind, k, waves, split = ctx.last_pass_config()
        assert kind == "unsorted" and (waves == 16) == (nt <= 6144 and ns <= 6144), (nt, ns, waves)
        ref = oracle.forces(P, tg, sr) if op == "forces" else oracle.gradient(P, af, tg, sr)
        got = gather(a, tg)
        rms, mx = stats(rel_errors(got, ref))
        assert rms <= RMS_TOL and mx <= MAX_TOL, (nt, ns, rms, mx)
        try:
            ctx.set_config(opc, "mixed", 1, 4, 0)
            c = run()
        finally:
            ctx.set_config(opc, "mixed", 0)
        rms, mx = stats(rel_errors(gather(c, tg), got))
        assert rms <= RMS_TOL and mx <= MAX_TOL, (nt, ns, rms, mx)


@pytest.mark.parametrize("op", ["forces", "gradient"])
def test_small_pass_kernel_fp64_parity(ctx, op):
    """FP64 passes of up to 6,144 targets and sources run as one launch that reads the sources
    straight from the masters (no pack, no reduction kernel): ragged and tiny shapes within the
    FP64 tolerance of the oracle (1e-12 of the magnitude sum), bitwise repeatable, and within
    that tolerance of the split kernels a forced configuration selects, softened and not."""
    d = _cluster(20000, 73)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    rng = np.random.default_rng(74)
    af = oracle.forces(P)
    ad = [torch.as_tensor(af[:, k].copy(), device="cuda") for k in range(3)]
    opc = bf.BF_OP_FORCES if op == "forces" else bf.BF_OP_GRADIENT
    for (nt, ns), eps2 in zip(((1, 5), (17, 1000), (333, 4097), (6144, 6144), (6145, 100)),
                              (0.0, 1e-6, 0.0, 1e-6, 0.0)):
        tg = np.sort(rng.choice(20000, nt, replace=False))
        sr = np.sort(rng.choice(20000, ns, replace=False))
        run = (lambda: ctx.forces(Pd, tg, sr, eps2=eps2, prec="fp64")) if op == "forces" else \
            (lambda: ctx.force_gradient(Pd, ad, tg, sr, eps2=eps2, prec="fp64"))
        a, b = run(), run()
        assert all(torch.equal(x, y) for x, y in zip(a, b))
        kind, k, waves, split = ctx.last_pass_config()
        assert kind == "unsorted" and (waves == 16) == (nt <= 6144 and ns <= 6144), (nt, ns, waves)
        if op == "forces":
            ref, mag, _ = oracle.forces(P, tg, sr, eps2=eps2, return_mag=True)
        else:
            ref, mag, _ = oracle.gradient(P, af, tg, sr, eps2=eps2, return_mag=True)
        got = gather(a, tg)
        assert np.all(np.linalg.norm(got - ref, axis=1) <= 1e-12 * mag), (nt, ns)
        try:
            ctx.set_config(opc, "fp64", 1, 4, 0)
            c = run()
            assert ctx.last_pass_config()[2] == 4
        finally:
            ctx.set_config(opc, "fp64", 0)
        assert np.all(np.linalg.norm(gather(c, tg) - got, axis=1) <= 1e-12 * mag), (nt, ns)
    assert ctx.read_flags(clear=True) & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0


def test_autotune_table_round_trip(ctx, tmp_path):
    """The autotuner times the kernel variants for one size bucket, stores the fastest in the
    context and in a JSON cache; a fresh context loading the cache plans the same variant, and
    results keep parity with the tuned variant in use."""
    n = 20000
    cache = str(tmp_path / "tune.json")
    for op in (bf.BF_OP_FORCES, bf.BF_OP_GRADIENT):
        ctx.autotune(op, "mixed", n, n, cache)
    tuned = [ctx.query_config(op, "mixed", n, n) for op in (bf.BF_OP_FORCES, bf.BF_OP_GRADIENT)]
    other = bf.Context(0)
    try:
        other.autotune_load(cache)
        assert [other.query_config(op, "mixed", n, n) for op in (bf.BF_OP_FORCES, bf.BF_OP_GRADIENT)] == tuned
    finally:
        other.close()
    d = ics.king_cluster(ics.rng_for(103), n, 6.0, 0.01)
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    T = np.sort(np.random.default_rng(13).choice(n, 400, replace=False))
    got = gather(ctx.forces(Pd, T, None, prec="mixed", r_fb=0.0), T)
    rms, mx = stats(rel_errors(got, oracle.forces(P, T, None)))
    assert rms <= RMS_TOL and mx <= MAX_TOL


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_degenerate_systems(ctx, prec):
    """One particle: no source but itself, so zero acceleration and gradient and infinite
    time-steps.  Two particles: the two-body closed form.  A massless test particle feels the
    field and exerts none."""
    one = {k: np.array([0.3]) for k in ("x", "y", "z", "vx", "vy", "vz")}
    one["m"] = np.array([1.0])
    P1 = _dev(one)
    a = ctx.forces(P1, prec=prec)
    g = ctx.force_gradient(P1, a, prec=prec)
    ff, fb = ctx.dt_min(P1, prec=prec)
    assert all(float(t[0]) == 0.0 for t in (*a, *g))
    assert torch.isinf(ff[0]) and torch.isinf(fb[0])
    two = {"x": np.array([0.0, 0.6]), "y": np.array([0.0, 0.8]), "z": np.zeros(2), "vx": np.zeros(2),
           "vy": np.zeros(2), "vz": np.zeros(2), "m": np.array([0.25, 0.75])}
    a = gather(ctx.forces(_dev(two), prec=prec), np.arange(2))
    u = np.array([0.6, 0.8, 0.0])  # unit vector from body 0 to body 1 at distance 1
    np.testing.assert_allclose(a[0], 0.75 * u, rtol=1e-6 if prec == "mixed" else 1e-14)
    np.testing.assert_allclose(a[1], -0.25 * u, rtol=1e-6 if prec == "mixed" else 1e-14)
    d = _cluster(2000, 41)
    d["m"][7] = 0.0
    P, Pd = oracle.Particles.from_dict(d), _dev(d)
    got = gather(ctx.forces(Pd, prec=prec, r_fb=0.0), np.arange(2000))
    ref = oracle.forces(P)
    without = oracle.forces(P, None, np.delete(np.arange(2000), 7))
    np.testing.assert_array_equal(ref, without)  # the oracle agrees the massless source adds nothing
    if prec == "fp64":
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    else:
        rms, mx = stats(rel_errors(got, ref))
        assert rms <= RMS_TOL and mx <= MAX_TOL


def test_size_limits_rejected(ctx):
    """Sizes beyond the int32 index range, sets outside [0, n), negative softening and bad
    precision are refused on the host before any launch."""
    d = _cluster(100, 42)
    Pd = _dev(d)
    with pytest.raises(bf.BifrostError):
        ctx.forces(Pd, bf.ParticleSet.range(90, 20), None)
    with pytest.raises(bf.BifrostError):
        ctx.forces(Pd, eps2=-1.0)
    with pytest.raises((bf.BifrostError, KeyError)):
        ctx.forces(Pd, prec="fp16")
    # n = 2^31 through the C ABI: the arrays are never touched, the size check fails first
    import ctypes
    from paper_2210_02472_amd import _binding as B
    big = Pd._c()
    big.n = 1 << 31
    rng = bf.ParticleSet.range(0, 10)._c()
    out = [torch.zeros(100, dtype=torch.float64, device="cuda") for _ in range(3)]
    rc = B._lib.bf_forces(ctx._h, ctypes.byref(big), ctypes.byref(rng), ctypes.byref(rng), 1.0, 0.0,
                          B.BF_PREC_MIXED, 0.0, *[B._ptr(t) for t in out])
    assert rc == -1  # BF_ERR_ARG
    assert all(torch.all(t == 0) for t in out)
