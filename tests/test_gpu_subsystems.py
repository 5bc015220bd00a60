"""GPU parity of the subsystem neighbour search, the subsystem labels and the exclusion of
intra-subsystem pairs from the pair passes (Sec. 3.3, Alg. 1) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2210_02472_amd import ics
from tests._parity import gather, rel_errors, stats

bf = pytest.importorskip("paper_2210_02472_amd")

pytestmark = pytest.mark.gpu

RMS_TOL, MAX_TOL = 1e-6, 1e-5
R_NGB = 2e-3


@pytest.fixture(scope="module")
def ctx():
    c = bf.Context(0)
    yield c
    c.close()


def _cluster_with_binaries(n, seed, n_bin=60):
    """Kroupa Plummer sphere in which n_bin particles get a close companion: bound pairs with
    semi-major axes log-uniform in [0.05, 5] r_ngb and eccentricities uniform in [0, 0.95], at a
    random phase, oriented at random; every fourth companion gets a bound companion of its own
    (hierarchical triples, some linked only through the middle particle)."""
    rng = ics.rng_for(310, seed)
    d = ics.plummer_cluster(rng, n, "kroupa")

    def attach(h, c):
        a = R_NGB * 10.0 ** rng.uniform(-1.3, 0.7)
        e = rng.uniform(0, 0.95)
        E = rng.uniform(0, 2 * np.pi)
        mu = d["m"][h] + d["m"][c]
        rel = np.array([a * (np.cos(E) - e), a * np.sqrt(1 - e * e) * np.sin(E), 0.0])
        r = a * (1 - e * np.cos(E))
        vrel = np.sqrt(mu * a) / r * np.array([-np.sin(E), np.sqrt(1 - e * e) * np.cos(E), 0.0])
        R = np.linalg.qr(rng.normal(size=(3, 3)))[0]
        rel, vrel = R @ rel, R @ vrel
        for k, ax in enumerate("xyz"):
            d[ax][c] = d[ax][h] + rel[k]
            d["v" + ax][c] = d["v" + ax][h] + vrel[k]

    host = rng.choice(n // 2, n_bin, replace=False)
    comp = n // 2 + np.arange(n_bin)
    for h, c in zip(host, comp):
        attach(h, c)
    for k, c in enumerate(comp[::4]):
        attach(c, n // 2 + n_bin + k)
    return d


def test_neighbours_and_subsystems_parity(ctx):
    n = 3000
    d = _cluster_with_binaries(n, 1)
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    kw = dict(r_ngb=R_NGB, r_max=0.05, C=0.5, tau=1e-3)
    ref = oracle.neighbours(P, **kw)
    got = ctx.neighbours(Pd, cap=16, **kw).cpu().numpy()  # too small at first: the binding retries
    assert len(ref) > 80
    np.testing.assert_array_equal(got, ref)
    lab_ref = oracle.subsystems(n, ref)
    lab, nsub = ctx.subsystems(n, torch.as_tensor(got, device="cuda"))
    np.testing.assert_array_equal(lab.cpu().numpy(), lab_ref)
    sizes = np.bincount(lab_ref, minlength=n)
    assert nsub == int(np.sum(sizes >= 2)) > 30
    assert np.any(sizes >= 3)
    assert ctx.read_flags() == 0


def test_neighbours_on_a_level_and_empty_graph(ctx):
    """Targets a level (index list), sources all; and a graph without edges."""
    n = 2000
    d = _cluster_with_binaries(n, 2, 30)
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    T = np.sort(np.random.default_rng(3).choice(n, 300, replace=False))
    kw = dict(r_ngb=R_NGB, r_max=0.05, C=0.5, tau=1e-3)
    ref = oracle.neighbours(P, T, None, **kw)
    got = ctx.neighbours(Pd, T, None, **kw).cpu().numpy()
    np.testing.assert_array_equal(got, ref)
    lab, nsub = ctx.subsystems(50, torch.zeros((0, 2), dtype=torch.int32, device="cuda"))
    assert np.array_equal(lab.cpu().numpy(), np.arange(50)) and nsub == 0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_exclusion_parity(ctx, prec):
    """Accelerations, gradient sums and time-steps with the subsystem labels set."""
    n = 2500
    d = _cluster_with_binaries(n, 4)
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    lab_ref = oracle.subsystems(n, oracle.neighbours(P, r_ngb=R_NGB, r_max=0.05))
    assert np.sum(np.bincount(lab_ref) >= 2) > 25
    lab = torch.as_tensor(lab_ref.astype(np.int32), device="cuda")
    idx = np.arange(n)
    try:
        ctx.set_subsystems(lab)
        a_ref, mag = oracle.forces(P, sub=lab_ref, return_mag=True)[:2]
        a = gather(ctx.forces(Pd, prec=prec, r_fb=0.0), idx)
        af = np.ascontiguousarray(a_ref)
        g_ref, gmag = oracle.gradient(P, af, sub=lab_ref, return_mag=True)[:2]
        g = gather(ctx.force_gradient(Pd, [torch.as_tensor(np.ascontiguousarray(af[:, k]), device="cuda")
                                           for k in range(3)], prec=prec, r_fb=0.0), idx)
        ff_ref, fb_ref = oracle.dt_min(P, eta_ff=0.2, eta_fb=0.2, sub=lab_ref)
        ff, fb = ctx.dt_min(Pd, eta_ff=0.2, eta_fb=0.2, prec=prec)
        ff, fb = ff.cpu().numpy(), fb.cpu().numpy()
        if prec == "fp64":
            assert np.all(np.linalg.norm(a - a_ref, axis=1) <= 1e-12 * mag)
            assert np.all(np.linalg.norm(g - g_ref, axis=1) <= 1e-12 * gmag)
            np.testing.assert_allclose(ff, ff_ref, rtol=1e-13)
            np.testing.assert_allclose(fb, fb_ref, rtol=1e-13)
        else:
            for got, ref in ((a, a_ref), (g, g_ref)):
                rms, mx = stats(rel_errors(got, ref))
                assert rms <= RMS_TOL and mx <= MAX_TOL, (rms, mx)
            np.testing.assert_allclose(ff, ff_ref, rtol=1e-6)
            np.testing.assert_allclose(fb, fb_ref, rtol=1e-6)
        with pytest.raises(bf.BifrostError):  # another particle count
            ctx.forces(bf.Particles.from_numpy({k: v[:100] for k, v in d.items()}), prec=prec)
    finally:
        ctx.set_subsystems(None)
    # cleared: back to all pairs
    a_all = gather(ctx.forces(Pd, prec="fp64"), idx)
    np.testing.assert_allclose(a_all, oracle.forces(P), rtol=1e-9, atol=1e-9 * np.abs(a_all).max())


def test_fsi_step_with_subsystems(ctx):
    n = 1500
    d = _cluster_with_binaries(n, 5, 40)
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    lab_ref = oracle.subsystems(n, oracle.neighbours(P, r_ngb=R_NGB, r_max=0.05))
    lab = torch.as_tensor(lab_ref.astype(np.int32), device="cuda")
    oracle.fsi_step(P, 1e-4, sub=lab_ref)
    try:
        ctx.set_subsystems(lab)
        ctx.fsi_step(Pd, 1e-4, prec="fp64")
    finally:
        ctx.set_subsystems(None)
    for k in ("x", "vx", "vy", "vz"):
        ref, got = getattr(P, k), getattr(Pd, k).cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), k
