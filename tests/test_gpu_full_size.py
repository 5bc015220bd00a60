"""Parity at the full sizes of the measured workloads, in the launch configuration bench.py
times (library defaults: spatially sorted mixed passes), on sampled outputs the oracle computes
one by one:

  * King W0 = 6, N = 2^20, all active (the headline sweep): acceleration and gradient;
  * Kroupa Plummer N = 65,536 with a random 10% level, eps = 1e-4: acceleration, gradient and
    time-steps of every active particle;
  * 256-cluster ensemble (about 3.9 million particles): batched accelerations of sampled
    clusters;
  * N = 262,144 cluster with 16 BHs and an IMBH: the deepest level's accelerations and PN1.0.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2210_02472_amd import ics
from tests._parity import gather, rel_errors, smooth_acc_field, stats

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
