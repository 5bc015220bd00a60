"""GPU parity of the batched ensemble path (one persistent launch over many clusters) and of its
HIP-graph replay, against the FP64 oracle cluster by cluster and against the unbatched path."""
import numpy as np
import pytest
import torch

import oracle
from paper_2210_02472_amd import ics
from tests._parity import rel_errors, stats

bf = pytest.importorskip("paper_2210_02472_amd")

pytestmark = pytest.mark.gpu

RMS_TOL, MAX_TOL = 1e-6, 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = bf.Context(0)
    yield c
    c.close()


def _ensemble(sizes, fracs, seed=0):
    parts, act = [], []
    off = [0]
    aoff = [0]
    for c, (n, f) in enumerate(zip(sizes, fracs)):
        rng = ics.rng_for(200 + seed, c)
        parts.append(ics.plummer_cluster(rng, n, "kroupa"))
        a = ics.random_subset(rng, n, f).astype(np.int64) + off[-1]
        act.append(a)
        off.append(off[-1] + n)
        aoff.append(aoff[-1] + a.size)
    d = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    return d, np.array(off, np.int64), np.concatenate(act).astype(np.int32), np.array(aoff, np.int64)


def _dev_lists(off, act, aoff):
    return (torch.as_tensor(off, device="cuda"), torch.as_tensor(act, device="cuda"),
            torch.as_tensor(aoff, device="cuda"))


SIZES = [1, 300, 4097, 1500, 9000, 2]
FRACS = [1.0, 0.5, 1 / 8, 1.0, 1 / 64, 1.0]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_forces_parity(ctx, prec):
    d, off, act, aoff = _ensemble(SIZES, FRACS)
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    co, ai, ao = _dev_lists(off, act, aoff)
    out = ctx.forces_batched(Pd, co, ai, ao, int(aoff[-1]), int(max(SIZES)), prec=prec)
    got_all = np.stack([t.cpu().numpy() for t in out], axis=1)
    assert ctx.read_flags() & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0
    for c in range(len(SIZES)):
        T = act[aoff[c]:aoff[c + 1]]
        S = np.arange(off[c], off[c + 1])
        ref, mag, _ = oracle.forces(P, T, S, return_mag=True)
        got = got_all[T]
        if SIZES[c] == 1:
            assert np.all(got == 0)
            continue
        if prec == "fp64":
            assert np.all(np.linalg.norm(got - ref, axis=1) <= 1e-12 * mag), c
        else:
            rms, mx = stats(rel_errors(got, ref))
            assert rms <= RMS_TOL and mx <= MAX_TOL, (c, rms, mx)
    # non-active particles untouched
    mask = np.ones(len(d["m"]), bool)
    mask[act] = False
    assert np.all(got_all[mask] == 0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_gradient_parity(ctx, prec):
    d, off, act, aoff = _ensemble(SIZES, FRACS, seed=1)
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    # a of every particle from its own cluster (oracle), as the input field
    a = np.zeros((len(d["m"]), 3))
    for c in range(len(SIZES)):
        S = np.arange(off[c], off[c + 1])
        a[S] = oracle.forces(P, S, S)
    acc = [torch.as_tensor(np.ascontiguousarray(a[:, k]), device="cuda") for k in range(3)]
    co, ai, ao = _dev_lists(off, act, aoff)
    out = ctx.force_gradient_batched(Pd, co, ai, ao, int(aoff[-1]), int(max(SIZES)), acc, prec=prec)
    got_all = np.stack([t.cpu().numpy() for t in out], axis=1)
    for c in range(len(SIZES)):
        if SIZES[c] == 1:
            continue
        T = act[aoff[c]:aoff[c + 1]]
        S = np.arange(off[c], off[c + 1])
        ref, mag, _ = oracle.gradient(P, a, T, S, return_mag=True)
        got = got_all[T]
        if prec == "fp64":
            assert np.all(np.linalg.norm(got - ref, axis=1) <= 1e-12 * mag), c
        else:
            rms, mx = stats(rel_errors(got, ref))
            assert rms <= RMS_TOL and mx <= MAX_TOL, (c, rms, mx)


def test_batched_matches_unbatched(ctx):
    d, off, act, aoff = _ensemble(SIZES, FRACS, seed=2)
    Pd = bf.Particles.from_numpy(d)
    co, ai, ao = _dev_lists(off, act, aoff)
    b = ctx.forces_batched(Pd, co, ai, ao, int(aoff[-1]), int(max(SIZES)), prec="fp64")
    for c in range(len(SIZES)):
        T = torch.as_tensor(act[aoff[c]:aoff[c + 1]], device="cuda")
        u = ctx.forces(Pd, T, bf.ParticleSet.range(int(off[c]), int(off[c + 1] - off[c])), prec="fp64")
        for x, y in zip(b, u):
            xs, ys = x[T.long()], y[T.long()]
            assert torch.allclose(xs, ys, rtol=1e-12, atol=1e-14 * float(ys.abs().max() + 1e-300))


def test_batched_fsi_graph_replays_match_eager(ctx):
    """Replays of the captured batched FSI cycle equal the eager sequence bit for bit, replay after
    replay, with eager work and synchronisations between replays and active sets that change."""
    sizes, fracs = [700, 2000, 1300, 64], [0.5, 0.25, 1.0, 1.0]
    d, off, act, aoff = _ensemble(sizes, fracs, seed=3)
    n = len(d["m"])
    A, B = bf.Particles.from_numpy(d), bf.Particles.from_numpy(d)
    max_active = n
    act_buf = torch.zeros(max_active, dtype=torch.int32, device="cuda")
    aoff_buf = torch.zeros(len(sizes) + 1, dtype=torch.int64, device="cuda")
    co = torch.as_tensor(off, device="cuda")

    def set_active(a_np, ao_np):
        act_buf[:a_np.size] = torch.as_tensor(a_np, device="cuda")
        aoff_buf.copy_(torch.as_tensor(ao_np, device="cuda"))

    set_active(act, aoff)
    # initial accelerations of every particle from its cluster
    accA = ctx.forces_batched(A, co, torch.arange(n, dtype=torch.int32, device="cuda"),
                              torch.as_tensor(off, device="cuda"), n, max(sizes), prec="mixed")
    accB = [t.clone() for t in accA]
    g = ctx.capture_batched_fsi(A, co, act_buf, aoff_buf, max_active, max(sizes), 1e-3, accA, prec="mixed")
    rng = np.random.default_rng(0)
    for rep in range(4):
        if rep == 2:  # new active sets, same buffers
            parts, ao = [], [0]
            for c in range(len(sizes)):
                a = np.sort(rng.choice(sizes[c], max(1, sizes[c] // 3), replace=False)) + off[c]
                parts.append(a)
                ao.append(ao[-1] + a.size)
            set_active(np.concatenate(parts).astype(np.int32), np.array(ao, np.int64))
        g.launch()
        torch.cuda.synchronize()
        ctx.fsi_step_batched(B, co, act_buf, aoff_buf, max_active, max(sizes), 1e-3, accB, prec="mixed")
        torch.cuda.synchronize()
        _ = (A.x * 2).sum().item()  # unrelated eager work between replays
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            assert torch.equal(getattr(A, k), getattr(B, k)), (rep, k)
        for x, y in zip(accA, accB):
            assert torch.equal(x, y), rep
    g.close()
    assert ctx.read_flags() & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0


def test_batched_fsi_matches_oracle(ctx):
    """A batched FSI cycle with all particles active equals the per-cluster oracle FSI cycle."""
    sizes = [500, 1200, 64]
    d, off, act, aoff = _ensemble(sizes, [1.0, 1.0, 1.0], seed=4)
    P, Pd = oracle.Particles.from_dict(d), bf.Particles.from_numpy(d)
    co, ai, ao = _dev_lists(off, act, aoff)
    acc = ctx.forces_batched(Pd, co, ai, ao, int(aoff[-1]), max(sizes), prec="fp64")
    ctx.fsi_step_batched(Pd, co, ai, ao, int(aoff[-1]), max(sizes), 2e-3, acc, prec="fp64")
    for c in range(len(sizes)):
        oracle.fsi_step(P, 2e-3, np.arange(off[c], off[c + 1]))
    for k in ("x", "vy"):
        ref = getattr(P, k)
        assert np.abs(getattr(Pd, k).cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
