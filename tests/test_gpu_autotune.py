"""GPU tests of the launch shapes the autotuner chooses between, and of the tuners themselves:
every pair-symmetric shape and every batched shape keeps parity with the FP64 oracle; the
tuners store their choice (directed, symmetric and batched entries of the table), the passes
then run it, and a fresh context loading the cache plans the same shapes."""
import json

import numpy as np
import pytest
import torch

import oracle
from paper_2210_02472_amd import ics
from tests._parity import gather, rel_errors, smooth_acc_field, stats

bf = pytest.importorskip("paper_2210_02472_amd")

pytestmark = pytest.mark.gpu

RMS_TOL, MAX_TOL = 1e-6, 1e-5


def _check_mixed(got, ref):
    rms, mx = stats(rel_errors(got, ref))
    assert rms <= RMS_TOL and mx <= MAX_TOL, (rms, mx)


def _field(af):
    return [torch.as_tensor(np.ascontiguousarray(af[:, k]), device="cuda") for k in range(3)]


@pytest.fixture(scope="module")
def king():
    n = 9000  # 141 tiles: 9 blocks of 16 tiles, the last one ragged
    d = ics.king_cluster(ics.rng_for(110), n, 6.0, 0.01)
    return d, oracle.Particles.from_dict(d)


@pytest.mark.parametrize("shape", [(1, 16), (2, 8), (4, 4)])
@pytest.mark.parametrize("rounds", [1, 4])
def test_symmetric_shapes_parity(king, shape, rounds):
    """Each shape of the pair-symmetric sweep (row tiles per wavefront x waves) and share count,
    forced, over every target of a King cluster against the oracle (acceleration and gradient)."""
    d, P = king
    n = len(d["m"])
    rows, waves = shape
    with bf.Context(0) as ctx:
        ctx.set_spatial_sort(True, True, any_size=True)
        Pd = bf.Particles.from_numpy(d)
        for op in (bf.BF_OP_FORCES, bf.BF_OP_GRADIENT):
            ctx.set_symmetric_config(op, rows, waves, rounds)
        a = ctx.forces(Pd, prec="mixed")
        kind, k, w, _ = ctx.last_pass_config()
        assert (kind, k, w) == ("symmetric", rows, waves)
        _check_mixed(gather(a, np.arange(n)), oracle.forces(P))
        af = smooth_acc_field(d)
        g = ctx.force_gradient(Pd, _field(af), prec="mixed")
        assert ctx.last_pass_config()[:3] == ("symmetric", rows, waves)
        _check_mixed(gather(g, np.arange(n)), oracle.gradient(P, af))
        assert ctx.read_flags() == 0


def _ensemble(sizes, fracs, seed):
    parts, act, off, aoff = [], [], [0], [0]
    for c, (n, f) in enumerate(zip(sizes, fracs)):
        rng = ics.rng_for(300 + seed, c)
        parts.append(ics.plummer_cluster(rng, n, "kroupa"))
        a = ics.random_subset(rng, n, f).astype(np.int64) + off[-1]
        act.append(a)
        off.append(off[-1] + n)
        aoff.append(aoff[-1] + a.size)
    d = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    return d, np.array(off, np.int64), np.concatenate(act).astype(np.int32), np.array(aoff, np.int64)


SIZES = [300, 9100, 2, 4500, 1]
FRACS = [1.0, 0.25, 1.0, 1 / 16, 1.0]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", [(1, 4, 2048), (2, 4, 4096), (4, 4, 8192), (1, 8, 2048), (2, 8, 4096),
                                   (4, 8, 8192)])
def test_batched_shapes_parity(prec, shape):
    """Each batched shape (targets per lane, waves, sources per work item), forced, over a mixed
    ensemble (a cluster larger than two work items, tiny clusters, ragged slabs) against the
    oracle per cluster: accelerations and gradient sums."""
    d, off, act, aoff = _ensemble(SIZES, FRACS, 0)
    P = oracle.Particles.from_dict(d)
    co, ai, ao = (torch.as_tensor(x, device="cuda") for x in (off, act, aoff))
    k, w, chunk = shape
    af = smooth_acc_field(d)
    with bf.Context(0) as ctx:
        Pd = bf.Particles.from_numpy(d)
        for op in (bf.BF_OP_FORCES, bf.BF_OP_GRADIENT):
            ctx.set_batched_config(op, prec, k, w, chunk)
        a = ctx.forces_batched(Pd, co, ai, ao, int(aoff[-1]), max(SIZES), prec=prec)
        g = ctx.force_gradient_batched(Pd, co, ai, ao, int(aoff[-1]), max(SIZES), _field(af), prec=prec)
        assert ctx.read_flags() & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0
    for c in range(len(SIZES)):
        if SIZES[c] == 1:
            continue
        T = act[aoff[c]:aoff[c + 1]]
        S = np.arange(off[c], off[c + 1])
        ra, ma, _ = oracle.forces(P, T, S, return_mag=True)
        rg, mg, _ = oracle.gradient(P, af, T, S, return_mag=True)
        for got, ref, mag in ((gather(a, T), ra, ma), (gather(g, T), rg, mg)):
            if prec == "fp64":
                assert np.all(np.linalg.norm(got - ref, axis=1) <= 1e-12 * mag), c
            else:
                _check_mixed(got, ref)


def test_autotune_pass_symmetric_and_directed(king, tmp_path):
    """Tuning on the caller's particles: a pass over one set stores a symmetric entry (its shape
    and rounds), a level against all particles a directed one (with its split); the next passes
    run the tuned shapes and keep parity; a fresh context loading the cache runs them too."""
    d, P = king
    n = len(d["m"])
    cache = str(tmp_path / "tune.json")
    lvl = np.sort(np.random.default_rng(2).choice(n, 1200, replace=False)).astype(np.int32)
    T = torch.as_tensor(lvl, device="cuda")
    af = smooth_acc_field(d)
    with bf.Context(0) as ctx:
        ctx.set_spatial_sort(True, True, any_size=True)
        Pd = bf.Particles.from_numpy(d)
        ctx.autotune_pass(bf.BF_OP_GRADIENT, "mixed", Pd, acc=_field(af), cache_path=cache)
        ctx.autotune_pass(bf.BF_OP_FORCES, "mixed", Pd, T, None, cache_path=cache)
        table = json.load(open(cache))
        sym = [e for e in table if e["sweep"] == 1 and e["op"] == bf.BF_OP_GRADIENT]
        dire = [e for e in table if e["sweep"] == 0 and e["op"] == bf.BF_OP_FORCES]
        assert len(sym) == 1 and len(dire) == 1, table
        g = ctx.force_gradient(Pd, _field(af), prec="mixed")
        assert ctx.last_pass_config()[:3] == ("symmetric", sym[0]["k"], sym[0]["waves"])
        _check_mixed(gather(g, np.arange(n)), oracle.gradient(P, af))
        a = ctx.forces(Pd, T, None, prec="mixed")
        kind, k, w, split = ctx.last_pass_config()
        assert (k, w) == (dire[0]["k"], dire[0]["waves"])
        if dire[0]["split"] > 0:
            assert split == dire[0]["split"]
        _check_mixed(gather(a, lvl), oracle.forces(P, lvl, None))
    with bf.Context(0) as other:
        other.set_spatial_sort(True, True, any_size=True)
        other.autotune_load(cache)
        Pd = bf.Particles.from_numpy(d)
        other.force_gradient(Pd, _field(af), prec="mixed")
        assert other.last_pass_config()[:3] == ("symmetric", sym[0]["k"], sym[0]["waves"])


def test_autotune_batched_round_trip(tmp_path):
    """Tuning the batched passes on the caller's ensemble stores batched entries; the passes use
    them (results keep parity), and the cache loads into a fresh context."""
    d, off, act, aoff = _ensemble(SIZES, FRACS, 1)
    P = oracle.Particles.from_dict(d)
    co, ai, ao = (torch.as_tensor(x, device="cuda") for x in (off, act, aoff))
    af = smooth_acc_field(d)
    cache = str(tmp_path / "tune_b.json")
    na = int(aoff[-1])
    with bf.Context(0) as ctx:
        Pd = bf.Particles.from_numpy(d)
        ctx.autotune_batched(bf.BF_OP_FORCES, "mixed", Pd, co, ai, ao, na, max(SIZES), cache_path=cache)
        ctx.autotune_batched(bf.BF_OP_GRADIENT, "mixed", Pd, co, ai, ao, na, max(SIZES), acc=_field(af),
                             cache_path=cache)
        table = json.load(open(cache))
        assert sorted(e["op"] for e in table if e["sweep"] == 2) == [bf.BF_OP_FORCES, bf.BF_OP_GRADIENT], table
        a = ctx.forces_batched(Pd, co, ai, ao, na, max(SIZES), prec="mixed")
        g = ctx.force_gradient_batched(Pd, co, ai, ao, na, max(SIZES), _field(af), prec="mixed")
    for c in range(len(SIZES)):
        if SIZES[c] == 1:
            continue
        T = act[aoff[c]:aoff[c + 1]]
        S = np.arange(off[c], off[c + 1])
        _check_mixed(gather(a, T), oracle.forces(P, T, S))
        _check_mixed(gather(g, T), oracle.gradient(P, af, T, S))
    with bf.Context(0) as other:
        other.autotune_load(cache)  # the entries parse and name existing shapes


def test_autotune_cache_of_directed_entries_without_sweep(tmp_path):
    """Tables written before the sweep kind existed (directed entries only) still load."""
    cache = tmp_path / "old.json"
    cache.write_text('[\n  {"op": 0, "prec": 1, "nt_log2": 14, "ns_log2": 14, "k": 1, "waves": 8, "split": 16}\n]\n')
    with bf.Context(0) as ctx:
        ctx.autotune_load(str(cache))
        assert ctx.query_config(bf.BF_OP_FORCES, "mixed", 20000, 20000) == (1, 8, 16)
