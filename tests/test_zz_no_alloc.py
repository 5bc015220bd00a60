"""The allocation-free entry point bf_forces_noalloc (its passes run in a static device array)
against bf_forces and the FP64 oracle: two calls in a row on one context, the second with a
smaller input, in mixed precision and in FP64; the context's own scratch stays empty; sizes
beyond the static array are rejected."""
import numpy as np
import pytest
import torch

import oracle
from paper_2210_02472_amd import ics
from tests._parity import gather, rel_errors, stats

bf = pytest.importorskip("paper_2210_02472_amd")

pytestmark = pytest.mark.gpu

RMS_TOL, MAX_TOL = 1e-6, 1e-5


def _zeros(n):
    return [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_noalloc_matches_forces_on_two_calls(prec):
    # 30,000 listed targets x 40,000 sources (several source chunks, ragged tiles), then 700 x 3,000
    cases = ((40000, 30000, 1), (3000, 700, 2))
    with bf.Context(0) as fresh, bf.Context(0) as ctx:
        for n, nt, seed in cases:
            d = ics.plummer_cluster(ics.rng_for(400, seed), n, "kroupa")
            P = bf.Particles.from_numpy(d)
            tg = np.sort(np.random.default_rng(seed).choice(n, nt, replace=False)).astype(np.int32)
            got = fresh.forces_noalloc(P, tg, None, eps2=1e-8, prec=prec, out=_zeros(n))
            ref = ctx.forces(P, tg, None, eps2=1e-8, prec=prec, out=_zeros(n))
            g, r = gather(got, tg), gather(ref, tg)
            # against the existing entry point, every target
            if prec == "fp64":
                assert np.all(np.linalg.norm(g - r, axis=1) <= 1e-12 * np.linalg.norm(r, axis=1)), (n, nt)
            else:
                rms, mx = stats(rel_errors(g, r))
                assert rms <= RMS_TOL and mx <= MAX_TOL, (n, nt, rms, mx)
            # against the oracle, on sampled targets
            sample = np.sort(np.random.default_rng(seed + 10).choice(nt, min(nt, 400), replace=False))
            Po = oracle.Particles.from_dict(d)
            a_ref, mag, _ = oracle.forces(Po, tg[sample], None, eps2=1e-8, return_mag=True)
            if prec == "fp64":
                assert np.all(np.linalg.norm(g[sample] - a_ref, axis=1) <= 1e-12 * mag), (n, nt)
            else:
                rms, mx = stats(rel_errors(g[sample], a_ref))
                assert rms <= RMS_TOL and mx <= MAX_TOL, (n, nt, rms, mx)
            # entries of non-targets untouched
            rest = np.setdiff1d(np.arange(n), tg)
            assert not got[0].cpu().numpy()[rest].any()
        # the pass took nothing from the context's own (allocated) buffers
        assert fresh.release_scratch() == 0
        assert fresh.read_flags() & (bf.BF_FLAG_NONFINITE | bf.BF_FLAG_BADINDEX) == 0


def test_noalloc_rejects_sizes_beyond_the_static_array():
    """2.2 million sources need 70 MB of packed sources alone: BF_ERR_ARG before any launch,
    outputs untouched."""
    n = 2_200_000
    g = torch.Generator(device="cuda").manual_seed(5)
    arrays = {k: torch.rand(n, dtype=torch.float64, device="cuda", generator=g) for k in bf.Particles.KEYS}
    P = bf.Particles(**arrays)
    out = _zeros(n)
    with bf.Context(0) as ctx:
        with pytest.raises(bf.BifrostError, match="static buffer"):
            ctx.forces_noalloc(P, np.arange(64, dtype=np.int32), None, prec="mixed", out=out)
        torch.cuda.synchronize()
        assert not any(t.any().item() for t in out)
        assert ctx.release_scratch() == 0
