"""The simplex refinement through the entry point that allocates nothing
(nm_refine_noalloc, state in a static device array) against nm_refine run in
the same launch configuration (64 lanes per trial point, no saved roots): bit
for bit, on two calls in a row, the second with fewer lightcurves, so that
the second call runs over what the first left in the array."""
import numpy as np
import pytest
import torch

from paper_1208_4830_amd import inputs
from tests.helpers import oracle_lightcurves

pytestmark = pytest.mark.gpu

LO, HI = inputs.PRIOR_LO, inputs.PRIOR_HI
MAX_LC = 9936  # lightcurves whose simplices fit the 8 MiB array


def _lightcurves(hip, lengths, seed):
    wl = inputs.uniform_workload(seed, len(lengths), max(max(lengths), 1))
    L0 = max(max(lengths), 1)
    ts, off = [], [0]
    for k, L in enumerate(lengths):
        ts.append(wl.t[k * L0:k * L0 + L])
        off.append(off[-1] + L)
    wl.t, wl.off = np.concatenate(ts), np.array(off, np.int64)
    wl.sfrac, wl.noise = wl.sfrac[:wl.t.size], wl.noise[:wl.t.size]
    y, w = oracle_lightcurves(wl)
    cu = lambda a, dt=torch.float64: torch.tensor(a, dtype=dt, device="cuda")
    lcs = hip.Lightcurves(cu(wl.off, torch.int64), cu(wl.t), cu(y), cu(w))
    rng = np.random.default_rng(seed + 1)
    x0 = np.clip((wl.theta - LO[:, None]) / (HI - LO)[:, None]
                 + rng.normal(scale=0.03, size=wl.theta.shape), 0, 1)
    return lcs, torch.tensor(x0, device="cuda")


def test_noalloc_refine_equals_refine(hip, monkeypatch):
    cfg = hip.nm_default_config()
    cfg.max_iter = 120
    # first call: 40 lightcurves (ragged, one empty); second: 7 lightcurves
    cases = [([300, 0, 257, 64] * 10, 51), ([120, 33, 0, 300, 5, 1, 200], 52)]
    for lengths, seed in cases:
        print(f"no-alloc simplex: {len(lengths)} lightcurves, seed {seed}", flush=True)
        lcs, x0 = _lightcurves(hip, lengths, seed)
        st_a, st_b = hip.new_stats(), hip.new_stats()
        got = hip.nm_refine_noalloc(lcs, LO, HI, x0, cfg, stats=st_a)
        torch.cuda.synchronize()
        monkeypatch.setenv("SBLM_NM_LANES", "64")
        ref = hip.nm_refine(lcs, LO, HI, x0, cfg, stats=st_b)
        monkeypatch.delenv("SBLM_NM_LANES")
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a.cpu().view(torch.uint8), b.cpu().view(torch.uint8))
        assert hip.stats_dict(st_a) == hip.stats_dict(st_b)
        assert hip.stats_dict(st_a)["n_unsettled"] == 0


def test_noalloc_refine_rejects_beyond_the_array(hip):
    # MAX_LC + 1 empty lightcurves: refused on the host, before any launch
    n = MAX_LC + 1
    cu = lambda a, dt=torch.float64: torch.tensor(a, dtype=dt, device="cuda")
    lcs = hip.Lightcurves(cu(np.zeros(n + 1, np.int64), torch.int64), cu(np.zeros(1)),
                          cu(np.zeros(1)), cu(np.zeros(1)))
    x0 = torch.full((6, n), 0.5, dtype=torch.float64, device="cuda")
    with pytest.raises(hip.SblmError, match="9936"):
        hip.nm_refine_noalloc(lcs, LO, HI, x0)
    # the largest batch it takes: MAX_LC empty lightcurves run to completion
    lcs = hip.Lightcurves(cu(np.zeros(MAX_LC + 1, np.int64), torch.int64), cu(np.zeros(1)),
                          cu(np.zeros(1)), cu(np.zeros(1)))
    x0 = torch.full((6, MAX_LC), 0.5, dtype=torch.float64, device="cuda")
    x, c, _, _, it = hip.nm_refine_noalloc(lcs, LO, HI, x0)
    assert torch.all(c == 0)
