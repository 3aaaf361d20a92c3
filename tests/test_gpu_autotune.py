"""The autotuner and its cache, through the C ABI.

tgw_plan_autotune times every distinct tile shape on a block of markers and
keeps the fastest; the choice is written to a JSON cache keyed by (device,
padded samples, column blocks, panels, precision), which later plans with the
same key read instead of timing.  Checked: the cache entry the call writes, a
later plan taking it, a plan following an edited entry, and the autotuned
plan's outputs equal bit for bit to a plan fixed to the chosen shape (and
within tolerance of the oracle).
"""
import json

import numpy as np
import pytest
import torch

from synth import cohort_spec
from tests.gpu_common import cohort_arrays, compare, lib, oracle_scan, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tgw():
    t = lib()
    t.init()
    return t


def _same(a: torch.Tensor, b: torch.Tensor) -> bool:
    return torch.equal(a.view(torch.int32), b.view(torch.int32))  # bitwise, NaN included


@pytest.mark.parametrize("precision", ["split8", "split"])
def test_autotune_cache_round_trip(tgw, precision, tmp_path, monkeypatch):
    cache = tmp_path / "tune" / "tune.json"  # the library creates the directory
    monkeypatch.setenv("TGW_TUNE_CACHE", str(cache))
    spec = cohort_spec("cfg1", n_markers=3000)
    codes, packed, C, Y = cohort_arrays(spec, np.arange(spec.n_markers))
    say(f"case: autotune {precision}, N={spec.n_samples} M={spec.n_markers} P={Y.shape[1]}")
    g = torch.from_numpy(packed).cuda()
    cov = tgw.fit_covariates(torch.from_numpy(C).cuda())
    panel = tgw.prepare_phenotypes(cov, torch.from_numpy(Y).cuda(), precision)
    M, P = codes.shape[0], Y.shape[1]

    plan = tgw.Plan([panel])
    assert not cache.exists()
    ms = plan.autotune(g, tgw.make_outputs([P], M), 0, M)
    assert ms > 0.0
    chosen = plan.info()["tile"]
    n_tiles = plan.info()["n_tiles"]
    entries = json.loads(cache.read_text())
    assert len(entries) == 1, entries
    (key, tile), = entries.items()
    assert tile == chosen and 0 <= chosen < n_tiles
    prec_id = {"split8": tgw.PREC_SPLIT_F8, "split": tgw.PREC_SPLIT}[precision]
    assert key.endswith(f"prec{prec_id}"), key
    say(f"autotune chose tile {chosen} ({ms:.3f} ms), cache key {key}")

    # a new plan with the same key takes the cached shape without timing
    assert tgw.Plan([panel]).info()["tile"] == chosen
    # and follows the cache when it changes
    other = (chosen + 1) % n_tiles
    cache.write_text(json.dumps({key: other}))
    assert tgw.Plan([panel]).info()["tile"] == other
    # an explicit tile overrides the cache
    assert tgw.Plan([panel], tile=chosen).info()["tile"] == chosen

    # the autotuned plan's outputs are those of the fixed shape it chose
    outs_a = tgw.scan(plan, g)
    outs_f = tgw.scan(tgw.Plan([panel], tile=chosen), g)
    for k in outs_a[0]:
        assert _same(outs_a[0][k], outs_f[0][k]), k
    ref = oracle_scan(codes, C, Y)
    compare({k: v.cpu().numpy() for k, v in outs_a[0].items()}, ref, ref["df"], f"autotuned {precision} ")
