"""Reduced outputs on the GPU: the per-phenotype best test and the thresholded
hit list, against the FP64 oracle, with the dense outputs switched off.

The best test of a column is unique up to near-ties: the GPU's -log10 p must
match the oracle's maximum within the -log10 p tolerance, and the marker it
names must reach that maximum within the same tolerance.  Hit lists are sets:
tests whose oracle -log10 p lies within the tolerance of the threshold may fall
either way; every other test must be in the list exactly when it reaches the
threshold, with its -log10 p and r within tolerance.
"""
import numpy as np
import pytest
import torch

from synth import cohort_spec, pack_codes_np, row_bytes_for
from tests.gpu_common import P_TOL, R_TOL, cohort_arrays, lib, oracle_scan, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tgw():
    t = lib()
    t.init()
    return t


def _tol(ref_nl):
    return P_TOL * np.maximum(ref_nl, 1.0)


def _workload():
    """cfg1 markers plus three planted markers strong enough for the FP64 tail (|t| > 40)."""
    spec = cohort_spec("cfg1")
    codes, _, C, Y = cohort_arrays(spec, np.arange(3000))
    rng = np.random.default_rng(11)
    n = spec.n_samples
    strong = rng.integers(0, 3, size=(3, n)).astype(np.uint8)
    codes = np.concatenate([codes, strong])
    Y = Y.astype(np.float64)
    Y[:, 0] += 6.0 * strong[0]
    Y[:, 5] += 4.0 * strong[1]
    Y[:, 9] += 0.9 * strong[2]
    return codes, C, Y.astype(np.float32)


def _check_best(nl, marker, ref):
    rn = np.where(np.isnan(ref["nlog10p"]), -np.inf, ref["nlog10p"])
    ref_max = rn.max(axis=0)
    tol = _tol(ref_max)
    assert np.all(np.abs(nl - ref_max) <= tol), float(np.max(np.abs(nl - ref_max) - tol))
    chosen = rn[marker, np.arange(rn.shape[1])]
    assert np.all(ref_max - chosen <= 2 * tol)
    return float(np.max(np.abs(nl - ref_max)))


def _check_hits(h, ref, thr, panel=0):
    rn = ref["nlog10p"]
    sel = h["panel"] == panel
    got = set(zip(h["marker"][sel].tolist(), h["pheno"][sel].tolist()))
    assert len(got) == int(sel.sum()), "duplicate hits"
    tol = _tol(np.nan_to_num(rn, nan=0.0))
    sure_in = set(zip(*np.nonzero(np.nan_to_num(rn, nan=-1.0) >= thr + tol)))
    maybe = set(zip(*np.nonzero(np.abs(np.nan_to_num(rn, nan=-1e9) - thr) <= tol)))
    missing = sure_in - got
    extra = got - sure_in - maybe
    assert not missing, sorted(missing)[:5]
    assert not extra, sorted(extra)[:5]
    m, p = h["marker"][sel], h["pheno"][sel]
    assert np.all(np.abs(h["nlog10p"][sel] - rn[m, p]) <= tol[m, p])
    assert np.all(np.abs(h["r"][sel] - ref["r"][m, p]) <= R_TOL)
    return len(got)


@pytest.mark.parametrize("precision", ["split8", "split", "fp32"])
def test_best_and_hits_without_dense_outputs(tgw, precision):
    codes, C, Y = _workload()
    m, n = codes.shape
    p = Y.shape[1]
    say(f"case: reduced outputs {precision}, N={n} M={m} P={p}")
    ref = oracle_scan(codes, C, Y)
    assert np.nanmax(ref["nlog10p"]) > 300  # the FP64 tail is exercised
    cov = tgw.fit_covariates(torch.from_numpy(C).cuda())
    panel = tgw.prepare_phenotypes(cov, torch.from_numpy(Y).cuda(), precision)
    plan = tgw.Plan([panel])
    thr = 6.0
    hits, count = tgw.make_hits(4096)
    plan.set_hits(hits, count, thr)
    best = tgw.make_best([p])
    g = torch.from_numpy(pack_codes_np(codes, row_bytes_for(n))).cuda()
    plan.scan(g, [{"best": best[0]}])
    n_tail = plan.check()
    assert n_tail == int(np.sum(np.abs(ref["t"]) > 40))
    nl, marker = tgw.unpack_best(best[0])
    err = _check_best(nl, marker, ref)
    h = tgw.read_hits(hits, count)
    assert h["count"] <= 4096
    nh = _check_hits(h, ref, thr)
    say(f"[reduced {precision}] best max |d -log10 p| {err:.3g}; {nh} hits at -log10 p >= {thr}")
    assert nh > 20


def test_reduced_outputs_split_over_calls_and_overflow(tgw):
    """Two marker ranges merge into the same best and the same hit set as one
    call; a short list is truncated but still counts every hit.  The ranges
    split at a multiple of 512 markers: the FP16 hi + FP8 lo form adds a
    fragment's FP8 term at a step that depends on the marker's row in the
    512-marker tile, so only tile-aligned splits are bitwise identical."""
    codes, C, Y = _workload()
    m, n = codes.shape
    p = Y.shape[1]
    say("case: reduced outputs over two calls, overflow")
    cov = tgw.fit_covariates(torch.from_numpy(C).cuda())
    panel = tgw.prepare_phenotypes(cov, torch.from_numpy(Y).cuda(), "split8")
    plan = tgw.Plan([panel])
    g = torch.from_numpy(pack_codes_np(codes, row_bytes_for(n))).cuda()
    hits1, count1 = tgw.make_hits(4096)
    plan.set_hits(hits1, count1, 5.0)
    best1 = tgw.make_best([p])
    plan.scan(g, [{"best": best1[0]}])
    hits2, count2 = tgw.make_hits(4096)
    plan.set_hits(hits2, count2, 5.0)
    best2 = tgw.make_best([p])
    plan.scan(g, [{"best": best2[0]}], 0, 1024)
    plan.scan(g, [{"best": best2[0]}], 1024, m)
    plan.check()
    assert torch.equal(best1[0], best2[0])
    h1, h2 = tgw.read_hits(hits1, count1), tgw.read_hits(hits2, count2)
    assert h1["count"] == h2["count"]
    key = lambda h: sorted(zip(h["marker"].tolist(), h["pheno"].tolist(), h["nlog10p"].tolist()))
    assert key(h1) == key(h2)
    # overflow: capacity 7
    hits3, count3 = tgw.make_hits(7)
    plan.set_hits(hits3, count3, 5.0)
    plan.scan(g, [{"best": tgw.make_best([p])[0]}])
    plan.check()
    h3 = tgw.read_hits(hits3, count3)
    assert h3["count"] == h1["count"] and len(h3["marker"]) == 7
    assert set(zip(h3["marker"].tolist(), h3["pheno"].tolist())) <= set(zip(h1["marker"].tolist(),
                                                                              h1["pheno"].tolist()))
    # off again: nothing appended, dense outputs agree with the hits
    plan.set_hits(None)
    outs = tgw.make_outputs([p], m, names=("nlog10p",))
    plan.scan(g, outs)
    plan.check()
    dense = outs[0]["nlog10p"].cpu().numpy()
    np.testing.assert_array_equal(dense[h1["marker"], h1["pheno"]], h1["nlog10p"])
    assert int(count1.item()) == h1["count"]


def test_reduced_outputs_batched_panels(tgw):
    """Two panels in one plan: hits carry their panel index; best per panel."""
    codes, C, Y = _workload()
    m, n = codes.shape
    say("case: reduced outputs, two panels")
    Y2 = Y[:, ::-1].copy()[:, :7]
    cov = tgw.fit_covariates(torch.from_numpy(C).cuda())
    panels = [tgw.prepare_phenotypes(cov, torch.from_numpy(Yp).cuda(), "split8") for Yp in (Y, Y2)]
    plan = tgw.Plan(panels)
    hits, count = tgw.make_hits(8192)
    plan.set_hits(hits, count, 6.0)
    best = tgw.make_best([Y.shape[1], Y2.shape[1]])
    plan.scan(torch.from_numpy(pack_codes_np(codes, row_bytes_for(n))).cuda(), [{"best": b} for b in best])
    plan.check()
    h = tgw.read_hits(hits, count)
    for j, Yp in enumerate((Y, Y2)):
        ref = oracle_scan(codes, C, Yp)
        nl, marker = tgw.unpack_best(best[j])
        _check_best(nl, marker, ref)
        _check_hits(h, ref, 6.0, panel=j)


@pytest.mark.parametrize("precision", ["split8", "fp32"])
def test_hit_threshold_above_table_range(tgw, precision):
    """A threshold above -log10 p at |t| = 40 keeps exactly the tail tests that
    reach it: the decision waits for the FP64 value."""
    codes, C, Y = _workload()
    m, n = codes.shape
    say(f"case: hit threshold 1000, {precision}")
    ref = oracle_scan(codes, C, Y)
    thr = 1000.0
    want = set(zip(*np.nonzero(np.nan_to_num(ref["nlog10p"], nan=-1.0) >= thr)))
    assert len(want) == 1
    cov = tgw.fit_covariates(torch.from_numpy(C).cuda())
    plan = tgw.Plan([tgw.prepare_phenotypes(cov, torch.from_numpy(Y).cuda(), precision)])
    hits, count = tgw.make_hits(16)
    plan.set_hits(hits, count, thr)
    plan.scan(torch.from_numpy(pack_codes_np(codes, row_bytes_for(n))).cuda(), [{}])
    plan.check()
    h = tgw.read_hits(hits, count)
    assert set(zip(h["marker"].tolist(), h["pheno"].tolist())) == want
    _check_hits(h, ref, thr)
