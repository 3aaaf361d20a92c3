"""Per-phenotype top-k lists (tgw_outputs.topk) against the FP64 oracle.

For each phenotype the list holds the k tests with the largest |t| (the
largest -log10 p at the panel's df) in decreasing order.  Against the oracle:
the i-th -log10 p equals the oracle's i-th largest within the -log10 p
tolerance, each listed marker's oracle value equals the listed one within it,
and every marker clearly inside the oracle's top k (above its k-th value by
more than the tolerance) is listed.  Lists are built concurrently by many
workgroups, so their order of insertion varies; the result may not: a scan
split over two calls must give the same words as one call, bit for bit.
"""
import numpy as np
import pytest
import torch

from synth import pack_codes_np, row_bytes_for
from tests.gpu_common import lib, oracle_scan, say
from tests.test_gpu_collinear import _workload as collinear_workload
from tests.test_gpu_reduced import _tol, _workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tgw():
    t = lib()
    t.init()
    return t


def _check_topk(nl, marker, ref, k):
    rn = np.where(np.isnan(ref["nlog10p"]), -np.inf, ref["nlog10p"])
    m, p = rn.shape
    order = np.argsort(-rn, axis=0, kind="stable")[:k]          # oracle top k per column
    ref_sorted = np.take_along_axis(rn, order, axis=0)            # (k, P)
    worst = 0.0
    for c in range(p):
        n_valid = int(np.isfinite(rn[:, c]).sum())
        kk = min(k, n_valid)
        assert np.all(marker[c, kk:] == -1) and np.all(np.isnan(nl[c, kk:])), c
        got_nl, got_m = nl[c, :kk], marker[c, :kk]
        want = ref_sorted[:kk, c]
        tol = _tol(want)
        assert np.all(np.abs(got_nl - want) <= tol), (c, got_nl, want)
        at_m = rn[got_m, c]
        assert np.all(np.abs(at_m - got_nl) <= _tol(at_m)), (c, at_m, got_nl)
        assert len(set(got_m.tolist())) == kk
        sure = set(order[:kk, c][want > want[-1] + tol[-1]].tolist())
        assert sure <= set(got_m.tolist()), (c, sorted(sure - set(got_m.tolist())))
        worst = max(worst, float(np.max(np.abs(got_nl - want))))
    return worst


@pytest.mark.parametrize("precision", ["split8", "split", "fp32"])
def test_topk_against_oracle_and_split_calls(tgw, precision):
    codes, C, Y = _workload()
    m, n = codes.shape
    p = Y.shape[1]
    k = 10
    say(f"case: top-{k} {precision}, N={n} M={m} P={p}")
    ref = oracle_scan(codes, C, Y)
    g = torch.from_numpy(pack_codes_np(codes, row_bytes_for(n))).cuda()
    cov = tgw.fit_covariates(torch.from_numpy(C).cuda())
    panel = tgw.prepare_phenotypes(cov, torch.from_numpy(Y).cuda(), precision)
    plan = tgw.Plan([panel])
    one = tgw.make_topk([p], k)[0]
    best = tgw.make_best([p])[0]
    plan.scan(g, [{"topk": one, "best": best}])
    plan.check()
    nl, marker = [x.cpu().numpy() for x in tgw.read_topk(panel, one)]
    worst = _check_topk(nl, marker, ref, k)
    # the first entry is the best test
    nlb, mb = tgw.unpack_best(best)
    assert np.array_equal(marker[:, 0], mb)
    assert np.all(np.abs(nl[:, 0] - nlb) <= _tol(nlb))
    # the same markers in two calls merge into the same words (a boundary at a
    # multiple of 512 markers keeps every test's arithmetic, so its |t|, unchanged)
    two = tgw.make_topk([p], k)[0]
    plan.scan(g, [{"topk": two}], 0, 1024)
    plan.scan(g, [{"topk": two}], 1024, m)
    plan.check()
    assert torch.equal(one, two)
    say(f"top-{k} {precision}: max |d -log10 p| {worst:.3g}; two calls equal one")


def test_topk_more_slots_than_markers(tgw):
    codes, C, Y = _workload()
    codes = codes[:40]
    m, n = codes.shape
    p = Y.shape[1]
    say(f"case: top-64 of {m} markers")
    ref = oracle_scan(codes, C, Y)
    g = torch.from_numpy(pack_codes_np(codes, row_bytes_for(n))).cuda()
    cov = tgw.fit_covariates(torch.from_numpy(C).cuda())
    panel = tgw.prepare_phenotypes(cov, torch.from_numpy(Y).cuda(), "split8")
    tk = tgw.make_topk([p], 64)[0]
    tgw.Plan([panel]).scan(g, [{"topk": tk}])
    nl, marker = [x.cpu().numpy() for x in tgw.read_topk(panel, tk)]
    _check_topk(nl, marker, ref, 64)


def test_topk_collinear_markers_and_two_panels(tgw):
    """Markers finished on the FP64 path enter the lists too; two panels in one plan."""
    codes, C, Y = collinear_workload(seed=406)
    m, n = codes.shape
    p = Y.shape[1]
    k = 5
    say(f"case: top-{k}, covariate-collinear markers, two panels")
    C2 = np.ascontiguousarray(C[:, -1:])
    refs = [oracle_scan(codes, C, Y), oracle_scan(codes, C2, Y)]
    covs = [tgw.fit_covariates(torch.from_numpy(np.ascontiguousarray(c)).cuda()) for c in (C, C2)]
    Yd = torch.from_numpy(Y).cuda()
    panels = [tgw.prepare_phenotypes(cv, Yd, "split8") for cv in covs]
    lists = tgw.make_topk([p, p], k)
    g = torch.from_numpy(pack_codes_np(codes, row_bytes_for(n))).cuda()
    tgw.Plan(panels, block_markers=1024).scan(g, [{"topk": lists[0]}, {"topk": lists[1]}])
    for j in range(2):
        nl, marker = [x.cpu().numpy() for x in tgw.read_topk(panels[j], lists[j])]
        worst = _check_topk(nl, marker, refs[j], k)
        say(f"panel {j}: max |d -log10 p| {worst:.3g}")
