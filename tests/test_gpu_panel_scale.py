"""Panel scale at full size: N = 23,000 samples, M = 1,000,000 markers,
P = 20,480 phenotypes (half of them from a rank-64 factor model), K = 10,
in the FP16 hi + FP8 lo form, against the FP64 oracle.

The full scan runs as the benchmark's panel-scale leg does (one plan, reduced
outputs: the per-phenotype best test and the hit list at -log10 p >= 7.3).
The oracle cannot redo 2e10 tests, so it is run on a sample of marker rows
times all 20,480 columns, and the GPU is checked there:
  - dense outputs of the sampled rows (start, middle and end of M, the causal
    markers, markers drawn from the full scan's hit list, and the best markers
    of a sample of columns), computed by the same plan over those rows;
  - the best test and the hit list of a scan restricted to the sampled rows;
  - the full scan's hit list on every sampled row (complete and exact there),
    and its best test per column: at least every sampled row's oracle value,
    and equal to the oracle's value at the marker it names.
"""
import numpy as np
import pytest
import torch

from synth import causal_markers, cohort_spec, geno_codes_np, pack_codes_np, packed_rows_torch, panel_inputs, \
    row_bytes_for
from tests.gpu_common import compare, lib, oracle_scan, say
from tests.test_gpu_reduced import _check_best, _check_hits, _tol

pytestmark = pytest.mark.gpu

THR = 7.3


@pytest.fixture(scope="module")
def tgw():
    t = lib()
    t.init()
    return t


def test_cfg4_panel_scale_sampled(tgw):
    spec = cohort_spec("cfg4")
    M, n = spec.n_markers, spec.n_samples
    say(f"case: cfg4 full scan split8 N={n} M={M}, reduced outputs; sampled parity")
    C, Y = panel_inputs(spec)
    P = Y.shape[1]
    g = torch.empty((M, row_bytes_for(n)), dtype=torch.uint8, device="cuda")
    packed_rows_torch(spec, 0, M, "cuda", out=g, chunk=8192)
    cov = tgw.fit_covariates(torch.from_numpy(C).cuda())
    panel = tgw.prepare_phenotypes(cov, torch.from_numpy(Y).cuda(), "split8")
    plan = tgw.Plan([panel])
    best = tgw.make_best([P])
    hits, count = tgw.make_hits(1 << 22)
    plan.set_hits(hits, count, THR)
    plan.scan(g, [{"best": best[0]}])
    n_tail = plan.check()
    h_full = tgw.read_hits(hits, count)
    nl_best, m_best = tgw.unpack_best(best[0])
    say(f"full scan: {len(h_full['marker'])} hits, {n_tail} tail tests")
    assert int(count.item()) <= (1 << 22)

    rng = np.random.default_rng(4)
    hit_rows = np.unique(h_full["marker"])
    cols = rng.choice(P, 64, replace=False)
    blocks = [np.arange(0, 256), np.arange(M // 2, M // 2 + 256), np.arange(M - 256, M)]
    rows = np.unique(np.concatenate(blocks + [causal_markers(spec),
                                              rng.choice(hit_rows, min(128, len(hit_rows)), replace=False),
                                              m_best[cols]]))
    say(f"sampled rows: {len(rows)} x {P} columns")
    codes = geno_codes_np(spec, rows)
    assert np.array_equal(g[torch.from_numpy(rows).cuda()].cpu().numpy(), pack_codes_np(codes, row_bytes_for(n)))
    ref = oracle_scan(codes, C, Y)

    # dense outputs of the sampled rows, same plan
    hits2, count2 = tgw.make_hits(1 << 20)
    plan.set_hits(hits2, count2, THR)
    sub = g[torch.from_numpy(rows).cuda()].contiguous()
    best2 = tgw.make_best([P])
    outs = tgw.make_outputs([P], len(rows))
    outs[0]["best"] = best2[0]
    plan.scan(sub, outs)
    plan.check()
    got = {k: v.cpu().numpy() for k, v in outs[0].items() if k != "best"}
    compare(got, ref, ref["df"], "cfg4 split8 sampled rows ")
    # reduced outputs of the restricted scan (marker indices are rows of `sub`)
    nl2, m2 = tgw.unpack_best(best2[0])
    err = _check_best(nl2, m2, ref)
    nh = _check_hits(tgw.read_hits(hits2, count2), ref, THR)
    say(f"restricted scan: best max error {err:.3g}, {nh} hits")

    # the full scan's reduced outputs on the sampled rows
    rn = np.where(np.isnan(ref["nlog10p"]), -np.inf, ref["nlog10p"])
    sampled_max = rn.max(axis=0)
    assert np.all(nl_best >= sampled_max - _tol(sampled_max)), "best below a sampled row's -log10 p"
    pos = np.searchsorted(rows, m_best[cols])
    at_best = rn[pos, cols]
    assert np.all(np.abs(nl_best[cols] - at_best) <= _tol(at_best)), float(np.max(np.abs(nl_best[cols] - at_best)))
    in_rows = np.isin(h_full["marker"], rows)
    h_rows = {k: v[in_rows] for k, v in h_full.items() if k != "count"}
    h_rows["marker"] = np.searchsorted(rows, h_rows["marker"])
    nh = _check_hits(h_rows, ref, THR)
    say(f"full scan on the sampled rows: {nh} hits checked, best checked on {len(cols)} columns")
