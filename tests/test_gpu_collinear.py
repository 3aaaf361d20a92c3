"""Markers nearly inside the covariate span, against the FP64 oracle.

Conditional analysis puts a lead marker's dosage among the covariates; markers
in strong LD with it then keep only a sliver of their variance after the
covariates are projected out (||g_res||^2 / ||g_c||^2 small).  The library
finishes every marker whose ratio is below one half on an FP64 path (explicit
residualization, FP64 contraction with the stored panel operand), so these
markers must meet the same tolerances as any other, down to the degenerate
threshold 1e-8 that the oracle uses; an exact covariate copy gives NaN.

Covariates c_k = g_k + eps_k z_k make marker k collinear to a chosen ratio;
phenotype columns that load on z_k give those markers strong associations
(|t| up to the FP64 tail), so r, t, beta, SE, -log10 p, the per-phenotype best
test and the hit list are all exercised on the FP64 path.
"""
import numpy as np
import pytest
import torch

from synth import dosage8_row_bytes_for, pack_codes_np, row_bytes_for
from tests.gpu_common import compare, decode_codes, gpu_scan, lib, oracle_scan, say
from tests.test_gpu_reduced import _check_best, _check_hits

pytestmark = pytest.mark.gpu

RATIOS = [1e-7, 1e-6, 1e-5, 3e-4, 1e-3, 1e-2, 0.1, 0.3, 0.45]


@pytest.fixture(scope="module")
def tgw():
    t = lib()
    t.init()
    return t


def _collinear_covariates(rng, g_imp, n):
    """Covariates that make markers 1, 4, 7, ... collinear to the ratios RATIOS,
    marker 40 an exact covariate, plus one ordinary covariate; phenotypes that
    load on the noise of each collinear covariate."""
    k_c = len(RATIOS)
    Z = rng.standard_normal((n, k_c))
    cols = []
    for k, rho in enumerate(RATIOS):
        g = g_imp[3 * k + 1]  # markers 1, 4, 7, ...: collinear to ratio about rho
        cols.append(g + np.sqrt(rho * g.var() / (1.0 - rho)) * Z[:, k])
    cols.append(g_imp[40].copy())          # marker 40 is a covariate: degenerate
    cols.append(rng.standard_normal(n))    # an ordinary covariate
    C = np.stack(cols, axis=1)
    p = 3 * k_c + 5
    Y = rng.standard_normal((n, p)) + C @ rng.standard_normal((C.shape[1], p)) * 0.1
    for k in range(k_c):  # columns 3k .. 3k+2 load on z_k: moderate, strong, extreme
        for i, b in enumerate((0.2, 1.0, 12.0)):
            Y[:, 3 * k + i] += b * Z[:, k]
    return C, Y.astype(np.float32)


def _workload(n=5000, m=700, seed=404):
    rng = np.random.default_rng(seed)
    maf = rng.uniform(0.05, 0.5, m)
    codes = rng.binomial(2, maf[:, None], size=(m, n)).astype(np.uint8)
    codes[rng.random((m, n)) < 0.01] = 3
    G = decode_codes(codes)
    g_imp = np.where(np.isnan(G), np.nanmean(G, axis=1)[:, None], G)
    C, Y = _collinear_covariates(rng, g_imp, n)
    return codes, C, Y


@pytest.mark.parametrize("precision", ["split", "split16", "split8", "fp32"])
def test_collinear_markers_dense(tgw, precision):
    codes, C, Y = _workload()
    say(f"case: covariate-collinear markers {precision} n={codes.shape[1]} m={codes.shape[0]} p={Y.shape[1]}")
    packed = pack_codes_np(codes, row_bytes_for(codes.shape[1]))
    ref = oracle_scan(codes, C, Y)
    ratio = ref["h"] ** 2 / ref["gc2"]
    planted = [3 * k + 1 for k in range(len(RATIOS))]
    say("planted ratios: " + ", ".join(f"{ratio[i]:.2g}" for i in planted) + f"; copy {ratio[40]:.2g}")
    assert np.all(np.isfinite(ref["r"][planted]))
    assert np.all(np.isnan(ref["r"][40]))
    # several marker blocks, so the FP64 list is rebuilt per block
    res, _, _ = gpu_scan(C, [Y], packed, precision, plan_kw={"block_markers": 512})
    got = res[0]
    assert np.all(np.isnan(got["r"][40]))
    for i in planted:
        assert np.all(np.isfinite(got["r"][i])), i
    errs = compare(got, ref, ref["df"], f"collinear {precision} ")
    dr = np.abs(got["r"][planted] - ref["r"][planted])
    say(f"collinear {precision}: max |dr| on the planted markers {dr.max():.3g}")
    assert errs["r"] <= 1e-5


def test_collinear_markers_reduced_two_panels(tgw):
    """Best test and hit list from the FP64 path, in a plan whose second panel
    has no collinear covariates (its list stays empty)."""
    codes, C, Y = _workload(seed=405)
    n = codes.shape[1]
    p = Y.shape[1]
    say(f"case: covariate-collinear markers, reduced outputs, two panels n={n} p={p}")
    C2 = C[:, -1:]
    ref1 = oracle_scan(codes, C, Y)
    ref2 = oracle_scan(codes, C2, Y)
    cov1 = tgw.fit_covariates(torch.from_numpy(C).cuda())
    cov2 = tgw.fit_covariates(torch.from_numpy(np.ascontiguousarray(C2)).cuda())
    Yd = torch.from_numpy(Y).cuda()
    panels = [tgw.prepare_phenotypes(cov1, Yd, "split8"), tgw.prepare_phenotypes(cov2, Yd, "split8")]
    plan = tgw.Plan(panels, block_markers=1024)
    best = tgw.make_best([p, p])
    hits, count = tgw.make_hits(1 << 16)
    thr = 7.3
    plan.set_hits(hits, count, thr)
    g = torch.from_numpy(pack_codes_np(codes, row_bytes_for(n))).cuda()
    plan.scan(g, [{"best": best[0]}, {"best": best[1]}])
    plan.check()
    h = tgw.read_hits(hits, count)
    for j, ref in enumerate((ref1, ref2)):
        nl, marker = tgw.unpack_best(best[j])
        err = _check_best(nl, marker, ref)
        nh = _check_hits(h, ref, thr, panel=j)
        say(f"panel {j}: best max error {err:.3g}, {nh} hits")
    planted = [3 * k + 1 for k in range(len(RATIOS))]
    nl, marker = tgw.unpack_best(best[0])
    # the extreme columns pick their collinear marker, through the FP64 path
    assert np.all(marker[[3 * k + 2 for k in range(len(RATIOS))]] == np.array(planted))


@pytest.mark.parametrize("precision", ["split16", "fp32"])
def test_collinear_markers_dosage8(tgw, precision):
    """The FP64 path reads 8-bit dosage rows too (q / 127 copies, 255 missing)."""
    n, m = 5000, 700
    rng = np.random.default_rng(407)
    maf = rng.uniform(0.05, 0.5, m)
    g = rng.binomial(2, maf[:, None], size=(m, n))
    q = np.clip(127 * g + rng.integers(-30, 31, size=(m, n)), 0, 254).astype(np.uint8)
    q[rng.random((m, n)) < 0.01] = 255
    G = np.where(q == 255, np.nan, q / 127.0)
    g_imp = np.where(np.isnan(G), np.nanmean(G, axis=1)[:, None], G)
    C, Y = _collinear_covariates(rng, g_imp, n)
    say(f"case: covariate-collinear markers, 8-bit dosages, {precision}")
    rows = np.zeros((m, dosage8_row_bytes_for(n)), dtype=np.uint8)
    rows[:, :n] = q
    ref = oracle_scan(G, C, Y)
    res, _, _ = gpu_scan(C, [Y], rows, precision, code=tgw.CODE_DOSAGE8, plan_kw={"block_markers": 512})
    planted = [3 * k + 1 for k in range(len(RATIOS))]
    for i in planted:
        assert np.all(np.isfinite(res[0]["r"][i])), i
    assert np.all(np.isnan(res[0]["r"][40]))
    compare(res[0], ref, ref["df"], f"collinear dosage8 {precision} ")


def test_collinear_markers_plink_coding(tgw):
    """The FP64 path decodes PLINK .bed codes (00 / 10 / 11 = 0 / 1 / 2, 01 missing)."""
    codes, C, Y = _workload(seed=408)
    n = codes.shape[1]
    say("case: covariate-collinear markers, PLINK coding, split8")
    plink = np.array([0, 2, 3, 1], dtype=np.uint8)[codes]  # allele count 0, 1, 2, missing -> .bed code
    ref = oracle_scan(codes, C, Y)
    res, _, _ = gpu_scan(C, [Y], pack_codes_np(plink, row_bytes_for(n)), "split8", code=tgw.CODE_PLINK_BED)
    compare(res[0], ref, ref["df"], "collinear plink split8 ")
