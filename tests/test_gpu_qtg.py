"""The covariate projections Q^T g across chunk counts, against the FP64 oracle.

The Q^T g contraction walks the samples in 64-sample chunks, four per round,
and copies the covariate operand of two chunks at a time; the last round may
hold one, two or three chunks.  These cases take N so that the chunk count
leaves each remainder (N = 1,000 / 1,050 / 1,100 / 1,180: 16 / 17 / 18 / 19
chunks), with covariates that carry a noisy copy of a few markers, so that
those markers' projections are large and an error in any chunk's contribution
to Q^T g shows in ||g_res|| and hence in r.  A K = 20 panel (two packed
covariate blocks) and the PLINK coding take the same paths.
"""
import numpy as np
import pytest

from synth import pack_codes_np, row_bytes_for
from tests.gpu_common import compare, gpu_scan, lib, oracle_scan, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tgw():
    t = lib()
    t.init()
    return t


def _cohort(n, m, k, seed):
    """Codes with 2 % missing calls; k covariates, two of them noisy copies of
    markers 5 and m - 7 (||g_res||^2 / ||g_c||^2 about 0.7), and phenotypes
    that load on the covariates and on those two markers."""
    rng = np.random.default_rng(seed)
    maf = rng.uniform(0.05, 0.5, m)
    codes = rng.binomial(2, maf[:, None], size=(m, n)).astype(np.uint8)
    codes[rng.random((m, n)) < 0.02] = 3
    G = np.where(codes == 3, np.nan, codes.astype(np.float64))
    g_imp = np.where(np.isnan(G), np.nanmean(G, axis=1)[:, None], G)
    C = rng.standard_normal((n, k))
    for j, i in enumerate((5, m - 7)):
        g = g_imp[i] - g_imp[i].mean()
        C[:, j] = g + np.sqrt(0.7 / 0.3) * g.std() * rng.standard_normal(n)
    Y = rng.standard_normal((n, 24)) + C @ rng.standard_normal((k, 24)) * 0.3
    Y[:, :4] += 0.5 * (g_imp[5] - g_imp[5].mean())[:, None]
    Y[:, 4:8] += 0.5 * (g_imp[m - 7] - g_imp[m - 7].mean())[:, None]
    return codes, C, Y.astype(np.float32)


@pytest.mark.parametrize("n", [1000, 1050, 1100, 1180])
@pytest.mark.parametrize("precision", ["split8", "split"])
def test_qtg_chunk_remainders(tgw, n, precision):
    m = 700  # three 256-marker tiles, the last ragged
    codes, C, Y = _cohort(n, m, 6, seed=n)
    chunks = -(-n // 64)
    say(f"case: Q^T g over {chunks} chunks (remainder {chunks % 4}) {precision} n={n} m={m} k=6")
    ref = oracle_scan(codes, C, Y)
    ratio = ref["h"] ** 2 / ref["gc2"]
    assert 0.5 < ratio[5] < 0.9 and 0.5 < ratio[m - 7] < 0.9, (ratio[5], ratio[m - 7])
    res, _, _ = gpu_scan(C, [Y], pack_codes_np(codes, row_bytes_for(n)), precision)
    compare(res[0], ref, ref["df"], f"Q^T g n={n} {precision} ")
    dr = np.abs(res[0]["r"][[5, m - 7]] - ref["r"][[5, m - 7]]).max()
    say(f"markers projected most: max |dr| {dr:.3g}")
    assert dr <= 1e-5


@pytest.mark.parametrize("n", [1050, 1180])
def test_qtg_two_blocks_and_plink(tgw, n):
    """K = 20 (q = 21: two packed covariate blocks per panel) beside a K = 6
    panel in one plan, on PLINK-coded rows."""
    m = 600
    codes, C, Y = _cohort(n, m, 20, seed=7 * n)
    _, C6, Y6 = _cohort(n, m, 6, seed=7 * n + 1)
    say(f"case: Q^T g two blocks + PLINK n={n} ({-(-n // 64)} chunks)")
    plink = np.array([0, 2, 3, 1], dtype=np.uint8)[codes]  # allele count 0, 1, 2, missing -> .bed code
    packed = pack_codes_np(plink, row_bytes_for(n))
    tg = lib()
    import torch
    cov20 = tg.fit_covariates(torch.from_numpy(C).cuda())
    cov6 = tg.fit_covariates(torch.from_numpy(C6).cuda())
    panels = [tg.prepare_phenotypes(cov20, torch.from_numpy(Y).cuda(), "split8"),
              tg.prepare_phenotypes(cov6, torch.from_numpy(Y6).cuda(), "split8")]
    plan = tg.Plan(panels)
    outs = tg.make_outputs([p.n_pheno for p in panels], m)
    plan.scan(torch.from_numpy(packed).cuda(), outs, 0, m, tg.CODE_PLINK_BED)
    plan.check()
    for j, (c, y) in enumerate(((C, Y), (C6, Y6))):
        ref = oracle_scan(codes, c, y)
        got = {k: v.cpu().numpy() for k, v in outs[j].items()}
        compare(got, ref, ref["df"], f"K = {c.shape[1]} panel, PLINK coding, n={n} ")
