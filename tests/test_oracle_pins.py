"""Pins of the FP64 oracle against values fixed by the mathematics.

None of these compare the oracle with itself: each pin is brute force, a
closed form, an independent library routine used as the definition of a
special case, or a statistical property.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import assoc


def _tiny_cohort(rng, n, k, m, p, miss):
    C = rng.standard_normal((n, k))
    maf = rng.uniform(0.1, 0.5, m)
    G = rng.binomial(2, maf[:, None], size=(m, n)).astype(np.float64)
    # a few strong effects so that r spans a useful range
    Y = rng.standard_normal((n, p)) + C @ rng.standard_normal((k, p)) + 0.8 * G[:3].T @ rng.standard_normal((3, p))
    if miss > 0:
        G[rng.random((m, n)) < miss] = np.nan
    return G, C, Y


def _nanmean_impute(G):
    """Mean imputation written out here with numpy's nanmean, row by row, so
    that the least-squares pins do not take the oracle's own imputation."""
    G = np.array(G, dtype=np.float64)
    for m in range(G.shape[0]):
        row = G[m]
        miss = np.isnan(row)
        if miss.any() and not miss.all():
            row[miss] = np.nanmean(row)
    return G


def _brute_ols(g, C, y):
    """OLS of y on [1, C, g] by least squares; returns beta, se, t, df."""
    n = len(y)
    X = np.column_stack([np.ones(n), C, g])
    coef, _, _, _ = np.linalg.lstsq(X, y, rcond=None)
    resid = y - X @ coef
    df = n - X.shape[1]
    sigma2 = resid @ resid / df
    cov = sigma2 * np.linalg.inv(X.T @ X)
    beta = coef[-1]
    se = math.sqrt(cov[-1, -1])
    return beta, se, beta / se, df


@pytest.mark.parametrize("n,k,miss", [(12, 0, 0.0), (12, 1, 0.1), (50, 4, 0.0), (50, 1, 0.2),
                                      (200, 4, 0.05), (200, 0, 0.2)])
def test_brute_force_ols(n, k, miss):
    rng = np.random.default_rng(1000 + n + k)
    G, C, Y = _tiny_cohort(rng, n, k, 20, 3, miss)
    out = oracle.scan(G, C, Y)
    G_imp = _nanmean_impute(G)
    assert out["df"] == n - k - 2
    checked = 0
    for m in range(G.shape[0]):
        if not out["marker_valid"][m]:
            continue
        for p in range(Y.shape[1]):
            beta, se, t, df = _brute_ols(G_imp[m], C, Y[:, p])
            assert df == out["df"]
            np.testing.assert_allclose(out["beta"][m, p], beta, rtol=1e-9, atol=1e-12)
            np.testing.assert_allclose(out["se"][m, p], se, rtol=1e-9)
            np.testing.assert_allclose(out["t"][m, p], t, rtol=1e-9, atol=1e-10)
            # r is the partial correlation: t / sqrt(df + t^2)
            np.testing.assert_allclose(out["r"][m, p], t / math.sqrt(df + t * t), rtol=1e-9, atol=1e-12)
            checked += 1
    assert checked > 30


def test_k0_is_pearson_and_paper_eq123_literal():
    """At K = 0 the paper's Eq. 1-3 (standardize, R = G~ Y~ / N, df = N-2) are exact."""
    rng = np.random.default_rng(7)
    n = 300
    G, _, Y = _tiny_cohort(rng, n, 1, 25, 4, 0.0)
    C = np.zeros((n, 0))
    out = oracle.scan(G, C, Y)
    assert out["df"] == n - 2
    # paper, literally: population standardization and R = G~ Y~ / N
    Gs = (G - G.mean(1, keepdims=True)) / G.std(1, keepdims=True)
    Ys = (Y - Y.mean(0, keepdims=True)) / Y.std(0, keepdims=True)
    R = Gs @ Ys / n
    T = R * np.sqrt((n - 2) / (1 - R ** 2))
    np.testing.assert_allclose(out["r"], R, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(out["t"], T, rtol=1e-10, atol=1e-12)
    for m in range(5):
        for p in range(4):
            np.testing.assert_allclose(out["r"][m, p], np.corrcoef(G[m], Y[:, p])[0, 1], rtol=1e-12)


def test_identities_t_r_beta_se():
    rng = np.random.default_rng(11)
    G, C, Y = _tiny_cohort(rng, 120, 3, 30, 5, 0.05)
    out = oracle.scan(G, C, Y)
    df = out["df"]
    r, t = out["r"], out["t"]
    ok = np.isfinite(r)
    np.testing.assert_allclose(t[ok], r[ok] * np.sqrt(df / (1 - r[ok] ** 2)), rtol=1e-13)
    np.testing.assert_allclose(out["beta"][ok] / out["se"][ok], t[ok], rtol=1e-12)


# ---------------------------------------------------------------------------
# p-values
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("t", [0.0, 1e-6, 0.3, 1.0, 2.5, 10.0, 1e3, 1e8, 1e150])
def test_pvalue_closed_forms(t):
    # df = 1 (Cauchy): p = (2/pi) atan(1/|t|)
    p1 = (2.0 / math.pi) * math.atan2(1.0, abs(t))
    got1 = oracle.nlog10p_two_sided(np.array([t]), 1)[0]
    np.testing.assert_allclose(got1, -math.log10(p1), rtol=1e-12, atol=1e-15)
    # df = 2: p = 1 - |t|/sqrt(2+t^2) = 2 / (sqrt(2+t^2) (sqrt(2+t^2) + |t|))
    s = math.sqrt(2.0 + t * t)
    p2 = 2.0 / (s * (s + abs(t)))
    got2 = oracle.nlog10p_two_sided(np.array([t]), 2)[0]
    np.testing.assert_allclose(got2, -math.log10(p2), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("t,df", [(5.0, 22988), (19.0, 22988), (40.0, 22988), (60.0, 22988),
                                  (150.0, 22988), (8.0, 1994), (45.0, 1994), (3.0, 30),
                                  (300.0, 30), (0.5, 22988), (1.5, 22988)])
def test_pvalue_mpmath(t, df):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    x = mpmath.mpf(df) / (mpmath.mpf(df) + mpmath.mpf(t) ** 2)
    p = mpmath.betainc(mpmath.mpf(df) / 2, mpmath.mpf(1) / 2, 0, x, regularized=True)
    ref = float(-mpmath.log10(p))
    got = oracle.nlog10p_two_sided(np.array([t]), df)[0]
    np.testing.assert_allclose(got, ref, rtol=1e-11)
    # the log-space continued fraction on its own, over the whole range
    cf = -oracle.ln_p_two_sided_cf(t, df) / math.log(10.0)
    np.testing.assert_allclose(cf, ref, rtol=1e-10)


def test_pvalue_normal_limit():
    from scipy import stats
    t = np.array([0.5, 2.0, 6.0])
    got = oracle.nlog10p_two_sided(t, 1e9)
    ref = -np.log10(2 * stats.norm.sf(t))
    np.testing.assert_allclose(got, ref, rtol=1e-6)


def test_pvalue_special_values():
    got = oracle.nlog10p_two_sided(np.array([np.inf, -np.inf, np.nan, 0.0]), 100)
    assert got[0] == np.inf and got[1] == np.inf and np.isnan(got[2]) and got[3] == 0.0


# ---------------------------------------------------------------------------
# null calibration
# ---------------------------------------------------------------------------
def test_null_calibration_uniform_p():
    from scipy import stats
    from synth import cohort_spec, geno_codes_np, panel_inputs
    spec = cohort_spec("cfg1", n_samples=400, n_markers=1600, n_causal=0, seed=99)
    spec = spec.__class__(**{**spec.__dict__, "panels": (spec.panels[0].__class__(64, 4),)})
    C, Y = panel_inputs(spec)
    codes = geno_codes_np(spec, np.arange(spec.n_markers))
    G = np.where(codes == 3, np.nan, codes.astype(np.float64))
    out = oracle.scan(G, C, Y.astype(np.float64))
    nl = out["nlog10p"][np.isfinite(out["nlog10p"])]
    p = 10.0 ** (-nl)
    assert p.size > 1e5
    ks = stats.kstest(p, "uniform")
    assert ks.pvalue > 1e-3, ks
    t2 = out["t"][np.isfinite(out["t"])] ** 2
    lam = np.median(t2) / stats.f.ppf(0.5, 1, out["df"])
    assert 0.97 < lam < 1.03, lam


# ---------------------------------------------------------------------------
# invariances
# ---------------------------------------------------------------------------
def test_invariances():
    rng = np.random.default_rng(5)
    n = 150
    G, C, Y = _tiny_cohort(rng, n, 3, 12, 4, 0.05)
    base = oracle.scan(G, C, Y)
    ok = np.isfinite(base["r"])
    # allele flip g -> 2 - g: r, beta, t change sign, p unchanged
    flip = oracle.scan(2.0 - G, C, Y)
    np.testing.assert_allclose(flip["r"][ok], -base["r"][ok], rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(flip["beta"][ok], -base["beta"][ok], rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(flip["nlog10p"][ok], base["nlog10p"][ok], rtol=1e-9, atol=1e-12)
    # phenotype y -> a y + C gamma + const: r, t, p unchanged; beta, se scaled by |a|
    a = -3.5
    Y2 = a * Y + C @ rng.standard_normal((3, 4)) + 7.0
    aff = oracle.scan(G, C, Y2)
    np.testing.assert_allclose(aff["r"][ok], np.sign(a) * base["r"][ok], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(aff["se"][ok], abs(a) * base["se"][ok], rtol=1e-9)
    np.testing.assert_allclose(aff["beta"][ok], a * base["beta"][ok], rtol=1e-9, atol=1e-12)
    # sample permutation
    perm = rng.permutation(n)
    per = oracle.scan(G[:, perm], C[perm], Y[perm])
    np.testing.assert_allclose(per["t"][ok], base["t"][ok], rtol=1e-9, atol=1e-12)
    # a different basis of the same covariate space (mixed, reordered columns)
    A = rng.standard_normal((3, 3)) + 3 * np.eye(3)
    C2 = (C @ A)[:, ::-1] + 2.0
    bas = oracle.scan(G, C2, Y)
    np.testing.assert_allclose(bas["t"][ok], base["t"][ok], rtol=1e-9, atol=1e-12)
    # duplicate phenotype columns give identical columns
    dup = oracle.scan(G, C, np.column_stack([Y, Y[:, 1]]))
    np.testing.assert_array_equal(dup["t"][:, -1], dup["t"][:, 1])


# ---------------------------------------------------------------------------
# decoding, degenerate cases, errors
# ---------------------------------------------------------------------------
def test_decode_brute_force():
    rng = np.random.default_rng(3)
    packed = rng.integers(0, 256, size=(7, 13), dtype=np.uint8)
    n = 50  # 2 padding samples in the last byte are ignored
    for code, table in ((oracle.CODE_DOSAGE, [0.0, 1.0, 2.0, None]),
                        (oracle.CODE_PLINK_BED, [0.0, None, 1.0, 2.0])):
        G = oracle.decode(packed, n, code)
        assert G.shape == (7, n)
        for m in range(7):
            for i in range(n):
                byte = int(packed[m, i // 4])
                v = (byte >> (2 * (i % 4))) & 3
                want = table[v]
                if want is None:
                    assert np.isnan(G[m, i])
                else:
                    assert G[m, i] == want


def test_decode_dosage8_brute_force():
    rng = np.random.default_rng(4)
    rows = rng.integers(0, 256, size=(5, 70), dtype=np.uint8)
    rows[0, :3] = [0, 254, 255]
    n = 61  # bytes past the last sample are ignored
    G = oracle.decode_dosage8(rows, n)
    assert G.shape == (5, n)
    for m in range(5):
        for i in range(n):
            q = int(rows[m, i])
            if q == 255:
                assert np.isnan(G[m, i])
            else:
                assert G[m, i] == q / 127.0
    assert G[0, 0] == 0.0 and G[0, 1] == 2.0


def test_brute_force_ols_fractional_dosages():
    """The same least-squares pin with 8-bit dosages (values q / 127) and
    missing bytes, including a marker whose observed dosages are all equal."""
    rng = np.random.default_rng(77)
    n, k = 90, 3
    G0, C, Y = _tiny_cohort(rng, n, k, 12, 2, 0.0)
    q = np.clip(np.rint(127 * (np.nan_to_num(G0) + rng.uniform(-0.3, 0.3, G0.shape))), 0, 254).astype(np.uint8)
    q[rng.random(q.shape) < 0.08] = 255
    q[0] = 127
    q[0, :4] = 255  # monomorphic among observed
    G = oracle.decode_dosage8(q, n)
    out = oracle.scan(G, C, Y)
    assert not out["marker_valid"][0] and np.all(np.isnan(out["t"][0]))
    G_imp = _nanmean_impute(G)
    checked = 0
    for m in range(1, G.shape[0]):
        assert out["marker_valid"][m]
        for p in range(Y.shape[1]):
            beta, se, t, df = _brute_ols(G_imp[m], C, Y[:, p])
            np.testing.assert_allclose(out["beta"][m, p], beta, rtol=1e-9, atol=1e-12)
            np.testing.assert_allclose(out["se"][m, p], se, rtol=1e-9)
            np.testing.assert_allclose(out["t"][m, p], t, rtol=1e-9, atol=1e-10)
            checked += 1
    assert checked == 22
    # scan_packed with the dosage code is the same computation
    out2 = oracle.scan_packed(q, n, C, Y, oracle.CODE_DOSAGE8)
    np.testing.assert_array_equal(out2["t"], out["t"])


def test_degenerate_markers_and_phenotypes():
    rng = np.random.default_rng(9)
    n = 80
    G, C, Y = _tiny_cohort(rng, n, 2, 6, 3, 0.0)
    G[0] = 1.0                 # monomorphic
    G[1] = np.nan              # all missing
    G[2, :] = 2.0
    G[2, :5] = np.nan          # monomorphic among observed
    G[3] = C[:, 0] * 0 + (C[:, 1] > 0)  # fine marker
    Y[:, 1] = 4.0 + C @ np.array([1.0, -2.0])  # inside the covariate space
    out = oracle.scan(G, C, Y)
    assert np.all(np.isnan(out["r"][:3]))
    assert np.all(np.isnan(out["t"][:, 1]))
    assert np.all(np.isfinite(out["t"][3:, [0, 2]]))


def _span_residual(v, C):
    """v minus its least-squares fit on [1 | C] (numpy lstsq, not a QR)."""
    X = np.column_stack([np.ones(len(v)), C])
    coef, _, _, _ = np.linalg.lstsq(X, v, rcond=None)
    return v - X @ coef


# ratio h^2 / ||g_c||^2 of each planted marker; the oracle tests a marker only
# above MARKER_TOL = 1e-8 (reading R10)
SPAN_RATIOS = (0.0, 0.0, 0.67e-8, 1.5e-8, 1e-6, 1e-4, 1e-2)


def test_markers_near_the_covariate_span():
    """Conditional analysis puts a lead marker's dosage among the covariates:
    that marker (and its allele flip) lies in the covariate span and gives
    NaN; markers a distance eps off the span keep exactly the planted share
    h^2 / ||g_c||^2 of their variance.  Below the threshold: NaN; above: the
    least-squares fit of y ~ 1 + C + g."""
    rng = np.random.default_rng(2024)
    n, k = 240, 3
    C0 = rng.standard_normal((n, k))
    lead = rng.binomial(2, 0.3, n).astype(np.float64)
    C = np.column_stack([C0, lead])
    Y = rng.standard_normal((n, 3)) + 0.4 * lead[:, None] + C0 @ rng.standard_normal((k, 3))
    Y[:, 2] += 0.5 * rng.standard_normal(n)
    z = _span_residual(rng.standard_normal(n), C)      # orthogonal to 1 and C
    lead_c = lead - lead.mean()
    rows = [lead, 2.0 - lead]
    for rho in SPAN_RATIOS[2:]:
        eps = math.sqrt(rho / (1.0 - rho)) * np.linalg.norm(lead_c) / np.linalg.norm(z)
        rows.append(lead + eps * z)
    G = np.array(rows)
    # the planted ratio, measured by lstsq residuals and plain centring
    for m, rho in enumerate(SPAN_RATIOS):
        h2 = np.sum(_span_residual(G[m], C) ** 2)
        gc2 = np.sum((G[m] - G[m].mean()) ** 2)
        assert abs(h2 / gc2 - rho) <= 1e-3 * rho + 1e-14, (m, h2 / gc2, rho)
    out = oracle.scan(G, C, Y)
    for m, rho in enumerate(SPAN_RATIOS):
        for name in ("r", "beta", "se", "t", "nlog10p"):
            if rho <= 1e-8:
                assert np.all(np.isnan(out[name][m])), (m, name)
            else:
                assert np.all(np.isfinite(out[name][m])), (m, name)
        if rho > 1e-8:
            for p in range(Y.shape[1]):
                beta, se, t, df = _brute_ols(G[m], C, Y[:, p])
                np.testing.assert_allclose(out["t"][m, p], t, rtol=1e-6, atol=1e-8)
                np.testing.assert_allclose(out["beta"][m, p], beta, rtol=1e-6)
                np.testing.assert_allclose(out["se"][m, p], se, rtol=1e-6)


def test_errors():
    rng = np.random.default_rng(1)
    C = rng.standard_normal((30, 3))
    C[:, 2] = C[:, 0] * 2 - C[:, 1]
    with pytest.raises(oracle.RankDeficient):
        oracle.covariate_basis(C)
    with pytest.raises(oracle.RankDeficient):
        oracle.covariate_basis(np.ones((30, 1)))  # collinear with the intercept
    C[0, 0] = np.nan
    with pytest.raises(oracle.NonFinite):
        oracle.covariate_basis(C)
    Q = oracle.covariate_basis(rng.standard_normal((30, 2)))
    Y = rng.standard_normal((30, 2))
    Y[3, 1] = np.inf
    with pytest.raises(oracle.NonFinite):
        oracle.prepare_panel(Y, Q)


# ---------------------------------------------------------------------------
# planted mistakes must be caught by the pins above (mutations in the oracle)
# ---------------------------------------------------------------------------
def test_planted_mistake_df_is_caught(monkeypatch):
    monkeypatch.setattr(assoc, "residual_df", lambda n, q: n - 2)
    with pytest.raises(AssertionError):
        test_brute_force_ols(50, 4, 0.0)


def test_planted_mistake_unresidualized_genotype_is_caught(monkeypatch):
    real_scan = assoc.scan

    def no_g_resid(G, C, Y, Q=None):
        # the paper's Eq. 2 read literally with covariates: centred-only G
        out = real_scan(G, np.zeros((G.shape[1], 0)), Y)
        out2 = real_scan(G, C, Y)
        out2["t"] = out["r"] * np.sqrt(out2["df"] / (1 - out["r"] ** 2))
        return out2

    monkeypatch.setattr(oracle, "scan", no_g_resid)
    with pytest.raises(AssertionError):
        test_brute_force_ols(200, 4, 0.05)


def test_planted_mistake_zero_imputation_is_caught(monkeypatch):
    def zero_fill(G):
        obs = ~np.isnan(G)
        n_obs = obs.sum(axis=1)
        with np.errstate(invalid="ignore", divide="ignore"):
            mu = np.where(obs, G, 0.0).sum(axis=1) / n_obs
        return np.where(obs, G, 0.0), n_obs, mu

    monkeypatch.setattr(assoc, "impute_mean", zero_fill)
    with pytest.raises(AssertionError):
        test_brute_force_ols(50, 1, 0.2)


def test_planted_mistake_median_imputation_is_caught(monkeypatch):
    def median_fill(G):
        obs = ~np.isnan(G)
        n_obs = obs.sum(axis=1)
        with np.errstate(invalid="ignore", divide="ignore"):
            mu = np.where(obs, G, 0.0).sum(axis=1) / n_obs
        med = np.nanmedian(G, axis=1)
        return np.where(obs, G, med[:, None]), n_obs, mu

    monkeypatch.setattr(assoc, "impute_mean", median_fill)
    with pytest.raises(AssertionError):
        test_brute_force_ols(200, 4, 0.05)


def test_planted_mistake_reversed_marker_rule_is_caught(monkeypatch):
    def reversed_rule(n_obs, mono, h2, gc2):
        return (n_obs > 0) & ~mono & (h2 < assoc.MARKER_TOL * gc2)

    monkeypatch.setattr(assoc, "marker_is_valid", reversed_rule)
    with pytest.raises(AssertionError):
        test_markers_near_the_covariate_span()


@pytest.mark.parametrize("tol", [0.0, 1e-4])
def test_planted_mistake_marker_threshold_is_caught(monkeypatch, tol):
    monkeypatch.setattr(assoc, "MARKER_TOL", tol)
    with pytest.raises(AssertionError):
        test_markers_near_the_covariate_span()
