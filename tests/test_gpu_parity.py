"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Every input is seeded and synthetic.  Sizes span several tiles plus ragged
tails in samples (N not a multiple of 64), markers and phenotypes.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from synth import (cohort_spec, causal_markers, geno_codes_np, pack_codes_np, packed_rows_torch, panel_inputs,
                   row_bytes_for)
from tests.gpu_common import (R_TOL, bf16_round, compare, cohort_arrays, decode_codes, gpu_scan, lib, oracle_scan,
                               recentre, say)

pytestmark = pytest.mark.gpu

PRECS = ["split", "split16", "split8", "fp32"]
F16_FORMS = ("split16", "split8")  # operands stored as 2^12 y


@pytest.fixture(scope="module")
def tgw():
    t = lib()
    t.init()
    return t


# ---------------------------------------------------------------------------
# contraction exactness (operand layout, decode, K order, tiling, padding)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("n,m,p,tile", [(300, 70, 40, 0), (2000, 1100, 130, 0), (2000, 1100, 130, 1),
                                        (2000, 1100, 300, 6)])
def test_contraction_exact_integers(tgw, precision, n, m, p, tile):
    say(f"case: exact contraction {precision} n={n} m={m} p={p} tile={tile}")
    rng = np.random.default_rng(17 + n)
    codes = rng.integers(0, 3, size=(m, n)).astype(np.uint8)
    codes[5, :] = 1                      # monomorphic: shift = 1 exactly
    V = rng.integers(-8, 9, size=(n, p)).astype(np.float32)
    packed = pack_codes_np(codes, row_bytes_for(n))
    cov = tgw.fit_covariates(None, n_samples=n)
    panel = tgw.prepare_phenotypes(cov, torch.randn(n, p, dtype=torch.float32, device="cuda"), precision)
    panel.debug_set_operand(torch.from_numpy(V).cuda())
    plan = tgw.Plan([panel], tile=tile)
    g = torch.from_numpy(packed).cuda()
    S = plan.debug_contract(g).cpu().numpy().astype(np.float64)
    shift, mean, gs = [x.cpu().numpy() for x in plan.debug_marker_stats(g)]
    np.testing.assert_array_equal(mean, codes.mean(axis=1))
    ok = np.ones(m, dtype=bool)
    ok[5] = False  # degenerate (monomorphic) markers are not re-centred
    # no missing calls: every marker takes the integer centring rint(mu)
    want_shift, want_gs, obs_val, _ = recentre(codes.mean(axis=1), ok, precision, complete=np.ones(m, dtype=bool))
    np.testing.assert_array_equal(shift, want_shift)
    assert np.all(shift == np.rint(shift))
    np.testing.assert_array_equal(gs, want_gs)
    if precision in F16_FORMS:
        S = S / tgw.F16_SCALE  # the FP16 forms store 2^12 times the operand
    A = np.take_along_axis(obs_val, codes.astype(np.int64), axis=1)  # gs (g - c), exact
    want = A @ V.astype(np.float64)
    assert np.array_equal(want, want.astype(np.float32).astype(np.float64))  # exactly representable
    np.testing.assert_array_equal(S, want)


@pytest.mark.parametrize("precision", PRECS)
def test_contraction_missing_value(tgw, precision):
    """Missing calls enter as (mu - c) rounded to the operand type."""
    say(f"case: contraction with missing calls {precision}")
    rng = np.random.default_rng(5)
    n, m, p = 777, 300, 33
    codes = rng.integers(0, 3, size=(m, n)).astype(np.uint8)
    codes[rng.random((m, n)) < 0.05] = 3
    V = rng.integers(-8, 9, size=(n, p)).astype(np.float32)
    cov = tgw.fit_covariates(None, n_samples=n)
    panel = tgw.prepare_phenotypes(cov, torch.randn(n, p, dtype=torch.float32, device="cuda"), precision)
    panel.debug_set_operand(torch.from_numpy(V).cuda())
    plan = tgw.Plan([panel])
    g = torch.from_numpy(pack_codes_np(codes, row_bytes_for(n))).cuda()
    S = plan.debug_contract(g).cpu().numpy().astype(np.float64)
    if precision in F16_FORMS:
        S = S / tgw.F16_SCALE
    shift, mean, gs = [x.cpu().numpy() for x in plan.debug_marker_stats(g)]
    obs = codes < 3
    mu = np.where(obs, codes, 0).sum(1) / obs.sum(1)
    np.testing.assert_allclose(mean, mu, rtol=1e-15)
    ok = np.array([len(set(row[row < 3].tolist())) > 1 for row in codes])
    want_shift, want_gs, obs_val, vm = recentre(mean, ok, precision, complete=obs.all(axis=1))
    np.testing.assert_array_equal(shift, want_shift)
    np.testing.assert_array_equal(gs, want_gs)
    if precision == "split":
        # at most 2^-9 |mu - c| per genotype unit; 2^-16 with the nearest multiple of 1/64
        vm_op, bound = bf16_round(vm), 2.0 ** -17 * gs
    elif precision in F16_FORMS:
        vm_op, bound = vm.astype(np.float16).astype(np.float64), 2.0 ** -21
    else:
        vm_op, bound = vm.astype(np.float32).astype(np.float64), 2.0 ** -30
    assert np.all(np.abs(vm - vm_op) <= bound)
    if precision == "split":
        err = np.abs(vm - vm_op) / gs
        say(f"BF16 missing-value error per genotype unit: max {err.max():.3g}, median {np.median(err):.3g}")
        assert np.median(err) < 2.0 ** -22
    A = np.where(obs, np.take_along_axis(obs_val, np.minimum(codes, 2).astype(np.int64), axis=1), vm_op[:, None])
    want = A @ V.astype(np.float64)
    scale = np.abs(A) @ np.abs(V.astype(np.float64)) + 1.0
    assert np.max(np.abs(S - want) / scale) < 1e-6


def _e4m3(x: np.ndarray) -> np.ndarray:
    """Round to OCP FP8 E4M3 (nearest even) and back, via torch's CPU conversion."""
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.float8_e4m3fn).to(
        torch.float64).numpy()


@pytest.mark.parametrize("k", [0, 31])
def test_contraction_fp8_lo_term(tgw, k):
    """FP16 hi + FP8 lo form on non-integer operands: the contraction equals
    A16 @ hi + A8 @ lo8 * 2^-s, with hi = fp16(2^12 v), lo8 = e4m3((2^12 v - hi) 2^s)
    for the column's shift s, A16 the re-centred genotypes g - c (exact in
    FP16) and A8 the genotypes centred on c8: g - c8, missing calls
    e4m3(mu - c8).  c8 = rint(c) (A8 exact for calls) when every panel of the
    plan has q <= 31, whose last correction slot then takes the shift; c8 = c
    at K = 31 (q = 32).  The lo term is ~2^-12 of the total, so a wrong
    sample order, decode, centring or scale in the FP8 pass fails the 1e-6
    bound."""
    say(f"case: FP8 lo term of the FP16 hi + FP8 lo contraction, K = {k}")
    rng = np.random.default_rng(61)
    n, m, p = 1000, 700, 70
    codes = rng.integers(0, 3, size=(m, n)).astype(np.uint8)
    codes[rng.random((m, n)) < 0.03] = 3
    V = (rng.standard_normal((n, p)) * np.exp(rng.uniform(-3, 3, size=p))[None, :] / np.sqrt(n)).astype(np.float32)
    C = torch.from_numpy(rng.standard_normal((n, k))).cuda() if k else None
    cov = tgw.fit_covariates(C, n_samples=n)
    panel = tgw.prepare_phenotypes(cov, torch.randn(n, p, dtype=torch.float32, device="cuda"), "split8")
    panel.debug_set_operand(torch.from_numpy(V).cuda())
    plan = tgw.Plan([panel])
    g = torch.from_numpy(pack_codes_np(codes, row_bytes_for(n))).cuda()
    S = plan.debug_contract(g).cpu().numpy().astype(np.float64)
    shift, _, _ = [x.cpu().numpy() for x in plan.debug_marker_stats(g)]
    obs = codes < 3
    mu = np.where(obs, codes, 0).sum(1) / obs.sum(1)
    A16 = np.where(obs, codes - shift[:, None], (mu - shift)[:, None].astype(np.float16).astype(np.float64))
    c8 = np.rint(shift) if k < 31 else shift  # the FP8 pass's centring
    A8 = _e4m3(np.where(obs, codes - c8[:, None], (mu - c8)[:, None]))
    vs = V.astype(np.float64) * tgw.F16_SCALE
    hi = vs.astype(np.float16).astype(np.float64)
    lo = vs - hi
    mx = np.abs(lo).max(axis=0)
    sh = np.where(mx > 0, np.floor(np.log2(448.0 / np.where(mx > 0, mx, 1.0))), 0.0)
    lo8 = _e4m3(lo * 2.0 ** sh[None, :]) * 2.0 ** -sh[None, :]
    want = A16 @ hi + A8 @ lo8
    scale = np.abs(A16) @ np.abs(vs)
    err = np.max(np.abs(S - want) / scale)
    lo_part = np.max(np.abs(A8 @ lo8) / scale)
    say(f"fp8 lo term: max rel err {err:.3g}, lo term up to {lo_part:.3g} of the scale")
    assert lo_part > 1e-5  # the lo term is visible at this tolerance
    assert err < 1e-6


# ---------------------------------------------------------------------------
# parity with the oracle
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", PRECS)
def test_cfg1_full(tgw, precision):
    """Small workload in full: N=2,000 M=5,000 P=16 K=4, 1% missing, 20 causal markers."""
    spec = cohort_spec("cfg1")
    say(f"case: cfg1 full {precision}")
    codes, packed, C, Y = cohort_arrays(spec, np.arange(spec.n_markers))
    res, n_tail, panels = gpu_scan(C, [Y], packed, precision)
    ref = oracle_scan(codes, C, Y)
    compare(res[0], ref, ref["df"], f"cfg1 {precision} ")
    assert n_tail == int(np.sum(np.abs(ref["t"]) > 40))
    # the causal markers carry real signal
    cm = causal_markers(spec)
    assert np.nanmax(res[0]["nlog10p"][cm]) > 10


@pytest.mark.parametrize("precision,tile", [("split", 1), ("split16", 1), ("split8", 1), ("split8", 6)])
def test_cfg1_other_wide_shapes(tgw, precision, tile):
    """cfg1 in full on the wide tiles with two waves per SIMD (tile 1) and,
    for the FP8 lo form, 256 x 256 with one wave per SIMD (tile 6)."""
    spec = cohort_spec("cfg1")
    say(f"case: cfg1 full {precision}, tile {tile}")
    codes, packed, C, Y = cohort_arrays(spec, np.arange(spec.n_markers))
    res, n_tail, _ = gpu_scan(C, [Y], packed, precision, plan_kw={"tile": tile})
    ref = oracle_scan(codes, C, Y)
    compare(res[0], ref, ref["df"], f"cfg1 {precision} tile {tile} ")
    assert n_tail == int(np.sum(np.abs(ref["t"]) > 40))


@pytest.mark.parametrize("precision", PRECS)
def test_edge_cases(tgw, precision):
    """Ragged N, K = 0, one phenotype, degenerate markers and phenotypes."""
    rng = np.random.default_rng(23)
    n, m = 130, 41
    say(f"case: edge cases {precision} n={n}")
    codes = rng.integers(0, 3, size=(m, n)).astype(np.uint8)
    codes[rng.random((m, n)) < 0.1] = 3
    codes[0, :] = 3                      # no observed call
    codes[1, :] = 1                      # monomorphic
    codes[2, :] = 2
    codes[2, :7] = 3                     # monomorphic among observed
    codes[3, :] = 0
    codes[3, 5] = 1                      # a single minor allele
    binc = (rng.random(n) < 0.5).astype(np.float64)
    codes[4, :] = binc.astype(np.uint8)  # identical to a covariate column -> degenerate
    C = np.column_stack([binc, rng.standard_normal(n)])
    Y = rng.standard_normal((n, 4)).astype(np.float32)
    Y[:, 1] = 1.0 + 3.0 * binc           # exactly inside the covariate space -> degenerate
    Y[:, 2] = 2.5                        # constant -> degenerate
    packed = pack_codes_np(codes, row_bytes_for(n))
    res, _, _ = gpu_scan(C, [Y], packed, precision)
    ref = oracle_scan(codes, C, Y)
    assert np.all(np.isnan(res[0]["r"][[0, 1, 2, 4]]))
    assert np.all(np.isnan(res[0]["r"][:, 1])) and np.all(np.isnan(res[0]["r"][:, 2]))
    assert np.all(np.isnan(ref["r"][:, 1])) and np.all(np.isnan(ref["r"][:, 2]))
    compare(res[0], ref, ref["df"], f"edge {precision} ")
    # K = 0, P = 1
    res0, _, _ = gpu_scan(None, [Y[:, :1]], packed, precision)
    ref0 = oracle_scan(codes, None, Y[:, :1])
    assert ref0["df"] == n - 2
    compare(res0[0], ref0, ref0["df"], f"edge K=0 {precision} ")


@pytest.mark.parametrize("precision,k", [(p, 31) for p in PRECS] + [("split8", 30)])
def test_plink_coding_and_k31(tgw, precision, k):
    """PLINK coding with the largest covariate counts: K = 31 fills every
    projection-correction slot; K = 30 leaves only the last one, which the
    FP16 + FP8 form then takes for its FP8 pass's change of centring."""
    rng = np.random.default_rng(31)
    n, m = 500, 600
    say(f"case: PLINK coding, K={k}, {precision}")
    plink_codes = rng.choice(4, size=(m, n), p=[0.4, 0.05, 0.35, 0.2]).astype(np.uint8)
    C = rng.standard_normal((n, k))
    Y = (rng.standard_normal((n, 37)) + C[:, :3] @ rng.standard_normal((3, 37))).astype(np.float32)
    packed = pack_codes_np(plink_codes, row_bytes_for(n))
    res, _, _ = gpu_scan(C, [Y], packed, precision, code=1)
    ref = oracle_scan(plink_codes, C, Y, plink=True)
    assert ref["df"] == n - k - 2
    compare(res[0], ref, ref["df"], f"plink K={k} {precision} ")


@pytest.mark.parametrize("n,k", [(34, 31), (40, 5), (500, 10), (23_000, 10)])
def test_covariate_basis(tgw, n, k):
    """Q of [1 | C] (Eq. 1) against numpy's Householder QR: orthonormal
    columns that rebuild [1 | C], equal to numpy's up to column signs; two
    fits give the same bits (fixed grid and summation order). At n = 34 and
    40 most of the row-parallel workgroups get no rows."""
    say(f"case: covariate basis n={n} K={k}")
    rng = np.random.default_rng(1000 + n + k)
    C = rng.standard_normal((n, k))
    X = np.hstack([np.ones((n, 1)), C])
    Q1 = tgw.fit_covariates(torch.from_numpy(C).cuda()).Q()
    Q2 = tgw.fit_covariates(torch.from_numpy(C).cuda()).Q()
    torch.cuda.synchronize()
    assert torch.equal(Q1, Q2)
    Q = Q1.cpu().numpy()
    assert np.abs(Q.T @ Q - np.eye(k + 1)).max() < 1e-11
    assert np.abs(X - Q @ (Q.T @ X)).max() < 1e-10 * np.abs(X).max()
    Qn, _ = np.linalg.qr(X)
    assert np.abs(np.abs(Q.T @ Qn) - np.eye(k + 1)).max() < 1e-10


def test_tiny_cohort(tgw):
    """A 40-sample cohort (one 64-sample chunk, most QR workgroups idle) in
    every precision against the oracle."""
    n, m, k = 40, 300, 5
    say(f"case: tiny cohort n={n}")
    rng = np.random.default_rng(40)
    codes = rng.choice(4, size=(m, n), p=[0.3, 0.4, 0.25, 0.05]).astype(np.uint8)
    C = rng.standard_normal((n, k))
    Y = (rng.standard_normal((n, 9)) + C[:, :2] @ rng.standard_normal((2, 9))).astype(np.float32)
    packed = pack_codes_np(codes, row_bytes_for(n))
    ref = oracle_scan(codes, C, Y)
    for precision in PRECS:
        res, _, _ = gpu_scan(C, [Y], packed, precision)
        compare(res[0], ref, ref["df"], f"tiny n={n} {precision} ")


@pytest.mark.parametrize("precision", PRECS)
def test_tail_fp64(tgw, precision):
    """|t| > 40 goes through the FP64 tail kernel."""
    rng = np.random.default_rng(41)
    n, m = 3000, 64
    say(f"case: extreme tail {precision}")
    codes = rng.integers(0, 3, size=(m, n)).astype(np.uint8)
    G = codes.astype(np.float64)
    C = rng.standard_normal((n, 2))
    Y = np.column_stack([G[0] * 3.0 + rng.standard_normal(n), G[1] * 0.6 + rng.standard_normal(n),
                         G[2] * 10.0 + rng.standard_normal(n), rng.standard_normal(n)]).astype(np.float32)
    packed = pack_codes_np(codes, row_bytes_for(n))
    res, n_tail, _ = gpu_scan(C, [Y], packed, precision)
    ref = oracle_scan(codes, C, Y)
    assert n_tail >= 2, n_tail
    assert ref["nlog10p"][2, 2] > 300
    compare(res[0], ref, ref["df"], f"tail {precision} ")


def test_errors(tgw):
    say("case: error statuses")
    n = 100
    rng = np.random.default_rng(3)
    C = rng.standard_normal((n, 3))
    C[:, 2] = C[:, 0] - 2 * C[:, 1]
    with pytest.raises(tgw.TgwError) as e:
        tgw.fit_covariates(torch.from_numpy(C).cuda())
    assert e.value.status == tgw.ERR_RANK_DEFICIENT
    C[0, 0] = np.nan
    with pytest.raises(tgw.TgwError) as e:
        tgw.fit_covariates(torch.from_numpy(C).cuda())
    assert e.value.status == tgw.ERR_NONFINITE
    with pytest.raises(tgw.TgwError) as e:
        tgw.fit_covariates(torch.zeros((n, 32), dtype=torch.float64, device="cuda"))
    assert e.value.status == tgw.ERR_SHAPE
    cov = tgw.fit_covariates(torch.from_numpy(rng.standard_normal((n, 2))).cuda())
    Y = torch.randn(n, 4, device="cuda")
    Y[7, 2] = float("inf")
    with pytest.raises(tgw.TgwError) as e:
        tgw.prepare_phenotypes(cov, Y, "split")
    assert e.value.status == tgw.ERR_NONFINITE
    panel = tgw.prepare_phenotypes(cov, torch.randn(n, 4, device="cuda"), "split")
    plan = tgw.Plan([panel])
    g = torch.zeros((10, 32), dtype=torch.uint8, device="cuda")
    outs = tgw.make_outputs([4], 12)
    with pytest.raises(tgw.TgwError) as e:
        plan.scan(g, outs, 0, 11)  # m_end > n_markers
    assert e.value.status == tgw.ERR_SHAPE
    with pytest.raises(tgw.TgwError) as e:
        plan.scan(torch.zeros((10, 16), dtype=torch.uint8, device="cuda"), outs)
    assert e.value.status == tgw.ERR_SHAPE  # row too short for n = 100
    plan.scan(g, outs, 3, 3)  # empty range is a no-op
    wide = torch.empty((1, (1 << 22) + 1), dtype=torch.float32, device="cuda")[:, :4]
    with pytest.raises(tgw.TgwError) as e:
        plan.scan(g, [{"r": wide}], 0, 1)  # output row stride above 2^22 elements
    assert e.value.status == tgw.ERR_SHAPE


# ---------------------------------------------------------------------------
# determinism, resume, graphs, batching
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision,cut", [("split", 1234), ("split8", 1024)])
def test_determinism_resume_graph(tgw, precision, cut):
    """Repeat, resume over two ranges (for the FP8 lo form at a 512-marker
    boundary, see tgw_scan), and graph replay give bitwise the same outputs."""
    spec = cohort_spec("cfg1")
    say(f"case: determinism / resume / graph replay {precision}")
    codes, packed, C, Y = cohort_arrays(spec, np.arange(3000))
    cov = tgw.fit_covariates(torch.from_numpy(C).cuda())
    panel = tgw.prepare_phenotypes(cov, torch.from_numpy(Y).cuda(), precision)
    plan = tgw.Plan([panel])
    g = torch.from_numpy(packed).cuda()
    a = tgw.scan(plan, g)
    b = tgw.scan(plan, g)
    for k in a[0]:
        assert torch.equal(torch.nan_to_num(a[0][k], nan=7.0), torch.nan_to_num(b[0][k], nan=7.0)), k
    # resume: two marker ranges
    p1 = tgw.scan(plan, g, m_begin=0, m_end=cut)
    p2 = tgw.scan(plan, g, m_begin=cut, m_end=3000)
    for k in a[0]:
        joined = torch.cat([p1[0][k], p2[0][k]])
        assert torch.equal(torch.nan_to_num(joined, nan=7.0), torch.nan_to_num(a[0][k], nan=7.0)), k
    # graph replays, with eager work in between
    outs = tgw.make_outputs([16], 3000)
    graph = plan.graph(g, outs)
    for rep in range(3):
        for o in outs[0].values():
            o.fill_(-1.0)
        graph.launch()
        torch.cuda.synchronize()
        for k in a[0]:
            assert torch.equal(torch.nan_to_num(outs[0][k], nan=7.0), torch.nan_to_num(a[0][k], nan=7.0)), (rep, k)
        x = torch.randn(256, 256, device="cuda")
        (x @ x).sum().item()
        tgw.scan(plan, g, m_begin=10, m_end=400)
        torch.cuda.synchronize()


def test_batching_equals_single(tgw):
    """Several uneven panels in one plan give the same bits as one plan each.
    The K=20 panel (q = 21) takes two packed covariate blocks in the Q^T g
    contraction, the others one."""
    spec = cohort_spec("cfg1")
    say("case: batching vs single panels")
    rng = np.random.default_rng(77)
    codes, packed, _, _ = cohort_arrays(spec, np.arange(2500))
    n = spec.n_samples
    sizes = [(20, 2), (70, 5), (5, 0), (33, 9), (12, 20)]
    Cs, Ys = [], []
    for p, k in sizes:
        Cs.append(rng.standard_normal((n, k)))
        Ys.append((rng.standard_normal((n, p))
                   + (Cs[-1] @ rng.standard_normal((k, p)) if k else 0.0)).astype(np.float32))
    tg = lib()
    g = torch.from_numpy(packed).cuda()
    covs = [tg.fit_covariates(torch.from_numpy(Cc).cuda() if Cc.shape[1] else None, n_samples=n) for Cc in Cs]
    panels = [tg.prepare_phenotypes(cv, torch.from_numpy(Yy).cuda(), "split") for cv, Yy in zip(covs, Ys)]
    plan_all = tg.Plan(panels)
    outs_all = tg.scan(plan_all, g)
    for j, pan in enumerate(panels):
        single = tg.scan(tg.Plan([pan]), g)
        for k in single[0]:
            assert torch.equal(torch.nan_to_num(single[0][k], nan=7.0),
                               torch.nan_to_num(outs_all[j][k], nan=7.0)), (j, k)
        ref = oracle_scan(codes, Cs[j] if Cs[j].shape[1] else None, Ys[j])
        compare({k: v.cpu().numpy() for k, v in outs_all[j].items()}, ref, ref["df"], f"batch panel {j} ")


@pytest.mark.parametrize("precision,tile", [("split8", 1), ("split8", 0), ("split8", 6), ("split", 1)])
def test_batching_wide_tiles(tgw, precision, tile):
    """Column tiles that straddle panels of different K (so different degrees
    of freedom and p-value tables) in each wide tile shape: the epilogue
    switches its per-row values and table copy between column blocks."""
    spec = cohort_spec("cfg1")
    say(f"case: batching across panels {precision} tile={tile}")
    rng = np.random.default_rng(78)
    codes, packed, _, _ = cohort_arrays(spec, np.arange(1100))
    n = spec.n_samples
    sizes = [(20, 2), (70, 5), (5, 0), (33, 9), (150, 1)]
    Cs, Ys = [], []
    for p, k in sizes:
        Cs.append(rng.standard_normal((n, k)))
        Ys.append((rng.standard_normal((n, p))
                   + (Cs[-1] @ rng.standard_normal((k, p)) if k else 0.0)).astype(np.float32))
    g = torch.from_numpy(packed).cuda()
    covs = [tgw.fit_covariates(torch.from_numpy(Cc).cuda() if Cc.shape[1] else None, n_samples=n) for Cc in Cs]
    panels = [tgw.prepare_phenotypes(cv, torch.from_numpy(Yy).cuda(), precision) for cv, Yy in zip(covs, Ys)]
    outs = tgw.scan(tgw.Plan(panels, tile=tile), g)
    for j in range(len(sizes)):
        ref = oracle_scan(codes, Cs[j] if Cs[j].shape[1] else None, Ys[j])
        compare({k: v.cpu().numpy() for k, v in outs[j].items()}, ref, ref["df"], f"{precision} tile {tile} panel {j} ")


# ---------------------------------------------------------------------------
# full-size workloads on sampled markers
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", PRECS)
def test_cfg2_sampled_blocks(tgw, precision):
    """N=23,000 P=2,048 K=10: three 512-marker blocks (start, middle, end of M) + causal markers."""
    spec = cohort_spec("cfg2")
    M = spec.n_markers
    markers = np.unique(np.concatenate([np.arange(0, 512), np.arange(M // 2, M // 2 + 512),
                                        np.arange(M - 512, M), causal_markers(spec)]))
    say(f"case: cfg2 sampled {precision} ({len(markers)} markers)")
    codes, packed, C, Y = cohort_arrays(spec, markers)
    res, n_tail, _ = gpu_scan(C, [Y], packed, precision)
    ref = oracle_scan(codes, C, Y)
    compare(res[0], ref, ref["df"], f"cfg2 {precision} ")


@pytest.mark.parametrize("precision", ["split", "split8"])
def test_cfg3_bench_configuration(tgw, precision):
    """Precision form at full size (N=23,000, M=1,000,000, P=2,048) in the benchmark's
    launch configuration; sampled rows are checked against the oracle."""
    spec = cohort_spec("cfg3")
    M, n = spec.n_markers, spec.n_samples
    say(f"case: cfg3 full scan {precision}, sampled parity")
    C, Y = panel_inputs(spec)
    g = torch.empty((M, row_bytes_for(n)), dtype=torch.uint8, device="cuda")
    packed_rows_torch(spec, 0, M, "cuda", out=g, chunk=8192)
    cov = tgw.fit_covariates(torch.from_numpy(C).cuda())
    panel = tgw.prepare_phenotypes(cov, torch.from_numpy(Y).cuda(), precision)
    plan = tgw.Plan([panel])
    outs = tgw.make_outputs([panel.n_pheno], M, names=("r", "nlog10p"))
    plan.scan(g, outs)
    plan.check()
    rows = np.unique(np.concatenate([np.arange(0, 256), np.arange(M // 2, M // 2 + 256),
                                     np.arange(M - 256, M), causal_markers(spec)]))
    got = {k: v[torch.from_numpy(rows).cuda()].cpu().numpy() for k, v in outs[0].items()}
    # the GPU-generated rows must be the generator's rows
    assert np.array_equal(g[torch.from_numpy(rows).cuda()].cpu().numpy(),
                          pack_codes_np(geno_codes_np(spec, rows), row_bytes_for(n)))
    codes = geno_codes_np(spec, rows)
    ref = oracle_scan(codes, C, Y)
    compare(got, ref, ref["df"], f"cfg3 {precision} ")


@pytest.mark.parametrize("precision", ["split", "split8"])
def test_cfg5_batching_form_sampled(tgw, precision):
    """Batching form at full size: 64 panels of uneven P (log-uniform 32..4096) and
    K (3..20) sharing N=23,000 x M=200,000 genotypes, all in one plan; sampled
    markers of every panel are checked against the oracle."""
    spec = cohort_spec("cfg5")
    M, n = spec.n_markers, spec.n_samples
    rows = np.unique(np.concatenate([np.arange(0, 24), np.arange(M // 2, M // 2 + 24),
                                     np.arange(M - 24, M), causal_markers(spec)[:8]]))
    say(f"case: cfg5 batching {precision}, {len(spec.panels)} panels, {len(rows)} sampled markers")
    codes = geno_codes_np(spec, rows)
    g = torch.from_numpy(pack_codes_np(codes, row_bytes_for(n))).cuda()
    Cs, Ys, panels = [], [], []
    for j in range(len(spec.panels)):
        C, Y = panel_inputs(spec, j)
        Cs.append(C)
        Ys.append(Y)
        cov = tgw.fit_covariates(torch.from_numpy(C).cuda())
        panels.append(tgw.prepare_phenotypes(cov, torch.from_numpy(Y).cuda(), precision))
    plan = tgw.Plan(panels)
    outs = tgw.scan(plan, g, names=("r", "t", "nlog10p"))
    plan.check()
    worst = 0.0
    for j in range(len(spec.panels)):
        ref = oracle_scan(codes, Cs[j], Ys[j])
        errs = compare({k: v.cpu().numpy() for k, v in outs[j].items()}, ref, ref["df"], f"cfg5 {precision} panel {j} ")
        worst = max(worst, errs["r"])
    say(f"cfg5 worst |dr| over panels: {worst:.3g}")


@pytest.mark.parametrize("precision", PRECS)
def test_markers_without_missing_calls(tgw, precision):
    """Markers with no missing call are centred on the integer rint(mu) in every
    form (they carry no missing value); beside markers with missing calls, in
    the same blocks, both kinds meet the oracle."""
    spec = cohort_spec("cfg1", n_markers=1500)
    say(f"case: markers without missing calls {precision}")
    codes, _, C, Y = cohort_arrays(spec, np.arange(spec.n_markers))
    rng = np.random.default_rng(71)
    whole = rng.random(codes.shape[0]) < 0.5
    codes = np.where(whole[:, None] & (codes == 3), rng.integers(0, 3, size=codes.shape, dtype=np.uint8), codes)
    packed = pack_codes_np(codes, row_bytes_for(spec.n_samples))
    res, _, panels = gpu_scan(C, [Y], packed, precision)
    ref = oracle_scan(codes, C, Y)
    compare(res[0], ref, ref["df"], f"without missing calls {precision} ")
    plan = tgw.Plan(panels)
    shift, mean, gs = [x.cpu().numpy() for x in plan.debug_marker_stats(torch.from_numpy(packed).cuda())]
    obs = codes < 3
    ok = ref["gc2"] > 0  # not monomorphic among observed calls
    want_shift, want_gs, _, _ = recentre(mean, ok, precision, complete=obs.all(axis=1))
    np.testing.assert_array_equal(shift, want_shift)
    np.testing.assert_array_equal(gs, want_gs)
    assert np.all(shift[whole & ok] == np.rint(mean[whole & ok]))


def _e4m3_lo_sums(Yt: np.ndarray, scale: float) -> np.ndarray:
    """Per column: the sum of the FP8 lo terms that the FP16 + FP8 form stores
    for the unit columns Yt (in units of 1 / scale), computed here from the
    form's definition (hi = fp16(scale y), lo = e4m3((scale y - hi) 2^s) 2^-s)."""
    vs = Yt * scale
    hi = vs.astype(np.float16).astype(np.float64)
    lo = vs - hi
    mx = np.abs(lo).max(axis=0)
    sh = np.where(mx > 0, np.floor(np.log2(448.0 / np.where(mx > 0, mx, 1.0))), 0.0)
    return (_e4m3(lo * 2.0 ** sh[None, :]) * 2.0 ** -sh[None, :]).sum(axis=0)


def test_fp8_lo_centring_shift_removed(tgw):
    """The FP8 pass of the FP16 + FP8 form runs on g - c8 with c8 = rint(c), which
    shifts the contraction by (c - c8) L_p, L_p the column's sum of FP8 lo
    terms; the last projection-correction slot removes it.  Two-valued phenotypes without covariates
    give every sample of a column one of two rounding residuals, so L_p is
    large: left in, the shift would move r by many times the tolerance
    (checked here from the form's definition); the scan meets the oracle."""
    say("case: FP8 lo centring shift, two-valued phenotypes, K = 0")
    rng = np.random.default_rng(72)
    n, m = 8001, 900
    maf = rng.uniform(0.05, 0.5, m)
    codes = rng.binomial(2, maf[:, None], size=(m, n)).astype(np.uint8)
    codes[rng.random((m, n)) < 0.02] = 3
    Y = np.stack([(rng.random(n) < f).astype(np.float32) for f in (0.1, 0.3, 0.5, 0.7, 0.9)] +
                 [rng.standard_normal(n).astype(np.float32)], axis=1)
    ref = oracle_scan(codes, None, Y)
    Yt = oracle.prepare_panel(Y.astype(np.float64), oracle.covariate_basis(np.zeros((n, 0))))[0]
    L = _e4m3_lo_sums(Yt, tgw.F16_SCALE)
    G = decode_codes(codes)
    mu = np.nanmean(G, axis=1)
    c = np.rint(512.0 * mu) / 512.0
    shift_r = np.abs(np.outer(c - np.rint(c), L)) / tgw.F16_SCALE / ref["h"][:, None]
    say(f"column lo sums {np.array2string(L, precision=3)}; uncorrected shift of r up to {shift_r.max():.3g}")
    assert shift_r.max() > 10 * R_TOL
    res, _, _ = gpu_scan(None, [Y], pack_codes_np(codes, row_bytes_for(n)), "split8")
    compare(res[0], ref, ref["df"], "lo centring shift ")


def test_fp8_lo_centring_off_with_a_k31_panel(tgw):
    """A plan holding a K = 31 panel (q = 32: no free correction slot) runs the
    FP8 pass of all its panels on c8 = c; each panel still meets the oracle,
    and the small-K panel agrees with its own plan (which centres on rint(c))
    to well inside the tolerance."""
    spec = cohort_spec("cfg1", n_markers=1500)
    say("case: FP16 + FP8 plan with a K = 31 panel beside a K = 4 panel")
    codes, packed, C, Y = cohort_arrays(spec, np.arange(spec.n_markers))
    rng = np.random.default_rng(73)
    n = spec.n_samples
    C31 = rng.standard_normal((n, 31))
    Y31 = (rng.standard_normal((n, 9)) + C31[:, :3] @ rng.standard_normal((3, 9))).astype(np.float32)
    res, _, _ = gpu_scan(C, [Y], packed, "split8")
    covs = [tgw.fit_covariates(torch.from_numpy(c).cuda()) for c in (C, C31)]
    panels = [tgw.prepare_phenotypes(cv, torch.from_numpy(y).cuda(), "split8") for cv, y in zip(covs, (Y, Y31))]
    outs = tgw.scan(tgw.Plan(panels), torch.from_numpy(packed).cuda())
    got = [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]
    for j, (c, y) in enumerate(((C, Y), (C31, Y31))):
        ref = oracle_scan(codes, c, y)
        compare(got[j], ref, ref["df"], f"K = {c.shape[1]} panel of the mixed plan ")
    dr = np.nanmax(np.abs(got[0]["r"] - res[0]["r"]))
    say(f"K = 4 panel, mixed plan vs its own plan: max |dr| {dr:.3g}")
    assert dr < 2e-6


@pytest.mark.parametrize("precision", PRECS)
def test_phenotype_dependent_missingness(tgw, precision):
    """Missing calls concentrated where one phenotype is high (up to 40 %): the
    imputed value's operand rounding is then aligned with that phenotype, the
    worst case for the re-centred missing value."""
    rng = np.random.default_rng(97)
    n, m = 3001, 200
    say(f"case: phenotype-dependent missingness {precision}")
    C = rng.standard_normal((n, 3))
    Y = rng.standard_normal((n, 5)) + C @ rng.standard_normal((3, 5))
    maf = rng.uniform(0.05, 0.5, m)
    codes = rng.binomial(2, maf[:, None], size=(m, n)).astype(np.uint8)
    high = Y[:, 0] > np.quantile(Y[:, 0], 0.5)
    rate = np.where(high, 0.4, 0.01)
    codes[rng.random((m, n)) < rate[None, :]] = 3
    Y = Y.astype(np.float32)
    packed = pack_codes_np(codes, row_bytes_for(n))
    res, _, _ = gpu_scan(C, [Y], packed, precision)
    ref = oracle_scan(codes, C, Y)
    if precision == "split":
        # BF16 carries the imputed value to within e_m per genotype unit (the
        # rounding of the re-centred missing value, per marker), so
        # |dr| <= e_m |sum_miss y~| / ||g_res|| plus the FP32 accumulation
        G = decode_codes(codes)
        miss = np.isnan(G)
        mu = np.nanmean(G, axis=1)
        _, gs, _, vm = recentre(mu, np.ones(m, dtype=bool), precision, complete=~miss.any(axis=1))
        e_m = np.abs(bf16_round(vm) - vm) / gs
        say(f"BF16 missing-value error per genotype unit: max {e_m.max():.3g} (nearest 1/64: <= {2.0 ** -16:.3g})")
        Yt = oracle.prepare_panel(Y.astype(np.float64), oracle.covariate_basis(C))[0]
        bound = e_m[:, None] * np.abs(miss.astype(np.float64) @ Yt) / ref["h"][:, None]
        dr = np.abs(res[0]["r"] - ref["r"])
        ok = np.isfinite(ref["r"])
        assert np.all(dr[ok] <= bound[ok] + 2e-6), float(np.max(dr[ok] - bound[ok]))
    compare(res[0], ref, ref["df"], f"dependent missingness {precision} ")


@pytest.fixture(scope="module")
def biobank_cohort():
    spec = cohort_spec("cfg1", n_samples=500_001, n_markers=640)
    codes, packed, C, Y = cohort_arrays(spec, np.arange(spec.n_markers))
    return spec, codes, packed, C, Y, oracle_scan(codes, C, Y)


@pytest.mark.parametrize("precision", ["split8", "fp32"])
def test_biobank_scale_cohort(tgw, biobank_cohort, precision):
    """N = 500,001 samples (a biobank-sized cohort, ragged against the 64-sample
    chunk), 640 markers (a ragged 512-marker tile), K = 4: every output against
    the oracle; the FP32 accumulation runs over 7,813 sample chunks."""
    spec, codes, packed, C, Y, ref = biobank_cohort
    n = spec.n_samples
    say(f"case: biobank-scale cohort {precision} N={n} M={spec.n_markers}")
    res, n_tail, _ = gpu_scan(C, [Y], packed, precision)
    assert ref["df"] == n - 6
    err = compare(res[0], ref, ref["df"], f"N=500001 {precision} ")
    assert n_tail == int(np.sum(np.abs(ref["t"]) > 40))
    say(f"[N=500001 {precision}] {err}")
