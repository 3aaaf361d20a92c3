"""8-bit dosage genotypes (TGW_CODE_DOSAGE8) on the GPU: the contraction's
operand exactly, then every output against the FP64 oracle on the decoded
dosages q / 127.  Sizes span several tiles and ragged sample counts."""
import numpy as np
import pytest
import torch

import oracle
from synth import cohort_spec, dosage8_row_bytes_for, dosage8_rows_np, dosage8_rows_torch, panel_inputs
from tests.gpu_common import compare, gpu_scan, lib, oracle_scan, say

pytestmark = pytest.mark.gpu

PRECS8 = ["split16", "split8", "fp32"]
F16_FORMS = ("split16", "split8")


@pytest.fixture(scope="module")
def tgw():
    t = lib()
    t.init()
    return t


def _rows(q: np.ndarray) -> np.ndarray:
    m, n = q.shape
    out = np.zeros((m, dosage8_row_bytes_for(n)), dtype=np.uint8)
    out[:, :n] = q
    return out


def _debug_plan(tgw, n, V, precision, tile=-1):
    cov = tgw.fit_covariates(None, n_samples=n)
    panel = tgw.prepare_phenotypes(cov, torch.randn(n, V.shape[1], dtype=torch.float32, device="cuda"), precision)
    panel.debug_set_operand(torch.from_numpy(V).cuda())
    return tgw.Plan([panel], tile=tile)


@pytest.mark.parametrize("precision", PRECS8)
@pytest.mark.parametrize("n,m,p,tile", [(300, 70, 40, 0), (2000, 1100, 130, 1), (2000, 1100, 130, 2),
                                        (2000, 1100, 130, 3), (1999, 700, 70, 4), (1999, 700, 70, 5),
                                        (1999, 1300, 300, 0)])
def test_dosage8_contraction_exact_integers(tgw, precision, n, m, p, tile):
    """q - c with the integer c = round(mu) is exact in FP16 and FP32: the raw
    contraction equals int64 arithmetic bit for bit (no missing bytes)."""
    say(f"case: dosage8 exact contraction {precision} n={n} m={m} p={p} tile={tile}")
    rng = np.random.default_rng(31 + n + tile)
    q = rng.integers(0, 255, size=(m, n)).astype(np.uint8)
    q[5, :] = 127                        # monomorphic: degenerate, not re-centred
    q[6, :] = rng.choice([0, 254], size=n)  # the extremes
    V = rng.integers(-8, 9, size=(n, p)).astype(np.float32)
    plan = _debug_plan(tgw, n, V, precision, tile)
    g = torch.from_numpy(_rows(q)).cuda()
    S = plan.debug_contract(g, code=tgw.CODE_DOSAGE8).cpu().numpy().astype(np.float64)
    shift, mean, _ = [x.cpu().numpy() for x in plan.debug_marker_stats(g, code=tgw.CODE_DOSAGE8)]
    np.testing.assert_array_equal(mean, q.astype(np.int64).sum(axis=1) / n)
    want_shift = np.rint(mean)
    want_shift[5] = 0.0
    np.testing.assert_array_equal(shift, want_shift)
    if precision in F16_FORMS:
        S = S / tgw.F16_SCALE
    want = (q.astype(np.float64) - shift[:, None]) @ V.astype(np.float64)
    assert np.array_equal(want, want.astype(np.float32).astype(np.float64))
    np.testing.assert_array_equal(S, want)


@pytest.mark.parametrize("precision", PRECS8)
def test_dosage8_contraction_missing_value(tgw, precision):
    """A missing byte enters as mu - c rounded to the operand type."""
    say(f"case: dosage8 contraction with missing bytes {precision}")
    rng = np.random.default_rng(8)
    n, m, p = 777, 300, 33
    q = rng.integers(0, 255, size=(m, n)).astype(np.uint8)
    q[rng.random((m, n)) < 0.05] = 255
    V = rng.integers(-8, 9, size=(n, p)).astype(np.float32)
    plan = _debug_plan(tgw, n, V, precision)
    g = torch.from_numpy(_rows(q)).cuda()
    S = plan.debug_contract(g, code=tgw.CODE_DOSAGE8).cpu().numpy().astype(np.float64)
    if precision in F16_FORMS:
        S = S / tgw.F16_SCALE
    shift, mean, _ = [x.cpu().numpy() for x in plan.debug_marker_stats(g, code=tgw.CODE_DOSAGE8)]
    obs = q < 255
    mu = np.where(obs, q, 0).astype(np.int64).sum(1) / obs.sum(1)
    np.testing.assert_allclose(mean, mu, rtol=1e-15)
    np.testing.assert_array_equal(shift, np.rint(mu))
    vm = mu - shift
    if precision in F16_FORMS:
        vm_op, bound = vm.astype(np.float16).astype(np.float64), 2.0 ** -12
    else:
        vm_op, bound = vm.astype(np.float32).astype(np.float64), 2.0 ** -25
    assert np.all(np.abs(vm - vm_op) <= bound)
    A = np.where(obs, q - shift[:, None], vm_op[:, None])
    want = A @ V.astype(np.float64)
    scale = np.abs(A) @ np.abs(V.astype(np.float64)) + 1.0
    assert np.max(np.abs(S - want) / scale) < 1e-6


def _e4m3(x: np.ndarray) -> np.ndarray:
    """Round to OCP FP8 E4M3 (nearest even) and back, via torch's CPU conversion."""
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.float8_e4m3fn).to(
        torch.float64).numpy()


@pytest.mark.parametrize("tile", [0, 1])
def test_dosage8_contraction_fp8_lo_term(tgw, tile):
    """FP16 + FP8 form on dosages with non-integer operands: the contraction
    equals A16 @ hi + A8 @ lo8 with A16 = q - c (a missing byte: mu - c in
    FP16), A8 = e4m3(A16) (converted from the FP16 values), hi = fp16(2^12 v)
    and lo8 the e4m3 lo term with the column's scale.  The lo term is about
    2^-12 of the total, so a wrong sample order, byte placement or scale in
    the converted FP8 operand fails the 1e-6 bound."""
    say(f"case: dosage8 FP8 lo term, tile {tile}")
    rng = np.random.default_rng(62 + tile)
    n, m, p = 1000, 1100, 70
    q = rng.integers(0, 255, size=(m, n)).astype(np.uint8)
    q[rng.random((m, n)) < 0.03] = 255
    V = (rng.standard_normal((n, p)) * np.exp(rng.uniform(-3, 3, size=p))[None, :] / np.sqrt(n)).astype(np.float32)
    plan = _debug_plan(tgw, n, V, "split8", tile)
    g = torch.from_numpy(_rows(q)).cuda()
    S = plan.debug_contract(g, code=tgw.CODE_DOSAGE8).cpu().numpy().astype(np.float64)
    shift, _, _ = [x.cpu().numpy() for x in plan.debug_marker_stats(g, code=tgw.CODE_DOSAGE8)]
    obs = q < 255
    mu = np.where(obs, q, 0).astype(np.int64).sum(1) / obs.sum(1)
    A16 = np.where(obs, q - shift[:, None], (mu - shift)[:, None].astype(np.float16).astype(np.float64))
    A8 = _e4m3(A16)
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
    say(f"dosage8 fp8 lo term: max rel err {err:.3g}, lo term up to {lo_part:.3g} of the scale")
    assert lo_part > 1e-5
    assert err < 1e-6


@pytest.mark.parametrize("precision", PRECS8)
def test_dosage8_cfg1_against_oracle(tgw, precision):
    spec = cohort_spec("cfg1")
    n = spec.n_samples
    rows = dosage8_rows_np(spec, np.arange(3000))
    C, Y = panel_inputs(spec, 0)
    say(f"case: dosage8 cfg1 {precision} N={n} M=3000 P={Y.shape[1]}")
    res, n_tail, _ = gpu_scan(C, [Y], rows, precision, code=tgw.CODE_DOSAGE8)
    ref = oracle_scan(oracle.decode_dosage8(rows, n), C, Y)
    assert n_tail == int(np.sum(np.abs(ref["t"]) > 40))
    err = compare(res[0], ref, ref["df"], f"dosage8 cfg1 {precision} ")
    say(f"[dosage8 cfg1 {precision}] {err}")


@pytest.mark.parametrize("precision", PRECS8)
def test_dosage8_edge_cases(tgw, precision):
    """Ragged N, K = 0, degenerate markers: no observed dosage, all equal,
    all equal among observed, a copy of a covariate; dosages 0 and 2."""
    rng = np.random.default_rng(29)
    n, m = 130, 41
    say(f"case: dosage8 edge cases {precision} n={n}")
    q = rng.integers(0, 255, size=(m, n)).astype(np.uint8)
    q[rng.random((m, n)) < 0.1] = 255
    q[0, :] = 255
    q[1, :] = 200
    q[2, :] = 3
    q[2, :9] = 255
    binc = (rng.random(n) < 0.5).astype(np.float64)
    q[3, :] = (254 * binc).astype(np.uint8)  # dosage 0 / 2, identical to a covariate column
    q[4, :] = 0
    q[4, 7] = 254
    C = np.column_stack([binc, rng.standard_normal(n)])
    Y = rng.standard_normal((n, 4)).astype(np.float32)
    rows = _rows(q)
    G = oracle.decode_dosage8(rows, n)
    res, _, _ = gpu_scan(C, [Y], rows, precision, code=tgw.CODE_DOSAGE8)
    ref = oracle_scan(G, C, Y)
    assert np.all(np.isnan(res[0]["r"][[0, 1, 2, 3]]))
    compare(res[0], ref, ref["df"], f"dosage8 edge {precision} ")
    res0, _, _ = gpu_scan(None, [Y[:, :1]], rows, precision, code=tgw.CODE_DOSAGE8)
    ref0 = oracle_scan(G, None, Y[:, :1])
    compare(res0[0], ref0, ref0["df"], f"dosage8 edge K=0 {precision} ")


def test_dosage8_unsupported_and_shape_errors(tgw):
    n = 100
    rows = _rows(np.full((4, n), 3, dtype=np.uint8))
    Y = np.random.default_rng(0).standard_normal((n, 3)).astype(np.float32)
    with pytest.raises(tgw.TgwError) as e:
        gpu_scan(None, [Y], rows, "split", code=tgw.CODE_DOSAGE8)
    assert e.value.status == tgw.ERR_UNSUPPORTED
    with pytest.raises(tgw.TgwError) as e:  # rows as short as 2-bit rows
        gpu_scan(None, [Y], rows[:, :32], "split16", code=tgw.CODE_DOSAGE8)
    assert e.value.status == tgw.ERR_SHAPE


@pytest.mark.parametrize("precision,tile", [("split16", 0), ("split16", 1), ("split16", 2), ("split8", 0),
                                            ("split8", 1), ("fp32", -1)])
def test_dosage8_full_width_against_oracle(tgw, precision, tile):
    """N = 23,000, P = 2,048: 1,536 markers (three 512-marker tiles) from the
    device generator, every output against the oracle; the FP16 split on the
    two wide tiles and a register-staged one, FP16 + FP8 on both wide tiles."""
    spec = cohort_spec("cfg3")
    n = spec.n_samples
    m0, m1 = 40_000, 41_536
    rows = dosage8_rows_torch(spec, m0, m1, "cuda").cpu().numpy()
    np.testing.assert_array_equal(rows[:64], dosage8_rows_np(spec, np.arange(m0, m0 + 64)))
    C, Y = panel_inputs(spec, 0)
    say(f"case: dosage8 N={n} P={Y.shape[1]} markers [{m0}, {m1}) {precision} tile {tile}")
    res, _, _ = gpu_scan(C, [Y], rows, precision, code=tgw.CODE_DOSAGE8, plan_kw={"tile": tile})
    ref = oracle_scan(oracle.decode_dosage8(rows, n), C, Y)
    err = compare(res[0], ref, ref["df"], f"dosage8 full width {precision} tile {tile} ")
    say(f"[dosage8 full width {precision} tile {tile}] {err}")
