"""Shared pieces of the GPU parity tests: run the library, run the oracle, compare.

Tolerances (the oracle is FP64):
  r        |dr| <= 1e-5
  -log10p  |d| <= 1e-4 * max(ref, 1)     (relative, floored at p = 0.1)
  t        |dt| <= 1e-5 sqrt(df) / (1 - r^2)^1.5 + 1e-6 |t|   (what |dr| <= 1e-5 implies)
  beta     |dbeta| / se_ref within the same bound as t
  se       relative |r| 1e-5 / (1 - r^2) + 1e-6   (what |dr| <= 1e-5 implies)
Markers are compared at every degree of collinearity with the covariates
(oracle ||g_res||^2 / ||g_c||^2), except within a factor 3 of the degenerate
threshold 1e-8 that oracle and library share, where either may call the
marker degenerate (NaN or finite output, either is accepted).
"""
from __future__ import annotations

import math
import sys

import numpy as np
import torch

import oracle
from synth import geno_codes_np, pack_codes_np, panel_inputs, row_bytes_for

R_TOL = 1e-5
P_TOL = 1e-4
ILL_LO, ILL_HI = 1e-8 / 3, 3e-8  # borderline band around the degenerate threshold


def lib():
    from paper_2604_21095_amd import tgw
    return tgw


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def decode_codes(codes: np.ndarray) -> np.ndarray:
    return np.where(codes == 3, np.nan, codes.astype(np.float64))


def gpu_scan(C: np.ndarray, Ys, packed: np.ndarray, precision: str, code: int = 0, m_begin: int = 0,
             m_end=None, plan_kw=None, names=("r", "beta", "se", "t", "nlog10p")):
    """Fit, prepare (one panel per entry of Ys) and scan; returns numpy outputs per panel."""
    tgw = lib()
    Cd = torch.from_numpy(np.ascontiguousarray(C)).cuda() if C is not None and C.size else None
    n = packed_n = Ys[0].shape[0]
    cov = tgw.fit_covariates(Cd, n_samples=n)
    panels = [tgw.prepare_phenotypes(cov, torch.from_numpy(np.ascontiguousarray(Y)).cuda(), precision) for Y in Ys]
    plan = tgw.Plan(panels, **(plan_kw or {}))
    g = torch.from_numpy(np.ascontiguousarray(packed)).cuda()
    m_end = packed.shape[0] if m_end is None else m_end
    outs = tgw.make_outputs([p.n_pheno for p in panels], m_end - m_begin, names)
    plan.scan(g, outs, m_begin, m_end, code)
    n_tail = plan.check()
    res = [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]
    del packed_n
    return res, n_tail, panels


def oracle_scan(codes_or_G: np.ndarray, C: np.ndarray, Y: np.ndarray, plink: bool = False):
    G = codes_or_G
    if G.dtype == np.uint8:
        if plink:
            G = np.array([0.0, np.nan, 1.0, 2.0])[G]
        else:
            G = decode_codes(G)
    Ck = C if C is not None else np.zeros((Y.shape[0], 0))
    return oracle.scan(G, Ck, Y.astype(np.float64))


def compare(got: dict, ref: dict, df: int, label: str = "", r_tol: float = R_TOL, p_tol: float = P_TOL,
            check=True) -> dict:
    """Elementwise comparison; NaN must match NaN.  Returns the max errors."""
    r_ref = ref["r"]
    nan_ref = np.isnan(r_ref)
    errs = {}
    ill = np.zeros(r_ref.shape[0], dtype=bool)
    if "h" in ref and "gc2" in ref:
        with np.errstate(invalid="ignore", divide="ignore"):
            ratio = ref["h"] ** 2 / ref["gc2"]
            ill = (ratio > ILL_LO) & (ratio < ILL_HI) & np.isfinite(ref["h"])
    for k in got:
        g = got[k].astype(np.float64)
        rr = ref[k]
        nan_g = np.isnan(g)
        if check:
            assert np.array_equal(nan_g[~ill], np.isnan(rr)[~ill]), f"{label}{k}: NaN pattern differs " \
                f"({int(nan_g[~ill].sum())} vs {int(np.isnan(rr)[~ill].sum())})"
    ok = ~nan_ref & ~ill[:, None]
    r = r_ref[ok]
    if "r" in got:
        dr = np.abs(got["r"][ok] - r)
        errs["r"] = float(dr.max(initial=0.0))
        errs["r_p999"] = float(np.quantile(dr, 0.999)) if dr.size else 0.0
    omr2 = np.maximum(1.0 - r * r, 1e-12)
    t_tol = r_tol * math.sqrt(df) / omr2 ** 1.5 + 1e-6 * np.abs(ref["t"][ok])
    if "t" in got:
        fin = np.isfinite(ref["t"][ok])
        dt = np.abs(got["t"][ok][fin] - ref["t"][ok][fin])
        errs["t_rel_to_tol"] = float((dt / t_tol[fin]).max(initial=0.0))
    if "beta" in got and "se" in got:
        se = ref["se"][ok]
        pos = se > 0
        db = np.abs(got["beta"][ok][pos] - ref["beta"][ok][pos]) / se[pos]
        errs["beta_rel_to_tol"] = float((db / t_tol[pos]).max(initial=0.0))
        dse = np.abs(got["se"][ok][pos] - se[pos]) / se[pos]
        rr = np.abs(r[pos])
        se_tol = rr * r_tol / omr2[pos] + 1e-6
        errs["se_rel_to_tol"] = float((dse / se_tol).max(initial=0.0))
    if "nlog10p" in got:
        nl = ref["nlog10p"][ok]
        fin = np.isfinite(nl)
        dp = np.abs(got["nlog10p"][ok][fin] - nl[fin]) / np.maximum(nl[fin], 1.0)
        errs["nlog10p_rel"] = float(dp.max(initial=0.0))
        if check:
            assert np.array_equal(np.isinf(got["nlog10p"][ok]), np.isinf(nl)), f"{label}inf pattern differs"
    say(f"[{label}] max errors: " + ", ".join(f"{k}={v:.3g}" for k, v in errs.items()))
    if check:
        if "r" in errs:
            assert errs["r"] <= r_tol, f"{label}|dr| = {errs['r']}"
        if "t_rel_to_tol" in errs:
            assert errs["t_rel_to_tol"] <= 1.0, f"{label}t error {errs['t_rel_to_tol']} x tol"
        if "beta_rel_to_tol" in errs:
            assert errs["beta_rel_to_tol"] <= 1.0, f"{label}beta error {errs['beta_rel_to_tol']} x tol"
            assert errs["se_rel_to_tol"] <= 1.0, f"{label}se error {errs['se_rel_to_tol']} x tol"
        if "nlog10p_rel" in errs:
            assert errs["nlog10p_rel"] <= p_tol, f"{label}-log10 p error {errs['nlog10p_rel']}"
    return errs


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even to bfloat16 (via float32), returned as float64."""
    f = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    f = (f + 0x7FFF + ((f >> 16) & 1)) >> 16 << 16
    return f.astype(np.uint32).view(np.float32).astype(np.float64)


GRID = {"split16": 512, "split8": 512, "fp32": 64}


def recentre(mu: np.ndarray, ok: np.ndarray, precision: str, complete=None):
    """Per-marker re-centring of the genotype operand as tgw_debug_marker_stats
    documents it: returns (c, gs, obs, miss) with obs[m, g] the exact operand
    value gs (g - c) of a call g = 0, 1, 2 and miss[m] the unrounded missing
    value gs (mu - c).  BF16 split: gs = K / 128, c = U / K over K = 1..256
    with U = rint(K mu) <= 256 and 2K - U <= 256, the K whose missing value
    rounds to BF16 with the least error / K (ties: larger K).  Degenerate
    markers (ok False): c = 0, gs = 1, missing value mu.  Markers without
    missing calls (complete True, ok True), every form: c = rint(mu), gs = 1."""
    c, gs, obs, miss = _recentre_partial(mu, ok, precision)
    if complete is not None:
        whole = np.asarray(complete, dtype=bool) & np.asarray(ok, dtype=bool)
        ci = np.rint(np.asarray(mu, dtype=np.float64))
        c = np.where(whole, ci, c)
        gs = np.where(whole, 1.0, gs)
        obs = np.where(whole[:, None], np.arange(3)[None, :] - ci[:, None], obs)
        miss = np.where(whole, mu - ci, miss)
    return c, gs, obs, miss


def _recentre_partial(mu, ok, precision):
    mu = np.asarray(mu, dtype=np.float64)
    m = mu.shape[0]
    c = np.zeros(m)
    gs = np.ones(m)
    obs = np.tile(np.array([0.0, 1.0, 2.0]), (m, 1))
    miss = mu.copy()
    if precision == "split":
        best = np.full(m, np.inf)
        bk = np.zeros(m)
        for K in range(256, 0, -1):
            km = K * mu
            U = np.rint(km)
            v = (km - U) * (1.0 / 128.0)
            err = np.abs(bf16_round(v) - v) / K
            valid = (U <= 256.0) & (2.0 * K - U <= 256.0)
            take = valid & (err < best)
            best[take] = err[take]
            bk[take] = K
        U = np.rint(bk * mu)
        cs = U / bk
        vals = (np.arange(3)[None, :] * bk[:, None] - U[:, None]) * (1.0 / 128.0)
        c = np.where(ok, cs, 0.0)
        gs = np.where(ok, bk / 128.0, 1.0)
        obs = np.where(ok[:, None], vals, obs)
        miss = np.where(ok, (bk * mu - U) * (1.0 / 128.0), mu)
    else:
        grid = GRID[precision]
        cs = np.rint(grid * mu) / grid
        c = np.where(ok, cs, 0.0)
        obs = np.arange(3)[None, :] - c[:, None]
        miss = mu - c
    return c, gs, obs, miss


def cohort_arrays(spec, markers, panel=0, cols=None):
    """Codes, packed rows, covariates and phenotypes of a synthetic cohort subset."""
    codes = geno_codes_np(spec, np.asarray(markers))
    packed = pack_codes_np(codes, row_bytes_for(spec.n_samples))
    C, Y = panel_inputs(spec, panel, cols)
    return codes, packed, C, Y
