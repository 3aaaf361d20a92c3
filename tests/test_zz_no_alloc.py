"""tgw_scan_static (the scan without a plan, allocating nothing) against tgw_scan.

Two calls in a row through the C ABI, the second with a smaller input (fewer
markers, one panel instead of 32, fewer samples): each must give bit for bit
the outputs, best words and tail count of tgw_scan with a plan of the same
tile shape, and the first is also checked against the FP64 oracle.  The
workload exercises every scratch-resident part: 32 panels of different P and
K (tables, per-panel constants), strong markers (tail list), a
covariate-collinear marker (the FP64 list), and more markers than one block of
the static workspace holds for 32 panels (two blocks in the first call)."""
import ctypes

import numpy as np
import pytest
import torch

from synth import pack_codes_np, row_bytes_for
from tests.gpu_common import compare, decode_codes, lib, oracle_scan, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tgw():
    t = lib()
    t.init()
    return t


def _cohort(n, m, sizes, seed):
    rng = np.random.default_rng(seed)
    maf = rng.uniform(0.05, 0.5, m)
    codes = rng.binomial(2, maf[:, None], size=(m, n)).astype(np.uint8)
    codes[rng.random((m, n)) < 0.01] = 3
    g_imp = decode_codes(codes)
    g_imp = np.where(np.isnan(g_imp), np.nanmean(g_imp, axis=1)[:, None], g_imp)
    Cs, Ys = [], []
    for j, (p, k) in enumerate(sizes):
        C = rng.standard_normal((n, k))
        if j == 0 and k:
            C[:, 0] = g_imp[3] + 0.01 * rng.standard_normal(n)  # marker 3: collinear with a covariate
        Y = rng.standard_normal((n, p)) + C @ rng.standard_normal((k, p)) * 0.2
        Y[:, 0] += 3.0 * g_imp[1]  # marker 1: a tail test (|t| > 40)
        Cs.append(C)
        Ys.append(Y.astype(np.float32))
    return codes, Cs, Ys


def _static_call(tgw, panels, g, outs, tile, n_tail):
    hs = (ctypes.c_void_p * len(panels))(*[p.handle.value for p in panels])
    arr = tgw._outs_array(outs, panels, g.shape[0])
    st = tgw._scan_static(hs, len(panels), g.data_ptr(), g.shape[0], g.shape[1], tgw.CODE_DOSAGE, 0, g.shape[0],
                          arr, tile, n_tail.data_ptr(), None)
    assert st == tgw.OK, tgw._last_error()


def _same(a, b):
    return torch.equal(a.view(torch.int32) if a.dtype == torch.float32 else a,
                       b.view(torch.int32) if b.dtype == torch.float32 else b)


@pytest.mark.parametrize("precision", ["split8", "fp32"])
def test_scan_static_matches_scan(tgw, precision):
    rng = np.random.default_rng(30)
    many = [(int(p), int(k)) for p, k in zip(rng.integers(4, 41, 32), rng.integers(1, 6, 32))]
    many[0] = (40, 4)
    # 32 panels: the static workspace then holds 13,824 markers, so call 1 runs two blocks
    cases = [(2000, 16000, many, 31), (1500, 900, [(33, 3)], 32)]  # the second call is smaller
    for call, (n, m, sizes, seed) in enumerate(cases):
        say(f"case: tgw_scan_static call {call + 1} {precision} n={n} m={m} panels={sizes}")
        codes, Cs, Ys = _cohort(n, m, sizes, seed)
        g = torch.from_numpy(pack_codes_np(codes, row_bytes_for(n))).cuda()
        panels = []
        for C, Y in zip(Cs, Ys):
            cov = tgw.fit_covariates(torch.from_numpy(C).cuda())
            panels.append(tgw.prepare_phenotypes(cov, torch.from_numpy(Y).cuda(), precision))
        Ps = [p for p, _ in sizes]
        # the existing entry point, tile 0
        plan = tgw.Plan(panels, tile=0)
        want = tgw.make_outputs(Ps, m)
        for o, b in zip(want, tgw.make_best(Ps)):
            o["best"] = b
        plan.scan(g, want)
        want_tail = plan.check()
        # the allocation-free one, same tile; outputs pre-filled with garbage
        got = tgw.make_outputs(Ps, m)
        for o, b in zip(got, tgw.make_best(Ps)):
            for v in o.values():
                v.fill_(123.0)
            o["best"] = b
        n_tail = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        _static_call(tgw, panels, g, got, 0, n_tail)
        torch.cuda.synchronize()
        assert int(n_tail.item()) == want_tail > 0
        for j in range(len(sizes)):
            for k in want[j]:
                assert _same(want[j][k], got[j][k]), (call, j, k)
        if call == 0:
            for j in (0, 1, 31):
                ref = oracle_scan(codes, Cs[j], Ys[j])
                compare({k: v.cpu().numpy() for k, v in got[j].items() if k != "best"}, ref, ref["df"],
                        f"scan_static {precision} panel {j} ")
        say(f"call {call + 1}: bitwise equal to tgw_scan, {want_tail} tail tests")


def test_scan_static_rejects_sizes_beyond_its_limits(tgw):
    n = 500
    cov = tgw.fit_covariates(None, n_samples=n)
    panel = tgw.prepare_phenotypes(cov, torch.randn(n, 8, dtype=torch.float32, device="cuda"), "split8")
    g = torch.zeros((64, row_bytes_for(n)), dtype=torch.uint8, device="cuda")
    many = [panel] * 33
    outs = tgw.make_outputs([8] * 33, 64)
    hs = (ctypes.c_void_p * 33)(*[p.handle.value for p in many])
    arr = tgw._outs_array(outs, many, 64)
    st = tgw._scan_static(hs, 33, g.data_ptr(), 64, g.shape[1], tgw.CODE_DOSAGE, 0, 64, arr, 0, None, None)
    assert st == tgw.ERR_SHAPE
    assert b"32 panels" in tgw._last_error()
