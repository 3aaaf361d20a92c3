"""The scan streamed from a PLINK 1 .bed file (tgw_scan_bed) on the GPU.

The file holds the cfg1 cohort's samples in shuffled order plus unrelated
extra samples; the phenotype table keeps the cohort order minus a dropped
subset, and .fam ID matching gives the selection.  The streamed scan must
equal, bit for bit, tgw_scan over the same selected rows (read on the host
by tgw_bed_read) in the plan's launch configuration, and match the FP64
oracle on the selected codes.  Blocks of the FP16 + FP8 form are multiples
of 512 markers (its accumulation order depends on a marker's row in the
512-marker tile); the BF16 split is bit-exact at any block size.
"""
import numpy as np
import pytest
import torch

from synth import DOSAGE_TO_PLINK, cohort_spec, geno_codes_np, panel_inputs, write_plink
from tests.gpu_common import compare, lib, oracle_scan, say

pytestmark = pytest.mark.gpu

N_EXTRA = 37
M = 5000


@pytest.fixture(scope="module")
def tgw():
    t = lib()
    t.init()
    return t


@pytest.fixture(scope="module")
def cohort(tmp_path_factory):
    spec = cohort_spec("cfg1")
    n = spec.n_samples
    codes = geno_codes_np(spec, np.arange(M))  # markers x cohort samples, 3 = missing
    C, Y = panel_inputs(spec, 0)
    rng = np.random.default_rng(2024)
    extra = rng.choice(4, size=(M, N_EXTRA), p=[0.3, 0.4, 0.25, 0.05]).astype(np.uint8)
    order = rng.permutation(n + N_EXTRA)  # file sample f holds pool sample order[f]
    pool = np.concatenate([codes, extra], axis=1)
    ids = [f"P{i}" if i < n else f"X{i}" for i in range(n + N_EXTRA)]
    prefix = str(tmp_path_factory.mktemp("bed") / "cohort")
    write_plink(prefix, pool[:, order], iids=[ids[i] for i in order])
    kept = np.sort(rng.permutation(n)[: n - 100])  # phenotype table: cohort order, 100 dropped
    return {"prefix": prefix, "n_file": n + N_EXTRA, "codes": codes, "C": C, "Y": Y, "kept": kept,
            "table_ids": [f"P{i}" for i in kept]}


def _plan(tgw, cohort, precision, rows=None):
    kept = cohort["kept"] if rows is None else rows
    cov = tgw.fit_covariates(torch.from_numpy(np.ascontiguousarray(cohort["C"][kept])).cuda())
    panel = tgw.prepare_phenotypes(cov, torch.from_numpy(np.ascontiguousarray(cohort["Y"][kept])).cuda(), precision)
    return tgw.Plan([panel])


def _open(tgw, cohort, table_ids):
    idx, n_file, n_found = tgw.fam_match(cohort["prefix"] + ".fam", table_ids)
    assert n_file == cohort["n_file"] and n_found == len(table_ids)
    bed = tgw.Bed(cohort["prefix"] + ".bed", cohort["n_file"])
    bed.select(idx)
    return bed


def _scan_rows(tgw, plan, bed, m0, m1, names):
    n_sel = bed.info()["n_selected"]
    rb = (n_sel + 63) // 64 * 16
    g = torch.from_numpy(bed.read(0, M, rb)).cuda()
    outs = tgw.make_outputs([plan.panels[0].n_pheno], m1 - m0, names)
    plan.scan(g, outs, m0, m1, tgw.CODE_PLINK_BED)
    plan.check()
    return outs


@pytest.mark.parametrize("precision,block", [("split8", 1536), ("split", 1000), ("fp32", 2048)])
def test_scan_bed_equals_scan_and_matches_oracle(tgw, cohort, precision, block):
    say(f"case: scan_bed {precision} block {block}, N={len(cohort['kept'])} of {cohort['n_file']} M={M}")
    names = ("r", "beta", "se", "t", "nlog10p")
    plan = _plan(tgw, cohort, precision)
    bed = _open(tgw, cohort, cohort["table_ids"])
    P = plan.panels[0].n_pheno
    outs = tgw.make_outputs([P], M, names)
    tgw.scan_bed(plan, bed, outs, 0, M, block_markers=block, n_threads=3)
    plan.check()
    want = _scan_rows(tgw, plan, bed, 0, M, names)
    for k in names:
        a, b = outs[0][k].cpu().numpy(), want[0][k].cpu().numpy()
        assert np.array_equal(a, b, equal_nan=True), k
    kept = cohort["kept"]
    ref = oracle_scan(DOSAGE_TO_PLINK[cohort["codes"][:, kept]], cohort["C"][kept], cohort["Y"][kept], plink=True)
    res = {k: v.cpu().numpy() for k, v in outs[0].items()}
    err = compare(res, ref, ref["df"], f"scan_bed {precision} ")
    say(f"[scan_bed {precision}] {err}")
    bed.close()


def test_scan_bed_range_reduced_outputs_and_reselect(tgw, cohort):
    """A marker range not starting at 0, best + hits only, then a second
    selection on the same handle."""
    say("case: scan_bed range, reduced outputs, reselect")
    plan = _plan(tgw, cohort, "split8")
    bed = _open(tgw, cohort, cohort["table_ids"])
    P = plan.panels[0].n_pheno
    m0, m1 = 700, 4100
    hits, count = tgw.make_hits(4096)
    plan.set_hits(hits, count, 4.0)
    best = tgw.make_best([P])
    tgw.scan_bed(plan, bed, [{"best": best[0]}], m0, m1, block_markers=1024)
    plan.check()
    h1 = tgw.read_hits(hits, count)
    hits2, count2 = tgw.make_hits(4096)
    plan.set_hits(hits2, count2, 4.0)
    best2 = tgw.make_best([P])
    n_sel = bed.info()["n_selected"]
    g = torch.from_numpy(bed.read(0, M, (n_sel + 63) // 64 * 16)).cuda()
    plan.scan(g, [{"best": best2[0]}], m0, m1, tgw.CODE_PLINK_BED)
    plan.check()
    assert torch.equal(best[0], best2[0])
    h2 = tgw.read_hits(hits2, count2)
    key = lambda h: sorted(zip(h["marker"].tolist(), h["pheno"].tolist(), h["nlog10p"].tolist()))
    assert h1["count"] == h2["count"] > 0 and key(h1) == key(h2)
    assert h1["marker"].min() >= m0 and h1["marker"].max() < m1
    # a different selection on the same handle: the device copy of it is replaced
    kept2 = cohort["kept"][50:]
    bed.select(tgw.fam_match(cohort["prefix"] + ".fam", [f"P{i}" for i in kept2])[0])
    plan2 = _plan(tgw, cohort, "split", rows=kept2)
    plan2.set_hits(None)
    outs = tgw.make_outputs([P], M, ("r", "t"))
    tgw.scan_bed(plan2, bed, outs, 0, M, block_markers=777)
    plan2.check()
    want = _scan_rows(tgw, plan2, bed, 0, M, ("r", "t"))
    for k in ("r", "t"):
        assert np.array_equal(outs[0][k].cpu().numpy(), want[0][k].cpu().numpy(), equal_nan=True), k
    bed.close()
