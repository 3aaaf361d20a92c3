"""The seeded generator: determinism, numpy/torch identity, packing layout."""
import numpy as np

from synth import (cohort_spec, geno_codes_np, geno_codes_torch, maf_thresholds, pack_codes_np,
                   packed_rows_np, packed_rows_torch, panel_inputs, row_bytes_for)


def test_numpy_torch_bit_identical():
    spec = cohort_spec("cfg1")
    a = geno_codes_np(spec, np.arange(4990, 5000), n_cols=2048)
    b = geno_codes_torch(spec, 4990, 5000, "cpu", n_cols=2048).numpy()
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(packed_rows_np(spec, 7, 40), packed_rows_torch(spec, 7, 40, "cpu").numpy())


def test_block_regeneration_and_determinism():
    spec = cohort_spec("cfg2")
    whole = geno_codes_np(spec, np.arange(100, 140))
    part = geno_codes_np(spec, np.array([120, 101]))
    np.testing.assert_array_equal(part, whole[[20, 1]])
    np.testing.assert_array_equal(whole, geno_codes_np(spec, np.arange(100, 140)))
    C1, Y1 = panel_inputs(cohort_spec("cfg1"))
    C2, Y2 = panel_inputs(cohort_spec("cfg1"), cols=[15, 2])
    np.testing.assert_array_equal(C1, C2)
    np.testing.assert_array_equal(Y1[:, [15, 2]], Y2)


def test_packing_layout_and_rates():
    codes = np.array([[0, 1, 2, 3, 3, 2]], dtype=np.uint8)
    packed = pack_codes_np(codes, 16)
    assert packed[0, 0] == (0 | 1 << 2 | 2 << 4 | 3 << 6)
    assert packed[0, 1] == (3 | 2 << 2)
    assert np.all(packed[0, 2:] == 0)
    spec = cohort_spec("cfg1")
    assert row_bytes_for(spec.n_samples) == 512
    g = geno_codes_np(spec, np.arange(0, 400))
    miss = np.mean(g == 3)
    assert 0.008 < miss < 0.012
    thr = maf_thresholds(spec, np.arange(0, 400)) / 2.0 ** 21
    assert thr.min() >= 0.05 and thr.max() < 0.5
    obs = g[g < 3].astype(float)
    assert abs(obs.mean() / 2 - thr.mean()) < 0.01


def test_dosage8_generator():
    """8-bit dosages: numpy and torch agree bit for bit, missing bytes are the
    2-bit generator's missing calls, observed bytes stay within the noise of
    127 x the allele count, padding is zero."""
    import torch
    from synth import cohort_spec, dosage8_rows_np, dosage8_rows_torch, geno_codes_np
    spec = cohort_spec("cfg1", n_samples=301)
    a = dosage8_rows_np(spec, np.arange(50, 90))
    b = dosage8_rows_torch(spec, 50, 90, "cpu", chunk=13).numpy()
    np.testing.assert_array_equal(a, b)
    assert a.shape == (40, 320) and np.all(a[:, 301:] == 0)
    g = geno_codes_np(spec, np.arange(50, 90)).astype(np.int64)
    q = a[:, :301].astype(np.int64)
    np.testing.assert_array_equal(q == 255, g == 3)
    obs = g != 3
    assert np.all(np.abs(q[obs] - 127 * g[obs]) <= 19) and q[obs].max() <= 254
