"""PLINK 1 .bed reader, sample selection and .fam ID matching (host calls of
the C ABI; no GPU).

Expected rows are built here from the written codes by plain numpy
unpacking, independently of the library's reader.
"""
import os

import numpy as np
import pytest

from synth import DOSAGE_TO_PLINK, write_plink


@pytest.fixture(scope="module")
def tgw():
    from paper_2604_21095_amd import tgw as t
    return t


def _unpack(rows: np.ndarray, n: int) -> np.ndarray:
    bits = np.stack([(rows >> (2 * k)) & 3 for k in range(4)], axis=-1)
    return bits.reshape(rows.shape[0], -1)[:, :n]


def _codes(m, n, seed=3):
    rng = np.random.default_rng(seed)
    return rng.choice(4, size=(m, n), p=[0.3, 0.4, 0.25, 0.05]).astype(np.uint8)


@pytest.mark.parametrize("n", [1, 4, 37, 64, 257])
def test_read_all_samples(tgw, tmp_path, n):
    codes = _codes(23, n)
    prefix = str(tmp_path / "g")
    write_plink(prefix, codes)
    bed = tgw.Bed(prefix + ".bed", n)
    assert bed.info() == {"n_file_samples": n, "n_markers": 23, "n_selected": n}
    rb = ((n + 63) // 64) * 16
    rows = bed.read(0, 23, rb)
    got = _unpack(rows, rb * 4)
    np.testing.assert_array_equal(got[:, :n], DOSAGE_TO_PLINK[codes])
    assert np.all(got[:, n:] == 1)  # padding reads as missing
    np.testing.assert_array_equal(_unpack(bed.read(5, 9, rb), n), DOSAGE_TO_PLINK[codes[5:9]])
    assert bed.read(7, 7, rb).shape == (0, rb)
    bed.close()


def test_selection_order_and_reset(tgw, tmp_path):
    n, m = 101, 40
    codes = _codes(m, n, seed=5)
    prefix = str(tmp_path / "g")
    write_plink(prefix, codes)
    bed = tgw.Bed(prefix + ".bed", n)
    sel = np.random.default_rng(1).permutation(n)[:77]
    bed.select(sel)
    assert bed.info()["n_selected"] == 77
    rows = bed.read(3, 31, 32)
    np.testing.assert_array_equal(_unpack(rows, 77), DOSAGE_TO_PLINK[codes[3:31][:, sel]])
    assert np.all(_unpack(rows, 128)[:, 77:] == 1)
    bed.select(None)
    np.testing.assert_array_equal(_unpack(bed.read(0, m, 32), n), DOSAGE_TO_PLINK[codes])


def test_reader_errors(tgw, tmp_path):
    codes = _codes(10, 9)
    prefix = str(tmp_path / "g")
    write_plink(prefix, codes)
    with pytest.raises(tgw.TgwError) as e:
        tgw.Bed(prefix + ".bed", 13)  # 4 bytes per marker do not divide the 30 body bytes
    assert e.value.status == tgw.ERR_SHAPE
    with pytest.raises(tgw.TgwError) as e:
        tgw.Bed(str(tmp_path / "missing.bed"), 9)
    assert e.value.status == tgw.ERR_INVALID_ARG
    bad = tmp_path / "samplemajor.bed"
    bad.write_bytes(bytes([0x6C, 0x1B, 0x00]) + bytes(3 * 10))
    with pytest.raises(tgw.TgwError) as e:
        tgw.Bed(str(bad), 9)
    assert e.value.status == tgw.ERR_INVALID_ARG
    bed = tgw.Bed(prefix + ".bed", 9)
    with pytest.raises(tgw.TgwError):
        bed.select([0, 9])  # out of range
    with pytest.raises(tgw.TgwError):
        bed.select([2, 2])  # twice
    with pytest.raises(tgw.TgwError):
        bed.select([])
    with pytest.raises(tgw.TgwError):
        bed.read(0, 11, 16)  # past the last marker
    with pytest.raises(tgw.TgwError):
        bed.read(0, 2, 2)  # row too short for 9 samples
    assert bed.info()["n_selected"] == 9  # failed selections change nothing


def test_fam_match(tgw, tmp_path):
    n = 12
    ids = [f"id{7 * i % 13}" for i in range(n)]
    prefix = str(tmp_path / "g")
    write_plink(prefix, _codes(2, n), iids=ids)
    with open(prefix + ".fam", "a") as f:
        f.write("\n")  # a trailing blank line is not a sample
    want = ["id5", "nope", ids[0], ids[11]]
    idx, n_file, n_found = tgw.fam_match(prefix + ".fam", want)
    assert n_file == n and n_found == 3
    assert idx == [ids.index("id5"), -1, 0, 11]
    with pytest.raises(tgw.TgwError):
        tgw.fam_match(prefix + ".fam", ["id5", "id5"])
    dup = tmp_path / "dup.fam"
    dup.write_text("a x 0 0 0 -9\nb y 0 0 0 -9\nc x 0 0 0 -9\n")
    with pytest.raises(tgw.TgwError):
        tgw.fam_match(str(dup), ["x"])
    assert tgw.fam_match(str(dup), ["y"])[0] == [1]
    assert tgw.fam_match(str(dup), [])[1:] == (3, 0)


def test_fam_match_drives_selection(tgw, tmp_path):
    """IDs in phenotype-table order -> selection -> rows in that order."""
    n, m = 50, 8
    codes = _codes(m, n, seed=9)
    ids = [f"P{1000 + i}" for i in range(n)]
    prefix = str(tmp_path / "g")
    write_plink(prefix, codes, iids=ids)
    table = [ids[i] for i in np.random.default_rng(4).permutation(n)[:33]] + ["absent"]
    idx, _, n_found = tgw.fam_match(prefix + ".fam", table)
    keep = [i for i in idx if i >= 0]
    assert n_found == 33 and len(keep) == 33
    bed = tgw.Bed(prefix + ".bed", n)
    bed.select(keep)
    got = _unpack(bed.read(0, m, 16), 33)
    np.testing.assert_array_equal(got, DOSAGE_TO_PLINK[codes[:, keep]])
    assert os.path.exists(prefix + ".fam")
