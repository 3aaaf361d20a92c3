"""Seeded synthetic cohorts: genotype codes, covariates and phenotype panels.

Workload shapes follow the paper's benchmark cohort (about 23,000 samples,
panels of 2,048 and 20,480 phenotypes; Results, Benchmark results) scaled in
the marker count.  Nothing here implements the association method.

Genotypes use a counter-based generator so that any marker block can be
regenerated alone, on the CPU (numpy, uint64) or on a GPU (torch, int64 with
wrapping arithmetic), with bit-identical codes.  The generator is the
SplitMix64 output function (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) applied to the counter
``base + (marker << 32 | sample)``.  Three 21-bit fields of each 64-bit
output give two Bernoulli(maf) allele draws and one Bernoulli(missing) draw.

Covariates and phenotypes are drawn with numpy's PCG64 from SeedSequence keys
``[seed, stream, panel, block]``; columns come in blocks of ``COL_BLOCK`` so a
subset of phenotype columns can be regenerated alone.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

SEED = 20260421
COL_BLOCK = 512
MASK64 = (1 << 64) - 1
FIELD = 21  # bits per uniform field
FIELD_MASK = (1 << FIELD) - 1

# genotype code values in the 2-bit "dosage" scheme: 0/1/2 copies of the
# counted allele, 3 = missing call
CODE_MISSING = 3


# ---------------------------------------------------------------------------
# SplitMix64 on Python ints (scalar keys)
# ---------------------------------------------------------------------------
_SM_GAMMA = 0x9E3779B97F4A7C15
_SM_M1 = 0xBF58476D1CE4E5B9
_SM_M2 = 0x94D049BB133111EB


def _sm64(x: int) -> int:
    z = (x + _SM_GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * _SM_M1) & MASK64
    z = ((z ^ (z >> 27)) * _SM_M2) & MASK64
    return z ^ (z >> 31)


def _stream_key(seed: int, stream: int) -> int:
    return _sm64(_sm64(seed & MASK64) ^ ((stream * 0xD1B54A32D192ED03) & MASK64))


def _signed(x: int) -> int:
    return x - (1 << 64) if x >= (1 << 63) else x


# ---------------------------------------------------------------------------
# cohort description
# ---------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class PanelSpec:
    n_pheno: int
    n_cov: int  # K: covariates excluding the intercept
    corr_frac: float = 0.0  # fraction of columns with shared low-rank factors
    factor_rank: int = 0


@dataclasses.dataclass(frozen=True)
class CohortSpec:
    name: str
    n_samples: int
    n_markers: int
    panels: tuple
    n_causal: int = 20
    causal_var: float = 0.05  # variance of each causal effect
    miss_rate: float = 0.01
    maf_lo: float = 0.05
    maf_hi: float = 0.5
    seed: int = SEED

    @property
    def miss_threshold(self) -> int:
        return int(round(self.miss_rate * (1 << FIELD)))


def n_pad_for(n: int) -> int:
    """Samples rounded up to whole 64-sample chunks."""
    return (n + 63) // 64 * 64


def row_bytes_for(n: int) -> int:
    return n_pad_for(n) // 4


def _cfg5_panels(seed: int, n_panels: int = 64) -> tuple:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 100])))
    ps = np.rint(np.exp(rng.uniform(math.log(32), math.log(4096), n_panels))).astype(int)
    ks = rng.integers(3, 21, n_panels)
    return tuple(PanelSpec(int(p), int(k)) for p, k in zip(ps, ks))


def cohort_spec(name: str, seed: int = SEED, **overrides) -> CohortSpec:
    """The five synthetic workloads (plus overrides for scaled-down tests).

    cfg1: N=2,000  M=5,000      P=16      K=4   (small, oracle in full)
    cfg2: N=23,000 M=100,000    P=2,048   K=10  (plain FP32 scan)
    cfg3: N=23,000 M=1,000,000  P=2,048   K=10  (split-precision scan)
    cfg4: N=23,000 M=1,000,000  P=20,480  K=10, half the columns with a
          rank-64 shared factor model
    cfg5: N=23,000 M=200,000, 64 panels, P log-uniform in [32, 4096],
          K uniform in {3..20}
    """
    if name == "cfg1":
        spec = CohortSpec("cfg1", 2000, 5000, (PanelSpec(16, 4),), seed=seed)
    elif name == "cfg2":
        spec = CohortSpec("cfg2", 23000, 100_000, (PanelSpec(2048, 10),), seed=seed)
    elif name == "cfg3":
        spec = CohortSpec("cfg3", 23000, 1_000_000, (PanelSpec(2048, 10),), seed=seed)
    elif name == "cfg4":
        spec = CohortSpec("cfg4", 23000, 1_000_000,
                          (PanelSpec(20480, 10, corr_frac=0.5, factor_rank=64),), seed=seed)
    elif name == "cfg5":
        spec = CohortSpec("cfg5", 23000, 200_000, _cfg5_panels(seed), seed=seed)
    else:
        raise ValueError(f"unknown cohort {name!r}")
    if overrides:
        spec = dataclasses.replace(spec, **overrides)
    return spec


# ---------------------------------------------------------------------------
# genotype codes: numpy path
# ---------------------------------------------------------------------------
def _sm64_np(z: np.ndarray) -> np.ndarray:
    u = np.uint64
    z = z + u(_SM_GAMMA)
    z = (z ^ (z >> u(30))) * u(_SM_M1)
    z = (z ^ (z >> u(27))) * u(_SM_M2)
    return z ^ (z >> u(31))


def maf_thresholds(spec: CohortSpec, markers: np.ndarray) -> np.ndarray:
    """Per-marker allele threshold t_m; the allele frequency is t_m / 2^21."""
    lo = int(math.floor(spec.maf_lo * (1 << FIELD)))
    span = int(math.floor((spec.maf_hi - spec.maf_lo) * (1 << FIELD)))
    base = np.uint64(_stream_key(spec.seed, 0))
    with np.errstate(over="ignore"):
        h = _sm64_np(base + np.asarray(markers, dtype=np.uint64))
    top = (h >> np.uint64(64 - FIELD)).astype(np.int64)
    return lo + ((top * span) >> FIELD)


def geno_codes_np(spec: CohortSpec, markers: Sequence[int], with_missing: bool = True,
                  n_cols: Optional[int] = None) -> np.ndarray:
    """Codes (len(markers), n_cols) uint8: 0/1/2 allele counts, 3 = missing.

    Columns at or beyond ``n_samples`` (padding) are 0.
    """
    markers = np.asarray(markers, dtype=np.int64)
    n = spec.n_samples
    n_cols = n if n_cols is None else n_cols
    thr = maf_thresholds(spec, markers).astype(np.uint64)[:, None]
    base = np.uint64(_stream_key(spec.seed, 1))
    i = np.arange(n_cols, dtype=np.uint64)[None, :]
    with np.errstate(over="ignore"):
        ctr = base + ((markers.astype(np.uint64)[:, None] << np.uint64(32)) | i)
        h = _sm64_np(ctr)
    fm = np.uint64(FIELD_MASK)
    u1 = h & fm
    u2 = (h >> np.uint64(FIELD)) & fm
    g = (u1 < thr).astype(np.uint8) + (u2 < thr).astype(np.uint8)
    if with_missing:
        u3 = (h >> np.uint64(2 * FIELD)) & fm
        g[u3 < np.uint64(spec.miss_threshold)] = CODE_MISSING
    if n_cols > n:
        g[:, n:] = 0
    return g


def pack_codes_np(codes: np.ndarray, row_bytes: int) -> np.ndarray:
    """Pack codes 4 per byte, sample i at bits 2*(i & 3) of byte i >> 2."""
    m, n = codes.shape
    width = row_bytes * 4
    assert width >= n
    full = np.zeros((m, width), dtype=np.uint8)
    full[:, :n] = codes
    q = full.reshape(m, row_bytes, 4)
    return (q[:, :, 0] | (q[:, :, 1] << 2) | (q[:, :, 2] << 4) | (q[:, :, 3] << 6)).astype(np.uint8)


# ---------------------------------------------------------------------------
# 8-bit dosages: imputed expected allele counts, q / 127 copies, 255 missing
# ---------------------------------------------------------------------------
DOSAGE8_MISSING = 255
DOSAGE8_NOISE = 19  # imputation noise: uniform integer in [-19, 19], i.e. +-0.15 copies


def dosage8_row_bytes_for(n: int) -> int:
    return n_pad_for(n)


def _dosage8_from(g_codes, noise_field, np_like):
    """q = clip(127 g + e, 0, 254) with e = (u * 39 >> 16) - 19 from a 16-bit
    uniform u; 255 where the code is missing.  Integer arithmetic only, so the
    numpy and torch generators agree bit for bit."""
    e = ((noise_field * (2 * DOSAGE8_NOISE + 1)) >> 16) - DOSAGE8_NOISE
    q = np_like.clip(127 * g_codes + e, 0, 254)
    return np_like.where(g_codes == CODE_MISSING, DOSAGE8_MISSING, q)


def dosage8_rows_np(spec: CohortSpec, markers: Sequence[int], row_bytes: Optional[int] = None) -> np.ndarray:
    """8-bit dosage rows (len(markers), row_bytes) uint8, sample i at byte i,
    drawn around the 2-bit generator's allele counts (same missing calls);
    padding bytes are 0."""
    markers = np.asarray(markers, dtype=np.int64)
    n = spec.n_samples
    rb = dosage8_row_bytes_for(n) if row_bytes is None else row_bytes
    g = geno_codes_np(spec, markers).astype(np.int64)
    base = np.uint64(_stream_key(spec.seed, 5))
    i = np.arange(n, dtype=np.uint64)[None, :]
    with np.errstate(over="ignore"):
        h = _sm64_np(base + ((markers.astype(np.uint64)[:, None] << np.uint64(32)) | i))
    u = (h & np.uint64(0xFFFF)).astype(np.int64)
    out = np.zeros((len(markers), rb), dtype=np.uint8)
    out[:, :n] = _dosage8_from(g, u, np).astype(np.uint8)
    return out


def dosage8_rows_torch(spec: CohortSpec, m0: int, m1: int, device, row_bytes: Optional[int] = None,
                       chunk: int = 4096, out=None):
    """dosage8_rows_np for markers [m0, m1), generated on ``device``."""
    import torch
    n = spec.n_samples
    rb = dosage8_row_bytes_for(n) if row_bytes is None else row_bytes
    if out is None:
        out = torch.zeros((m1 - m0, rb), dtype=torch.uint8, device=device)
    for a in range(m0, m1, chunk):
        b = min(m1, a + chunk)
        g = geno_codes_torch(spec, a, b, device).to(torch.int64)
        markers = torch.arange(a, b, dtype=torch.int64, device=device)
        i = torch.arange(n, dtype=torch.int64, device=device)[None, :]
        h = _sm64_torch(((markers[:, None] << 32) | i) + _signed(_stream_key(spec.seed, 5)))
        u = h & 0xFFFF
        del h
        out[a - m0:b - m0, :n] = _dosage8_from(g, u, torch).to(torch.uint8)
        if rb > n:
            out[a - m0:b - m0, n:] = 0
    return out


# genotype code (0, 1, 2 copies; 3 missing) -> PLINK 1 .bed 2-bit code
# (00 / 10 / 11 = 0 / 1 / 2 copies of the second allele, 01 missing)
DOSAGE_TO_PLINK = np.array([0, 2, 3, 1], dtype=np.uint8)


def write_plink(prefix: str, codes: np.ndarray, iids: Optional[Sequence[str]] = None) -> None:
    """Write codes (markers x samples, 0/1/2 copies, 3 missing) as a
    variant-major PLINK 1 .bed and a .fam with the given IIDs (default
    S0, S1, ...); FID = IID, parents 0, sex 0, phenotype -9."""
    m, n = codes.shape
    raw = pack_codes_np(DOSAGE_TO_PLINK[codes], (n + 3) // 4)
    with open(prefix + ".bed", "wb") as f:
        f.write(bytes([0x6C, 0x1B, 0x01]))
        f.write(np.ascontiguousarray(raw).tobytes())
    ids = [f"S{i}" for i in range(n)] if iids is None else list(iids)
    assert len(ids) == n
    with open(prefix + ".fam", "w") as f:
        for i in ids:
            f.write(f"{i} {i} 0 0 0 -9\n")


def packed_rows_np(spec: CohortSpec, m0: int, m1: int, row_bytes: Optional[int] = None) -> np.ndarray:
    rb = row_bytes_for(spec.n_samples) if row_bytes is None else row_bytes
    codes = geno_codes_np(spec, np.arange(m0, m1))
    return pack_codes_np(codes, rb)


# ---------------------------------------------------------------------------
# genotype codes: torch path (GPU generation of large cohorts)
# ---------------------------------------------------------------------------
def _lsr(t, k: int):
    """Logical right shift of an int64 tensor."""
    return (t >> k) & ((1 << (64 - k)) - 1)


def _sm64_torch(z):
    z = z + _signed(_SM_GAMMA)
    z = (z ^ _lsr(z, 30)) * _signed(_SM_M1)
    z = (z ^ _lsr(z, 27)) * _signed(_SM_M2)
    return z ^ _lsr(z, 31)


def geno_codes_torch(spec: CohortSpec, m0: int, m1: int, device, n_cols: Optional[int] = None):
    import torch
    n = spec.n_samples
    n_cols = n if n_cols is None else n_cols
    markers = torch.arange(m0, m1, dtype=torch.int64, device=device)
    lo = int(math.floor(spec.maf_lo * (1 << FIELD)))
    span = int(math.floor((spec.maf_hi - spec.maf_lo) * (1 << FIELD)))
    hm = _sm64_torch(markers + _signed(_stream_key(spec.seed, 0)))
    thr = (lo + ((_lsr(hm, 64 - FIELD) * span) >> FIELD))[:, None]
    i = torch.arange(n_cols, dtype=torch.int64, device=device)[None, :]
    h = _sm64_torch(((markers[:, None] << 32) | i) + _signed(_stream_key(spec.seed, 1)))
    g = ((h & FIELD_MASK) < thr).to(torch.uint8) + ((_lsr(h, FIELD) & FIELD_MASK) < thr).to(torch.uint8)
    miss = (_lsr(h, 2 * FIELD) & FIELD_MASK) < spec.miss_threshold
    del h
    g = torch.where(miss, torch.full_like(g, CODE_MISSING), g)
    if n_cols > n:
        g[:, n:] = 0
    return g


def pack_codes_torch(codes, row_bytes: int):
    import torch
    m, n = codes.shape
    width = row_bytes * 4
    if width > n:
        codes = torch.nn.functional.pad(codes, (0, width - n))
    q = codes.reshape(m, row_bytes, 4)
    return (q[:, :, 0] | (q[:, :, 1] << 2) | (q[:, :, 2] << 4) | (q[:, :, 3] << 6)).contiguous()


def packed_rows_torch(spec: CohortSpec, m0: int, m1: int, device, row_bytes: Optional[int] = None,
                      chunk: int = 4096, out=None):
    """Packed genotype rows [m0, m1) generated on ``device`` in marker chunks."""
    import torch
    rb = row_bytes_for(spec.n_samples) if row_bytes is None else row_bytes
    if out is None:
        out = torch.empty((m1 - m0, rb), dtype=torch.uint8, device=device)
    for a in range(m0, m1, chunk):
        b = min(m1, a + chunk)
        out[a - m0:b - m0] = pack_codes_torch(geno_codes_torch(spec, a, b, device), rb)
    return out


# ---------------------------------------------------------------------------
# covariates and phenotypes
# ---------------------------------------------------------------------------
def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def causal_markers(spec: CohortSpec) -> np.ndarray:
    if spec.n_causal == 0:
        return np.zeros(0, dtype=np.int64)
    return np.sort(_rng(spec.seed, 4).choice(spec.n_markers, spec.n_causal, replace=False)).astype(np.int64)


def panel_inputs(spec: CohortSpec, panel: int = 0, cols: Optional[Sequence[int]] = None):
    """Covariates C (N x K, float64) and phenotypes Y (N x len(cols), float32).

    Y = G_causal B + C Gamma + E (+ F W on the correlated fraction), where
    G_causal holds the true allele counts (before missingness) of the causal
    markers, B ~ N(0, causal_var), Gamma ~ N(0, 1), E ~ N(0, 1), F ~ N(0, 1)
    (N x rank) and W ~ N(0, 1/rank).  The phenotypes are returned in float32,
    the precision handed to the GPU; consumers that work in float64 widen
    the same float32 values.
    """
    ps: PanelSpec = spec.panels[panel]
    n, k, p = spec.n_samples, ps.n_cov, ps.n_pheno
    cols = np.arange(p) if cols is None else np.asarray(cols, dtype=np.int64)
    C = _rng(spec.seed, 2, panel).standard_normal((n, k))
    cm = causal_markers(spec)
    Gc = geno_codes_np(spec, cm, with_missing=False).astype(np.float64).T if len(cm) else np.zeros((n, 0))
    n_corr = int(round(ps.corr_frac * p))
    F = _rng(spec.seed, 5, panel).standard_normal((n, ps.factor_rank)) if n_corr else None
    Y = np.empty((n, len(cols)), dtype=np.float32)
    blocks = np.unique(cols // COL_BLOCK)
    for b in blocks:
        c0 = int(b) * COL_BLOCK
        w = min(COL_BLOCK, p - c0)
        rng = _rng(spec.seed, 3, panel, int(b))
        Bm = rng.standard_normal((len(cm), w)) * math.sqrt(spec.causal_var)
        Gm = rng.standard_normal((k, w))
        E = rng.standard_normal((n, w))
        Yb = Gc @ Bm + C @ Gm + E
        if n_corr:
            W = rng.standard_normal((ps.factor_rank, w)) / math.sqrt(ps.factor_rank)
            sel = np.arange(c0, c0 + w) < n_corr
            Yb[:, sel] += F @ W[:, sel]
        want = (cols >= c0) & (cols < c0 + w)
        Y[:, want] = Yb[:, cols[want] - c0].astype(np.float32)
    return C, Y
