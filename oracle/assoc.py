"""Plain FP64 oracle of the phenotype-panel linear association scan.

Test infrastructure only (see the package docstring).

For every marker m and phenotype p the oracle returns the ordinary
least-squares statistics of the marker coefficient in y_p ~ 1 + C + g_m,
missing genotype calls replaced by the marker's mean over observed calls.
The steps follow Methods 2.2 (Association kernel) of the paper, in its order:

1. mean-centre each phenotype and remove the covariate space with an
   orthonormal basis Q of [1 | C] (Eq. 1), then scale each column to unit
   length (the standardization that follows Eq. 1);
2. take each marker, covariate-adjusted, and scale it to unit length
   (the per-marker standardization before Eq. 2);
3. r = correlation of the two unit vectors (Eq. 2 with the 1/N folded into
   the unit-length scaling);
4. t = r sqrt(df / (1 - r^2)) (Eq. 3) with df = N - q - 1 residual degrees of
   freedom, q = K + 1 columns in Q; at K = 0 this is the paper's N - 2;
5. two-sided p from t (the sentence after Eq. 3), reported as -log10 p.

Unlike the GPU path, the oracle residualizes the genotypes explicitly
(G_res = G - (G Q) Q^T) instead of using a norm identity.
"""
from __future__ import annotations

import numpy as np

from .pvalue import nlog10p_two_sided

CODE_DOSAGE = 0
CODE_PLINK_BED = 1
CODE_DOSAGE8 = 2  # one byte per sample: q / 127 copies for q <= 254, 255 missing
DOSAGE8_UNIT = 127.0

# value of each 2-bit code under each coding scheme; NaN = missing call
_LUT = {
    CODE_DOSAGE: np.array([0.0, 1.0, 2.0, np.nan]),
    CODE_PLINK_BED: np.array([0.0, np.nan, 1.0, 2.0]),
}

RANK_TOL = 1e-10        # |R_jj| <= RANK_TOL * max |R_ii|  -> rank deficient
PHENO_TOL = 1e-12       # s_p <= PHENO_TOL * ||Y_c,p||      -> degenerate column
MARKER_TOL = 1e-8       # h^2 <= MARKER_TOL * ||g_c||^2     -> degenerate marker


class RankDeficient(ValueError):
    pass


class NonFinite(ValueError):
    pass


def decode(packed: np.ndarray, n_samples: int, code: int = CODE_DOSAGE) -> np.ndarray:
    """Unpack 2-bit rows: sample i sits at bits 2*(i & 3) of byte i >> 2.

    Returns (M, n_samples) float64 genotype values, NaN for missing calls.
    """
    packed = np.asarray(packed, dtype=np.uint8)
    m, nb = packed.shape
    if nb * 4 < n_samples:
        raise ValueError("row too short for n_samples")
    codes = np.empty((m, nb, 4), dtype=np.uint8)
    for k in range(4):
        codes[:, :, k] = (packed >> (2 * k)) & 3
    codes = codes.reshape(m, nb * 4)[:, :n_samples]
    return _LUT[code][codes]


def decode_dosage8(rows: np.ndarray, n_samples: int) -> np.ndarray:
    """8-bit dosage rows (sample i at byte i): q / 127 expected copies for
    q = 0..254, NaN for 255.  The paper's BGEN input carries such imputed
    dosages (Abstract, Introduction); the byte format is the library's.

    Returns (M, n_samples) float64.
    """
    rows = np.asarray(rows, dtype=np.uint8)
    if rows.shape[1] < n_samples:
        raise ValueError("row too short for n_samples")
    q = rows[:, :n_samples].astype(np.float64)
    return np.where(q == 255.0, np.nan, q / DOSAGE8_UNIT)


def impute_mean(G: np.ndarray):
    """Mean imputation of missing calls (NaN), marker by marker.

    Returns (G_imp, n_obs, mu).  Markers with no observed call keep NaN.
    """
    obs = ~np.isnan(G)
    n_obs = obs.sum(axis=1)
    s = np.where(obs, G, 0.0).sum(axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        mu = s / n_obs
    G_imp = np.where(obs, G, mu[:, None])
    return G_imp, n_obs, mu


def covariate_basis(C: np.ndarray) -> np.ndarray:
    """Orthonormal basis Q (N x q) of [1 | C] by Householder QR (LAPACK).

    The intercept is always included.  Raises RankDeficient when
    |R_jj| <= 1e-10 max_i |R_ii|, NonFinite on NaN/Inf covariates.
    """
    C = np.asarray(C, dtype=np.float64)
    if C.ndim == 1:
        C = C[:, None]
    if not np.all(np.isfinite(C)):
        raise NonFinite("non-finite covariate")
    n = C.shape[0]
    X0 = np.concatenate([np.ones((n, 1)), C], axis=1)
    Q, R = np.linalg.qr(X0, mode="reduced")
    d = np.abs(np.diag(R))
    if d.min() <= RANK_TOL * d.max():
        raise RankDeficient("covariate matrix is rank deficient")
    return Q


def prepare_panel(Y: np.ndarray, Q: np.ndarray):
    """Eq. 1 and the column standardization that follows it.

    Y_c = Y - mean(Y); Y_res = (I - Q Q^T) Y_c; s_p = ||Y_res,p||;
    Y~ = Y_res / s_p.  Columns with s_p <= 1e-12 ||Y_c,p|| are degenerate
    (valid = False, Y~ = NaN).
    """
    Y = np.asarray(Y, dtype=np.float64)
    if not np.all(np.isfinite(Y)):
        raise NonFinite("non-finite phenotype")
    Yc = Y - Y.mean(axis=0, keepdims=True)
    Yres = Yc - Q @ (Q.T @ Yc)
    s = np.linalg.norm(Yres, axis=0)
    nc = np.linalg.norm(Yc, axis=0)
    valid = s > PHENO_TOL * nc
    with np.errstate(invalid="ignore", divide="ignore"):
        Yt = np.where(valid[None, :], Yres / s[None, :], np.nan)
    return Yt, s, valid


def marker_is_valid(n_obs: np.ndarray, mono: np.ndarray, h2: np.ndarray, gc2: np.ndarray) -> np.ndarray:
    """Which markers are tested (a reading: the paper does not say).

    A marker is tested when it has at least one observed call, its observed
    calls are not all equal, and the covariate projection leaves more than
    MARKER_TOL of its centred sum of squares (h2 > MARKER_TOL * gc2); a marker
    inside the covariate span has no residual variation to correlate.
    """
    return (n_obs > 0) & ~mono & (h2 > MARKER_TOL * gc2)


def residual_df(n_samples: int, q: int) -> int:
    """Residual degrees of freedom of y ~ [Q | g]: N - q - 1."""
    return n_samples - q - 1


def scan(G: np.ndarray, C: np.ndarray, Y: np.ndarray, Q: np.ndarray = None):
    """Association statistics for every (marker, phenotype) pair.

    G: (M, N) genotype values with NaN for missing calls.
    C: (N, K) covariates (intercept added here).  Y: (N, P) phenotypes.
    Returns a dict of (M, P) float64 arrays r, beta, se, t, nlog10p and the
    scalars df, q.  Degenerate markers or phenotypes give NaN.
    """
    if Q is None:
        Q = covariate_basis(C)
    n, q = Q.shape
    df = residual_df(n, q)
    Yt, s, yvalid = prepare_panel(Y, Q)

    G = np.asarray(G, dtype=np.float64)
    G_imp, n_obs, mu = impute_mean(G)
    obs = ~np.isnan(G)
    # monomorphic: every observed value equal (exact for any value set)
    gmax = np.where(obs, G, -np.inf).max(axis=1)
    gmin = np.where(obs, G, np.inf).min(axis=1)
    mono = gmax == gmin
    G_c = G_imp - G_imp.mean(axis=1, keepdims=True)
    gc2 = np.einsum("ij,ij->i", G_c, G_c)
    G_res = G_imp - (G_imp @ Q) @ Q.T
    h2 = np.einsum("ij,ij->i", G_res, G_res)
    mvalid = marker_is_valid(n_obs, mono, h2, gc2)
    h = np.sqrt(h2)

    with np.errstate(invalid="ignore", divide="ignore"):
        r = (G_res @ np.nan_to_num(Yt)) / h[:, None]
        r = np.clip(r, -1.0, 1.0)
        one_m_r2 = (1.0 - r) * (1.0 + r)
        t = r * np.sqrt(df / one_m_r2)
        beta = r * s[None, :] / h[:, None]
        se = s[None, :] * np.sqrt(one_m_r2 / df) / h[:, None]
    bad = ~(mvalid[:, None] & yvalid[None, :])
    for a in (r, t, beta, se):
        a[bad] = np.nan
    nl = nlog10p_two_sided(t, df)
    return dict(r=r, beta=beta, se=se, t=t, nlog10p=nl, df=df, q=q,
                mu=mu, n_obs=n_obs, h=h, gc2=gc2, scale=s, marker_valid=mvalid, pheno_valid=yvalid)


def scan_packed(packed: np.ndarray, n_samples: int, C: np.ndarray, Y: np.ndarray,
                code: int = CODE_DOSAGE):
    """scan() on 2-bit packed rows, or on 8-bit dosage rows (CODE_DOSAGE8)."""
    if code == CODE_DOSAGE8:
        return scan(decode_dosage8(packed, n_samples), C, Y)
    return scan(decode(packed, n_samples, code), C, Y)
