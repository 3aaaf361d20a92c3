"""FP64 CPU oracle of the phenotype-panel linear association scan.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plainly written
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
library itself never does, and it shares no code with the GPU path.

Pinned by the CPU test suite against things other than itself:
  * brute-force per-pair OLS with covariates (Frisch-Waugh-Lovell equality),
  * Pearson correlation and the paper's Eq. 1-3 taken literally at K = 0,
  * t = r sqrt(df/(1-r^2)) and beta/SE = t,
  * closed-form Student-t p-values (df = 1, 2) and 50-digit mpmath values
    of the regularized incomplete beta function in the extreme tail,
  * uniform p-values under simulated null cohorts,
  * invariances (allele flip, phenotype affine maps, sample permutation,
    basis choice),
  * brute-force decoding of random 2-bit rows and 8-bit dosage rows.

Readings of points the paper leaves open (degrees of freedom, divisor of the
standardization, missing genotypes, sidedness of p) are listed in the
module docstrings.
"""
from .assoc import (  # noqa: F401
    CODE_DOSAGE,
    CODE_DOSAGE8,
    CODE_PLINK_BED,
    DOSAGE8_UNIT,
    MARKER_TOL,
    NonFinite,
    PHENO_TOL,
    RANK_TOL,
    RankDeficient,
    covariate_basis,
    decode,
    decode_dosage8,
    impute_mean,
    marker_is_valid,
    prepare_panel,
    residual_df,
    scan,
    scan_packed,
)
from .pvalue import ln_p_two_sided_cf, nlog10p_two_sided  # noqa: F401
