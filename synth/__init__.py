"""Seeded synthetic cohorts for the association scan.

This package only draws random inputs (genotype codes, covariates and
phenotype panels), packs genotype codes into 2-bit rows and writes them as
PLINK 1 binary files.  It holds none of
the scan's arithmetic, so that both the FP64 oracle and the GPU path can take
their inputs from it without sharing any of the method.
"""
from .cohort import (  # noqa: F401
    CohortSpec,
    DOSAGE_TO_PLINK,
    dosage8_row_bytes_for,
    dosage8_rows_np,
    dosage8_rows_torch,
    PanelSpec,
    causal_markers,
    SEED,
    cohort_spec,
    geno_codes_np,
    geno_codes_torch,
    maf_thresholds,
    pack_codes_np,
    pack_codes_torch,
    panel_inputs,
    packed_rows_np,
    packed_rows_torch,
    row_bytes_for,
    n_pad_for,
    write_plink,
)
