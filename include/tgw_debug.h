/*
 * tgw_debug.h -- test hooks of the tgw library (include/tgw.h).
 *
 * Not part of the scan's interface: these calls expose intermediate values
 * (the raw contraction, the per-marker re-centring constant) and let a test
 * overwrite a prepared panel with chosen values, so that the contraction can
 * be checked bit for bit against integer arithmetic.  Same conventions as
 * tgw.h (device pointers, status codes, thread-local error message).
 */
#ifndef TGW_DEBUG_H
#define TGW_DEBUG_H

#include "tgw.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---- test hook (exactness of the contraction) -------------------------------
 * Writes the raw FP32 contraction S[m][c] = sum_i a_m(i) * v_c(i) of markers
 * [m_begin, m_end) with the panel's stored operand columns v_c (the prepared
 * Y~ in its operand precision, hi + lo for the split forms; for
 * TGW_PREC_SPLIT_F16 and TGW_PREC_SPLIT_F8 the stored columns are scaled by
 * 2^12), where a_m(i) is
 * the re-centred genotype operand described at tgw_scan.  d_S is row-major
 * with leading dim lds >= n_pheno.  Used by tests with integer operands. */
tgw_status tgw_debug_contract(tgw_plan* plan, const uint8_t* d_geno, int64_t n_markers, int64_t row_bytes,
                              tgw_geno_code code, int64_t m_begin, int64_t m_end, float* d_S, int64_t lds,
                              void* stream);
/* Overwrites a panel's stored operand columns with raw values (no centring,
 * residualization or unit scaling): d_V device FP32 column-major n x p (ld
 * ldv).  For TGW_PREC_SPLIT, hi = bf16(v) and lo = bf16(v - hi); for
 * TGW_PREC_SPLIT_F16 the same in FP16 of 2^12 v; for TGW_PREC_SPLIT_F8,
 * hi = fp16(2^12 v) and lo = e4m3 of (2^12 v - hi) with the column's scale.
 * Test use only. */
tgw_status tgw_debug_set_operand(tgw_panel* panel, const float* d_V, int64_t ldv, void* stream);
/* Per-marker re-centring constant c (round(64 mu)/64 for TGW_PREC_SPLIT,
 * round(512 mu)/512 for TGW_PREC_SPLIT_F16 and TGW_PREC_SPLIT_F8, as for
 * TGW_PREC_SPLIT for FP32)
 * and mean mu of markers
 * [m_begin, m_end) (device FP64 arrays, may be NULL).  Test use only. */
tgw_status tgw_debug_marker_stats(tgw_plan* plan, const uint8_t* d_geno, int64_t n_markers, int64_t row_bytes,
                                  tgw_geno_code code, int64_t m_begin, int64_t m_end, double* d_shift,
                                  double* d_mean, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* TGW_DEBUG_H */
