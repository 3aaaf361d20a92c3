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
 * the re-centred genotype operand described at tgw_scan, times the marker's
 * operand scale gs (see tgw_debug_marker_stats); for TGW_PREC_SPLIT_F8 the
 * FP8 lo pass takes the genotypes centred on c8 = rint(c) instead when
 * every panel of the plan has q <= 31 (the scan removes that shift with the
 * projection correction, this raw contraction keeps it).  d_S is row-major
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
/* Per-marker re-centring constant c, mean mu and operand scale gs of markers
 * [m_begin, m_end) (device FP64 arrays, each may be NULL); a call g enters
 * the contraction as gs (g - c), a missing call as gs (mu - c) rounded to
 * the operand type.  TGW_PREC_SPLIT: gs = K / 128 and c = U / K, with
 * U = rint(K mu) and K the integer in [1, 256] with U <= 256 and
 * 2K - U <= 256 (the largest among equals) for which the BF16 rounding error
 * of (K mu - U) / 128 (rounded to FP32 first), divided by K, is smallest.  TGW_PREC_SPLIT_F16 and TGW_PREC_SPLIT_F8: gs = 1,
 * c = rint(512 mu) / 512.  TGW_PREC_FP32: gs = 1, c = rint(64 mu) / 64.
 * A marker without missing calls, in every form: gs = 1, c = rint(mu).
 * 8-bit dosages: gs = 1, c = rint(mu) in units of 1/127.  Degenerate
 * markers: c = 0, gs = 1.  Test use only. */
tgw_status tgw_debug_marker_stats(tgw_plan* plan, const uint8_t* d_geno, int64_t n_markers, int64_t row_bytes,
                                  tgw_geno_code code, int64_t m_begin, int64_t m_end, double* d_shift,
                                  double* d_mean, double* d_scale, void* stream);
/* A counting allocator for tgw_set_allocator: hipMalloc / hipFree, with the
 * calls and bytes recorded in the tgw_debug_alloc_counts that ctx points to
 * (updated atomically).  Test use only. */
typedef struct {
  int64_t n_alloc;   /* successful allocations */
  int64_t n_free;    /* frees */
  int64_t bytes;     /* bytes allocated in total */
} tgw_debug_alloc_counts;
void* tgw_debug_counting_alloc(size_t bytes, void* stream, void* ctx);
void tgw_debug_counting_free(void* ptr, void* stream, void* ctx);

#ifdef __cplusplus
}
#endif
#endif /* TGW_DEBUG_H */
