/*
 * tgw.h -- C ABI of the MI355X (gfx950) phenotype-panel linear association scan.
 *
 * The library computes, for every marker m and phenotype p of one or more
 * phenotype panels, the ordinary least-squares statistics of the marker
 * coefficient in  y_p ~ 1 + C + g_m  (r, beta, SE, t and -log10 p), with
 * missing genotype calls replaced by the marker's mean over observed calls.
 * It follows the paper's Methods 2.2 (Association kernel):
 *   - the phenotype panel is mean-centred, projected off an orthonormal basis
 *     Q of the covariate space and scaled to unit columns ONCE (Eq. 1 and the
 *     standardization after it)                  -> tgw_prepare_phenotypes
 *   - genotypes are then streamed in marker blocks, each block contracted
 *     with the prepared panel (Eq. 2) and turned into t-statistics (Eq. 3)
 *     and p-values                                -> tgw_scan
 *   - Q comes from a Householder QR of [1 | C]    -> tgw_fit_covariates
 * Readings of points the paper leaves open (used throughout):
 *   - genotypes are covariate-adjusted as well (exact Frisch-Waugh-Lovell
 *     partial correlation); at K = 0 this is exactly the paper's Eq. 2-3;
 *   - df = N - q - 1 with q = K + 1 columns in Q (the paper's N - 2 at K = 0);
 *   - p-values are two-sided Student t with df degrees of freedom;
 *   - missing calls are imputed with the marker mean over observed calls.
 *
 * Conventions
 *   - "device" pointers point to memory on the current HIP device; the caller
 *     owns every buffer it passes in (covariates, phenotypes, genotypes,
 *     outputs).  Handles own their device memory, taken at creation from the
 *     registered allocator (tgw_set_allocator; default hipMalloc), and give
 *     it back in tgw_*_free.
 *   - "stream" is a hipStream_t passed as void*; NULL means the default stream.
 *   - All functions return a tgw_status; TGW_OK is 0.  On error nothing is
 *     enqueued and tgw_last_error() gives a thread-local message.  C++
 *     exceptions never cross this boundary.
 *   - Handles are immutable after creation except tgw_plan (see tgw_scan).
 */
#ifndef TGW_H
#define TGW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TGW_ABI_VERSION 7

typedef enum {
  TGW_OK = 0,
  TGW_ERR_INVALID_ARG = 1,    /* null pointer, negative size, bad enum */
  TGW_ERR_SHAPE = 2,          /* inconsistent sizes / strides / alignment */
  TGW_ERR_RANK_DEFICIENT = 3, /* [1 | C] rank deficient: |R_jj| <= 1e-10 max|R_ii| */
  TGW_ERR_NONFINITE = 4,      /* NaN or Inf in covariates or phenotypes */
  TGW_ERR_DEVICE = 5,         /* HIP runtime error (incl. earlier async faults) */
  TGW_ERR_OUT_OF_MEMORY = 6,
  TGW_ERR_UNSUPPORTED = 7,    /* e.g. more than 31 covariates, wrong GPU */
  TGW_ERR_TAIL_OVERFLOW = 8   /* more extreme-tail tests than the plan's list holds */
} tgw_status;

/* Arithmetic of the genotype x phenotype contraction (Eq. 2).  The scan's
 * statistics are computed from what the operands actually hold (the column
 * norms and covariate projections of the stored, rounded panel), so the
 * rounding of the panel perturbs r by about its relative residual / sqrt(3).
 *  TGW_PREC_FP32      : FP32 operands on the FP32 matrix cores, FP32 accumulate.
 *  TGW_PREC_SPLIT     : the prepared panel is split into BF16 hi + lo terms
 *                       (relative residual <= 2^-16); the genotype operand is
 *                       exact in BF16: a call g enters as gs (g - c) with a
 *                       per-marker scale gs = K / 128 and c = U / K (K, U
 *                       integers, 1 <= K <= 256, chosen per marker so that
 *                       the missing value gs (mu - c) rounds to BF16 with
 *                       the least error), a missing call as gs (mu - c) to
 *                       within about 2^-9 |mu - c| (at most about 2^-18,
 *                       typically below 2^-24, in genotype units); two BF16
 *                       matrix-core passes, FP32 accumulate.
 *  TGW_PREC_SPLIT_F16 : the same with FP16 hi + lo terms (panel scaled by 2^12
 *                       before the split, relative residual <= 2^-22) and
 *                       c = round(512 mu)/512 (missing calls to within 2^-21);
 *                       two FP16 matrix-core passes at the BF16 rate.
 *  TGW_PREC_SPLIT_F8  : FP16 hi term of 2^12 y~ against the FP16 genotype
 *                       operand of TGW_PREC_SPLIT_F16, plus the lo term
 *                       2^12 y~ - hi in FP8 e4m3 (OCP), scaled per column by
 *                       a power of two (E8M0 block scale of the matrix core)
 *                       against the genotypes centred on the integer c8
 *                       nearest c (g - c8 exact in e4m3, a missing call
 *                       mu - c8 rounded to e4m3; the change of centring,
 *                       (c - c8) times the column's sum of lo terms, is
 *                       removed with the projection correction; when a
 *                       panel of the plan has K = 31, c8 = c and the
 *                       genotype operand is rounded to e4m3 instead):
 *                       relative residual of the panel <= about 2^-16, one
 *                       FP16 pass plus one FP8 pass at twice the FP16 rate.
 * In every form a marker without missing calls takes gs = 1 and the integer
 * c = rint(mu) instead (no missing value to carry).
 *                       Runs on the wide tile shapes only (tiles 1 and 6
 *                       select their own; every other index selects tile 0).
 * Covariate QR, phenotype norms and the extreme-tail p-values stay FP64. */
typedef enum {
  TGW_PREC_FP32 = 0,
  TGW_PREC_SPLIT = 1,
  TGW_PREC_SPLIT_F16 = 2,
  TGW_PREC_SPLIT_F8 = 3
} tgw_precision;

/* Genotype row formats.  The 2-bit codes put sample i of a row at bits
 * 2*(i & 3) of byte i >> 2, as in PLINK .bed rows:
 *  TGW_CODE_DOSAGE    : 0, 1, 2 = copies of the counted allele, 3 = missing.
 *  TGW_CODE_PLINK_BED : 0 -> 0, 1 -> missing, 2 -> 1, 3 -> 2 (copies of the
 *                       second allele).
 *  TGW_CODE_DOSAGE8   : one byte per sample (sample i at byte i): q = 0..254
 *                       is the expected allele count q / 127 (the imputed
 *                       dosages that the paper's BGEN input carries; Abstract,
 *                       Introduction), 255 = missing.  Runs in TGW_PREC_FP32,
 *                       TGW_PREC_SPLIT_F16 and TGW_PREC_SPLIT_F8 (whose e4m3
 *                       genotype operand is the FP16 value q - c rounded to
 *                       e4m3); TGW_PREC_SPLIT gives TGW_ERR_UNSUPPORTED.  beta
 *                       and SE are per unit dosage. */
typedef enum { TGW_CODE_DOSAGE = 0, TGW_CODE_PLINK_BED = 1, TGW_CODE_DOSAGE8 = 2 } tgw_geno_code;

typedef struct tgw_covariates tgw_covariates; /* Q of one covariate matrix   */
typedef struct tgw_panel tgw_panel;           /* one prepared phenotype panel */
typedef struct tgw_plan tgw_plan;             /* panels + scan workspace      */
typedef struct tgw_graph tgw_graph;           /* a captured tgw_scan call     */

/* Output buffers of one panel for one tgw_scan call.  Each array is
 * (m_end - m_begin) rows x n_pheno columns, row-major with row stride `ld`
 * elements (n_pheno <= ld <= 2^22; a larger stride is TGW_ERR_SHAPE when a
 * dense array is given): element (m - m_begin, p) holds the statistic of
 * marker m and phenotype p.  Any pointer may be NULL (not computed/written).
 *   r        partial correlation of g_m and y_p given [1 | C], in [-1, 1]
 *   beta     OLS coefficient of g_m (phenotype units per allele)
 *   se       its standard error
 *   t        beta / se = r sqrt(df / (1 - r^2))
 *   nlog10p  -log10 of the two-sided Student-t p-value (df degrees)
 * Degenerate markers (no observed call, monomorphic among observed calls, or
 * ||g_res||^2 <= 1e-8 ||g_c||^2 in FP64, i.e. the covariates explain all but
 * 1e-8 of the marker's variance) and degenerate phenotypes (residual norm
 * <= 1e-12 of the centred norm) give NaN in every output.  Markers with
 * ||g_res||^2 < ||g_c||^2 / 2 are finished on an FP64 path (explicit
 * residualization, FP64 contraction with the stored panel operand).
 *   best     optional reduced output (Methods 2.2, after Eq. 3: the
 *            statistics feed locus ranking and phenotype-level
 *            prioritization): device array of
 *            n_pheno entries holding, for each phenotype p, the test with the
 *            largest -log10 p over every marker scanned into it, packed as
 *            (IEEE bits of that -log10 p) << 32 | (0xffffffff - marker), with
 *            the absolute marker index (the smallest one among equal maxima).
 *            Within a call the test is chosen by |t|, on which -log10 p at
 *            the panel's fixed df is increasing; its -log10 p is FP64 for
 *            |t| > 40.
 *            The caller zeroes it before the first scan; scans merge by
 *            maximum, so marker ranges may be split over calls (markers
 *            < 2^32).  NaN tests never enter; 0 means none.  Independent of
 *            the dense arrays, which may all be NULL.
 *   topk     optional reduced output (same passage: ranking loci per
 *            phenotype): device array of n_pheno x topk_k words, row p
 *            holding phenotype p's topk_k tests with the largest |t| (hence
 *            the largest -log10 p at the panel's fixed df) over every marker
 *            scanned into it, in decreasing order, each packed as
 *            (IEEE bits of |t|) << 32 | (0xffffffff - marker) with the
 *            absolute marker index (equal |t|: the smaller marker first);
 *            0 = empty slot.  tgw_topk_read turns the words into -log10 p
 *            (FP64) and marker indices.  The caller zeroes it before the
 *            first scan; later scans merge into it, so marker ranges may be
 *            split over calls, but must not overlap (a marker scanned twice
 *            would be listed twice).  NaN tests never enter; |t| is exact
 *            for |t| > 40 as well (FP32).  1 <= topk_k <= 64.
 *   topk_k   entries per phenotype of topk (ignored when topk is NULL). */
typedef struct {
  float* r;
  float* beta;
  float* se;
  float* t;
  float* nlog10p;
  int64_t ld;
  unsigned long long* best;
  unsigned long long* topk;
  int32_t topk_k;
  int32_t reserved;
} tgw_outputs;

/* One entry of a thresholded hit list (see tgw_plan_set_hits). */
typedef struct {
  int64_t marker;  /* absolute marker index */
  int32_t panel;   /* panel index in the plan */
  int32_t pheno;   /* phenotype column of that panel */
  float nlog10p;   /* -log10 p (FP64-finished for |t| > 40) */
  float r;         /* partial correlation */
} tgw_hit;

/* Scan plan options; zero-initialise and set what you need. */
typedef struct {
  int64_t block_markers; /* markers per internal block (0 = automatic)          */
  int64_t tail_capacity; /* extreme-tail list entries (0 = 1<<20)                */
  int32_t tile;          /* tile shape index, < 0 = default (see tgw_plan_info);
                            also the shape of 8-bit dosage scans, where the wide
                            shapes run the register-staged shape 2             */
  int32_t reserved;
} tgw_plan_options;

/* ---- device memory ---------------------------------------------------------
 * The phenotype panel is prepared once and its operand, like the covariate
 * basis and the scan workspace, stays resident on the device (Methods 2.1:
 * preprocessing is reused across the panel).  That memory, and the temporary
 * buffers of tgw_fit_covariates and tgw_prepare_phenotypes, comes from the
 * allocator registered here, so that a framework's caching allocator can
 * supply it:
 *   alloc_fn(bytes, stream, ctx) returns device memory of the current device,
 *     aligned to at least 256 bytes, or NULL (-> TGW_ERR_OUT_OF_MEMORY);
 *     `stream` is the hipStream_t of the call that allocates (NULL for
 *     tgw_plan_create and the .bed streamer);
 *   free_fn(ptr, stream, ctx) takes it back; the library has synchronized
 *     the device before, so no enqueued work still uses it.
 * Both NULL restores hipMalloc / hipFree; exactly one NULL is
 * TGW_ERR_INVALID_ARG.  A handle keeps the allocator (and ctx) registered
 * when it was made and frees through it, so ctx must outlive the handles
 * made under it.  The functions are called on the thread of the tgw call
 * that needs memory, never from inside a kernel or a stream callback.
 * Thread-safe; applies to handles made after the call. */
typedef void* (*tgw_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*tgw_free_fn)(void* ptr, void* stream, void* ctx);
tgw_status tgw_set_allocator(tgw_alloc_fn alloc_fn, tgw_free_fn free_fn, void* ctx);

/* An allocator over one device buffer that the caller owns (for example a
 * framework tensor): register it with
 *   tgw_set_allocator(tgw_arena_alloc, tgw_arena_free, arena)
 * and the handles made afterwards take their device memory (the resident
 * panel operand and covariate basis of Methods 2.1, the scan workspace, the
 * temporaries of fit and preparation) from that buffer.
 *   tgw_arena_create: d_base is a device address aligned to 256 bytes, bytes
 *     its size (rounded down to a multiple of 256, at least 256).  The
 *     buffer stays owned by the caller and must outlive the arena; the arena
 *     never reads or writes it (bookkeeping is on the host).
 *     TGW_ERR_INVALID_ARG for NULL pointers, TGW_ERR_SHAPE for a misaligned
 *     or too small buffer.
 *   tgw_arena_alloc / tgw_arena_free: tgw_alloc_fn / tgw_free_fn with the
 *     arena as ctx.  Blocks are whole multiples of 256 bytes at 256-byte
 *     aligned addresses, placed best fit (smallest free range that holds the
 *     request, lowest address among equals); freed blocks merge with free
 *     neighbours.  A request the arena cannot hold returns NULL (the tgw call
 *     then fails with TGW_ERR_OUT_OF_MEMORY) and counts in n_failed; a
 *     pointer that is not a live block of the arena is ignored and counts in
 *     n_bad_free.  The stream argument is not used: the library frees only
 *     memory that no enqueued work still uses.
 *   tgw_arena_info: occupancy and counters (below).
 *   tgw_arena_destroy: frees the bookkeeping; TGW_ERR_INVALID_ARG (and the
 *     arena stays valid) while blocks are in use, i.e. while handles made
 *     under it are alive.  NULL is a no-op.
 * Thread-safe (one lock per arena). */
typedef struct tgw_arena tgw_arena;
typedef struct {
  size_t capacity;       /* usable bytes                                  */
  size_t in_use;         /* bytes in live blocks                          */
  size_t peak;           /* largest in_use so far                         */
  size_t largest_free;   /* largest request that would succeed now        */
  int64_t n_blocks;      /* live blocks                                   */
  int64_t n_free_ranges; /* free ranges (1 when nothing is in use)        */
  int64_t n_failed;      /* requests refused                              */
  int64_t n_bad_free;    /* frees of pointers that were not live blocks   */
} tgw_arena_stats;
tgw_status tgw_arena_create(void* d_base, size_t bytes, tgw_arena** out);
void* tgw_arena_alloc(size_t bytes, void* stream, void* ctx);
void tgw_arena_free(void* ptr, void* stream, void* ctx);
tgw_status tgw_arena_info(tgw_arena* arena, tgw_arena_stats* out);
tgw_status tgw_arena_destroy(tgw_arena* arena);

/* ---- library ---------------------------------------------------------- */
const char* tgw_status_string(tgw_status s);
const char* tgw_last_error(void);      /* thread-local detail of the last error */
int32_t tgw_abi_version(void);
/* Checks that the current device is gfx950 and caches its properties. */
tgw_status tgw_init(void);

/* ---- covariates (paper Methods 2.2, Eq. 1: Q spans the covariate space) --
 * Builds Q (n_samples x q, q = n_cov + 1, orthonormal columns) by an FP64
 * Householder QR of X0 = [1 | C] on the GPU.  The intercept is always added.
 * The reductions run over a fixed grid in a fixed order, so the same C gives
 * the same Q bit for bit in every call.
 *   d_C   device FP64, column-major n_samples x n_cov, leading dim ldc >= n_samples
 *         (may be NULL when n_cov == 0).  Not retained.
 * Synchronizes `stream` once to report:
 *   TGW_ERR_NONFINITE if C holds NaN/Inf; TGW_ERR_RANK_DEFICIENT if
 *   |R_jj| <= 1e-10 max_i |R_ii|; TGW_ERR_SHAPE unless n_samples >= n_cov + 3
 *   and 0 <= n_cov <= 31. */
tgw_status tgw_fit_covariates(int64_t n_samples, int32_t n_cov, const double* d_C, int64_t ldc,
                              void* stream, tgw_covariates** out);
void tgw_covariates_free(tgw_covariates* cov);
/* Copies Q (FP64, column-major n x q, leading dim ldq >= n) to device memory. */
tgw_status tgw_covariates_q(const tgw_covariates* cov, double* d_Q, int64_t ldq, void* stream);

/* ---- phenotype panel (paper Methods 2.2, Eq. 1 + standardization) -------
 * Once per panel: Y_c = Y - mean(Y); Y_res = (I - Q Q^T) Y_c;
 * s_p = ||Y_res,p|| (FP64); Y~ = Y_res / s_p; then Y~ is stored in the
 * scan's operand layout (FP32, or the hi + lo terms of the split forms) together
 * with per-column FP64-derived constants and the p-value table for
 * df = n_samples - q - 1.
 *   d_Y   device, column-major n_samples x n_pheno, FP32 (y_is_fp64 = 0) or
 *         FP64 (y_is_fp64 = 1), leading dim ldy >= n_samples.  Not retained.
 * The panel keeps a reference to `cov`; free panels before their covariates.
 * Synchronizes `stream` once; TGW_ERR_NONFINITE on NaN/Inf in Y. */
tgw_status tgw_prepare_phenotypes(const tgw_covariates* cov, int64_t n_pheno, const void* d_Y,
                                  int32_t y_is_fp64, int64_t ldy, tgw_precision prec,
                                  void* stream, tgw_panel** out);
void tgw_panel_free(tgw_panel* panel);
/* n = samples, p = phenotypes, q = columns of Q, df = residual degrees of freedom. */
tgw_status tgw_panel_info(const tgw_panel* panel, int64_t* n, int64_t* p, int32_t* q, int64_t* df);

/* ---- scan plan ------------------------------------------------------------
 * Groups one or more prepared panels that share n_samples and precision
 * (the batching form: uneven P and K run through one persistent launch over
 * the virtual concatenation of all their columns) and allocates the scan
 * workspace.  `panels` must stay alive while the plan is used. */
tgw_status tgw_plan_create(const tgw_panel* const* panels, int32_t n_panels,
                           const tgw_plan_options* opts, tgw_plan** out);
void tgw_plan_free(tgw_plan* plan);
/* tile = chosen tile shape index; n_tiles = number of shapes;
 * block_markers = markers per internal block. */
tgw_status tgw_plan_info(const tgw_plan* plan, int32_t* tile, int32_t* n_tiles, int64_t* block_markers);
/* Tile shape idx as (markers per workgroup tile, columns per tile, waves). */
tgw_status tgw_tile_shape(int32_t idx, int32_t* tile_markers, int32_t* tile_cols, int32_t* waves);
/* Autotuner: times every tile shape on markers [m_begin, m_end) of d_geno
 * (one block at most) with HIP events, keeps the fastest for this plan and
 * records it in a JSON cache keyed by (arch, padded samples, column blocks,
 * panels, precision): $TGW_TUNE_CACHE, default ~/.cache/tgw/tune.json.  A
 * later plan with the same key takes the cached shape without timing.
 * Writes scratch results into `outs` (it scans the markers several times, so
 * zero best and topk again before the real scan); synchronizes `stream`.
 * best_ms may be NULL. */
tgw_status tgw_plan_autotune(tgw_plan* plan, const uint8_t* d_geno, int64_t n_markers, int64_t row_bytes,
                             tgw_geno_code code, int64_t m_begin, int64_t m_end, const tgw_outputs* outs,
                             void* stream, double* best_ms);

/* ---- the scan (paper Methods 2.2, Eq. 2-3 and the p-value conversion) ----
 * Streams markers [m_begin, m_end) of the packed genotype matrix through
 * every panel of the plan and writes each panel's outputs.
 *   d_geno     device, n_markers rows of row_bytes bytes (see tgw_geno_code);
 *              16-byte aligned, row_bytes a multiple of 16 and >= 16 *
 *              ceil(n_samples / 64) for 2-bit codes, >= 64 * ceil(n_samples /
 *              64) for 8-bit dosages.  Bytes past sample n_samples-1 are
 *              ignored.
 *   outs       n_panels entries, in the plan's panel order (see tgw_outputs).
 * Per marker: exact integer counts give the mean mu; each call g is fed to
 * the matrix cores as gs (g - c), exact in the operand type (FP32: gs = 1,
 * c = round(64 mu)/64; FP16 forms: gs = 1, c = round(512 mu)/512; BF16: see
 * TGW_PREC_SPLIT), a missing call as gs (mu - c) rounded to the operand type
 * (error <= about 2^-18 in BF16, 2^-21 in FP16); the intercept of the
 * covariate projection removes c exactly and the epilogue divides by gs.  8-bit dosages enter as q - c with the integer c = round(mu) in
 * units of 1/127 (exact in FP16 and FP32), a missing one as mu - c (error <=
 * 2^-12 / 127 in FP16).  They run the register-staged tile shapes; the
 * autotuner keeps a separate choice for them.
 * Results are deterministic run to run.  A scan split into several marker
 * ranges gives bitwise the same outputs as one call when every boundary is a
 * multiple of 512 markers from m_begin (any boundary for FP32 and the 16-bit
 * split forms; the FP16 hi + FP8 lo form orders its FP32 accumulation by a
 * marker's row in the 512-marker tile).
 * Asynchronous: enqueues kernels on `stream`, allocates nothing and does not
 * synchronize; capturable in a HIP graph.  The plan's workspace is reused, so
 * calls with the same plan must not run concurrently on different streams.
 * Extreme tails (|t| > 40) are finished in FP64 by a follow-up kernel; if
 * more than tail_capacity such tests occur in one call, the excess keep a
 * lower bound and tgw_plan_check reports TGW_ERR_TAIL_OVERFLOW. */
tgw_status tgw_scan(tgw_plan* plan, const uint8_t* d_geno, int64_t n_markers, int64_t row_bytes,
                    tgw_geno_code code, int64_t m_begin, int64_t m_end, const tgw_outputs* outs,
                    void* stream);
/* Thresholded hit list (reduced output; Methods 2.2, after Eq. 3: ranking
 * associated loci)
 * for the following tgw_scan calls on this plan and for graphs captured
 * afterwards: every test with -log10 p >= threshold is appended to d_hits
 * (device, `capacity` entries) at index atomicAdd(d_count, 1), in no
 * particular order; for |t| > 40 the decision is taken on the FP64 value.
 * Entries past `capacity` are dropped but still counted:
 * *d_count > capacity after a scan means the list is truncated.  The caller
 * owns both buffers and zeroes *d_count; successive scans keep appending.
 * d_hits == NULL turns the list off.  The autotuner never appends. */
tgw_status tgw_plan_set_hits(tgw_plan* plan, tgw_hit* d_hits, int64_t capacity, unsigned long long* d_count,
                             float threshold);

/* Per-phenotype top-k words of `panel` (tgw_outputs.topk, n_pheno x k) as
 * -log10 p (FP64 from |t| at the panel's df, rounded to FP32; NaN for an
 * empty slot) and absolute marker indices (-1 for an empty slot), both
 * device arrays of n_pheno x k, row-major.  Asynchronous on `stream`. */
tgw_status tgw_topk_read(const tgw_panel* panel, const unsigned long long* d_words, int32_t k, float* d_nlog10p,
                         int64_t* d_marker, void* stream);

/* Synchronizes `stream` and reports device errors / tail overflow of the
 * last tgw_scan on this plan; n_tail receives the number of tail tests. */
tgw_status tgw_plan_check(tgw_plan* plan, void* stream, int64_t* n_tail);

/* ---- kernel timing ----------------------------------------------------------
 * With profiling on, every tgw_scan on this plan records HIP events on its
 * stream around each launch of the main contraction kernel (the dominant
 * kernel).  tgw_plan_profile_read synchronizes `stream`, returns the summed
 * kernel time in ms and the number of launches since the last read, and
 * clears the record.  Not for use inside graph capture. */
tgw_status tgw_plan_profile(tgw_plan* plan, int32_t enable);
tgw_status tgw_plan_profile_read(tgw_plan* plan, void* stream, double* main_ms, int64_t* launches);

/* ---- scan without a plan, allocating nothing --------------------------------
 * For callers that cannot allocate device memory at scan time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * tgw_scan over the given panels without a plan.  Everything a plan holds
 * (column-block tables, per-panel constants, output table, per-block
 * workspace, the FP64 list of collinear markers, the tail list) lives in a
 * static device array of 64 MiB that every GPU the library runs on holds
 * until the process ends; the call allocates nothing and does not
 * synchronize.  Same arguments and results as tgw_scan (the panels' order is
 * the outputs' order), with these differences:
 *   - at most 32 panels and 2^20 phenotype columns in all (TGW_ERR_SHAPE);
 *     the marker block is the largest multiple of 512 markers whose
 *     workspace fits (330,240 markers for one panel, 13,824 for 32);
 *   - tile: the tile shape index (< 0: shape 0; 8-bit dosages: shape 2);
 *     no autotuning, no hit list, no profiling;
 *   - the tail list holds 65,536 tests; d_n_tail (device, may be NULL)
 *     receives the number of tail tests the call found: above 65,536 the
 *     excess keep the table's lower bound at |t| = 40;
 *   - calls on one GPU share the array and leave its contents behind: two
 *     calls that overlap on one GPU (streams, threads) race; host threads
 *     are serialized while they enqueue. */
tgw_status tgw_scan_static(const tgw_panel* const* panels, int32_t n_panels, const uint8_t* d_geno,
                           int64_t n_markers, int64_t row_bytes, tgw_geno_code code, int64_t m_begin, int64_t m_end,
                           const tgw_outputs* outs, int32_t tile, unsigned long long* d_n_tail, void* stream);

/* ---- graph capture ---------------------------------------------------------
 * Captures one tgw_scan call (same arguments) into an instantiated HIP graph;
 * tgw_graph_launch replays it on `stream`.  The graph refers to the plan's
 * workspace and to the given buffers, which must outlive it. */
tgw_status tgw_graph_create(tgw_plan* plan, const uint8_t* d_geno, int64_t n_markers, int64_t row_bytes,
                            tgw_geno_code code, int64_t m_begin, int64_t m_end,
                            const tgw_outputs* outs, tgw_graph** out);
tgw_status tgw_graph_launch(tgw_graph* graph, void* stream);
void tgw_graph_free(tgw_graph* graph);

/* ---- PLINK 1 binary genotype input ----------------------------------------
 * The paper's workflow reads PLINK (and BGEN, NumPy) genotype inputs directly
 * and aligns phenotype and covariate tables to the genotypes by sample ID
 * (Abstract; Introduction), and notes that end-to-end speed then depends on
 * the reader and storage bandwidth (Methods 2.4; Discussion).  These calls
 * read a variant-major .bed file (3 magic bytes 6c 1b 01, then per marker
 * ceil(n/4) bytes, sample s at bits 2(s & 3) of byte s >> 2, codes 00 / 01 /
 * 10 / 11 = 0 / missing / 1 / 2 copies of the second allele, i.e.
 * TGW_CODE_PLINK_BED), and stream it through the scan.  A tgw_bed handle is
 * not thread-safe: one call at a time. */
typedef struct tgw_bed tgw_bed;

/* Opens `path` (host) holding n_samples samples (the lines of its .fam).
 * Errors: TGW_ERR_INVALID_ARG (cannot open / not a variant-major .bed),
 * TGW_ERR_SHAPE (file size is not 3 + n_markers * ceil(n_samples / 4)).
 * All samples are selected, in file order. */
tgw_status tgw_bed_open(const char* path, int64_t n_samples, tgw_bed** out);
/* Waits for the handle's pending streamed work, frees its buffers, closes. */
void tgw_bed_close(tgw_bed* bed);
tgw_status tgw_bed_info(const tgw_bed* bed, int64_t* n_file_samples, int64_t* n_markers, int64_t* n_selected);
/* Sample selection (host array): scan sample j is file sample idx[j],
 * 0 <= idx[j] < n_file_samples, all distinct; the caller's phenotype and
 * covariate rows follow the same order.  idx == NULL selects every sample
 * in file order. */
tgw_status tgw_bed_select(tgw_bed* bed, const int64_t* idx, int64_t n);
/* Host read of markers [m_begin, m_end) with the selection applied: row m -
 * m_begin of `dst` (host, row_bytes >= ceil(n_selected / 4) bytes per row)
 * holds scan sample j at bits 2(j & 3) of byte j >> 2, and code 01
 * (missing) past the last selected sample. */
tgw_status tgw_bed_read(const tgw_bed* bed, int64_t m_begin, int64_t m_end, uint8_t* dst, int64_t row_bytes);
/* Sample-ID matching against a PLINK sample table (.fam: whitespace-separated
 * FID IID ... per line): idx[i] = the line (0-based, blank lines skipped) whose
 * IID equals ids[i], or -1 if none.  Errors if an id is requested twice or a
 * requested id occurs on several lines.  n_file_samples receives the number
 * of sample lines, n_found the number of matched ids (each may be NULL). */
tgw_status tgw_fam_match(const char* fam_path, const char* const* ids, int64_t n_ids, int64_t* idx,
                         int64_t* n_file_samples, int64_t* n_found);
/* tgw_scan over markers [m_begin, m_end) of the file (output row m - m_begin,
 * as for tgw_scan with TGW_CODE_PLINK_BED), streamed in blocks of
 * block_markers (0: 65,536) through two pinned host buffers and two device
 * buffers owned by the handle (made on the first call, kept until close):
 * n_threads host threads (0: 4) read block k while the device copies and
 * scans block k - 1; a gather kernel applies the sample selection on the
 * device.  The plan's n_samples must equal the selection's size.  Returns
 * when every read and host-to-device copy is done; the scan itself may still
 * run on `stream` (tgw_plan_check waits for it).  On error the outputs are
 * undefined. */
tgw_status tgw_scan_bed(tgw_plan* plan, tgw_bed* bed, int64_t m_begin, int64_t m_end, const tgw_outputs* outs,
                        int64_t block_markers, int32_t n_threads, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* TGW_H */
