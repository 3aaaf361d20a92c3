// Internal declarations shared by the gfx950 kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tgw {

// ---- operand layout -------------------------------------------------------
// Samples are processed in chunks of 64 (the contraction's K chunk).  A
// prepared panel (and the covariate columns used for Q^T g) is stored as
// column blocks of 32 columns; block (cb, ch) holds columns 32cb..32cb+31
// for samples 64ch..64ch+63, arranged exactly as the matrix core reads them
// (see kernels: operand_index_split / operand_index_fp32 / operand_index_lo8):
// 8 KiB for FP32 and the 16-bit splits, 6 KiB for FP16 hi + FP8 lo.
constexpr int kChunk = 64;
constexpr int kColBlock = 32;
constexpr int kBlockBytes = 8192;
constexpr int kBlockBytes8 = 6144;
constexpr int kSlots = 32;      // correction slots per (marker, panel): dmu, Q^T g
// the last slot, free when q <= 31, carries the FP8 lo pass's change of centring
// (FP16 + FP8 form): (c - c8) per marker against -(sum of lo terms) per column
constexpr int kLoSlot = kSlots - 1;
constexpr int kMaxCov = 31;     // K <= 31 so that q = K + 1 <= 32 slots
constexpr int kMaxPanelsPerBind = 32;
// Covariate-collinear markers.  The contraction's FP32 rounding error scales
// with ||g_c|| while the statistic scales with ||g_res||, so the error in r
// grows as (||g_res||^2 / ||g_c||^2)^-1/2.  A marker whose ||g_res||^2 (from
// the FP32-accumulated Q^T g, good to about 1e-6 ||g_c||^2) is below
// kRedoTol ||g_c||^2 is not finished by the main kernel (its rows there are
// NaN) but by an FP64 kernel that residualizes it explicitly and contracts
// it with the stored panel operand; that kernel calls it degenerate (NaN)
// when its FP64 ||g_res||^2 <= kCollinearTol ||g_c||^2.
constexpr double kRedoTol = 0.5;
constexpr double kCollinearTol = 1e-8;
constexpr int kRedoGroup = 16;   // listed markers per work item of the FP64 kernel
constexpr int kRedoCols = 256;   // columns per work item (one per thread)

// ---- p-value table ----------------------------------------------------------
constexpr float kTMax = 40.0f;        // |t| beyond this goes to the FP64 tail
constexpr int kTabPerUnit = 32;       // nodes per unit of |t|
constexpr int kTabNodes = 40 * 32 + 2;
constexpr int kTabIntervals = kTabNodes - 1;  // one cubic per interval between nodes

// kSplit8: FP16 hi term of 2^12 y against FP16 genotypes, plus the FP8 e4m3
// lo term (scaled per column by a power of two) against FP8 genotypes
enum Prec { kFP32 = 0, kSplit = 1, kSplit16 = 2, kSplit8 = 3 };
constexpr int kNumPrec = 4;
// the FP16 forms store 2^12 y (and 2^12 q_k) so that unit-norm columns stay
// in FP16's normal range; statistics are invariant to the scale
constexpr float kF16Scale = 4096.0f;
// 8-bit dosage q in 0..254 stands for q / 127 copies (255 = missing)
constexpr float kDosage8Unit = 127.0f;
__host__ __device__ constexpr int block_bytes(int prec) { return prec == kSplit8 ? kBlockBytes8 : kBlockBytes; }
// precision of the Q^T g contraction (the FP8 form has no covariate operand
// of its own: Q^T g runs on the FP16 split)
__host__ __device__ constexpr int wprec(int prec) { return prec == kSplit8 ? kSplit16 : prec; }
__host__ __device__ constexpr bool f16_scaled(int prec) { return prec == kSplit16 || prec == kSplit8; }
// kRaw: raw FP32 products; kTest: the fused test epilogue; kRawHL: raw
// products of a split operand whose hi parts sit in columns 0..15 and lo parts
// in columns 16..31 of the hi half (one matrix-core pass), summed per slot
// (the Q^T g contraction of the split forms)
enum Mode { kRaw = 0, kTest = 1, kRawHL = 2 };
constexpr int kHLSlots = 16;  // covariate slots per packed hi|lo operand block
// packed hi|lo blocks of a covariate basis with q columns
__host__ __device__ constexpr int hl_blocks(int q) { return q <= kHLSlots ? 1 : 2; }

// per-marker statistics of one marker block
struct MarkerStat {
  double gc2;    // ||g_c||^2 of the mean-imputed marker (exact from integer counts)
  float dmu;     // gs (mu - c): the operand value of a missing call before rounding
  int32_t flags; // 1 = degenerate (no observed call or monomorphic)
  double mu;
  double shift;  // c: mu rounded to U / K (BF16), 1/512 (FP16 forms, FP32: 1/64); 8-bit dosages: to an integer
  float gscale;  // gs: operand units per genotype unit of this marker (K / 128 for BF16, else 1)
  float dlo;     // c - c8, c8 the centring of the FP8 lo pass (FP16 + FP8 form), else 0
};

struct PanelDev {
  const float* scale;   // s_p = ||Y_res,p||
  const float* invny;   // 1 / ||(I - QQ^T) y_op,p||  (NaN for degenerate columns)
  const float* cw;      // [P_pad][32]: (-sum_i y_op, -q_k^T y_op for k >= 1, 0 ...)
  const float4* table;  // per interval k: -log10 p(|t|) = c0 + c1 s + c2 s^2 + c3 s^3, s = 32|t| - k
  const uint8_t* lscale; // FP8 form: E8M0 scale of each column's lo term (NULL otherwise)
  const double* Q;      // covariate basis, [q][n_pad] FP64 (the FP64 path of collinear markers)
  const void* yop;      // operand base (column 0, chunk 0)
  const void* wop;      // the covariates' Q^T g operand of this precision (packed hi|lo blocks, or FP32)
  int64_t n_pheno;
  float df;
  float sqrt_df;
  float inv_sqrt_df;
  int32_t q;
};

// largest output row stride: a workgroup's rows of one column block then lie
// within 2^31 bytes of its first element, so stores take 32-bit offsets
constexpr int64_t kMaxOutLd = int64_t(1) << 22;

struct OutDev {
  float* r;
  float* beta;
  float* se;
  float* t;
  float* nl;
  int64_t ld;
  unsigned long long* best;  // per column: (bits of max -log10 p) << 32 | (0xffffffff - marker)
  unsigned long long* topk;  // per column: topk_k words (bits of |t|) << 32 | (0xffffffff - marker), decreasing
  int32_t topk_k;
  int32_t pad;
};
constexpr int kTopKMax = 64;

// thresholded hit list (layout of tgw_hit)
struct Hit {
  int64_t marker;
  int32_t panel;
  int32_t pheno;
  float nl;
  float r;
};

struct HitDev {
  Hit* entries;               // NULL: no hit list
  unsigned long long* count;
  int64_t capacity;
  float threshold;            // -log10 p
  float t_floor;              // |t| below this cannot reach the threshold at any df
};

// one 32-column block of the virtual concatenation of all panels' columns
struct ColBlock {
  const char* op;  // operand base of this block: chunk ch at op + ch * block_bytes(prec)
  int32_t panel;   // owning panel
  int32_t col0;    // local column of the block's first column (RAW: output column)
  int32_t ncol;    // valid columns in this block
  int32_t pad;
};

struct TailEntry {
  int64_t row;  // output row (marker - m_begin)
  int32_t panel;
  int32_t col;
  float r;
  int32_t pad;
};

struct TailDev {
  TailEntry* entries;
  unsigned long long* count;  // [0] = entries requested in the current call
  int64_t capacity;
};

struct GemmArgs {
  const uint8_t* geno;
  int64_t row_bytes;
  int64_t m0;        // row of the block's first marker in geno
  int64_t nm;        // markers in the block
  int64_t out_row0;  // output row of the block's first marker
  int32_t n_chunks;
  int32_t n_cblocks;
  int32_t n_mtiles;
  int32_t n_ctiles;
  int32_t n_panels;
  float gunit;           // operand units per genotype unit (1; 127 for 8-bit dosages): scales beta and SE
  const ColBlock* cblocks;
  const PanelDev* panels;
  const OutDev* outs;
  const uint4* mlut;     // [nm] decode table of each marker (2-bit codes, 16-bit forms: x lo bytes, y hi
                         // bytes, z FP8 bytes; FP32: the four values; 8-bit dosages: see kG8Lut)
  const float* wws;      // [nm][n_panels][32]
  const float2* invh;    // [nm][n_panels]: 1 / (gs ||g_res||), 1 / ||g_res||
  float* raw_out;        // RAW mode destination
  int64_t raw_ld;
  TailDev tail;
  HitDev hits;
  int64_t m_begin;   // absolute index of output row 0
};

struct StatsArgs {
  const uint8_t* geno;
  int64_t row_bytes;
  int64_t m0;
  int64_t nm;
  int64_t n;           // samples
  int32_t code;        // tgw_geno_code
  int32_t prec;        // Prec
  uint4* mlut;
  MarkerStat* mstat;
  uint32_t* redo_count;  // [n_panels]: zeroed by the block's first workgroup
  int32_t n_panels;
  int32_t lo_int;        // FP16 + FP8 form: the FP8 lo pass centres on the integer c8 = rint(c)
};

// markers left to the FP64 kernel, per panel: rows (within the marker block)
// at entries[j * stride + k], k < count[j]
struct RedoDev {
  int32_t* entries;
  uint32_t* count;
  int64_t stride;
};

struct RedoArgs {
  const uint8_t* geno;
  int64_t row_bytes;
  int64_t m0;        // row of the block's first marker in geno
  int64_t n;         // samples
  int64_t n_pad;
  int32_t n_chunks;
  int32_t code;      // tgw_geno_code
  int32_t prec;
  int32_t n_panels;
  int32_t max_chunks;  // column chunks of kRedoCols in the widest panel
  float gunit;
  int64_t out_row0;
  int64_t m_begin;
  const MarkerStat* mstat;
  const PanelDev* panels;
  const OutDev* outs;
  HitDev hits;
  RedoDev redo;
};

struct BindArgs {
  OutDev outs[kMaxPanelsPerBind];
  OutDev* dst;
  int32_t first;
  int32_t count;
};

// ---- launchers (kernels.hip) -------------------------------------------------
// covariate QR: row-parallel passes over kQrGrid workgroups; scratch holds
// kQrScratch doubles (the partial sums and the per-step coefficients)
constexpr int kQrGrid = 128;
constexpr int kQrScratch = kQrGrid * kSlots + 2 * kSlots;
hipError_t launch_qr(const double* C, int64_t ldc, int64_t n, int64_t n_pad, int q, double* X, double* Q,
                     double* rdiag, double* scratch, int32_t* flags, hipStream_t s);
hipError_t launch_cov_operands(const double* Q, int64_t n, int64_t n_pad, int q, void* wop_fp32,
                               void* const* wop_hl, hipStream_t s);
hipError_t launch_prep(const void* Y, int y_fp64, int64_t ldy, int64_t n, int64_t n_pad, int64_t P,
                       const double* Q, int q, int prec, void* yop, float* scale, float* invny, float* cw,
                       uint8_t* lscale, int32_t* flags, hipStream_t s);
hipError_t launch_set_operand(const float* V, int64_t ldv, int64_t n, int64_t n_pad, int64_t P, int prec,
                              void* yop, uint8_t* lscale, hipStream_t s);
hipError_t launch_table(float4* table, double df, hipStream_t s);
hipError_t launch_stats(const StatsArgs& a, hipStream_t s);
hipError_t launch_finalize(const MarkerStat* ms, float* wws, float2* invh, int64_t nm, int n_panels, float wscale,
                           int lo_slot, RedoDev redo, hipStream_t s);
hipError_t launch_redo(const RedoArgs& a, int grid, hipStream_t s);
hipError_t launch_bind(const BindArgs& a, hipStream_t s);
hipError_t launch_tail_reset(TailDev t, hipStream_t s);
hipError_t launch_tail(TailDev t, const PanelDev* panels, const OutDev* outs, HitDev hits, int64_t m_begin,
                       hipStream_t s);
hipError_t launch_topk_read(const unsigned long long* words, int64_t n, int k, double df, float* nl, int64_t* marker,
                            hipStream_t s);
hipError_t launch_debug_stats(const MarkerStat* ms, int64_t nm, double* shift, double* mean, double* scale,
                              hipStream_t s);

// main contraction; `tile` selects one of the compiled tile shapes
struct TileShape {
  int waves;     // waves per workgroup (all along the marker dimension)
  int wm_frags;  // 32-row fragments per wave
  int wn_frags;  // 32-column blocks per workgroup tile
  int tm() const { return waves * wm_frags * 32; }
  int tp() const { return wn_frags * 32; }
};
int n_tile_shapes();
TileShape tile_shape(int idx);
// g8: the genotype rows hold 8-bit dosages (one byte per sample), which the
// register-staged kernel decodes; the wide shapes run shape 2 for them
TileShape tile_shape_for(int idx, int prec, bool g8 = false);  // the shape a precision actually runs
// largest resident grid for a tile shape (occupancy x CUs), rounded to 8 XCDs
int gemm_grid(int idx, int prec, int mode, int n_cu, bool g8 = false);
int tile_alias(int idx, int prec, bool g8 = false);  // smallest tile index that runs the same kernel
hipError_t launch_gemm(int idx, int prec, int mode, const GemmArgs& a, int grid, hipStream_t s, bool g8 = false);
// precisions that 8-bit dosages run in (exact re-centred operand: FP32 and the FP16 split)
__host__ __device__ constexpr bool g8_supported(int prec) { return prec == kFP32 || prec == kSplit16 || prec == kSplit8; }
int wgemm_tile();  // tile shape used for the Q^T g contraction

}  // namespace tgw
