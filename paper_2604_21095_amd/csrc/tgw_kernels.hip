// gfx950 kernels of the phenotype-panel linear association scan.
//
//  qr_*_kernel        FP64 Householder QR of [1 | C] -> Q (Methods 2.2: Q
//                     spans the covariate space and has orthonormal columns)
//  prep_kernel        Eq. 1 + column standardization, once per panel, FP64;
//                     writes the contraction operand (FP32 or BF16 hi + lo)
//  table_kernel       -log10 p nodes for |t| in [0, 40] at the panel's df
//  stats_kernel       exact integer per-marker counts -> mean, ||g_c||^2,
//                     re-centring constant and the 2-bit decode table
//  gemm_kernel        the contraction of Eq. 2 on the matrix cores with the
//                     fused epilogue (r, t of Eq. 3, beta, SE, -log10 p)
//  finalize_kernel    ||g_res||^2 = ||g_c||^2 - sum_k (q_k^T g)^2
//  tail_kernel        FP64 -log10 p for |t| > 40
#include "tgw_internal.h"

#include <math.h>

#include <type_traits>

namespace tgw {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ inline uint32_t bf16_bits_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ inline float bf16_to_float(uint32_t b) { return __uint_as_float(b << 16); }

__device__ inline uint32_t pack_bf16x2(float lo, float hi) {
  return bf16_bits_rne(lo) | (bf16_bits_rne(hi) << 16);
}

template <int NT>
__device__ inline double block_max(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double m = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) m = fmax(m, sh[i]);
  return m;
}

template <int NT>
__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += sh[i];
  return s;
}

// reduce NV values at once; sh holds (NT/64) * NV doubles
template <int NT, int NV>
__device__ inline void block_sum_vec(double* v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k)
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[w * NV + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int i = 0; i < NT / 64; ++i) s += sh[i * NV + k];
    v[k] = s;
  }
}

// ---------------------------------------------------------------------------
// operand layout (must match the matrix-core fragment reads in gemm_kernel)
//
// BF16 split: block (cb, ch) holds 4096 bf16: [hl][j][lane][e], hl = 0 for
// hi, 1 for lo; j = K16 step; lane = 32 h + column; e = element.  The sample
// fed at (j, h, e) is 64 ch + 32 h + 16 (j >> 1) + 4 (j & 1) + (e >> 1) +
// 8 (e & 1), which is the order in which gemm_kernel decodes packed codes.
// FP32: block (cb, ch) holds 2048 floats: [j >> 2][lane][j & 3], j = K2 step,
// sample 64 ch + 32 h + j.
// ---------------------------------------------------------------------------
// stride: 16-bit elements per block (4096 for the 16-bit splits; 3072 for
// FP16 hi + FP8 lo, whose block keeps only the hi half in this layout)
__device__ inline int64_t operand_index_split(int64_t col, int64_t i, int n_chunks, int hl,
                                              int64_t stride = 4096) {
  const int64_t cb = col >> 5;
  const int c = (int)(col & 31);
  const int64_t ch = i >> 6;
  const int s = (int)(i & 63);
  const int h = s >> 5;
  const int rem = s & 31;
  const int jhi = rem >> 4;
  const int b = (rem >> 3) & 1;
  const int jlo = (rem >> 2) & 1;
  const int d = rem & 3;
  const int j = 2 * jhi + jlo;
  const int e = 2 * d + b;
  const int lane = 32 * h + c;
  return (cb * n_chunks + ch) * stride + hl * 2048 + j * 512 + lane * 8 + e;
}

__device__ inline int64_t operand_index_fp32(int64_t col, int64_t i, int n_chunks) {
  const int64_t cb = col >> 5;
  const int c = (int)(col & 31);
  const int64_t ch = i >> 6;
  const int s = (int)(i & 63);
  const int h = s >> 5;
  const int j = s & 31;
  const int lane = 32 * h + c;
  return (cb * n_chunks + ch) * 2048 + (j >> 2) * 256 + lane * 4 + (j & 3);
}

// FP16 hi + FP8 lo: block (cb, ch) = 6 KiB.  Bytes [0, 4096) hold the FP16
// hi terms in the split layout's hi half; bytes [4096, 6144) the e4m3 lo
// terms as [part][lane][16 bytes].  A lane (32 h + column) holds 32 bytes,
// dword D = 4 part + t, byte k; it feeds sample 64 ch + 32 h + 16 part +
// 4 k + t, the order in which the genotype FP8 decode emits them.
__device__ inline int64_t operand_index_lo8(int64_t col, int64_t i, int n_chunks) {
  const int64_t cb = col >> 5;
  const int c = (int)(col & 31);
  const int64_t ch = i >> 6;
  const int s = (int)(i & 63);
  const int h = s >> 5;
  const int part = (s >> 4) & 1;
  const int k = (s >> 2) & 3;
  const int t = s & 3;
  const int lane = 32 * h + c;
  return (cb * n_chunks + ch) * kBlockBytes8 + 4096 + part * 1024 + lane * 16 + 4 * t + k;
}

__device__ inline uint32_t f16_bits_rn(float f) {
  const _Float16 h = (_Float16)f;  // round to nearest even
  return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
__device__ inline float f16_to_float(uint32_t b) { return (float)__builtin_bit_cast(_Float16, (uint16_t)b); }

// OCP FP8 E4M3 (bias 7, no infinities, largest finite 448, subnormals
// m * 2^-9), round to nearest even.  |x| must not exceed 448.
__device__ inline uint32_t e4m3_bits_rne(double x) {
  const uint32_t sign = x < 0.0 ? 0x80u : 0u;
  const double a = fabs(x);
  if (a < 0x1p-6) {
    const double m = rint(a * 0x1p9);  // subnormal step 2^-9; m = 8 is the smallest normal
    return sign | (uint32_t)m;
  }
  int e = ilogb(a);
  double q = rint(ldexp(a, 3 - e)) - 8.0;  // 3 fraction bits
  if (q >= 8.0) {
    q = 0.0;
    ++e;
  }
  return sign | (uint32_t)((e + 7) << 3) | (uint32_t)q;
}
__device__ inline double e4m3_value(uint32_t b) {
  const int e = (b >> 3) & 15, m = b & 7;
  const double v = e == 0 ? ldexp((double)m, -9) : ldexp(1.0 + m / 8.0, e - 7);
  return (b & 0x80u) ? -v : v;
}

// power-of-two shift that brings a column's largest FP8 lo term near the top
// of the e4m3 range (0 for a column without lo terms)
__device__ inline int lo_shift(double maxlo) {
  if (!(maxlo > 0.0)) return 0;
  int s = ilogb(448.0 / maxlo);
  return s < -100 ? -100 : (s > 100 ? 100 : s);
}

// lsh: the column's FP8 lo shift (FP16 hi + FP8 lo form only)
// the hi and lo parts of a value in the BF16 split, or of 2^12 times it in
// the FP16 split (round to nearest even, then the rounded remainder)
__device__ inline void split_parts(int prec, double v, uint32_t* hb, uint32_t* lb) {
  if (prec == kSplit16) {
    const double vs = v * (double)kF16Scale;
    *hb = f16_bits_rn((float)vs);
    *lb = f16_bits_rn((float)(vs - (double)f16_to_float(*hb)));
  } else {
    *hb = bf16_bits_rne((float)v);
    *lb = bf16_bits_rne((float)(v - (double)bf16_to_float(*hb)));
  }
}

// stored: the value the operand now holds (in 2^12 units for the FP16
// forms); lo: its FP8 lo term alone (FP16 + FP8 form; 0 otherwise)
__device__ inline void store_operand(void* op, int prec, int64_t col, int64_t i, int n_chunks, double v,
                                     double* stored, int lsh = 0, double* lo = nullptr) {
  if (lo) *lo = 0.0;
  if (prec == kSplit8) {
    const double vs = v * (double)kF16Scale;
    const uint32_t hb = f16_bits_rn((float)vs);
    const double hi = (double)f16_to_float(hb);
    const uint32_t qb = e4m3_bits_rne(ldexp(vs - hi, lsh));
    ((uint16_t*)op)[operand_index_split(col, i, n_chunks, 0, kBlockBytes8 / 2)] = (uint16_t)hb;
    ((uint8_t*)op)[operand_index_lo8(col, i, n_chunks)] = (uint8_t)qb;
    const double lv = ldexp(e4m3_value(qb), -lsh);
    *stored = hi + lv;
    if (lo) *lo = lv;
  } else if (prec == kSplit16 || prec == kSplit) {
    uint32_t hb, lb;
    split_parts(prec, v, &hb, &lb);
    uint16_t* p = (uint16_t*)op;
    p[operand_index_split(col, i, n_chunks, 0)] = (uint16_t)hb;
    p[operand_index_split(col, i, n_chunks, 1)] = (uint16_t)lb;
    *stored = prec == kSplit16 ? (double)f16_to_float(hb) + (double)f16_to_float(lb)
                               : (double)bf16_to_float(hb) + (double)bf16_to_float(lb);
  } else {
    const float f = (float)v;
    ((float*)op)[operand_index_fp32(col, i, n_chunks)] = f;
    *stored = (double)f;
  }
}

// ---------------------------------------------------------------------------
// FP64 Student-t tail: ln of the two-sided p-value
//   p = I_x(df/2, 1/2), x = df / (df + t^2)
// I_x(a, b) = x^a (1 - x)^b / (a B(a, b)) * F, F the continued fraction of
// the incomplete beta function (Abramowitz & Stegun 26.5.8), evaluated with
// the modified Lentz method; valid for x < (a + 1) / (a + b + 2), otherwise
// I_x(a, b) = 1 - I_{1-x}(b, a).
// ---------------------------------------------------------------------------
__device__ double beta_cf(double x, double a, double b) {
  const double tiny = 1e-300, eps = 4e-16;
  double f = tiny, c = tiny, d = 0.0;
  for (int j = 0; j < 20000; ++j) {
    double num;
    if (j == 0) {
      num = 1.0;
    } else {
      const double m = (double)(j >> 1);
      if (j & 1)
        num = -(a + m) * (a + b + m) * x / ((a + 2.0 * m) * (a + 2.0 * m + 1.0));
      else
        num = m * (b - m) * x / ((a + 2.0 * m - 1.0) * (a + 2.0 * m));
    }
    d = 1.0 + num * d;
    if (fabs(d) < tiny) d = tiny;
    c = 1.0 + num / c;
    if (fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = c * d;
    f *= del;
    if (j > 0 && fabs(del - 1.0) < eps) break;
  }
  return f;
}

__device__ double ln_betai_cf(double x, double a, double b) {
  const double lbeta = lgamma(a) + lgamma(b) - lgamma(a + b);
  return a * log(x) + b * log1p(-x) - log(a) - lbeta + log(beta_cf(x, a, b));
}

__device__ double ln_p_two_sided(double t, double df) {
  t = fabs(t);
  if (isinf(t)) return -INFINITY;
  if (t == 0.0) return 0.0;
  const double a = 0.5 * df, b = 0.5;
  const double t2 = t * t;
  const double x = df / (df + t2);
  const double omx = t2 / (df + t2);
  if (x < (a + 1.0) / (a + b + 2.0)) return ln_betai_cf(x, a, b);
  return log1p(-exp(ln_betai_cf(omx, b, a)));
}

__device__ double ln_pdf_t(double t, double df) {
  return lgamma(0.5 * (df + 1.0)) - lgamma(0.5 * df) - 0.5 * log(df * M_PI) -
         0.5 * (df + 1.0) * log1p(t * t / df);
}

// -log10 p of |t| and its derivative in |t|, in FP64
__device__ void nlog10p_and_slope(double t, double df, double& f, double& fp) {
  const double lnp = ln_p_two_sided(t, df);
  f = -lnp / M_LN10;
  fp = 2.0 * exp(ln_pdf_t(t, df) - lnp) / M_LN10;
}

// the cubic Hermite interpolant of -log10 p on interval k (nodes k and k + 1,
// values and slopes), written as its power-series coefficients in the local
// variable s in [0, 1] so that the epilogue evaluates it with three FMAs
__global__ void table_kernel(float4* table, double df) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kTabIntervals) return;
  double f0, d0, f1, d1;
  nlog10p_and_slope((double)k / kTabPerUnit, df, f0, d0);
  nlog10p_and_slope((double)(k + 1) / kTabPerUnit, df, f1, d1);
  d0 /= kTabPerUnit;  // slopes per unit of s
  d1 /= kTabPerUnit;
  table[k] = make_float4((float)f0, (float)d0, (float)(3.0 * (f1 - f0) - 2.0 * d0 - d1),
                         (float)(2.0 * (f0 - f1) + d0 + d1));
}

// interval coefficients as a plain vector type (HIP's float4 class has no
// copy from an LDS reference); the wide kernel's epilogue reads a copy of the
// table in LDS
typedef float tab4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(3))) tab4* LdsTable;

// cubic Hermite interpolation of -log10 p at |t| <= kTMax (TabPtr: the global
// table or its LDS copy)
template <class TabPtr>
__device__ inline float table_nlog10p(TabPtr tab, float at) {
  const float x = at * (float)kTabPerUnit;
  int k = (int)x;
  k = k > kTabIntervals - 1 ? kTabIntervals - 1 : k;
  const float s = x - (float)k;
  const tab4 c = tab[k];
  return fmaf(fmaf(fmaf(c.w, s, c.z), s, c.y), s, c.x);
}

// ---------------------------------------------------------------------------
// covariate QR: Householder reflections on the (q x n_pad) column-major work
// copy X of [1 | C].  Each step is three launches: row-parallel partial dot
// products (kQrGrid workgroups, one contiguous row range each), one small
// workgroup that sums the partials in workgroup order and forms the
// reflection's coefficients, and a row-parallel update; so every pass over
// the samples is spread over the GPU.  On exit X holds the Householder
// vectors and Q (q x n_pad) the orthonormal basis.  Fixed grid and fixed
// summation order: the result is the same in every run.
// ---------------------------------------------------------------------------
constexpr int kQrThreads = 256;
constexpr int kQrCB = 4;  // columns reduced together

__global__ __launch_bounds__(kQrThreads) void qr_load_kernel(const double* __restrict__ C, int64_t ldc, int64_t n,
                                                             int64_t n_pad, int q, double* __restrict__ X,
                                                             int32_t* flags) {
  const int64_t total = n_pad * q;
  int bad = 0;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx / n_pad);
    const int64_t i = idx - (int64_t)k * n_pad;
    double v = 0.0;  // pad rows are zero
    if (i < n) {
      v = (k == 0) ? 1.0 : C[(int64_t)(k - 1) * ldc + i];
      if (!isfinite(v)) bad = 1;
    }
    X[idx] = v;
  }
  if (bad) flags[0] = 1;
}

// part[b][k] = sum over workgroup b's rows i >= i0 of v[i] * W[k][i], for
// k0 <= k < q (zero for a workgroup with no such rows)
__global__ __launch_bounds__(kQrThreads) void qr_dots_kernel(const double* __restrict__ v,
                                                             const double* __restrict__ W, int64_t n,
                                                             int64_t n_pad, int q, int k0, int64_t i0,
                                                             double* __restrict__ part) {
  __shared__ double sh[(kQrThreads / 64) * kQrCB];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  int64_t rb = (int64_t)blockIdx.x * per;
  const int64_t re = rb + per < n ? rb + per : n;
  rb = rb > i0 ? rb : i0;
  for (int c0 = k0; c0 < q; c0 += kQrCB) {
    double d[kQrCB];
#pragma unroll
    for (int t = 0; t < kQrCB; ++t) d[t] = 0.0;
    for (int64_t i = rb + threadIdx.x; i < re; i += kQrThreads) {
      const double vi = v[i];
#pragma unroll
      for (int t = 0; t < kQrCB; ++t) {
        const int64_t col = c0 + t < q ? c0 + t : q - 1;  // clamped: a valid address, value unused
        d[t] += vi * W[col * n_pad + i];
      }
    }
    block_sum_vec<kQrThreads, kQrCB>(d, sh);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int t = 0; t < kQrCB; ++t)
        if (c0 + t < q) part[(int64_t)blockIdx.x * kSlots + c0 + t] = d[t];
    }
  }
}

// step j's sums dv[k] (k >= j) from the partials, then the coefficients.
// forward: dv[j] = squares of x_j below row j, dv[k > j] = x_j . x_k below
// row j; the reflection maps x_j to alpha e_j (rdiag[j] = alpha), v_j = x_j
// with v_j[j] = x_j[j] - alpha, and fv[k] = 2 (v_j . x_k) / (v_j . v_j).
// backward (forming Q): dv[k] = v_j . Q_k from row j on, fv[k] = 2 dv[k] / vtv[j].
// (one workgroup of kQrThreads; the partials are staged in LDS with
// coalesced loads, then lane k sums column k's in workgroup order)
__global__ __launch_bounds__(kQrThreads) void qr_coef_kernel(double* X, int64_t n_pad, int q, int j, int forward,
                                                             const double* __restrict__ part, double* rdiag,
                                                             double* fv, double* vtv) {
  __shared__ double ps[kQrGrid * kSlots];
  __shared__ double dv[kSlots];
  for (int idx = threadIdx.x; idx < kQrGrid * kSlots; idx += kQrThreads) ps[idx] = part[idx];
  __syncthreads();
  const int k = threadIdx.x;
  if (k >= j && k < q) {
    double s = 0.0;
    for (int b = 0; b < kQrGrid; ++b) s += ps[b * kSlots + k];
    dv[k] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (forward) {
    double* xj = X + (int64_t)j * n_pad;
    const double xjj = xj[j];
    const double below = dv[j];
    const double nrm = sqrt(xjj * xjj + below);
    const double alpha = xjj > 0.0 ? -nrm : nrm;
    const double v0 = xjj - alpha;
    const double t = below + v0 * v0;
    xj[j] = v0;
    rdiag[j] = alpha;
    vtv[j] = t;
    for (int c = j + 1; c < q; ++c) fv[c] = t > 0.0 ? 2.0 * (dv[c] + v0 * X[(int64_t)c * n_pad + j]) / t : 0.0;
  } else {
    const double t = vtv[j];
    for (int c = j; c < q; ++c) fv[c] = t > 0.0 ? 2.0 * dv[c] / t : 0.0;
  }
}

// W[k][i] -= fv[k] * v[i] for rows i0 <= i < n and k0 <= k < q
__global__ __launch_bounds__(kQrThreads) void qr_reflect_kernel(const double* v, double* W, int64_t n, int64_t n_pad,
                                                                int q, int k0, int64_t i0,
                                                                const double* __restrict__ fv) {
  __shared__ double f_s[kSlots];
  if (threadIdx.x < kSlots) f_s[threadIdx.x] = (int)threadIdx.x >= k0 && (int)threadIdx.x < q ? fv[threadIdx.x] : 0.0;
  __syncthreads();
  for (int64_t i = i0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double vi = v[i];
    for (int k = k0; k < q; ++k) W[(int64_t)k * n_pad + i] -= f_s[k] * vi;
  }
}

// Q = [I_q; 0] before the reflections are applied from the last
__global__ void qr_qinit_kernel(double* Q, int64_t n_pad, int q) {
  const int64_t total = n_pad * q;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx / n_pad);
    Q[idx] = (idx - (int64_t)k * n_pad == k) ? 1.0 : 0.0;
  }
}

// rank check: every |R_jj| above 1e-10 max |R_ii|
__global__ void qr_rank_kernel(const double* rdiag, int q, int32_t* flags) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double mx = 0.0;
  for (int j = 0; j < q; ++j) mx = fmax(mx, fabs(rdiag[j]));
  int rd = 0;
  for (int j = 0; j < q; ++j)
    if (!(fabs(rdiag[j]) > 1e-10 * mx)) rd = 1;
  flags[1] = rd;
}


// operand blocks of the covariate columns used for Q^T g: slot k <- Q[:, k]
// for 1 <= k < q, slot 0 and slots >= q are zero.  FP32: one 32-column
// block.  The split forms take packed blocks (hl), one per 16 slots (one
// block when q <= 16, else two): slot k goes to block k / 16, its hi part in
// column k % 16 and its lo part in column k % 16 + 16 of the hi half, the lo
// half zero, so that one matrix-core pass forms both products.
__global__ void cov_operand_kernel(const double* __restrict__ Q, int64_t n, int64_t n_pad, int q, void* wop_fp32,
                                   void* hl_split, void* hl_split16) {
  const int n_chunks = (int)(n_pad / kChunk);
  const int64_t total = n_pad * kColBlock;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / kColBlock;
    const int k = (int)(idx % kColBlock);
    const double v = (k >= 1 && k < q && i < n) ? Q[(int64_t)k * n_pad + i] : 0.0;
    double st;
    store_operand(wop_fp32, kFP32, k, i, n_chunks, v, &st);
    if (k < hl_blocks(q) * kHLSlots) {
      const int64_t ch = 32 * (k / kHLSlots) + k % kHLSlots;  // hi column; lo column ch + 16
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        uint16_t* p = (uint16_t*)(f == 0 ? hl_split : hl_split16);
        uint32_t hb, lb;
        split_parts(f == 0 ? kSplit : kSplit16, v, &hb, &lb);
        p[operand_index_split(ch, i, n_chunks, 0)] = (uint16_t)hb;
        p[operand_index_split(ch + kHLSlots, i, n_chunks, 0)] = (uint16_t)lb;
        p[operand_index_split(ch, i, n_chunks, 1)] = 0;
        p[operand_index_split(ch + kHLSlots, i, n_chunks, 1)] = 0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// phenotype preparation (Eq. 1 + standardization): one workgroup per CPW
// columns, so that each element of Q read from L2 serves CPW columns; QS >= q
// slots of the projections are kept per column.  Every column's arithmetic
// and summation order is that of a workgroup running it alone.
// ---------------------------------------------------------------------------
constexpr int kPrepThreads = 256;

template <int QS, int CPW>
__global__ __launch_bounds__(kPrepThreads) void prep_kernel(const void* __restrict__ Y, int y_fp64, int64_t ldy,
                                                            int64_t n, int64_t n_pad, int64_t P,
                                                            const double* __restrict__ Q, int q, int prec,
                                                            void* yop, float* scale, float* invny, float* cw,
                                                            uint8_t* lscale, int32_t* flags) {
  static_assert(QS <= kSlots, "projection slots");
  constexpr int NV = CPW * (QS + 2);
  __shared__ double sh[(kPrepThreads / 64) * NV];
  __shared__ double qty_s[CPW][QS];
  const int tid = threadIdx.x;
  const int n_chunks = (int)(n_pad / kChunk);
  const int64_t p0 = (int64_t)blockIdx.x * CPW;
  // columns past P repeat the last one; nothing of theirs is stored
  int64_t pc[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) pc[c] = p0 + c < P ? p0 + c : P - 1;
  auto yval = [&](int c, int64_t i) -> double {
    return y_fp64 ? ((const double*)Y)[pc[c] * ldy + i] : (double)((const float*)Y)[pc[c] * ldy + i];
  };
  // slots k >= q hold zero: every slot is loaded (past q, column q - 1
  // again) and multiplied without a branch, which adds exact zeros only, so
  // the loads of a sample issue together
  auto load_q = [&](int64_t i, double* qv) {
#pragma unroll
    for (int k = 0; k < QS; ++k) {
      const double v = Q[(int64_t)(k < q ? k : q - 1) * n_pad + i];
      qv[k] = k < q ? v : 0.0;
    }
  };

  // pass 1: means (and finiteness)
  double mean[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) mean[c] = 0.0;
  int bad = 0;
  for (int64_t i = tid; i < n; i += kPrepThreads) {
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const double v = yval(c, i);
      if (!isfinite(v)) bad = 1;
      mean[c] += v;
    }
  }
  bad = __syncthreads_or(bad);
  if (bad) {
    if (tid == 0) atomicOr(flags, 1);
    return;
  }
  block_sum_vec<kPrepThreads, CPW>(mean, sh);
#pragma unroll
  for (int c = 0; c < CPW; ++c) mean[c] /= (double)n;

  // pass 2: Q^T y_c and ||y_c||^2 (slot QS)
  double acc[CPW][QS + 2];
#pragma unroll
  for (int c = 0; c < CPW; ++c)
#pragma unroll
    for (int k = 0; k < QS + 2; ++k) acc[c][k] = 0.0;
  for (int64_t i = tid; i < n; i += kPrepThreads) {
    double qv[QS];
    load_q(i, qv);
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const double yc = yval(c, i) - mean[c];
      acc[c][QS] += yc * yc;
#pragma unroll
      for (int k = 0; k < QS; ++k) acc[c][k] += qv[k] * yc;
    }
  }
  block_sum_vec<kPrepThreads, NV>(&acc[0][0], sh);
  double yc2[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    yc2[c] = acc[c][QS];
#pragma unroll
    for (int k = 0; k < QS; ++k)
      if (tid == k) qty_s[c][k] = acc[c][k];
  }
  __syncthreads();

  // y_res of column c at sample i, given Q's column i
  auto yres = [&](int c, int64_t i, const double* qv) {
    double v = yval(c, i) - mean[c];
#pragma unroll
    for (int k = 0; k < QS; ++k) v -= qv[k] * qty_s[c][k];
    return v;
  };

  // pass 3: ||y_res||^2
  double r2[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) r2[c] = 0.0;
  for (int64_t i = tid; i < n; i += kPrepThreads) {
    double qv[QS];
    load_q(i, qv);
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const double v = yres(c, i, qv);
      r2[c] += v * v;
    }
  }
  block_sum_vec<kPrepThreads, CPW>(r2, sh);
  double sp[CPW], inv[CPW];
  bool valid[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    sp[c] = sqrt(r2[c]);
    valid[c] = sp[c] > 1e-12 * sqrt(yc2[c]);
    inv[c] = valid[c] ? 1.0 / sp[c] : 0.0;
  }

  // pass 3b (FP8 lo form): each column's largest lo term sets its scale
  int lsh[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) lsh[c] = 0;
  if (prec == kSplit8) {
    double mx[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) mx[c] = 0.0;
    for (int64_t i = tid; i < n; i += kPrepThreads) {
      double qv[QS];
      load_q(i, qv);
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const double vs = yres(c, i, qv) * inv[c] * (double)kF16Scale;
        mx[c] = fmax(mx[c], fabs(vs - (double)f16_to_float(f16_bits_rn((float)vs))));
      }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      lsh[c] = lo_shift(block_max<kPrepThreads>(mx[c], sh));
      if (tid == 0 && p0 + c < P) lscale[p0 + c] = (uint8_t)(127 - lsh[c]);
    }
  }

  // pass 4: y~ = y_res / s_p into the operand; accumulate what the stored
  // (rounded) operand actually holds: Q^T y_op, sum (slot QS), norm^2 (QS + 1),
  // and (FP16 + FP8 form) the sum of the FP8 lo terms alone
#pragma unroll
  for (int c = 0; c < CPW; ++c)
#pragma unroll
    for (int k = 0; k < QS + 2; ++k) acc[c][k] = 0.0;
  double lsum[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) lsum[c] = 0.0;
  for (int64_t i = tid; i < n; i += kPrepThreads) {
    double qv[QS];
    load_q(i, qv);
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      if (p0 + c >= P) continue;
      double st, lo;
      store_operand(yop, prec, p0 + c, i, n_chunks, yres(c, i, qv) * inv[c], &st, lsh[c], &lo);
      lsum[c] += lo;
      acc[c][QS] += st;
      acc[c][QS + 1] += st * st;
#pragma unroll
      for (int k = 0; k < QS; ++k) acc[c][k] += qv[k] * st;
    }
  }
  block_sum_vec<kPrepThreads, NV>(&acc[0][0], sh);
  // FP16 + FP8 form with q <= 31: the last correction slot takes minus the
  // column's sum of lo terms (a plan whose markers centre their FP8 pass on
  // c8 = rint(c) puts c - c8 against it)
  const bool lo_slot = prec == kSplit8 && q <= kLoSlot;
  if (lo_slot) block_sum_vec<kPrepThreads, CPW>(lsum, sh);
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int64_t p = p0 + c;
    if (p >= P) break;
    if (tid == 0) {
      double proj = 0.0;
#pragma unroll
      for (int k = 0; k < QS; ++k)
        if (k < q) proj += acc[c][k] * acc[c][k];
      const double ny2 = acc[c][QS + 1] - proj;
      scale[p] = (float)sp[c];
      invny[p] = (valid[c] && ny2 > 0.0) ? (float)(1.0 / sqrt(ny2)) : __builtin_nanf("");
    }
    if (tid < kSlots) {
      float v = tid == 0 ? (float)(-acc[c][QS]) : 0.0f;
#pragma unroll
      for (int k = 1; k < QS; ++k)
        if (tid == k && k < q) v = (float)(-acc[c][k]);
      if (lo_slot && tid == kLoSlot) v = (float)(-lsum[c]);
      cw[p * kSlots + tid] = v;
    }
  }
}

// test hook: raw operand columns (no centring / scaling)
__global__ __launch_bounds__(kPrepThreads) void set_lscale_kernel(const float* __restrict__ V, int64_t ldv,
                                                                  int64_t n, uint8_t* lscale) {
  __shared__ double sh[kPrepThreads / 64];
  const int64_t p = blockIdx.x;
  double mx = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kPrepThreads) {
    const double vs = (double)V[p * ldv + i] * (double)kF16Scale;
    mx = fmax(mx, fabs(vs - (double)f16_to_float(f16_bits_rn((float)vs))));
  }
  mx = block_max<kPrepThreads>(mx, sh);
  if (threadIdx.x == 0) lscale[p] = (uint8_t)(127 - lo_shift(mx));
}

__global__ void set_operand_kernel(const float* __restrict__ V, int64_t ldv, int64_t n, int64_t n_pad,
                                   int64_t P, int prec, void* yop, const uint8_t* lscale) {
  const int n_chunks = (int)(n_pad / kChunk);
  const int64_t total = n_pad * P;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = idx / n_pad;
    const int64_t i = idx % n_pad;
    const double v = i < n ? (double)V[p * ldv + i] : 0.0;
    double st;
    store_operand(yop, prec, p, i, n_chunks, v, &st, prec == kSplit8 ? 127 - (int)lscale[p] : 0);
  }
}

// 0xff in every byte of d that is 0xff (the 8-bit dosage missing code), 0
// elsewhere: bit 7 of ((d & 0x7f) + 1) & d is set exactly for 0xff bytes
// (no carry leaves a byte); 2t - (t >> 7) spreads each marked bit over its byte
__device__ __forceinline__ uint32_t ff_bytes(uint32_t d) {
  const uint32_t t = ((d & 0x7f7f7f7fu) + 0x01010101u) & d & 0x80808080u;
  return (t << 1) - (t >> 7);
}

// Decode table of a marker of 8-bit dosages (q = 0..254, 255 missing),
// operand value q - c with an integer c = rint(mu), missing -> mu - c:
//   x = FP16 pair of -(1024 + c)    (1024 + q is built exactly by byte insertion)
//   y = FP16 pair of mu - c
//   z = FP32 bits of c, w = FP32 bits of mu - c   (the FP32 form)
__device__ void stats_dosage8(const StatsArgs& a, int64_t m, int lane) {
  const uint32_t* row = (const uint32_t*)(a.geno + (a.m0 + m) * a.row_bytes);
  const int64_t nd = (a.n + 3) / 4;
  uint32_t nmiss = 0;
  uint64_t S1 = 0, S2 = 0;
  for (int64_t d = lane; d < nd; d += 64) {
    const uint32_t w = row[d];
    const int64_t nv = a.n - 4 * d;
    const uint32_t vm = nv >= 4 ? 0xffffffffu : ((1u << (8 * nv)) - 1u);
    const uint32_t miss = ff_bytes(w) & vm;
    const uint32_t obs = w & ~miss & vm;
    nmiss += __popc(miss) >> 3;
    S1 += __builtin_amdgcn_udot4(obs, 0x01010101u, 0u, false);
    S2 += __builtin_amdgcn_udot4(obs, obs, 0u, false);
  }
  uint64_t M = nmiss;
  for (int o = 32; o > 0; o >>= 1) {
    M += __shfl_xor(M, o);
    S1 += __shfl_xor(S1, o);
    S2 += __shfl_xor(S2, o);
  }
  if (lane != 0) return;
  const int64_t n_obs = a.n - (int64_t)M;
  const int64_t sg = (int64_t)S1, sg2 = (int64_t)S2;
  const __int128 num128 = (__int128)n_obs * sg2 - (__int128)sg * sg;  // n_obs * sum (q - mu)^2
  const bool ok = n_obs > 0 && num128 != 0;
  MarkerStat st;
  st.flags = ok ? 0 : 1;
  const double mu = n_obs > 0 ? (double)sg / (double)n_obs : 0.0;
  const double c = ok ? rint(mu) : 0.0;
  st.mu = mu;
  st.shift = c;
  st.gscale = 1.0f;
  st.dlo = 0.0f;
  st.gc2 = n_obs > 0 ? (double)num128 / (double)n_obs : 0.0;
  st.dmu = (float)(mu - c);
  const uint32_t nc = f16_bits_rn((float)(-1024.0 - c));
  const uint32_t dm = f16_bits_rn((float)(mu - c));
  a.mlut[m] = make_uint4(nc | (nc << 16), dm | (dm << 16), __float_as_uint((float)c), __float_as_uint((float)(mu - c)));
  a.mstat[m] = st;
}

// ---------------------------------------------------------------------------
// per-marker statistics (one wave per marker)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void stats_kernel(StatsArgs a) {
  if (blockIdx.x == 0 && a.redo_count)  // the FP64 list of this block starts empty
    for (int j = threadIdx.x; j < a.n_panels; j += blockDim.x) a.redo_count[j] = 0u;
  const int lane = threadIdx.x & 63;
  const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= a.nm) return;
  if (a.code == 2) {
    stats_dosage8(a, m, lane);
    return;
  }
  // 16 bytes (64 samples) per lane and load; rows are 16-byte aligned and
  // hold at least ceil(n / 64) such pieces
  const uint4* row = (const uint4*)(a.geno + (a.m0 + m) * a.row_bytes);
  const int64_t n16 = (a.n + 63) / 64;
  // three popcounts per word: codes with the low bit set (pl), with the high
  // bit set (ph), with both (pb); codes past n are masked to 00, which counts
  // in none of them.  The tallies follow from these per coding below.
  int pl = 0, ph = 0, pb = 0;
  for (int64_t d4 = lane; d4 < n16; d4 += 64) {
    const uint4 w4 = row[d4];
    const uint32_t ws[4] = {w4.x, w4.y, w4.z, w4.w};
    const bool full = 64 * (d4 + 1) <= a.n;  // all 64 samples of this piece are real
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t w = ws[q];
      if (!full) {
        const int64_t nv = a.n - 16 * (4 * d4 + q);  // samples in this word
        w &= nv >= 16 ? 0xffffffffu : (nv <= 0 ? 0u : ((1u << (2 * nv)) - 1u));
      }
      const uint32_t lo = w & 0x55555555u;
      const uint32_t hi = (w >> 1) & 0x55555555u;
      pl += __popc(lo);
      ph += __popc(hi);
      pb += __popc(lo & hi);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    pl += __shfl_xor(pl, o);
    ph += __shfl_xor(ph, o);
    pb += __shfl_xor(pb, o);
  }
  int nmiss, c1, c2;
  if (a.code == 0) {  // dosage: 0, 1, 2, 3 = missing (low bit only: 1; high bit only: 2)
    nmiss = pb;
    c1 = pl - pb;
    c2 = ph - pb;
  } else {  // PLINK .bed: 00 -> 0, 01 -> missing, 10 -> 1, 11 -> 2
    c2 = pb;
    nmiss = pl - pb;
    c1 = ph - pb;
  }
  const int64_t n_obs = a.n - nmiss;
  const int64_t sg = c1 + 2 * (int64_t)c2;
  const int64_t sg2 = c1 + 4 * (int64_t)c2;
  const int64_t num = n_obs * sg2 - sg * sg;  // n_obs * sum (g - mu)^2
  const bool ok = n_obs > 0 && num != 0;
  const double mu = n_obs > 0 ? (double)sg / (double)n_obs : 0.0;
  // operand value of a call g: gs (g - c); of a missing call: gs (mu - c)
  // rounded to the operand type.  FP16 forms: gs = 1, c on the 1/512 grid
  // (g - c exact in 11 bits, missing value to 2^-21).  FP32: gs = 1, c on
  // the 1/64 grid.  BF16 (8 significant bits): gs = K / 128 and c = U / K
  // with integers K >= 1 and U = rint(K mu) such that the calls' values
  // (-U, K - U, 2K - U) / 128 have magnitude <= 2, hence are exact; of those
  // K, the one whose missing value (K mu - U) / 128 rounds to BF16 with the
  // smallest error per genotype unit (ties: the larger K).  The error is
  // about 2^-9 |mu - U / K|: at most about 2^-18 (mu within 1/512 of a
  // simple fraction such as 1/2 or 1), typically below 2^-24, against up
  // to 2^-16 for the nearest multiple of 1/64.  The 256 candidates are
  // spread over the wave's lanes.
  // A marker without missing calls carries no missing value: every form
  // takes gs = 1 and the integer c = rint(mu), so that its operand holds
  // small integers, whose few changing bits cost the matrix cores less
  // power than fractional values (the contraction's clock is power-bound).
  const bool whole = ok && nmiss == 0;
  double c = 0.0, gs = 1.0, vmiss = mu, vg[3] = {0.0, 1.0, 2.0};  // degenerate: not re-centred
  if (whole) {
    c = rint(mu);
    vmiss = mu - c;
    for (int g = 0; g < 3; ++g) vg[g] = (double)g - c;
  } else if (ok && a.prec == kSplit) {
    double best = INFINITY;
    int bk = 0;
    for (int K = 256 - lane; K >= 1; K -= 64) {
      const double km = (double)K * mu;
      const double U = rint(km);
      if (U > 256.0 || 2.0 * K - U > 256.0) continue;
      const double v = (km - U) * (1.0 / 128.0);
      const double err = fabs((double)bf16_to_float(bf16_bits_rne((float)v)) - v) / (double)K;
      if (err < best) {  // K descends: ties keep the larger K
        best = err;
        bk = K;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o);
      const int ok2 = __shfl_xor(bk, o);
      if (ob < best || (ob == best && ok2 > bk)) {
        best = ob;
        bk = ok2;
      }
    }
    const double Kd = (double)bk, U = rint(Kd * mu);
    gs = Kd / 128.0;
    c = U / Kd;
    vmiss = (Kd * mu - U) * (1.0 / 128.0);
    for (int g = 0; g < 3; ++g) vg[g] = ((double)g * Kd - U) * (1.0 / 128.0);
  } else if (ok) {
    const double grid = f16_scaled(a.prec) ? 512.0 : 64.0;
    c = rint(grid * mu) / grid;
    vmiss = mu - c;
    for (int g = 0; g < 3; ++g) vg[g] = (double)g - c;
  }
  if (lane != 0) return;
  MarkerStat st;
  st.flags = ok ? 0 : 1;
  st.mu = mu;
  st.shift = c;
  st.gscale = (float)gs;
  // the FP8 lo pass of the FP16 + FP8 form may centre on the integer c8 =
  // rint(c): its calls' values g - c8 are then exact in e4m3 and, being
  // small integers, cheaper in matrix-core power; a missing call's mu - c8
  // rounds to e4m3, an error that the lo term of y~ (about 2^-12 of y~)
  // keeps below about 2^-17 of a genotype unit.  The shift (c - c8) times
  // the column's sum of lo terms leaves through the last correction slot.
  const double c8 = (a.prec == kSplit8 && a.lo_int) ? rint(c) : c;
  st.dlo = (float)(c - c8);  // a multiple of 1/512 in [-1/2, 1/2]: exact
  st.gc2 = n_obs > 0 ? (double)num / (double)n_obs : 0.0;
  st.dmu = (float)vmiss;
  // operand value of each 2-bit code, in the coding scheme's code order
  double val[4];
  if (a.code == 0) {
    val[0] = vg[0]; val[1] = vg[1]; val[2] = vg[2]; val[3] = vmiss;
  } else {
    val[0] = vg[0]; val[1] = vmiss; val[2] = vg[1]; val[3] = vg[2];
  }
  uint4 lut;
  if (a.prec != kFP32) {
    uint32_t lo8 = 0, hi8 = 0, f8 = 0;
    for (int k = 0; k < 4; ++k) {
      const uint32_t b = a.prec == kSplit ? bf16_bits_rne((float)val[k]) : f16_bits_rn((float)val[k]);
      lo8 |= (b & 0xffu) << (8 * k);
      hi8 |= (b >> 8) << (8 * k);
      f8 |= e4m3_bits_rne(val[k] + (c - c8)) << (8 * k);  // g - c8, or mu - c8, rounded to e4m3
    }
    lut = make_uint4(lo8, hi8, f8, 0u);
  } else {
    lut = make_uint4(__float_as_uint((float)val[0]), __float_as_uint((float)val[1]),
                     __float_as_uint((float)val[2]), __float_as_uint((float)val[3]));
  }
  a.mlut[m] = lut;
  a.mstat[m] = st;
}

__global__ void debug_stats_kernel(const MarkerStat* ms, int64_t nm, double* shift, double* mean, double* scale) {
  const int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (m >= nm) return;
  if (shift) shift[m] = ms[m].shift;
  if (mean) mean[m] = ms[m].mu;
  if (scale) scale[m] = (double)ms[m].gscale;
}

// ---------------------------------------------------------------------------
// ||g_res||^2 per (marker, panel) from Q^T g; slot 0 <- mu - c
// ---------------------------------------------------------------------------
// The slots and the contraction are in operand units (gs per genotype unit),
// so r takes 1 / (gs ||g_res||) and beta, SE take 1 / ||g_res||.  Markers
// whose ||g_res||^2 here is below kRedoTol ||g_c||^2 get NaN (the main
// kernel then writes NaN rows and no reduced outputs) and go to the FP64
// list of their panel.
__global__ void finalize_kernel(const MarkerStat* __restrict__ ms, float* __restrict__ wws,
                                float2* __restrict__ invh, int64_t nm, int n_panels, float wscale, int lo_slot,
                                RedoDev redo) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= nm * n_panels) return;
  const int64_t m = idx / n_panels;
  const MarkerStat st = ms[m];
  float* ws = wws + idx * kSlots;
  const double igs = 1.0 / (double)st.gscale;  // exact: gs is K / 128 or 1
  double h2 = st.gc2;
  for (int k = 1; k < kSlots; ++k) {
    const float wf = ws[k] * wscale;  // undo the operand scale of the Q columns
    ws[k] = wf;
    const double w = (double)wf * igs;
    h2 -= w * w;
  }
  const bool ok = st.flags == 0 && h2 > kRedoTol * st.gc2;
  if (st.flags == 0 && !ok) {
    const int j = (int)(idx - m * n_panels);
    const uint32_t k = atomicAdd(redo.count + j, 1u);
    redo.entries[j * redo.stride + k] = (int32_t)m;  // at most one entry per (marker, panel): never full
  }
  const double ih = 1.0 / sqrt(h2);
  invh[idx] = ok ? make_float2((float)(ih * igs), (float)ih) : make_float2(__builtin_nanf(""), __builtin_nanf(""));
  ws[0] = st.dmu;
  if (lo_slot) ws[kLoSlot] = st.dlo;  // the slot's Q^T g is 0 (q <= 31 in every panel of the plan)
}

// ---------------------------------------------------------------------------
// per-call output table, tail list
// ---------------------------------------------------------------------------
__global__ void bind_kernel(BindArgs a) {
  const int i = threadIdx.x;
  if (i < a.count) a.dst[a.first + i] = a.outs[i];
}

__global__ void tail_reset_kernel(TailDev t) {
  if (threadIdx.x == 0 && blockIdx.x == 0) t.count[0] = 0ull;
}

// per-column best test: max -log10 p in the high word, the complement of
// the marker index in the low word (so equal maxima keep the first marker)
__device__ inline unsigned long long best_pack(float nl, int64_t marker) {
  return ((unsigned long long)__float_as_uint(nl > 0.f ? nl : 0.f) << 32) |
         (unsigned long long)(0xffffffffu - (uint32_t)marker);
}

// per-column top-k lists: words (bits of |t|) << 32 | (0xffffffff - marker),
// kept in decreasing order; 0 is an empty slot
__device__ inline unsigned long long topk_pack(float at, int64_t marker) {
  return ((unsigned long long)__float_as_uint(at) << 32) | (unsigned long long)(0xffffffffu - (uint32_t)marker);
}

// Inserts w into the decreasing list s[0..k) that other lanes and workgroups
// update at the same time.  Every slot only grows (atomicMax), and a value
// reaches slot i + 1 only by being pushed out of slot i or by starting there
// after slot i was seen >= it, so s[i] >= s[i + 1] holds at every moment.
// The search for the first slot below w on plain (possibly stale) reads is
// therefore safe: every slot it skips is >= w for good.  From there each
// atomicMax keeps the larger of (slot, w) and w carries the smaller one on,
// until it lands in an empty slot or drops off the end, below the k-th value.
__device__ inline void topk_insert(unsigned long long* s, int k, unsigned long long w) {
  int lo = 0, hi = k;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (__atomic_load_n(s + mid, __ATOMIC_RELAXED) >= w)
      lo = mid + 1;
    else
      hi = mid;
  }
  for (int i = lo; i < k && w != 0ull; ++i) {
    const unsigned long long old = atomicMax(s + i, w);
    w = old < w ? old : w;
  }
}

__device__ inline void append_hit(const HitDev& hits, int64_t marker, int j, int64_t p, float nl, float r) {
  const unsigned long long idx = atomicAdd(hits.count, 1ull);
  if (idx < (unsigned long long)hits.capacity) {
    Hit h;
    h.marker = marker;
    h.panel = j;
    h.pheno = (int32_t)p;
    h.nl = nl;
    h.r = r;
    hits.entries[idx] = h;
  }
}

__global__ void tail_kernel(TailDev t, const PanelDev* __restrict__ panels, const OutDev* __restrict__ outs,
                            HitDev hits, int64_t m_begin) {
  const unsigned long long cnt = t.count[0];
  const int64_t n = cnt < (unsigned long long)t.capacity ? (int64_t)cnt : t.capacity;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const TailEntry e = t.entries[idx];
    const double df = (double)panels[e.panel].df;
    const double r = (double)e.r;
    const double tt = r * sqrt(df / ((1.0 - r) * (1.0 + r)));
    const double lnp = ln_p_two_sided(tt, df);
    const float nl = (float)(-lnp / M_LN10);
    const OutDev o = outs[e.panel];
    if (o.nl) o.nl[e.row * o.ld + e.col] = nl;
    if (o.best) atomicMax(o.best + e.col, best_pack(nl, m_begin + e.row));  // replaces the lower bound
    if (hits.entries && nl >= hits.threshold) append_hit(hits, m_begin + e.row, e.panel, e.col, nl, e.r);
  }
}

// ---------------------------------------------------------------------------
// FP64 path of covariate-collinear markers (the ones finalize_kernel lists):
// each listed marker is mean-imputed and residualized explicitly against its
// panel's FP64 Q, g_res = g_imp - Q (Q^T g_imp), then contracted in FP64 with
// the stored panel operand, so that r = g_res^T y_op / (||g_res|| ||(I -
// QQ^T) y_op||) carries no cancellation; t, beta, SE as in the main epilogue
// (Eq. 3), -log10 p in FP64 for every test, and the reduced outputs.  A
// marker with ||g_res||^2 <= kCollinearTol ||g_c||^2 gives NaN rows.  One
// work item: up to kRedoGroup listed markers of one panel x kRedoCols of its
// columns (one per thread), walked by a persistent grid; the work list comes
// from the per-panel counts, so a block without listed markers costs one
// short launch.
// ---------------------------------------------------------------------------
constexpr int kRedoThreads = kRedoCols;
static_assert(kRedoGroup % (kRedoThreads / 64) == 0 && kRedoGroup * kChunk == 4 * kRedoThreads, "redo shape");

// the operand value stored for (column, sample), in the units the main kernel
// contracts (2^12 y~ for the FP16 forms), i.e. what prep_kernel accumulated
// into the column's norm and projections
__device__ inline double load_operand(const void* op, int prec, int64_t col, int64_t i, int n_chunks, int lsh) {
  if (prec == kSplit8) {
    const uint32_t hb = ((const uint16_t*)op)[operand_index_split(col, i, n_chunks, 0, kBlockBytes8 / 2)];
    const uint32_t qb = ((const uint8_t*)op)[operand_index_lo8(col, i, n_chunks)];
    return (double)f16_to_float(hb) + ldexp(e4m3_value(qb), -lsh);
  }
  if (prec == kSplit16 || prec == kSplit) {
    const uint16_t* p = (const uint16_t*)op;
    const uint32_t hb = p[operand_index_split(col, i, n_chunks, 0)];
    const uint32_t lb = p[operand_index_split(col, i, n_chunks, 1)];
    return prec == kSplit16 ? (double)f16_to_float(hb) + (double)f16_to_float(lb)
                            : (double)bf16_to_float(hb) + (double)bf16_to_float(lb);
  }
  return (double)((const float*)op)[operand_index_fp32(col, i, n_chunks)];
}

// sample i of a genotype row in genotype units (8-bit dosages: q), NaN if missing
__device__ inline double geno_value(const uint8_t* row, int code, int64_t i) {
  if (code == 2) {  // 8-bit dosages
    const uint32_t q = row[i];
    return q == 255u ? __builtin_nan("") : (double)q;
  }
  const uint32_t v = (row[i >> 2] >> (2 * (i & 3))) & 3u;
  if (code == 0) return v == 3u ? __builtin_nan("") : (double)v;
  return v == 1u ? __builtin_nan("") : (v == 0u ? 0.0 : (double)(v - 1u));  // PLINK .bed order
}

__global__ __launch_bounds__(kRedoThreads) void redo_kernel(RedoArgs a) {
  constexpr int NW = kRedoThreads / 64;
  constexpr int PPT = kRedoGroup / NW;  // (marker, sample) pairs per thread in a chunk
  __shared__ double w_s[kRedoGroup][kSlots];
  __shared__ double gr_s[kRedoGroup][kChunk];
  __shared__ double h2_s[kRedoGroup];
  __shared__ double sh[NW * kSlots];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int64_t total = 0;
  for (int j = 0; j < a.n_panels; ++j)
    total += (int64_t)((a.redo.count[j] + kRedoGroup - 1) / kRedoGroup) * a.max_chunks;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    int64_t rem = w;
    int j = 0;
    uint32_t cnt = 0;
    for (; j < a.n_panels; ++j) {
      cnt = a.redo.count[j];
      const int64_t items = (int64_t)((cnt + kRedoGroup - 1) / kRedoGroup) * a.max_chunks;
      if (rem < items) break;
      rem -= items;
    }
    const int gi = (int)(rem / a.max_chunks);
    const int cc = (int)(rem - (int64_t)gi * a.max_chunks);
    const PanelDev pd = a.panels[j];
    if ((int64_t)cc * kRedoCols >= pd.n_pheno) continue;  // uniform over the workgroup
    const int ng = min(kRedoGroup, (int)cnt - gi * kRedoGroup);
    const int32_t* ent = a.redo.entries + j * a.redo.stride + (int64_t)gi * kRedoGroup;
    const int q = pd.q;
    // w = Q^T g_imp of each listed marker
    for (int e = 0; e < ng; ++e) {
      const int64_t m = ent[e];
      const double mu = a.mstat[m].mu;
      const uint8_t* row = a.geno + (a.m0 + m) * a.row_bytes;
      double acc[kSlots];
#pragma unroll
      for (int k = 0; k < kSlots; ++k) acc[k] = 0.0;
      for (int64_t i = tid; i < a.n; i += kRedoThreads) {
        double g = geno_value(row, a.code, i);
        if (g != g) g = mu;
#pragma unroll
        for (int k = 0; k < kSlots; ++k)
          if (k < q) acc[k] += pd.Q[(int64_t)k * a.n_pad + i] * g;
      }
      block_sum_vec<kRedoThreads, kSlots>(acc, sh);
#pragma unroll
      for (int k = 0; k < kSlots; ++k)
        if (tid == k) w_s[e][k] = acc[k];
    }
    // chunks of 64 samples: residualized genotypes into LDS, then each thread
    // contracts them with its column of the operand
    const int64_t p = (int64_t)cc * kRedoCols + tid;
    const bool colok = p < pd.n_pheno;
    const int lsh = (a.prec == kSplit8 && colok) ? 127 - (int)pd.lscale[p] : 0;
    double S[kRedoGroup], h2r[PPT];
#pragma unroll
    for (int e = 0; e < kRedoGroup; ++e) S[e] = 0.0;
#pragma unroll
    for (int r = 0; r < PPT; ++r) h2r[r] = 0.0;
    for (int ch = 0; ch < a.n_chunks; ++ch) {
      __syncthreads();  // w_s written; the previous chunk's gr_s read
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        const int e = wave + NW * r;
        const int64_t i = (int64_t)ch * kChunk + lane;
        double v = 0.0;
        if (e < ng && i < a.n) {
          const int64_t m = ent[e];
          double g = geno_value(a.geno + (a.m0 + m) * a.row_bytes, a.code, i);
          if (g != g) g = a.mstat[m].mu;
          v = g;
          for (int k = 0; k < q; ++k) v -= pd.Q[(int64_t)k * a.n_pad + i] * w_s[e][k];
          h2r[r] += v * v;
        }
        gr_s[e][lane] = v;
      }
      __syncthreads();
      if (colok) {
        const int ns = (int)min((int64_t)kChunk, a.n - (int64_t)ch * kChunk);
        for (int s = 0; s < ns; ++s) {
          const double y = load_operand(pd.yop, a.prec, p, (int64_t)ch * kChunk + s, a.n_chunks, lsh);
#pragma unroll
          for (int e = 0; e < kRedoGroup; ++e) S[e] += gr_s[e][s] * y;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      double v = h2r[r];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0) h2_s[wave + NW * r] = v;
    }
    __syncthreads();
    if (colok) {
      const double invny = (double)pd.invny[p];
      const double sp = (double)pd.scale[p] * (double)a.gunit;
      const double df = (double)pd.df;
      const OutDev od = a.outs[j];
#pragma unroll
      for (int e = 0; e < kRedoGroup; ++e) {
        if (e >= ng) break;
        const int64_t m = ent[e];
        const int64_t row = a.out_row0 + m;
        const double h2 = h2_s[e];
        const bool ok = h2 > kCollinearTol * a.mstat[m].gc2 && invny == invny;
        double r = __builtin_nan(""), t = r, beta = r, se = r, nl = r;
        if (ok) {
          const double ih = 1.0 / sqrt(h2);
          r = S[e] * invny * ih;
          r = r > 1.0 ? 1.0 : (r < -1.0 ? -1.0 : r);
          const double omr2 = (1.0 - r) * (1.0 + r);
          t = omr2 > 0.0 ? r * sqrt(df / omr2) : (r > 0.0 ? INFINITY : -INFINITY);
          beta = r * sp * ih;
          se = sp * ih * sqrt(omr2 / df);
          nl = -ln_p_two_sided(t, df) / M_LN10;
        }
        const int64_t o = row * od.ld + p;
        if (od.r) od.r[o] = (float)r;
        if (od.beta) od.beta[o] = (float)beta;
        if (od.se) od.se[o] = (float)se;
        if (od.t) od.t[o] = (float)t;
        if (od.nl) od.nl[o] = (float)nl;
        if (ok && od.best) atomicMax(od.best + p, best_pack((float)nl, a.m_begin + row));
        if (ok && od.topk) topk_insert(od.topk + p * od.topk_k, od.topk_k, topk_pack((float)fabs(t), a.m_begin + row));
        if (ok && a.hits.entries && (float)nl >= a.hits.threshold)
          append_hit(a.hits, a.m_begin + row, j, p, (float)nl, (float)r);
      }
    }
    __syncthreads();  // h2_s and w_s are rewritten by the next work item
  }
}

// Tile order of the persistent kernels: super-tiles of kGroupM marker tiles
// x kGroupC column tiles, walked column group by column group, marker group
// by marker group; within a super-tile, column tile fastest.  The 32
// workgroups an XCD runs at once (wide kernel) then work on about one
// super-tile, so a genotype chunk is fetched once for kGroupC workgroups and
// an operand chunk once for kGroupM (column-tile-major order fetches the
// genotypes once per column tile).  w in [0, n_mtiles * n_ctiles) maps one
// to one; edge groups are ragged.
constexpr int kGroupM = 8, kGroupC = 4;
__device__ __forceinline__ void grouped_tile(int64_t w, int nm, int nc, int& mtile, int& ctile) {
  const int64_t full = (int64_t)nm * kGroupC;  // tiles of a full column group
  const int cg = (int)(w / full);
  const int64_t u = w - (int64_t)cg * full;
  const int c = nc - cg * kGroupC < kGroupC ? nc - cg * kGroupC : kGroupC;
  const int64_t sg = (int64_t)kGroupM * c;  // tiles of a full marker group in this column group
  const int mg = (int)(u / sg);
  const int r = (int)(u - (int64_t)mg * sg);
  const int mi = r / c;
  mtile = mg * kGroupM + mi;
  ctile = cg * kGroupC + (r - mi * c);
}

// ---------------------------------------------------------------------------
// the contraction (Eq. 2) with the fused epilogue
//
// Workgroup tile: TM = NW * WMF * 32 markers x TP = WN * 32 columns; every
// wave owns WMF 32-row fragments across all WN column blocks.  K loop over
// 64-sample chunks: the column tile's operand chunk is double-buffered in
// LDS; each wave reads its markers' packed codes straight from global memory
// and decodes them in registers with v_perm_b32 and the per-marker table.
// Persistent: the grid is resident and walks the (marker tile, column tile)
// list; the list is cut into 8 contiguous ranges, one per XCD (workgroups
// are dispatched round-robin to XCDs), so that the workgroups of an XCD
// share column tiles in their L2.
// ---------------------------------------------------------------------------
template <int NW>
struct GWords {
  typedef uint32_t type __attribute__((ext_vector_type(NW)));
};
template <>
struct GWords<1> {
  typedef uint32_t type;
};
// load through a global-address-space pointer (global_load_*, not flat_load_*)
template <class T>
__device__ __forceinline__ T gload(const void* p) {
  static_assert(sizeof(T) % 4 == 0, "gload of whole words only");
  typedef typename GWords<sizeof(T) / 4>::type V;
  const V v = *(const __attribute__((address_space(1))) V*)p;
  return __builtin_bit_cast(T, v);
}
template <class T>
__device__ __forceinline__ void gstore(void* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
// a store no kernel of the scan reads back (the dense outputs): marked
// non-temporal, so the written lines do not displace operand and genotype
// lines that later tiles fetch through L2
template <class T>
__device__ __forceinline__ void gstore_nt(void* p, T v) {
  __builtin_nontemporal_store(v, (__attribute__((address_space(1))) T*)p);
}

// one 32x32x16 matrix-core step on 16-bit operands given as raw bits
template <int PREC>
__device__ __forceinline__ f32x16 mfma16(const u32x4& a, const u32x4& b, const f32x16& c) {
  if constexpr (f16_scaled(PREC)) {
    typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                  0, 0, 0);
  }
}

// the rare part of a test's epilogue: |t| > 40 goes to the FP64 tail list
// (its -log10 p written as +inf until the tail kernel replaces it; with the
// list full, the table's value at 40 stands as a lower bound and the call
// reports the overflow), and a test at or above the hit threshold is
// appended to the hit list (for tail entries the tail kernel decides).
template <class TabPtr>
__device__ __forceinline__ void epilogue_rare(bool to_tail, float nl, float at, float r, TabPtr tab, float* nl_out,
                                           int64_t row, int j, int64_t p, const TailDev& tail, const HitDev& hits,
                                           int64_t marker) {
  if (to_tail) {
    const unsigned long long idx = atomicAdd(tail.count, 1ull);
    if (idx < (unsigned long long)tail.capacity) {
      TailEntry e;
      e.row = row;
      e.panel = j;
      e.col = (int32_t)p;
      e.r = r;
      e.pad = 0;
      tail.entries[idx] = e;
      if (nl_out) gstore(nl_out, INFINITY);
      return;
    }
    nl = table_nlog10p(tab, kTMax);
    if (nl_out) gstore(nl_out, nl);
  }
  if (hits.entries && at >= hits.t_floor && nl >= hits.threshold) append_hit(hits, marker, j, p, nl, r);
}

// finish one 32-column block of a wave's staged accumulators (stage holds
// rows 0 .. 32*WMF-1 of the wave's fragments, 32 columns each): lanes run
// along columns, two rows at a time; the per-column best over the rows is
// reduced in registers and merged with one atomic per column.
// invny and sp are this lane's column values (sp already per genotype unit).
// IhPtr: GlobalRows reads each row's 1/||g_res|| from global memory; an LDS
// pointer gives the wave's rows, copied there ahead of the output stores
// (on this chip a load issued after stores waits for them to complete, so
// loads inside the row loop would serialise behind the previous row's stores).
struct GlobalRows {};
__device__ __forceinline__ float* at_byte(float* base, uint32_t ob) { return (float*)((char*)base + ob); }
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(3))) f32x2* LdsRows;

template <int WMF, class TabPtr, class IhPtr>
__device__ __forceinline__ void finish_block(const float* stage, const GemmArgs& a, const ColBlock& blk,
                                             int64_t rowbase, int h, int r32, TabPtr tab, IhPtr ih, float invny,
                                             float sp) {
  if constexpr (!std::is_same<IhPtr, GlobalRows>::value) {
    // the lane's place from a fresh v_mbcnt: a lane index kept in a register
    // across the whole kernel gets spilled, and its reload just before the row
    // loop makes the compiler wait in every iteration for the earlier stores
    int lane;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(lane));
    h = lane >> 5;
    r32 = lane & 31;
  }
  static_assert(WMF <= 4, "rows of a block within 32-bit store offsets");
  const int j = blk.panel;
  const PanelDev pd = a.panels[j];
  const OutDev od = a.outs[j];
  const int64_t p = blk.col0 + r32;
  const bool colok = r32 < blk.ncol;
  // dense outputs rebased at (first row, first column) of the block: with
  // ld <= 2^22 and at most 128 rows every store is within 2^31 bytes of it
  // (held in scalar registers, so that a store is scalar base + vector offset)
  OutDev odb = od;
  {
    const int64_t base = (a.out_row0 + rowbase) * od.ld + blk.col0;
    auto rebase = [base](float* q) {
      const uint64_t v = q ? (uint64_t)(q + base) : 0;
      const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
      const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
      return (float*)(((uint64_t)hi << 32) | lo);
    };
    odb.r = rebase(od.r);
    odb.beta = rebase(od.beta);
    odb.se = rebase(od.se);
    odb.t = rebase(od.t);
    odb.nl = rebase(od.nl);
  }
  // top-k of this lane's column: the list and its current last word (rows
  // whose word is not above it cannot enter)
  const bool tk_on = od.topk != nullptr;  // uniform: one panel per column block
  unsigned long long* tkp = (tk_on && colok) ? od.topk + p * od.topk_k : nullptr;
  unsigned long long tk_last = tkp ? __atomic_load_n(tkp + od.topk_k - 1, __ATOMIC_RELAXED) : ~0ull;
  if constexpr (!std::is_same<IhPtr, GlobalRows>::value) {
    // the loads above (vector loads: the kernel writes global memory, so
    // they cannot go through the scalar cache) are waited for once here;
    // waited for at their first use they would put a full wait for the
    // previous rows' stores into every iteration
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt and lgkmcnt unconstrained
  }
  float bv = -1.0f;  // largest |t| of this lane's rows (-log10 p is increasing in |t| at fixed df)
  int64_t bm = 0;
  // -log10 p is needed for the dense output, for hit candidates, and (in
  // FP64, from the tail kernel) for |t| > 40 whenever any reduced output or
  // the dense output asks for it
  const bool need_p = od.nl || od.best || a.hits.entries;
  const bool need_tab = od.nl || a.hits.entries;
  const float hit_floor = a.hits.entries ? a.hits.t_floor : __builtin_nanf("");  // NaN: no |t| reaches it
  const float sqrt_df = pd.sqrt_df, inv_sqrt_df = pd.inv_sqrt_df;
  // R rows at a time: their LDS reads and table reads are in flight together
  constexpr int R = 4;
  static_assert((WMF * 16) % R == 0, "row groups");
  for (int g = 0; g < WMF * 16; g += R) {
    float Sv[R];
    f32x2 ihv[R];  // 1 / (gs ||g_res||) for r, 1 / ||g_res|| for beta and SE
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int rr = h + 2 * (g + i);
      Sv[i] = stage[rr * 32 + r32];
      if constexpr (std::is_same<IhPtr, GlobalRows>::value) {
        int64_t mr = rowbase + rr;
        mr = mr < a.nm ? mr : a.nm - 1;
        const float2 v = gload<float2>(a.invh + mr * a.n_panels + j);
        ihv[i] = f32x2{v.x, v.y};
      } else {
        ihv[i] = ih[rr];
      }
    }
    float rv[R], atv[R];
    bool okv[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int rr = h + 2 * (g + i);
      okv[i] = colok && rowbase + rr < a.nm;
      const float invh = ihv[i].y;
      float r = Sv[i] * ihv[i].x * invny;
      if (r > 1.0f) r = 1.0f;
      if (r < -1.0f) r = -1.0f;
      // 1 - r^2 is 0 or at least about 2^-24, never subnormal: the hardware
      // square root and reciprocal square root (1 ulp) serve as they are
      const float omr2 = (1.0f - r) * (1.0f + r);
      const float t = r * sqrt_df * __builtin_amdgcn_rsqf(omr2);
      const uint32_t ob = ((uint32_t)rr * (uint32_t)od.ld + (uint32_t)r32) * 4u;
      if (okv[i]) {
        if (odb.r) gstore_nt(at_byte(odb.r, ob), r);
        if (odb.beta) gstore_nt(at_byte(odb.beta, ob), r * sp * invh);
        if (odb.se) gstore_nt(at_byte(odb.se, ob), sp * invh * __builtin_amdgcn_sqrtf(omr2) * inv_sqrt_df);
        if (odb.t) gstore_nt(at_byte(odb.t, ob), t);
      }
      rv[i] = r;
      atv[i] = fabsf(t);
      if (okv[i] && atv[i] > bv) {  // NaN never enters
        bv = atv[i];
        bm = a.m_begin + a.out_row0 + rowbase + rr;
      }
    }
    if (need_p) {
      float nlv[R];
      if (need_tab) {  // the table at min(|t|, 40) (NaN reads the last interval): R reads in flight together
        tab4 cv[R];
        float sv[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const float x = fminf(atv[i], kTMax) * (float)kTabPerUnit;
          int k = (int)x;
          k = k > kTabIntervals - 1 ? kTabIntervals - 1 : k;
          sv[i] = x - (float)k;
          cv[i] = tab[k];
        }
#pragma unroll
        for (int i = 0; i < R; ++i) nlv[i] = fmaf(fmaf(fmaf(cv[i].w, sv[i], cv[i].z), sv[i], cv[i].y), sv[i], cv[i].x);
      } else {
#pragma unroll
        for (int i = 0; i < R; ++i) nlv[i] = 0.0f;
      }
      uint32_t rare = 0;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const float at = atv[i];
        // |t| <= 40: the table; NaN and +inf carry over; 40 < |t| < inf: the tail
        const bool to_tail = okv[i] && at > kTMax && at != INFINITY;
        const float nl = at <= kTMax ? nlv[i] : at;
        nlv[i] = nl;
        if (okv[i] && !to_tail && odb.nl) gstore_nt(at_byte(odb.nl, ((uint32_t)(h + 2 * (g + i)) * (uint32_t)od.ld + (uint32_t)r32) * 4u), nl);
        const bool hit = okv[i] && !to_tail && at >= hit_floor && nl >= a.hits.threshold;
        rare |= (to_tail || hit) ? 1u << i : 0u;
      }
      if (__builtin_amdgcn_ballot_w64(rare != 0)) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
          if (rare & (1u << i)) {
            const int rr = h + 2 * (g + i);
            const int64_t row = a.out_row0 + rowbase + rr;
            const uint32_t ob = ((uint32_t)rr * (uint32_t)od.ld + (uint32_t)r32) * 4u;
            const float at = atv[i];
            epilogue_rare(at > kTMax && at != INFINITY, nlv[i], at, rv[i], tab,
                          odb.nl ? at_byte(odb.nl, ob) : (float*)nullptr, row, j, p, a.tail, a.hits, a.m_begin + row);
          }
        }
      }
    }
    if (tk_on) {
      unsigned long long tw[R];
      uint32_t tkm = 0;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        tw[i] = topk_pack(atv[i], a.m_begin + a.out_row0 + rowbase + h + 2 * (g + i));
        tkm |= (okv[i] && atv[i] == atv[i] && tw[i] > tk_last) ? 1u << i : 0u;
      }
      if (__builtin_amdgcn_ballot_w64(tkm != 0)) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
          if (tkm & (1u << i)) {
            topk_insert(tkp, od.topk_k, tw[i]);
            tk_last = __atomic_load_n(tkp + od.topk_k - 1, __ATOMIC_RELAXED);
          }
        }
      }
    }
  }
  if (od.best) {  // uniform: one panel per column block
    const float ov = __shfl_xor(bv, 32);
    const int64_t om = __shfl_xor(bm, 32);
    if (ov > bv || (ov == bv && om < bm)) {
      bv = ov;
      bm = om;
    }
    if (h == 0 && colok && bv >= 0.0f) {
      // beyond |t| = 40 the table's value at 40 is a lower bound that the
      // FP64 tail kernel replaces
      const float nl = bv == INFINITY ? INFINITY : table_nlog10p(tab, bv <= kTMax ? bv : kTMax);
      atomicMax(od.best + p, best_pack(nl, bm));
    }
  }
}

// ---------------------------------------------------------------------------
// the contraction (Eq. 2) with the fused epilogue
//
// Workgroup tile: TM = NW * WMF * 32 markers x TP = WN * 32 columns; every
// wave owns WMF 32-row fragments across all WN column blocks.  K loop over
// 64-sample chunks: the column tile's operand chunk is double-buffered in
// LDS; each wave reads its markers' packed codes straight from global memory
// and decodes them in registers with v_perm_b32 and the per-marker table.
// Persistent: the grid is resident and walks the (marker tile, column tile)
// list; the list is cut into 8 contiguous ranges, one per XCD (workgroups
// are dispatched round-robin to XCDs), so that the workgroups of an XCD
// share column tiles in their L2.
// ---------------------------------------------------------------------------
//
// G8: the rows hold 8-bit dosages, one byte per sample; each lane half reads
// its 32 bytes of the chunk and builds FP16 q - c by inserting the byte under
// the exponent of 1024 and subtracting 1024 + c (exact for integers below
// 2048), or FP32 q - c; a missing byte takes the marker's mu - c.
template <int PREC, int NW, int WMF, int WN, int MODE, bool G8 = false>
__global__ __launch_bounds__(NW * 64, (WN == 1 && MODE == kRawHL) ? 4 : 1) void gemm_kernel(GemmArgs a) {
  static_assert(!G8 || PREC == kFP32 || PREC == kSplit16, "8-bit dosages run the FP32 and FP16 split forms here");
  static_assert(MODE != kRawHL || (PREC != kFP32 && WN == 1), "the packed hi|lo operand is one split block");
  constexpr bool LO_PASS = MODE != kRawHL;
  constexpr int NT = NW * 64;
  constexpr int TM = NW * WMF * 32;
  constexpr int TILE_BYTES = WN * kBlockBytes;
  constexpr int RPB = kBlockBytes / 16 / NT;  // 16-byte pieces per thread per block
  static_assert(kBlockBytes % (16 * NT) == 0, "block copy must divide evenly");
  constexpr int STAGE_BYTES = MODE == kTest ? NW * WMF * 32 * 32 * 4 : 0;
  constexpr int LDS_BYTES = 2 * TILE_BYTES > STAGE_BYTES ? 2 * TILE_BYTES : STAGE_BYTES;
  __shared__ __attribute__((aligned(16))) char smem[LDS_BYTES];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int h = lane >> 5;
  const int r32 = lane & 31;

  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int xcd = b & 7;
  const int slot = b >> 3;
  const int nslots = G >> 3;
  const int64_t W = (int64_t)a.n_mtiles * a.n_ctiles;
  const int64_t wlo = W * xcd / 8;
  const int64_t whi = W * (xcd + 1) / 8;

  for (int64_t w = wlo + slot; w < whi; w += nslots) {
    int mtile, ctile;
    grouped_tile(w, a.n_mtiles, a.n_ctiles, mtile, ctile);

    // operand blocks of this column tile; blocks past the end alias the
    // first one (their columns are never written)
    const char* bop[WN];
#pragma unroll
    for (int fn = 0; fn < WN; ++fn) {
      const int cb = ctile * WN + fn;
      bop[fn] = a.cblocks[cb < a.n_cblocks ? cb : ctile * WN].op;
    }
    const int64_t rowbase = (int64_t)mtile * TM + wave * (WMF * 32);
    const uint8_t* ap[WMF];
    uint4 lut[WMF];
#pragma unroll
    for (int fm = 0; fm < WMF; ++fm) {
      int64_t mr = rowbase + fm * 32 + r32;
      mr = mr < a.nm ? mr : a.nm - 1;
      ap[fm] = a.geno + (a.m0 + mr) * a.row_bytes + (G8 ? 32 : 8) * h;
      lut[fm] = gload<uint4>(a.mlut + mr);
    }

    f32x16 acc[WMF][WN];
#pragma unroll
    for (int fm = 0; fm < WMF; ++fm)
#pragma unroll
      for (int fn = 0; fn < WN; ++fn)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[fm][fn][i] = 0.0f;

    u32x4 breg[WN][RPB];
    // this lane's genotype bytes of the chunk: 8 (2-bit codes) or 32 (dosages).
    // The 32-column shape (the Q^T g contraction) does little work per
    // chunk, so it keeps a ring of AD chunks of its rows in flight to cover
    // the memory latency (the chunk loop is unrolled by AD so that the ring
    // is indexed statically); the others keep one chunk ahead.
    constexpr int AD = WN == 1 ? (G8 ? 2 : 4) : 1;
    struct ARow {
      u32x4 q[G8 ? 2 : 1];
    };
    auto load_b = [&](int ch) {
#pragma unroll
      for (int fn = 0; fn < WN; ++fn)
#pragma unroll
        for (int q = 0; q < RPB; ++q)
          breg[fn][q] = gload<u32x4>(bop[fn] + (int64_t)ch * kBlockBytes + (q * NT + tid) * 16);
    };
    auto store_b = [&](int buf) {
#pragma unroll
      for (int fn = 0; fn < WN; ++fn)
#pragma unroll
        for (int q = 0; q < RPB; ++q) *(u32x4*)(smem + buf * TILE_BYTES + fn * kBlockBytes + (q * NT + tid) * 16) = breg[fn][q];
    };
    auto load_a = [&](int ch, ARow* dst) {
#pragma unroll
      for (int fm = 0; fm < WMF; ++fm) {
        if constexpr (G8) {
          dst[fm].q[0] = gload<u32x4>(ap[fm] + (int64_t)ch * 64);
          dst[fm].q[1] = gload<u32x4>(ap[fm] + (int64_t)ch * 64 + 16);
        } else {
          const uint2 v = gload<uint2>(ap[fm] + (int64_t)ch * 16);
          dst[fm].q[0][0] = v.x;
          dst[fm].q[0][1] = v.y;
        }
      }
    };
    // dword k (4 samples) of this lane's dosage bytes
    auto dword8 = [&](const ARow& r, int k) -> uint32_t { return k < 4 ? r.q[0][k] : r.q[G8 ? 1 : 0][k & 3]; };

    // one chunk's decode and matrix-core steps on the staged operand tile cur
    auto compute = [&](const int cur, const ARow* areg, const int half) __attribute__((always_inline)) {
      const char* tile = smem + cur * TILE_BYTES + half * (kBlockBytes / 2);
      if constexpr (PREC != kFP32) {
        u32x4 bh[WN], bl[WN];
#pragma unroll
        for (int fn = 0; fn < WN; ++fn) {
          bh[fn] = *(const u32x4*)(tile + fn * kBlockBytes + (lane * 8) * 2);
          if constexpr (LO_PASS) bl[fn] = *(const u32x4*)(tile + fn * kBlockBytes + (2048 + lane * 8) * 2);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          u32x4 A[WMF];
#pragma unroll
          for (int fm = 0; fm < WMF; ++fm) {
            if constexpr (G8) {
              // slots (2d, 2d+1) of step j take samples 16 (j >> 1) + 4 (j & 1) + d
              // and that + 8 of this lane half: byte d of dwords k0 and k0 + 2
              const int k0 = 4 * (j >> 1) + (j & 1);
              const uint32_t D0 = dword8(areg[fm], k0), D1 = dword8(areg[fm], k0 + 2);
              const uint32_t M0 = ff_bytes(D0), M1 = ff_bytes(D1);
#pragma unroll
              for (int d = 0; d < 4; ++d) {
                const uint32_t x = __builtin_amdgcn_perm(D1, D0, 0x0c000c00u | ((4u + d) << 16) | d) | 0x64006400u;
                const uint32_t v = __builtin_bit_cast(uint32_t, __builtin_bit_cast(f16x2, x) +
                                                                    __builtin_bit_cast(f16x2, lut[fm].x));
                const uint32_t mk = __builtin_amdgcn_perm(M1, M0, d | (d << 8) | ((4u + d) << 16) | ((4u + d) << 24));
                A[fm][d] = (mk & lut[fm].y) | (~mk & v);
              }
            } else {
              const uint32_t src = (j < 2) ? areg[fm].q[0][0] : areg[fm].q[0][1];
#pragma unroll
              for (int d = 0; d < 4; ++d) {
                const int t = 4 * (j & 1) + d;
                const uint32_t R = (src >> (2 * t)) & 0x00030003u;
                const uint32_t sel = R * 0x101u + 0x04000400u;
                A[fm][d] = __builtin_amdgcn_perm(lut[fm].y, lut[fm].x, sel);
              }
            }
          }
          u32x4 nh[WN], nl[WN];
          if (j < 3) {
#pragma unroll
            for (int fn = 0; fn < WN; ++fn) {
              nh[fn] = *(const u32x4*)(tile + fn * kBlockBytes + ((j + 1) * 512 + lane * 8) * 2);
              if constexpr (LO_PASS)
                nl[fn] = *(const u32x4*)(tile + fn * kBlockBytes + (2048 + (j + 1) * 512 + lane * 8) * 2);
            }
          }
#pragma unroll
          for (int fn = 0; fn < WN; ++fn)
#pragma unroll
            for (int fm = 0; fm < WMF; ++fm) acc[fm][fn] = mfma16<PREC>(A[fm], bh[fn], acc[fm][fn]);
          if constexpr (LO_PASS) {
#pragma unroll
            for (int fn = 0; fn < WN; ++fn)
#pragma unroll
              for (int fm = 0; fm < WMF; ++fm) acc[fm][fn] = mfma16<PREC>(A[fm], bl[fn], acc[fm][fn]);
          }
          if (j < 3) {
#pragma unroll
            for (int fn = 0; fn < WN; ++fn) {
              bh[fn] = nh[fn];
              if constexpr (LO_PASS) bl[fn] = nl[fn];
            }
          }
        }
      } else {
        uint64_t bits[WMF];
#pragma unroll
        for (int fm = 0; fm < WMF; ++fm) bits[fm] = (uint64_t)areg[fm].q[0][0] | ((uint64_t)areg[fm].q[0][1] << 32);
#pragma unroll
        for (int j4 = 0; j4 < 8; ++j4) {
          float4 bv[WN];
#pragma unroll
          for (int fn = 0; fn < WN; ++fn)
            bv[fn] = *(const float4*)(tile + fn * kBlockBytes + (j4 * 256 + lane * 4) * 4);
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const int j = j4 * 4 + jj;
            float av[WMF];
#pragma unroll
            for (int fm = 0; fm < WMF; ++fm) {
              if constexpr (G8) {  // sample 32 h + j: byte j of this lane half's 32
                const uint32_t q = (dword8(areg[fm], j >> 2) >> (8 * (j & 3))) & 0xffu;
                av[fm] = q == 0xffu ? __uint_as_float(lut[fm].w) : (float)q - __uint_as_float(lut[fm].z);
              } else {
                const uint32_t c = (uint32_t)(bits[fm] >> (2 * j)) & 3u;
                const uint32_t lo = (c & 1u) ? lut[fm].y : lut[fm].x;
                const uint32_t hi = (c & 1u) ? lut[fm].w : lut[fm].z;
                av[fm] = __uint_as_float((c & 2u) ? hi : lo);
              }
            }
#pragma unroll
            for (int fn = 0; fn < WN; ++fn) {
              const float bb = jj == 0 ? bv[fn].x : jj == 1 ? bv[fn].y : jj == 2 ? bv[fn].z : bv[fn].w;
#pragma unroll
              for (int fm = 0; fm < WMF; ++fm)
                acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[fm], bb, acc[fm][fn], 0, 0, 0);
            }
          }
        }
      }
    };

    const int nch = a.n_chunks;
    if constexpr (AD == 1) {
      ARow areg[WMF], anext[WMF];
      load_b(0);
      load_a(0, areg);
      store_b(0);
      __syncthreads();
      for (int ch = 0; ch < nch; ++ch) {
        const int cur = ch & 1;
        const bool more = ch + 1 < nch;
        if (more) {
          load_b(ch + 1);
          load_a(ch + 1, anext);
        }
        compute(cur, areg, 0);
        if (more) store_b(cur ^ 1);
        __syncthreads();
#pragma unroll
        for (int fm = 0; fm < WMF; ++fm) areg[fm] = anext[fm];
      }
    } else if constexpr (MODE == kRawHL && AD == 4 && WN == 1 && RPB == 1) {
      // A packed hi|lo block fills the first half of its 8 KiB chunk (the
      // split layout's lo half is zero and never read), so the used halves
      // of two chunks fill one LDS buffer: chunks 2P and 2P + 1 sit in
      // buffer P & 1, thread t copies piece t & 255 of chunk 2P + (t >> 8),
      // and one barrier serves two chunks.  The rows go by pairs of chunks
      // too: the lane pair of a row (h = 0, 1) reads chunks 2p and 2p + 1
      // whole, one 16-byte piece each, and the two lanes swap halves, so a
      // row's 128-byte line is requested in four pieces, not eight.  rraw[v]
      // holds the pieces of the row pair ch0 + 2v, ch0 + 2v + 1; pring[v]
      // the operand pair after the one in LDS whose index is v mod 2.  Both
      // are requested four chunks ahead (the last chunk again past the end: a
      // valid address whose bytes are not used), and the loop runs whole
      // rounds of four chunks without branches, so a wait covers only
      // requests a round old (the wait counter is in order).
      constexpr int HB = kBlockBytes / 2;
      auto clamp = [&](int ch) { return ch < nch ? ch : nch - 1; };
      auto load_pair = [&](int P, u32x4& dst) {
        dst = gload<u32x4>(bop[0] + (int64_t)clamp(2 * P + (tid >> 8)) * kBlockBytes + (tid & 255) * 16);
      };
      auto store_pair = [&](int buf, const u32x4& src) {
        *(u32x4*)(smem + buf * TILE_BYTES + (tid >> 8) * HB + (tid & 255) * 16) = src;
      };
      // ap[fm] points at this lane half's 8 bytes of chunk 0; the row starts 8 h before
      auto load_rows = [&](int c, u32x4* dst) {  // c even: chunk c + h whole
#pragma unroll
        for (int fm = 0; fm < WMF; ++fm) dst[fm] = gload<u32x4>(ap[fm] - 8 * h + (int64_t)clamp(c + h) * 16);
      };
      // this lane half's 8 bytes of chunks c and c + 1: lane h = 0 holds chunk
      // c and passes its second half to lane 32 + r32, which holds chunk c + 1
      // and passes back that chunk's first half
      auto split_rows = [&](const u32x4* src, ARow* first, ARow* second) {
#pragma unroll
        for (int fm = 0; fm < WMF; ++fm) {
          const uint32_t s0 = h ? src[fm][0] : src[fm][2];
          const uint32_t s1 = h ? src[fm][1] : src[fm][3];
          const uint32_t r0 = (uint32_t)__shfl_xor((int)s0, 32);
          const uint32_t r1 = (uint32_t)__shfl_xor((int)s1, 32);
          first[fm].q[0][0] = h ? r0 : src[fm][0];
          first[fm].q[0][1] = h ? r1 : src[fm][1];
          second[fm].q[0][0] = h ? src[fm][2] : r0;
          second[fm].q[0][1] = h ? src[fm][3] : r1;
        }
      };
      u32x4 rraw[2][WMF];
      u32x4 pring[2];
      ARow a0[WMF], a1[WMF];
      // requests in the order a round makes them (rows, pair, rows, pair),
      // so that the counts the compiler waits for at the loop head hold for
      // the first round as for the others
      load_pair(0, pring[0]);
      store_pair(0, pring[0]);
      load_rows(0, rraw[0]);
      __builtin_amdgcn_sched_barrier(0);
      load_pair(1, pring[1]);
      __builtin_amdgcn_sched_barrier(0);
      load_rows(2, rraw[1]);
      __builtin_amdgcn_sched_barrier(0);
      load_pair(2, pring[0]);
      __syncthreads();
      const int nfull = nch / 4 * 4;
      for (int ch0 = 0; ch0 < nfull; ch0 += 4) {
        const int P = ch0 / 2;
        split_rows(rraw[0], a0, a1);
        compute(0, a0, 0);
        compute(0, a1, 1);
        load_rows(ch0 + 4, rraw[0]);
        store_pair(1, pring[1]);  // pair P + 1: chunks ch0 + 2, ch0 + 3
        load_pair(P + 3, pring[1]);
        __syncthreads();
        split_rows(rraw[1], a0, a1);
        compute(1, a0, 0);
        compute(1, a1, 1);
        load_rows(ch0 + 6, rraw[1]);
        store_pair(0, pring[0]);  // pair P + 2: the next round's first two chunks
        load_pair(P + 4, pring[0]);
        __syncthreads();
      }
      // the last nch - nfull < 4 chunks: the first two in buffer 0 and
      // rraw[0], the third's operand pair in pring[1] and rows in rraw[1]
      const int r = nch - nfull;
      if (r > 0) {
        split_rows(rraw[0], a0, a1);
        compute(0, a0, 0);
        if (r > 1) compute(0, a1, 1);
      }
      if (r > 2) {
        store_pair(1, pring[1]);
        __syncthreads();
        split_rows(rraw[1], a0, a1);
        compute(1, a0, 0);
      }
      __syncthreads();  // every wave is done with the buffers before the next tile's copies
    } else {
      // ring[u] holds the rows of chunk ch0 + u and bring[v] the operand
      // block of the chunk after it that is v mod AD (ch0 a multiple of AD,
      // so chunk ch sits in LDS buffer ch & 1).  Each is refilled once used,
      // with the chunk AD later (the last chunk again past the end: a valid
      // address whose bytes are not used).  A chunk's operand block is
      // requested AD chunks before it is copied to LDS, after that chunk's
      // rows: waiting for it waits only for requests AD chunks old, so AD
      // chunks of rows stay in flight (the wait counter is in order).
      ARow ring[AD][WMF];
      u32x4 bring[AD][WN][RPB];
      // a packed hi|lo block uses the first half of its chunk (the split
      // layout's lo half is zero and never read): only that half is copied
      constexpr int B_USED = MODE == kRawHL ? kBlockBytes / 2 : kBlockBytes;
      auto load_b_to = [&](int ch, u32x4 (*dst)[RPB]) {
#pragma unroll
        for (int fn = 0; fn < WN; ++fn)
#pragma unroll
          for (int q = 0; q < RPB; ++q)
            if ((q * NT + tid) * 16 < B_USED)
              dst[fn][q] = gload<u32x4>(bop[fn] + (int64_t)ch * kBlockBytes + (q * NT + tid) * 16);
      };
      auto store_b_from = [&](int buf, u32x4 (*src)[RPB]) {
#pragma unroll
        for (int fn = 0; fn < WN; ++fn)
#pragma unroll
          for (int q = 0; q < RPB; ++q)
            if ((q * NT + tid) * 16 < B_USED)
              *(u32x4*)(smem + buf * TILE_BYTES + fn * kBlockBytes + (q * NT + tid) * 16) = src[fn][q];
      };
      auto clamp = [&](int ch) { return ch < nch ? ch : nch - 1; };
      load_b_to(0, bring[0]);
      store_b_from(0, bring[0]);
#pragma unroll
      for (int u = 0; u < AD; ++u) {
        load_a(clamp(u), ring[u]);
        load_b_to(clamp(u + 1), bring[(u + 1) % AD]);
      }
      __syncthreads();
      // whole rounds of AD chunks, with no branch inside a round (a branch
      // per chunk left the compiler waiting for every request in flight)
      const int nfull = nch / AD * AD;
      for (int ch0 = 0; ch0 < nfull; ch0 += AD) {
#pragma unroll
        for (int u = 0; u < AD; ++u) {
          const int ch = ch0 + u;
          compute(u & 1, ring[u], 0);
          load_a(clamp(ch + AD), ring[u]);
          store_b_from((u & 1) ^ 1, bring[(u + 1) % AD]);  // chunk ch + 1 (a repeat of the last past the end)
          load_b_to(clamp(ch + 1 + AD), bring[(u + 1) % AD]);
          __syncthreads();
        }
      }
      // the last nch - nfull < AD chunks (chunk nfull + u in ring[u], its
      // successor's operand block in bring[(u + 1) % AD])
#pragma unroll
      for (int u = 0; u < AD - 1; ++u) {
        const int ch = nfull + u;
        if (ch < nch) {
          compute(u & 1, ring[u], 0);
          if (ch + 1 < nch) store_b_from((u & 1) ^ 1, bring[(u + 1) % AD]);
          __syncthreads();
        }
      }
    }

    // ---------------------------------------------------------------- epilogue
    if constexpr (MODE == kRawHL) {
      // slot col0 + r32, r32 < 16: the hi product (column r32) plus the lo
      // product (column r32 + 16, held by lane r32 + 16 of this lane half);
      // a block of 32 columns (ncol = 32: the panel's only block) also
      // writes zeros to the 16 slots after its own
      if (ctile < a.n_cblocks) {
        const ColBlock blk = a.cblocks[ctile];
#pragma unroll
        for (int fm = 0; fm < WMF; ++fm)
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const float v = acc[fm][0][i];
            const float o = __shfl_xor(v, kHLSlots);
            const int64_t mr = rowbase + fm * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
            if (mr < a.nm && r32 < blk.ncol)
              gstore(a.raw_out + mr * a.raw_ld + blk.col0 + r32, r32 < kHLSlots ? v + o : 0.0f);
          }
      }
    } else if constexpr (MODE == kRaw) {
#pragma unroll
      for (int fn = 0; fn < WN; ++fn) {
        const int cb = ctile * WN + fn;
        if (cb >= a.n_cblocks) continue;
        const ColBlock blk = a.cblocks[cb];
        if (r32 >= blk.ncol) continue;
#pragma unroll
        for (int fm = 0; fm < WMF; ++fm)
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int64_t mr = rowbase + fm * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
            if (mr < a.nm) gstore(a.raw_out + mr * a.raw_ld + blk.col0 + r32, acc[fm][fn][i]);
          }
      }
    } else {
      // correction: acc += sum_slot w[m][slot] * cw[p][slot]
      //   = -(mu - c) sum_i y_op,i - sum_{k>=1} (q_k^T g)(q_k^T y_op)
      // i.e. the intercept and covariate components of the projection
      // (I - QQ^T) applied to the stored operand.  Small term: one BF16
      // matrix-core pass over 32 slots.
#pragma unroll
      for (int fn = 0; fn < WN; ++fn) {
        const int cb = ctile * WN + fn;
        const ColBlock blk = a.cblocks[cb < a.n_cblocks ? cb : ctile * WN];
        const float* cwp = a.panels[blk.panel].cw + (int64_t)(blk.col0 + r32) * kSlots + 8 * h;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          const float4 c0 = gload<float4>(cwp + 16 * ks);
          const float4 c1 = gload<float4>(cwp + 16 * ks + 4);
          u32x4 bo;
          bo[0] = pack_bf16x2(c0.x, c0.y);
          bo[1] = pack_bf16x2(c0.z, c0.w);
          bo[2] = pack_bf16x2(c1.x, c1.y);
          bo[3] = pack_bf16x2(c1.z, c1.w);
          const bf16x8 B = __builtin_bit_cast(bf16x8, bo);
#pragma unroll
          for (int fm = 0; fm < WMF; ++fm) {
            int64_t mr = rowbase + fm * 32 + r32;
            mr = mr < a.nm ? mr : a.nm - 1;
            const float* wp = a.wws + (mr * a.n_panels + blk.panel) * kSlots + 16 * ks + 8 * h;
            const float4 w0 = gload<float4>(wp);
            const float4 w1 = gload<float4>(wp + 4);
            u32x4 ao;
            ao[0] = pack_bf16x2(w0.x, w0.y);
            ao[1] = pack_bf16x2(w0.z, w0.w);
            ao[2] = pack_bf16x2(w1.x, w1.y);
            ao[3] = pack_bf16x2(w1.z, w1.w);
            acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ao), B,
                                                                  acc[fm][fn], 0, 0, 0);
          }
        }
      }
      // stage one 32-column slice of the accumulators at a time through this
      // wave's 8 KiB of LDS (the B buffers are free now), then finish the
      // tests in a plain loop: lanes run along columns, so every output row
      // segment is one 128-byte store per half-wave.
      float* stage = (float*)smem + wave * (WMF * 32 * 32);
#pragma unroll
      for (int fn = 0; fn < WN; ++fn) {
        const int cb = ctile * WN + fn;
        if (cb >= a.n_cblocks) break;
#pragma unroll
        for (int fm = 0; fm < WMF; ++fm)
#pragma unroll
          for (int i = 0; i < 16; ++i)
            stage[(fm * 32 + 8 * (i >> 2) + 4 * h + (i & 3)) * 32 + r32] = acc[fm][fn][i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const ColBlock blk = a.cblocks[cb];
        const PanelDev& pdb = a.panels[blk.panel];
        const bool colok = r32 < blk.ncol;
        const float invny = colok ? gload<float>(pdb.invny + blk.col0 + r32) : 0.f;
        const float sp = colok ? gload<float>(pdb.scale + blk.col0 + r32) * a.gunit : 0.f;
        finish_block<WMF>(stage, a, blk, rowbase, h, r32, (const tab4*)pdb.table, GlobalRows{}, invny, sp);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      __syncthreads();  // the next tile's prologue overwrites the staging area
    }
  }
}

// ---------------------------------------------------------------------------
// wide split-precision contraction: one wave per SIMD, each wave owns a
// 128 x 128 accumulator tile (256 FP32 accumulators, AGPRs); workgroup tile
// 512 markers x 128 columns.
//
// Operands move through an LDS ring, one 64-sample chunk per stage: the
// column tile's operand chunk and the packed codes of the tile's 512 markers
// (8 KiB), both copied with direct-to-LDS loads.  A chunk is requested
// NSTAGE - 1 chunks before it is used.  Within a chunk, step j's matrix-core
// instructions are interleaved with the LDS reads of step j+1's operand
// fragments and the decode of its genotypes, into the register set of the
// other parity.  One barrier per chunk, ahead of its last step: after it the
// next chunk has landed and every wave is done with this chunk's stage,
// which is refilled at once.
//
// Forms: the 16-bit splits run 2 x WMF x 4 MFMA 32x32x16 per step (hi and lo
// terms); FP16 hi + FP8 lo runs WMF x 4 FP16 MFMA per step plus a quarter of
// the chunk's block-scaled FP8 MFMA 32x32x64 (E8M0 scale of each column's lo
// term on the B side): with WMF = 4 those of marker fragment j, with WMF = 2
// those of column block j.
//
// Shapes: NW = 4, WMF = 4 (one wave per SIMD, 128 x 128 per wave, 256 AGPR
// accumulators) or NW = 8, WMF = 2 (two waves per SIMD, 64 x 128 per wave),
// so that one wave's genotype decode and epilogue overlap the other wave's
// matrix-core work.
// ---------------------------------------------------------------------------
typedef int i32x8 __attribute__((ext_vector_type(8)));

// s_waitcnt immediate: vmcnt(vm), lgkmcnt(0), expcnt unconstrained
constexpr int waitcnt_vm_lgkm0(int vm) { return (vm & 15) | ((vm >> 4) << 14) | (0x7 << 4); }
// vmcnt(vm) only (expcnt and lgkmcnt unconstrained)
constexpr int waitcnt_vm_only(int vm) { return waitcnt_vm_lgkm0(vm) | (0xF << 8); }

// G8: 8-bit dosage rows (FP16 split only): each stage holds the tile's 64
// bytes per marker; a lane reads the two dwords of its row that each K16 step
// needs and builds FP16 q - c as the register-staged kernel does.
// Two FP16 values (the halves of v) to OCP e4m3, round to nearest even,
// into bytes 0 and 1 (lo) or 2 and 3 (hi) of old, the other two kept.
// Written as the instruction itself: this compiler's builtin for it, given
// several calls that differ only in v, emitted the conversion of the first v
// for all of them.
__device__ __forceinline__ uint32_t cvt_pk_e4m3_lo(uint32_t old, uint32_t v) {
  asm("v_cvt_scalef32_pk_fp8_f16 %0, %1, 1.0" : "+v"(old) : "v"(v));
  return old;
}
__device__ __forceinline__ uint32_t cvt_pk_e4m3_hi(uint32_t old, uint32_t v) {
  asm("v_cvt_scalef32_pk_fp8_f16 %0, %1, 1.0 op_sel:[0,0,1]" : "+v"(old) : "v"(v));
  return old;
}

template <int PREC, int MODE, int NW, int WMF, int WN = 4, bool G8 = false>
__global__ __launch_bounds__(NW * 64) void gemm_wide_kernel(GemmArgs a) {
  static_assert(PREC != kFP32, "the wide kernel runs the split forms");
  static_assert(!G8 || PREC == kSplit16 || PREC == kSplit8, "8-bit dosages run the FP16 split forms here");
  static_assert((NW * WMF == 16 && WN == 4 && (WMF == 4 || WMF == 2)) ||
                    (NW == 4 && WMF == 2 && WN == 8 && PREC == kSplit8),
                "512 x 128 tiles, or 256 x 256 for the FP8 lo form");
  constexpr bool F8 = PREC == kSplit8;
  // 8-bit dosages in the FP16 + FP8 form: the FP8 lo operand is converted from
  // the FP16 values of the hi pass, a step at a time, and the chunk's lo
  // MFMAs run together at its last step
  constexpr bool GF = F8 && G8;
  constexpr bool W2 = WMF == 2;  // FP8 lo MFMAs by column block: both fragments, WN / 4 blocks per step
  constexpr int FNS = WN / 4;    // column blocks whose FP8 lo term runs at each step (WMF = 2)
  constexpr int NT = NW * 64;
  constexpr int TM = NW * WMF * 32;
  constexpr int BB = block_bytes(PREC);
  constexpr int NSTAGE = G8 ? 2 : (F8 ? (WN == 8 ? 3 : 4) : 3);
  constexpr int B_BYTES = WN * BB;  // operand chunk of the column tile
  constexpr int AB = G8 ? 64 : 16;  // bytes of a marker's chunk: 64 two-bit codes or 64 dosage bytes
  constexpr int A_BYTES = TM * AB;
  constexpr int STAGE_BYTES = B_BYTES + A_BYTES;
  constexpr int LDS_BYTES = NSTAGE * STAGE_BYTES;
  constexpr int PPB = BB / 1024;                // 1 KiB pieces per operand block
  constexpr int B_OPS = B_BYTES / (NT * 16);    // direct-to-LDS loads per wave per chunk
  constexpr int A_OPS = A_BYTES / (NT * 16);
  constexpr int CHUNK_OPS = B_OPS + A_OPS;
  constexpr int HI_MFMA = F8 ? WMF * WN : 2 * WMF * WN;  // 16-bit MFMA per step
  constexpr int DS_STEP = F8 ? WN : 2 * WN;              // fragment reads per step
  static_assert(NW * WMF * 32 * 32 * 4 <= LDS_BYTES, "epilogue staging must fit");
  static_assert((NSTAGE - 2) * CHUNK_OPS < 64, "vmcnt range");
  // past the stages: each row's 1/||g_res|| of the current column panel and,
  // where it fits, that panel's p-value table; the epilogue then reads
  // nothing from global memory between its output stores
  constexpr int IH_BYTES = TM * 8;
  constexpr int TAB_BYTES = kTabIntervals * 16;
  constexpr bool LT = LDS_BYTES + IH_BYTES + TAB_BYTES <= 160 * 1024;
  static_assert(WMF % 2 == 0 && LDS_BYTES + IH_BYTES <= 160 * 1024, "epilogue rows in LDS");
  __shared__ __attribute__((aligned(16))) char smem[LDS_BYTES + IH_BYTES + (LT ? TAB_BYTES : 0)];
  int tab_panel = -1;  // panel whose table is in LDS (uniform)

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int h = lane >> 5;
  const int r32 = lane & 31;

  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int xcd = b & 7;
  const int slot = b >> 3;
  const int nslots = G >> 3;
  const int64_t W = (int64_t)a.n_mtiles * a.n_ctiles;
  const int64_t wlo = W * xcd / 8;
  const int64_t whi = W * (xcd + 1) / 8;

  for (int64_t w = wlo + slot; w < whi; w += nslots) {
    int mtile, ctile;
    grouped_tile(w, a.n_mtiles, a.n_ctiles, mtile, ctile);
    const char* bop[WN];
    int bscale[WN];  // FP8 form: E8M0 scale of this lane's column, per block
#pragma unroll
    for (int fn = 0; fn < WN; ++fn) {
      const int cb = ctile * WN + fn;
      const ColBlock blk = a.cblocks[cb < a.n_cblocks ? cb : ctile * WN];
      bop[fn] = blk.op;
      bscale[fn] = 127;
      if constexpr (F8) {
        if (cb < a.n_cblocks && r32 < blk.ncol) bscale[fn] = a.panels[blk.panel].lscale[blk.col0 + r32];
      }
    }
    const int64_t rowbase = (int64_t)mtile * TM + wave * (WMF * 32);
    uint2 lut[WMF];
    uint32_t lut8[WMF];
#pragma unroll
    for (int fm = 0; fm < WMF; ++fm) {
      int64_t mr = rowbase + fm * 32 + r32;
      mr = mr < a.nm ? mr : a.nm - 1;
      if constexpr (F8) {
        const uint4 l4 = gload<uint4>(a.mlut + mr);
        lut[fm] = make_uint2(l4.x, l4.y);
        lut8[fm] = l4.z;
      } else {
        lut[fm] = gload<uint2>(a.mlut + mr);
        lut8[fm] = 0u;
      }
    }
    // code rows copied by this lane: markers rowbase + 64 k + lane (rows
    // past the end read the last row; their results are never stored)
    // (8-bit dosages: 16-byte piece 64 k + lane of the wave's rows, i.e.
    // quarter (64 k + lane) & 3 of marker rowbase + (64 k + lane) / 4)
    const uint8_t* arow[A_OPS];
#pragma unroll
    for (int k = 0; k < A_OPS; ++k) {
      const int piece = 64 * k + lane;
      int64_t mr = rowbase + (G8 ? piece >> 2 : piece);
      mr = mr < a.nm ? mr : a.nm - 1;
      arow[k] = a.geno + (a.m0 + mr) * a.row_bytes + (G8 ? (piece & 3) * 16 : 0);
    }

    f32x16 acc[WMF][WN];
#pragma unroll
    for (int fm = 0; fm < WMF; ++fm)
#pragma unroll
      for (int fn = 0; fn < WN; ++fn)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[fm][fn][i] = 0.0f;

    const int nch = a.n_chunks;
    // chunk ch (clamped to the last one: the surplus copies land in stages
    // nobody reads again) into stage st
    auto dma = [&](int ch, int st) {
      ch = ch < nch ? ch : nch - 1;
      char* stage = smem + st * STAGE_BYTES;
#pragma unroll
      for (int q = 0; q < B_OPS; ++q) {
        const int piece = q * NW + wave;  // 1 KiB piece of the operand chunk
        const int fn = piece / PPB;
        const int off = (piece % PPB) * 1024;
        __builtin_amdgcn_global_load_lds(
            (const __attribute__((address_space(1))) void*)(bop[fn] + (int64_t)ch * BB + off + lane * 16),
            (__attribute__((address_space(3))) void*)(stage + fn * BB + off), 16, 0, 0);
      }
#pragma unroll
      for (int k = 0; k < A_OPS; ++k)
        __builtin_amdgcn_global_load_lds(
            (const __attribute__((address_space(1))) void*)(arow[k] + (int64_t)ch * AB),
            (__attribute__((address_space(3))) void*)(stage + B_BYTES + wave * (WMF * 32 * AB) + k * 1024), 16, 0,
            0);
    };
    // whole 16-byte rows, this lane's half picked in registers (paired
    // 8-byte reads would be fused into one read that the compiler then holds
    // until every direct-to-LDS copy in flight has landed)
    auto read_a_raw = [&](int st, u32x4* raw) {
      const char* ab = smem + st * STAGE_BYTES + B_BYTES + wave * (WMF * 32 * 16);
#pragma unroll
      for (int fm = 0; fm < WMF; ++fm) raw[fm] = *(const u32x4*)(ab + (fm * 32 + r32) * 16);
    };
    auto pick_a = [&](const u32x4* raw, uint2* dst) {
#pragma unroll
      for (int fm = 0; fm < WMF; ++fm) dst[fm] = h ? make_uint2(raw[fm][2], raw[fm][3]) : make_uint2(raw[fm][0], raw[fm][1]);
    };
    auto read_a = [&](int st, uint2* dst) {
      u32x4 raw[WMF];
      read_a_raw(st, raw);
      pick_a(raw, dst);
    };
    // 8-bit dosages: dwords k0 and k0 + 2 (k0 = 4 (j >> 1) + (j & 1)) of this
    // lane half's 32 bytes of each fragment row, the two that K16 step j needs
    auto read_g8 = [&](int st, int j, uint2* dst) {
      const char* ab = smem + st * STAGE_BYTES + B_BYTES + wave * (WMF * 32 * 64) + h * 32;
      const int k0 = 4 * (j >> 1) + (j & 1);
#pragma unroll
      for (int fm = 0; fm < WMF; ++fm) {
        const char* row = ab + (fm * 32 + r32) * 64;
        dst[fm] = make_uint2(*(const uint32_t*)(row + 4 * k0), *(const uint32_t*)(row + 4 * (k0 + 2)));
      }
    };
    // slots (2d, 2d + 1) of step j take samples 16 (j >> 1) + 4 (j & 1) + d and
    // that + 8 of this lane half: byte d of the two dwords read above; FP16
    // q - c by inserting the byte under the exponent of 1024, a missing byte
    // takes mu - c
    auto decode_g8 = [&](const uint2* D, u32x4* A) {
#pragma unroll
      for (int fm = 0; fm < WMF; ++fm) {
        const uint32_t D0 = D[fm].x, D1 = D[fm].y;
        const uint32_t M0 = ff_bytes(D0), M1 = ff_bytes(D1);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const uint32_t x = __builtin_amdgcn_perm(D1, D0, 0x0c000c00u | ((4u + d) << 16) | d) | 0x64006400u;
          const uint32_t v =
              __builtin_bit_cast(uint32_t, __builtin_bit_cast(f16x2, x) + __builtin_bit_cast(f16x2, lut[fm].x));
          const uint32_t mk = __builtin_amdgcn_perm(M1, M0, d | (d << 8) | ((4u + d) << 16) | ((4u + d) << 24));
          A[fm][d] = (mk & lut[fm].y) | (~mk & v);
        }
      }
    };
    // 16-bit values of K16 step j: two per dword via the per-marker table
    auto decode = [&](const uint2* src2, int j, u32x4* A) {
#pragma unroll
      for (int fm = 0; fm < WMF; ++fm) {
        const uint32_t src = (j < 2) ? src2[fm].x : src2[fm].y;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const int t = 4 * (j & 1) + d;
          const uint32_t R = (src >> (2 * t)) & 0x00030003u;
          const uint32_t sel = R * 0x101u + 0x04000400u;
          A[fm][d] = __builtin_amdgcn_perm(lut[fm].y, lut[fm].x, sel);
        }
      }
    };
    // e4m3 values of fragment fm over the whole chunk: four per dword
    auto decode8 = [&](const uint2* src2, int fm, i32x8& A8) {
#pragma unroll
      for (int part = 0; part < 2; ++part) {
        const uint32_t src = part ? src2[fm].y : src2[fm].x;
#pragma unroll
        for (int t = 0; t < 4; ++t)
          A8[4 * part + t] = (int)__builtin_amdgcn_perm(lut8[fm], lut8[fm], (src >> (2 * t)) & 0x03030303u);
      }
    };
    // FP16 hi + FP8 lo with WMF = 2: the 2-bit fields of a code dword spread
    // one per byte, Y[d] = (src >> 2d) & 0x03030303 for d = 0..3, are the e4m3
    // table selectors as they stand and, paired byte by byte with Y + 0x04040404
    // by one v_perm_b32, the FP16 table selectors; both decodes share one field
    // extraction.  Y of the first code dword (K16 steps 0, 1) is made at the
    // previous chunk's step 3, that of the second (steps 2, 3) at step 0.
    auto spread = [&](const uint2* src2, int p, uint32_t (*Y)[4]) {
#pragma unroll
      for (int fm = 0; fm < WMF; ++fm) {
        const uint32_t src = p ? src2[fm].y : src2[fm].x;
#pragma unroll
        for (int d = 0; d < 4; ++d) Y[fm][d] = (src >> (2 * d)) & 0x03030303u;
      }
    };
    // step j (of the dword that Y spreads): samples t = 4 (j & 1) + d and t + 8
    // sit in bytes (j & 1) and 2 + (j & 1) of Y[d]
    auto decode_y = [&](const uint32_t (*Y)[4], int j, u32x4* A) {
#pragma unroll
      for (int fm = 0; fm < WMF; ++fm)
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const uint32_t y = Y[fm][d];
          const uint32_t sel = __builtin_amdgcn_perm(y + 0x04040404u, y, (j & 1) ? 0x07030501u : 0x06020400u);
          A[fm][d] = __builtin_amdgcn_perm(lut[fm].y, lut[fm].x, sel);
        }
    };
    auto decode8_y = [&](const uint32_t (*Y0)[4], const uint32_t (*Y1)[4], int fm, i32x8& A8) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        A8[k] = (int)__builtin_amdgcn_perm(lut8[fm], lut8[fm], Y0[fm][k]);
        A8[4 + k] = (int)__builtin_amdgcn_perm(lut8[fm], lut8[fm], Y1[fm][k]);
      }
    };
    auto read_b = [&](int st, int j, u32x4* bh, u32x4* bl) {
      const char* tile = smem + st * STAGE_BYTES;
#pragma unroll
      for (int fn = 0; fn < WN; ++fn) {
        bh[fn] = *(const u32x4*)(tile + fn * BB + (j * 512 + lane * 8) * 2);
        if constexpr (!F8) bl[fn] = *(const u32x4*)(tile + fn * BB + (2048 + j * 512 + lane * 8) * 2);
      }
    };
    auto read_b8_one = [&](int st, int fn, i32x8& B8f) {
      const char* tile = smem + st * STAGE_BYTES;
      const u32x4 p0 = *(const u32x4*)(tile + fn * BB + 4096 + lane * 16);
      const u32x4 p1 = *(const u32x4*)(tile + fn * BB + 4096 + 1024 + lane * 16);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        B8f[t] = (int)p0[t];
        B8f[4 + t] = (int)p1[t];
      }
    };
    auto read_b8 = [&](int st, i32x8* B8) {
#pragma unroll
      for (int fn = 0; fn < WN; ++fn) read_b8_one(st, fn, B8[fn]);
    };
    // 8-bit dosages, FP16 + FP8 form: the FP16 values of K16 step s (as
    // decode_g8 leaves them, dword d holds samples 16 (s >> 1) + 4 (s & 1) + d
    // and that + 8 of this lane half) converted to e4m3 in the lo operand's
    // layout, where dword 4 p + t holds sample 16 p + 4 k + t in byte k.  Step
    // 2p writes bytes 0 and 1 of dword 4p + d (k = 0 and 2), step 2p + 1 bytes
    // 2 and 3 (k = 1 and 3); one byte permutation then puts k in byte k.
    auto cvt8 = [&](const u32x4* Av, int s, i32x8* A8v) {
      const int p = s >> 1;
#pragma unroll
      for (int fm = 0; fm < WMF; ++fm)
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          uint32_t w = (uint32_t)A8v[fm][4 * p + d];
          if (s & 1) {
            w = cvt_pk_e4m3_hi(w, Av[fm][d]);
            w = __builtin_amdgcn_perm(w, w, 0x03010200u);
          } else {
            w = cvt_pk_e4m3_lo(w, Av[fm][d]);
          }
          A8v[fm][4 * p + d] = (int)w;
        }
    };

    // prologue: chunks 0..NSTAGE-1 requested, chunk 0 awaited
#pragma unroll
    for (int c = 0; c < NSTAGE; ++c) dma(c, c);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    u32x4 bh[2][WN], bl[2][WN], A[2][WMF];
    i32x8 A8[GF ? WMF : 2], B8[WN];
    uint2 acur[WMF], anext[WMF];
    u32x4 araw[WMF];  // FP8 form: the next chunk's code rows, read a step early
    constexpr bool SY = F8 && W2 && !G8;  // shared selectors (spread / decode_y / decode8_y)
    uint32_t Y0[SY ? WMF : 1][4], Y1[SY ? WMF : 1][4];  // selectors of the first / second code dword
    uint2 dg8[WMF];  // 8-bit dosages: the two dwords of the step being decoded
    if constexpr (G8) {
      read_b(0, 0, bh[0], bl[0]);
      read_g8(0, 0, dg8);
      decode_g8(dg8, A[0]);
    } else {
      read_a(0, acur);
      read_b(0, 0, bh[0], bl[0]);
    }
    if constexpr (SY) {
      spread(acur, 0, Y0);
      decode_y(Y0, 0, A[0]);
    } else if constexpr (!G8) {
      decode(acur, 0, A[0]);
    }
    if constexpr (F8 && !W2 && !G8) decode8(acur, 0, A8[0]);
    if constexpr (GF) {
#pragma unroll
      for (int fm = 0; fm < WMF; ++fm)
#pragma unroll
        for (int i = 0; i < 8; ++i) A8[fm][i] = 0;
      cvt8(A[0], 0, A8);
    }

    // the prologue's reads are complete before the loop; saying so keeps
    // the compiler from waiting for all LDS reads at the loop head
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), vmcnt and expcnt unconstrained

    int st = 0;  // stage of chunk ch
    for (int ch = 0; ch < nch; ++ch) {
      const int st1 = st + 1 < NSTAGE ? st + 1 : 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int cs = j & 1, ns = cs ^ 1;
        if constexpr (F8 && !W2 && !G8) {
          if (j == 0) read_b8(st, B8);  // this chunk's lo fragments, used by all four steps
        }
        if constexpr (GF) {
          if (j == 3) {
            // the chunk's FP8 lo term, every fragment against every column
            // block (its e4m3 operand was completed at step 2), before the
            // barrier after which the stage is refilled
#pragma unroll
            for (int fn = 0; fn < WN; ++fn) {
              i32x8 b8;
              read_b8_one(st, fn, b8);
#pragma unroll
              for (int fm = 0; fm < WMF; ++fm)
                acc[fm][fn] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A8[fm], b8, acc[fm][fn], 0, 0, 0, 127,
                                                                              0, bscale[fn]);
            }
          }
        }
        if constexpr (F8 && W2 && !G8) {
#pragma unroll
          for (int q = 0; q < FNS; ++q) read_b8_one(st, j * FNS + q, B8[j * FNS + q]);  // used by this step
          if (j == 0) {
            spread(acur, 1, Y1);
#pragma unroll
            for (int fm = 0; fm < WMF; ++fm) decode8_y(Y0, Y1, fm, A8[fm]);  // both fragments, whole chunk
          }
        }
        if (F8 && !G8 && j == 2) {
          // the next chunk's codes are this wave's own copies: they need
          // only its own copy of chunk ch+1 to have landed, not the barrier
          __builtin_amdgcn_s_waitcnt(waitcnt_vm_only((NSTAGE - 2) * CHUNK_OPS));
          read_a_raw(st1, araw);  // this lane's halves are picked at step 3
        }
        if (j < 3) {
          read_b(st, j + 1, bh[ns], bl[ns]);
          if constexpr (G8) {
            read_g8(st, j + 1, dg8);
            decode_g8(dg8, A[ns]);
            if constexpr (GF) cvt8(A[ns], j + 1, A8);
          } else if constexpr (SY) {
            decode_y(j + 1 < 2 ? Y0 : Y1, j + 1, A[ns]);
          } else {
            decode(acur, j + 1, A[ns]);
          }
        } else {
          // own copies of chunk ch+1 done (the NSTAGE-2 later chunks may
          // still be in flight) and own LDS reads of this chunk done; then
          // every wave's (a plain s_barrier: a workgroup fence here would
          // wait for every copy in flight)
          __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0((NSTAGE - 2) * CHUNK_OPS));
          if constexpr (!F8 && !G8) read_a(st1, anext);  // this wave's own copies: no barrier needed
          if constexpr (F8 && !G8) pick_a(araw, anext);
          asm volatile("s_barrier" ::: "memory");
          // LDS reads before the copies: a read issued after a
          // direct-to-LDS load is held until that load completes
          read_b(st1, 0, bh[ns], bl[ns]);
          if constexpr (G8) read_g8(st1, 0, dg8);  // own copies of chunk ch + 1 have landed
          if constexpr (!F8 || G8) dma(ch + NSTAGE, st);  // the 2-bit FP8 form copies beside its lo MFMAs
          if constexpr (G8) {
            decode_g8(dg8, A[ns]);
          } else if constexpr (SY) {
            spread(anext, 0, Y0);
            decode_y(Y0, 0, A[ns]);
          } else {
            decode(anext, 0, A[ns]);
          }
        }
#pragma unroll
        for (int fn = 0; fn < WN; ++fn)
#pragma unroll
          for (int fm = 0; fm < WMF; ++fm) acc[fm][fn] = mfma16<PREC>(A[cs][fm], bh[cs][fn], acc[fm][fn]);
        if constexpr (!F8) {
#pragma unroll
          for (int fn = 0; fn < WN; ++fn)
#pragma unroll
            for (int fm = 0; fm < WMF; ++fm) acc[fm][fn] = mfma16<PREC>(A[cs][fm], bl[cs][fn], acc[fm][fn]);
        }
        // issue order: copies and LDS reads early, each behind one
        // matrix-core instruction, then the decode, a few VALU ops per MFMA
        if (GF) {
          // 8-bit dosages, FP16 + FP8: no group hints
        } else if (F8 && W2) {  // WMF x WN FP16 MFMA; WN hi + 2 FNS lo fragment reads (+ code rows at step 2)
          constexpr int NDS = W2 ? WN + 2 * FNS : 0;
#pragma unroll
          for (int q = 0; q < NDS; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);  // VALU
          }
#pragma unroll
          for (int q = 0; q < HI_MFMA - NDS; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);  // VALU
          }
        } else if (j == 3 && F8) {
#pragma unroll
          for (int q = 0; q < DS_STEP; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);  // VALU
          }
#pragma unroll
          for (int q = 0; q < HI_MFMA - DS_STEP; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);  // VALU
          }
        } else if (j == 3) {
#pragma unroll
          for (int q = 0; q < DS_STEP + WMF; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
          }
#pragma unroll
          for (int q = 0; q < CHUNK_OPS; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);  // VMEM (direct-to-LDS)
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);  // VALU
          }
#pragma unroll
          for (int q = 0; q < HI_MFMA - CHUNK_OPS - DS_STEP - WMF; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);  // VALU
          }
        } else {
          if (F8 && j == 0) {  // plus the chunk's lo fragment reads
#pragma unroll
            for (int q = 0; q < 3 * WN; ++q) {
              __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
              __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);  // VALU
            }
#pragma unroll
            for (int q = 0; q < HI_MFMA - 3 * WN; ++q) {
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
              __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);  // VALU
            }
          } else {
            constexpr int VPD = F8 ? 3 : 0, VREST = F8 ? 5 : 3;
#pragma unroll
            for (int q = 0; q < DS_STEP; ++q) {
              __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
              if (VPD) __builtin_amdgcn_sched_group_barrier(0x002, VPD, 0);  // VALU
            }
#pragma unroll
            for (int q = 0; q < HI_MFMA - DS_STEP; ++q) {
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
              __builtin_amdgcn_sched_group_barrier(0x002, VREST, 0);  // VALU
            }
          }
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (GF) {
          if (j == 3) cvt8(A[ns], 0, A8);  // the next chunk's first step (after the lo MFMAs that read A8)
        }
        if constexpr (F8 && W2 && !G8) {
          // FP8 lo term of column blocks j FNS .. (j + 1) FNS - 1, both fragments, whole chunk
          if (j == 3) dma(ch + NSTAGE, st);  // the stage of chunk ch is free since the barrier
#pragma unroll
          for (int q = 0; q < FNS; ++q) {
            const int fn = j * FNS + q;
#pragma unroll
            for (int fm = 0; fm < WMF; ++fm)
              acc[fm][fn] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A8[fm], B8[fn], acc[fm][fn], 0, 0, 0,
                                                                            127, 0, bscale[fn]);
          }
          if (j == 3) {
#pragma unroll
            for (int q = 0; q < WMF * FNS; ++q) {
              __builtin_amdgcn_sched_group_barrier(0x010, (CHUNK_OPS + WMF * FNS - 1) / (WMF * FNS), 0);  // VMEM
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                                       // MFMA
              __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);                                       // VALU
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (F8 && !W2 && !G8) {
          // FP8 lo term of fragment fm = j over the whole chunk, after the
          // step's FP16 work (its operands were read at step 0); the decode
          // of the next fragment's e4m3 values rides along
          if (j < 3) {
            decode8(acur, j + 1, A8[ns]);
          } else {
            dma(ch + NSTAGE, st);  // the stage of chunk ch is free since the barrier
            decode8(anext, 0, A8[ns]);
          }
#pragma unroll
          for (int fn = 0; fn < WN; ++fn)
            acc[j][fn] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A8[cs], B8[fn], acc[j][fn], 0, 0, 0, 127,
                                                                         0, bscale[fn]);
          if (j == 3) {
#pragma unroll
            for (int q = 0; q < WN; ++q) {
              __builtin_amdgcn_sched_group_barrier(0x010, CHUNK_OPS / WN, 0);  // VMEM (direct-to-LDS)
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);               // MFMA
              __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);              // VALU
            }
          } else {
#pragma unroll
            for (int q = 0; q < WN; ++q) {
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
              __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);  // VALU
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
#pragma unroll
      for (int fm = 0; fm < WMF; ++fm) acur[fm] = anext[fm];
      st = st1;
      // the next chunk's first fragments landed long ago; saying so here
      // keeps the compiler from waiting for all LDS reads at the loop head
      __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), vmcnt and expcnt unconstrained
    }
    __builtin_amdgcn_s_waitcnt(0);  // surplus copies have landed
    __syncthreads();                // all waves are done with the stages

    if constexpr (MODE == kRaw) {
#pragma unroll
      for (int fn = 0; fn < WN; ++fn) {
        const int cb = ctile * WN + fn;
        if (cb >= a.n_cblocks) continue;
        const ColBlock blk = a.cblocks[cb];
        if (r32 >= blk.ncol) continue;
#pragma unroll
        for (int fm = 0; fm < WMF; ++fm)
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int64_t mr = rowbase + fm * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
            if (mr < a.nm) gstore(a.raw_out + mr * a.raw_ld + blk.col0 + r32, acc[fm][fn][i]);
          }
      }
    } else {
      // this lane's column values of each block, read ahead of the stores
      float cinv[WN], csp[WN];
#pragma unroll
      for (int fn = 0; fn < WN; ++fn) {
        const int cb = ctile * WN + fn;
        const ColBlock blk = a.cblocks[cb < a.n_cblocks ? cb : ctile * WN];
        const PanelDev& pdb = a.panels[blk.panel];
        const bool colok = cb < a.n_cblocks && r32 < blk.ncol;
        cinv[fn] = colok ? gload<float>(pdb.invny + blk.col0 + r32) : 0.f;
        csp[fn] = colok ? gload<float>(pdb.scale + blk.col0 + r32) * a.gunit : 0.f;
      }
      // the wave's rows' 1/||g_res|| for panel j, one or two rows per lane
      float2* ihl = (float2*)(smem + LDS_BYTES) + __builtin_amdgcn_readfirstlane(wave) * (WMF * 32);
      auto load_rows = [&](int j) {
#pragma unroll
        for (int k = 0; k < WMF / 2; ++k) {
          int64_t mr = rowbase + 64 * k + lane;
          mr = mr < a.nm ? mr : a.nm - 1;
          ihl[64 * k + lane] = gload<float2>(a.invh + mr * a.n_panels + j);
        }
      };
      // panel j's table into LDS (all threads; the caller brackets it with barriers)
      auto load_table = [&](int j) {
        tab4* tl = (tab4*)(smem + LDS_BYTES + IH_BYTES);
        const tab4* tg = (const tab4*)a.panels[j].table;
        for (int k = tid; k < kTabIntervals; k += NT) tl[k] = gload<tab4>(tg + k);
      };
      int ih_panel = a.cblocks[ctile * WN].panel;
      load_rows(ih_panel);
      if constexpr (LT) {
        if (ih_panel != tab_panel) {  // the last tile's epilogue ended at the barrier below
          load_table(ih_panel);
          tab_panel = ih_panel;
          __syncthreads();
        }
      }
      // projection correction (see gemm_kernel)
#pragma unroll
      for (int fn = 0; fn < WN; ++fn) {
        const int cb = ctile * WN + fn;
        const ColBlock blk = a.cblocks[cb < a.n_cblocks ? cb : ctile * WN];
        const float* cwp = a.panels[blk.panel].cw + (int64_t)(blk.col0 + r32) * kSlots + 8 * h;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          const float4 c0 = gload<float4>(cwp + 16 * ks);
          const float4 c1 = gload<float4>(cwp + 16 * ks + 4);
          u32x4 bo;
          bo[0] = pack_bf16x2(c0.x, c0.y);
          bo[1] = pack_bf16x2(c0.z, c0.w);
          bo[2] = pack_bf16x2(c1.x, c1.y);
          bo[3] = pack_bf16x2(c1.z, c1.w);
          const bf16x8 B = __builtin_bit_cast(bf16x8, bo);
#pragma unroll
          for (int fm = 0; fm < WMF; ++fm) {
            int64_t mr = rowbase + fm * 32 + r32;
            mr = mr < a.nm ? mr : a.nm - 1;
            const float* wp = a.wws + (mr * a.n_panels + blk.panel) * kSlots + 16 * ks + 8 * h;
            const float4 w0 = gload<float4>(wp);
            const float4 w1 = gload<float4>(wp + 4);
            u32x4 ao;
            ao[0] = pack_bf16x2(w0.x, w0.y);
            ao[1] = pack_bf16x2(w0.z, w0.w);
            ao[2] = pack_bf16x2(w1.x, w1.y);
            ao[3] = pack_bf16x2(w1.z, w1.w);
            acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ao), B,
                                                                  acc[fm][fn], 0, 0, 0);
          }
        }
      }
      // SB column blocks are staged at once (as many as the stages hold), so
      // that their accumulators are dead before the row loops run
      constexpr int SB = LDS_BYTES / (NW * WMF * 32 * 32 * 4) < WN ? LDS_BYTES / (NW * WMF * 32 * 32 * 4) : WN;
      static_assert(SB >= 1 && WN % SB == 0, "staged column blocks");
      const int wv = __builtin_amdgcn_readfirstlane(wave);  // uniform: LDS bases in scalar registers
      float* stage = (float*)smem + wv * (SB * WMF * 32 * 32);
#pragma unroll
      for (int f0 = 0; f0 < WN; f0 += SB) {
        if (ctile * WN + f0 >= a.n_cblocks) break;
#pragma unroll
        for (int s = 0; s < SB; ++s)
#pragma unroll
          for (int fm = 0; fm < WMF; ++fm)
#pragma unroll
            for (int i = 0; i < 16; ++i)
              stage[(s * WMF * 32 + fm * 32 + 8 * (i >> 2) + 4 * h + (i & 3)) * 32 + r32] = acc[fm][f0 + s][i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int s = 0; s < SB; ++s) {
          const int fn = f0 + s;
          const int cb = ctile * WN + fn;
          if (cb >= a.n_cblocks) break;
          const ColBlock blk = a.cblocks[cb];
          if (blk.panel != ih_panel) {  // a column tile across a panel boundary
            ih_panel = blk.panel;
            load_rows(ih_panel);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          }
          if constexpr (LT) {
            if (blk.panel != tab_panel) {
              __syncthreads();
              load_table(blk.panel);
              tab_panel = blk.panel;
              __syncthreads();
            }
          }
          const float* sb = stage + s * (WMF * 32 * 32);
          const LdsRows ihr = (LdsRows)ihl;
          if constexpr (LT)
            finish_block<WMF>(sb, a, blk, rowbase, h, r32, (LdsTable)(smem + LDS_BYTES + IH_BYTES), ihr, cinv[fn],
                              csp[fn]);
          else
            finish_block<WMF>(sb, a, blk, rowbase, h, r32, (const tab4*)a.panels[blk.panel].table, ihr, cinv[fn],
                              csp[fn]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __syncthreads();  // the next tile's prologue overwrites the staging area
  }
}

// ---------------------------------------------------------------------------
// tile shapes and launchers
// ---------------------------------------------------------------------------
// {waves, 32-row fragments per wave, 32-column blocks per tile}
static const TileShape kShapes[] = {
    {4, 4, 4},  // 0: 512 x 128, wide, one wave per SIMD (split forms)
    {8, 2, 4},  // 1: 512 x 128, wide, two waves per SIMD (split forms)
    {8, 2, 4},  // 2: 512 x 128
    {4, 2, 4},  // 3: 256 x 128
    {8, 1, 4},  // 4: 256 x 128, 8 waves
    {8, 2, 2},  // 5: 512 x 64
    {4, 2, 8},  // 6: 256 x 256, wide, one wave per SIMD (FP8 lo form; others run shape 0)
    {8, 1, 1},  // 7: 256 x 32 (Q^T g contraction)
};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
constexpr int kWShape = 7;

int n_tile_shapes() { return kNumShapes - 1; }
TileShape tile_shape(int idx) { return kShapes[idx]; }
int wgemm_tile() { return kWShape; }

template <int PREC, int MODE>
static const void* gemm_fn_g8(int idx) {  // 8-bit dosages: wide tiles 0 and 1 for the FP16 splits
  if constexpr (PREC == kSplit16 || PREC == kSplit8) {
    if (idx == 1) return (const void*)gemm_wide_kernel<PREC, MODE, 8, 2, 4, true>;
    if (idx == 0 || PREC == kSplit8) return (const void*)gemm_wide_kernel<PREC, MODE, 4, 4, 4, true>;
  }
  if constexpr (PREC == kFP32 || PREC == kSplit16) {  // the register-staged shapes
    switch (idx) {
      case 3: return (const void*)gemm_kernel<PREC, 4, 2, 4, MODE, true>;
      case 4: return (const void*)gemm_kernel<PREC, 8, 1, 4, MODE, true>;
      case 5: return (const void*)gemm_kernel<PREC, 8, 2, 2, MODE, true>;
      case kWShape: return (const void*)gemm_kernel<PREC, 8, 1, 1, MODE, true>;
      default: return (const void*)gemm_kernel<PREC, 8, 2, 4, MODE, true>;
    }
  }
  return nullptr;
}

template <int PREC, int MODE>
static const void* gemm_fn(int idx) {
  if constexpr (PREC == kSplit8) {  // the FP8 lo form exists only as the wide kernel
    if (idx == 1) return (const void*)gemm_wide_kernel<PREC, MODE, 8, 2>;
    if (idx == 6) return (const void*)gemm_wide_kernel<PREC, MODE, 4, 2, 8>;
    return (const void*)gemm_wide_kernel<PREC, MODE, 4, 4>;
  } else {
    switch (idx) {
      case 0:  // the wide kernels exist for the split forms; FP32 uses shape 2
        if constexpr (PREC != kFP32) return (const void*)gemm_wide_kernel<PREC, MODE, 4, 4>;
        return (const void*)gemm_kernel<PREC, 8, 2, 4, MODE>;
      case 1:
        if constexpr (PREC != kFP32) return (const void*)gemm_wide_kernel<PREC, MODE, 8, 2>;
        return (const void*)gemm_kernel<PREC, 8, 2, 4, MODE>;
      case 2: return (const void*)gemm_kernel<PREC, 8, 2, 4, MODE>;
      case 3: return (const void*)gemm_kernel<PREC, 4, 2, 4, MODE>;
      case 4: return (const void*)gemm_kernel<PREC, 8, 1, 4, MODE>;
      case 5: return (const void*)gemm_kernel<PREC, 8, 2, 2, MODE>;
      case 6:  // the 256 x 256 wide shape exists for the FP8 lo form only
        if constexpr (PREC != kFP32) return (const void*)gemm_wide_kernel<PREC, MODE, 4, 4>;
        return (const void*)gemm_kernel<PREC, 8, 2, 4, MODE>;
      case kWShape: return (const void*)gemm_kernel<PREC, 8, 1, 1, MODE>;
    }
    return nullptr;
  }
}

static TileShape effective_shape(int idx, int prec, bool g8 = false) {
  const bool wide = idx <= 1 || idx == 6;
  if (g8 && prec == kSplit8) return kShapes[idx == 1 ? 1 : 0];
  if (g8 && prec == kSplit16 && idx <= 1) return kShapes[idx];
  if (g8) return kShapes[wide ? 2 : idx];
  if (prec == kSplit8) return kShapes[(idx == 1 || idx == 6) ? idx : 0];
  if (wide && prec == kFP32) return kShapes[2];
  if (idx == 6) return kShapes[0];
  return kShapes[idx];
}
TileShape tile_shape_for(int idx, int prec, bool g8) { return effective_shape(idx, prec, g8); }

static const void* gemm_fn_any(int idx, int prec, int mode, bool g8 = false) {
  if (mode == kRawHL) {  // the Q^T g shape with the packed hi|lo covariate operand
    if (idx != kWShape) return nullptr;
    if (prec == kSplit16)
      return g8 ? (const void*)gemm_kernel<kSplit16, 8, 1, 1, kRawHL, true>
                : (const void*)gemm_kernel<kSplit16, 8, 1, 1, kRawHL>;
    if (prec == kSplit && !g8) return (const void*)gemm_kernel<kSplit, 8, 1, 1, kRawHL>;
    return nullptr;
  }
  if (g8) {
    if (prec == kSplit16) return mode == kRaw ? gemm_fn_g8<kSplit16, kRaw>(idx) : gemm_fn_g8<kSplit16, kTest>(idx);
    if (prec == kFP32) return mode == kRaw ? gemm_fn_g8<kFP32, kRaw>(idx) : gemm_fn_g8<kFP32, kTest>(idx);
    if (prec == kSplit8) return mode == kRaw ? gemm_fn_g8<kSplit8, kRaw>(idx) : gemm_fn_g8<kSplit8, kTest>(idx);
    return nullptr;
  }
  if (prec == kSplit) return mode == kRaw ? gemm_fn<kSplit, kRaw>(idx) : gemm_fn<kSplit, kTest>(idx);
  if (prec == kSplit16) return mode == kRaw ? gemm_fn<kSplit16, kRaw>(idx) : gemm_fn<kSplit16, kTest>(idx);
  if (prec == kSplit8) return mode == kRaw ? gemm_fn<kSplit8, kRaw>(idx) : gemm_fn<kSplit8, kTest>(idx);
  return mode == kRaw ? gemm_fn<kFP32, kRaw>(idx) : gemm_fn<kFP32, kTest>(idx);
}

int tile_alias(int idx, int prec, bool g8) {
  const void* fn = gemm_fn_any(idx, prec, kTest, g8);
  for (int i = 0; i < idx; ++i)
    if (gemm_fn_any(i, prec, kTest, g8) == fn) return i;
  return idx;
}

int gemm_grid(int idx, int prec, int mode, int n_cu, bool g8) {
  const void* fn = gemm_fn_any(idx, prec, mode, g8);
  if (!fn) return 8;
  int occ = 0;
  const int threads = effective_shape(idx, prec, g8).waves * 64;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, threads, 0) != hipSuccess || occ < 1) occ = 1;
  int g = occ * n_cu;
  g = (g / 8) * 8;
  return g < 8 ? 8 : g;
}

hipError_t launch_gemm(int idx, int prec, int mode, const GemmArgs& a, int grid, hipStream_t s, bool g8) {
  const void* fn = gemm_fn_any(idx, prec, mode, g8);
  if (!fn) return hipErrorInvalidValue;
  const int threads = effective_shape(idx, prec, g8).waves * 64;
  GemmArgs arg = a;
  void* params[] = {&arg};
  return hipLaunchKernel(fn, dim3(grid), dim3(threads), params, 0, s);
}

hipError_t launch_qr(const double* C, int64_t ldc, int64_t n, int64_t n_pad, int q, double* X, double* Q,
                     double* rdiag, double* scratch, int32_t* flags, hipStream_t s) {
  if (q < 1 || q > kSlots) return hipErrorInvalidValue;
  double* part = scratch;
  double* fv = scratch + kQrGrid * kSlots;
  double* vtv = fv + kSlots;
  const dim3 g(kQrGrid), b(kQrThreads);
  hipLaunchKernelGGL(qr_load_kernel, g, b, 0, s, C, ldc, n, n_pad, q, X, flags);
  for (int j = 0; j < q; ++j) {
    const double* xj = X + (int64_t)j * n_pad;
    hipLaunchKernelGGL(qr_dots_kernel, g, b, 0, s, xj, (const double*)X, n, n_pad, q, j, (int64_t)j + 1, part);
    hipLaunchKernelGGL(qr_coef_kernel, dim3(1), b, 0, s, X, n_pad, q, j, 1, (const double*)part, rdiag, fv, vtv);
    if (j + 1 < q) hipLaunchKernelGGL(qr_reflect_kernel, g, b, 0, s, xj, X, n, n_pad, q, j + 1, (int64_t)j, (const double*)fv);
  }
  hipLaunchKernelGGL(qr_qinit_kernel, g, b, 0, s, Q, n_pad, q);
  for (int j = q - 1; j >= 0; --j) {
    const double* xj = X + (int64_t)j * n_pad;
    hipLaunchKernelGGL(qr_dots_kernel, g, b, 0, s, xj, (const double*)Q, n, n_pad, q, j, (int64_t)j, part);
    hipLaunchKernelGGL(qr_coef_kernel, dim3(1), b, 0, s, X, n_pad, q, j, 0, (const double*)part, rdiag, fv, vtv);
    hipLaunchKernelGGL(qr_reflect_kernel, g, b, 0, s, xj, Q, n, n_pad, q, j, (int64_t)j, (const double*)fv);
  }
  hipLaunchKernelGGL(qr_rank_kernel, dim3(1), dim3(64), 0, s, (const double*)rdiag, q, flags);
  return hipGetLastError();
}

hipError_t launch_cov_operands(const double* Q, int64_t n, int64_t n_pad, int q, void* wop_fp32,
                               void* const* wop_hl, hipStream_t s) {
  if (!wop_fp32 || !wop_hl[kSplit] || !wop_hl[kSplit16]) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cov_operand_kernel, dim3(256), dim3(256), 0, s, Q, n, n_pad, q, wop_fp32, wop_hl[kSplit],
                     wop_hl[kSplit16]);
  return hipGetLastError();
}

hipError_t launch_prep(const void* Y, int y_fp64, int64_t ldy, int64_t n, int64_t n_pad, int64_t P,
                       const double* Q, int q, int prec, void* yop, float* scale, float* invny, float* cw,
                       uint8_t* lscale, int32_t* flags, hipStream_t s) {
  // q <= QS slots; two columns per workgroup (at P = 2,048 and q = 11 this
  // beats four, which leaves two waves per SIMD, and one), one for q > 24
  auto go = [&](auto kern, int cpw) {
    hipLaunchKernelGGL(kern, dim3((unsigned)((P + cpw - 1) / cpw)), dim3(kPrepThreads), 0, s, Y, y_fp64, ldy, n,
                       n_pad, P, Q, q, prec, yop, scale, invny, cw, lscale, flags);
  };
  if (q <= 4)
    go(prep_kernel<4, 2>, 2);
  else if (q <= 8)
    go(prep_kernel<8, 2>, 2);
  else if (q <= 12)
    go(prep_kernel<12, 2>, 2);
  else if (q <= 16)
    go(prep_kernel<16, 2>, 2);
  else if (q <= 24)
    go(prep_kernel<24, 2>, 2);
  else
    go(prep_kernel<kSlots, 1>, 1);
  return hipGetLastError();
}

hipError_t launch_set_operand(const float* V, int64_t ldv, int64_t n, int64_t n_pad, int64_t P, int prec,
                              void* yop, uint8_t* lscale, hipStream_t s) {
  if (prec == kSplit8) {
    hipLaunchKernelGGL(set_lscale_kernel, dim3((unsigned)P), dim3(kPrepThreads), 0, s, V, ldv, n, lscale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(set_operand_kernel, dim3(1024), dim3(256), 0, s, V, ldv, n, n_pad, P, prec, yop,
                     (const uint8_t*)lscale);
  return hipGetLastError();
}

hipError_t launch_table(float4* table, double df, hipStream_t s) {
  hipLaunchKernelGGL(table_kernel, dim3((kTabIntervals + 255) / 256), dim3(256), 0, s, table, df);
  return hipGetLastError();
}

hipError_t launch_stats(const StatsArgs& a, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.nm + 3) / 4);
  hipLaunchKernelGGL(stats_kernel, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finalize(const MarkerStat* ms, float* wws, float2* invh, int64_t nm, int n_panels, float wscale,
                           int lo_slot, RedoDev redo, hipStream_t s) {
  const int64_t total = nm * n_panels;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, ms, wws, invh, nm,
                     n_panels, wscale, lo_slot, redo);
  return hipGetLastError();
}

__global__ void topk_read_kernel(const unsigned long long* __restrict__ words, int64_t n, double df,
                                 float* __restrict__ nl, int64_t* __restrict__ marker) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long w = words[i];
    if (w == 0ull) {
      if (nl) nl[i] = __builtin_nanf("");
      if (marker) marker[i] = -1;
      continue;
    }
    const double at = (double)__uint_as_float((uint32_t)(w >> 32));
    if (nl) nl[i] = (float)(-ln_p_two_sided(at, df) / M_LN10);
    if (marker) marker[i] = (int64_t)(0xffffffffu - (uint32_t)w);
  }
}

hipError_t launch_topk_read(const unsigned long long* words, int64_t n, int k, double df, float* nl, int64_t* marker,
                            hipStream_t s) {
  (void)k;
  const int64_t blocks = std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(topk_read_kernel, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, s, words, n, df, nl,
                     marker);
  return hipGetLastError();
}

hipError_t launch_redo(const RedoArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(redo_kernel, dim3((unsigned)grid), dim3(kRedoThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bind(const BindArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(bind_kernel, dim3(1), dim3(kMaxPanelsPerBind), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_tail_reset(TailDev t, hipStream_t s) {
  hipLaunchKernelGGL(tail_reset_kernel, dim3(1), dim3(64), 0, s, t);
  return hipGetLastError();
}

hipError_t launch_tail(TailDev t, const PanelDev* panels, const OutDev* outs, HitDev hits, int64_t m_begin,
                       hipStream_t s) {
  hipLaunchKernelGGL(tail_kernel, dim3(64), dim3(64), 0, s, t, panels, outs, hits, m_begin);
  return hipGetLastError();
}

hipError_t launch_debug_stats(const MarkerStat* ms, int64_t nm, double* shift, double* mean, double* scale,
                              hipStream_t s) {
  hipLaunchKernelGGL(debug_stats_kernel, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, s, ms, nm, shift, mean,
                     scale);
  return hipGetLastError();
}

}  // namespace tgw
