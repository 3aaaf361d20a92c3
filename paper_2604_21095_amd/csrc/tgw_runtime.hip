// Host runtime behind the C ABI in include/tgw.h: handles, argument checks,
// workspace, the per-block launch sequence, autotuner and graph capture.
#include "tgw_host.h"
#include "tgw_internal.h"

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <sys/stat.h>
#include <vector>

using namespace tgw;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

tgw_status tgw::fail(tgw_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

tgw_status tgw::hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? TGW_ERR_OUT_OF_MEMORY : TGW_ERR_DEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// device properties
// ---------------------------------------------------------------------------
struct DevInfo {
  int n_cu = 0;
  std::string arch;
  bool gfx950 = false;
  char* scratch = nullptr;  // this device's copy of `scratch` (tgw_scan_static)
};

static std::mutex g_dev_mu;
static hipError_t static_scratch_address(char** p);  // with the device current
static std::map<int, DevInfo> g_dev;

static tgw_status device_info(int* dev_out, DevInfo* info) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_dev.find(dev);
  if (it == g_dev.end()) {
    hipDeviceProp_t p;
    HIP_TRY(hipGetDeviceProperties(&p, dev));
    DevInfo d;
    d.n_cu = p.multiProcessorCount;
    d.arch = p.gcnArchName;
    d.gfx950 = d.arch.rfind("gfx950", 0) == 0;
    if (d.gfx950) HIP_TRY(static_scratch_address(&d.scratch));
    it = g_dev.emplace(dev, d).first;
  }
  if (!it->second.gfx950)
    return fail(TGW_ERR_UNSUPPORTED, "device architecture " + it->second.arch + " is not gfx950");
  if (dev_out) *dev_out = dev;
  if (info) *info = it->second;
  return TGW_OK;
}

// the current device's CU count and static scratch, without copying DevInfo
static tgw_status device_basics(int* dev, int* n_cu, char** scratch) {
  tgw_status st = device_info(dev, nullptr);
  if (st != TGW_OK) return st;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  const DevInfo& d = g_dev.find(*dev)->second;
  *n_cu = d.n_cu;
  *scratch = d.scratch;
  return TGW_OK;
}

static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------
static std::mutex g_alloc_mu;
static DevAllocator g_alloc;

DevAllocator tgw::current_allocator() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc;
}

hipError_t tgw::dev_alloc(const DevAllocator& a, void** p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  if (bytes == 0) bytes = 1;
  if (!a.alloc) return hipMalloc(p, bytes);
  *p = a.alloc(bytes, (void*)s, a.ctx);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

void tgw::dev_free(const DevAllocator& a, void* p, hipStream_t s) {
  if (!p) return;
  if (!a.free) {
    (void)hipFree(p);
    return;
  }
  a.free(p, (void*)s, a.ctx);
}

void tgw::dev_release_begin(const DevAllocator& a) {
  if (a.free) (void)hipDeviceSynchronize();
}

extern "C" tgw_status tgw_set_allocator(tgw_alloc_fn alloc_fn, tgw_free_fn free_fn, void* ctx) {
  if ((alloc_fn == nullptr) != (free_fn == nullptr))
    return fail(TGW_ERR_INVALID_ARG, "give both allocator functions or neither");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc.alloc = alloc_fn;
  g_alloc.free = free_fn;
  g_alloc.ctx = alloc_fn ? ctx : nullptr;
  return TGW_OK;
}

extern "C" void* tgw_debug_counting_alloc(size_t bytes, void* stream, void* ctx) {
  (void)stream;
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  auto* c = (tgw_debug_alloc_counts*)ctx;
  __atomic_add_fetch(&c->n_alloc, 1, __ATOMIC_RELAXED);
  __atomic_add_fetch(&c->bytes, (int64_t)bytes, __ATOMIC_RELAXED);
  return p;
}

extern "C" void tgw_debug_counting_free(void* ptr, void* stream, void* ctx) {
  (void)stream;
  (void)hipFree(ptr);
  __atomic_add_fetch(&((tgw_debug_alloc_counts*)ctx)->n_free, 1, __ATOMIC_RELAXED);
}

template <class T>
static hipError_t dmalloc(const DevAllocator& a, T** p, size_t count, hipStream_t s = nullptr) {
  void* v = nullptr;
  const hipError_t e = dev_alloc(a, &v, (count ? count : 1) * sizeof(T), s);
  *p = (T*)v;
  return e;
}

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct tgw_covariates {
  DevAllocator mem;
  int device = 0;
  int64_t n = 0, n_pad = 0;
  int q = 0, n_chunks = 0;
  double* Q = nullptr;       // [q][n_pad]
  void* wop_fp32 = nullptr;     // Q^T g operand block of the FP32 form
  void* wop_hl[kNumPrec] = {};  // packed hi|lo Q^T g blocks of the split forms (hl_blocks(q) of them; the
                                // FP8 form uses the FP16 split's)
};

struct tgw_panel {
  DevAllocator mem;
  const tgw_covariates* cov = nullptr;
  int64_t P = 0, P_pad = 0;
  int prec = 0;
  int64_t df = 0;
  void* yop = nullptr;
  float* scale = nullptr;
  float* invny = nullptr;
  float* cw = nullptr;
  float4* table = nullptr;
  uint8_t* lscale = nullptr;  // FP8 lo form: E8M0 scale per column
  PanelDev* d_dev = nullptr;  // its PanelDev on the device (tables of tgw_scan_static)
};

// the per-panel constants the kernels read
static PanelDev panel_dev(const tgw_panel* p) {
  PanelDev d{};
  d.scale = p->scale;
  d.invny = p->invny;
  d.cw = p->cw;
  d.table = p->table;
  d.lscale = p->lscale;
  d.Q = p->cov->Q;
  d.yop = p->yop;
  d.wop = wprec(p->prec) != kFP32 ? p->cov->wop_hl[wprec(p->prec)] : p->cov->wop_fp32;
  d.n_pheno = p->P;
  d.df = (float)p->df;
  d.sqrt_df = (float)std::sqrt((double)p->df);
  d.inv_sqrt_df = (float)(1.0 / std::sqrt((double)p->df));
  d.q = p->cov->q;
  return d;
}

struct tgw_plan {
  DevAllocator mem;
  std::vector<const tgw_panel*> panels;
  int device = 0, prec = 0, n_cu = 0;
  std::string arch;
  int64_t n = 0, n_pad = 0;
  int n_chunks = 0, n_panels = 0, n_cb = 0;
  int64_t MB = 0;
  ColBlock* d_cb_main = nullptr;
  ColBlock* d_cb_w = nullptr;
  PanelDev* d_panels = nullptr;
  OutDev* d_outs = nullptr;
  uint4* mlut = nullptr;
  MarkerStat* mstat = nullptr;
  float* wws = nullptr;
  float2* invh = nullptr;
  int32_t* redo_entries = nullptr;  // FP64 list of covariate-collinear markers: [n_panels][MB]
  uint32_t* redo_count = nullptr;   // [n_panels]
  int max_chunks = 0;               // kRedoCols-column chunks of the widest panel
  TailEntry* tail_entries = nullptr;
  unsigned long long* tail_count = nullptr;
  int64_t tail_cap = 0;
  HitDev hits{};  // thresholded hit list of the following scans (entries NULL: off)
  int tile = 0;
  std::vector<int> grid_main;  // per tile shape
  int grid_w = 0;
  int w_mode = kRaw;  // kRawHL for the split forms (packed hi|lo covariate operand)
  int n_cb_w = 0;     // column blocks of the Q^T g contraction
  // 8-bit dosage rows (the FP32 and FP16 split forms): own tile choice and grids
  int tile8 = 2;
  // FP16 + FP8 form with q <= 31 in every panel: the FP8 lo pass centres on
  // the integer rint(c), its shift removed through the last correction slot
  bool lo_int = false;
  std::vector<int> grid_main8;
  int grid_w8 = 0;
  bool profile = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
};

struct tgw_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// ---------------------------------------------------------------------------
// library
// ---------------------------------------------------------------------------
extern "C" const char* tgw_status_string(tgw_status s) {
  switch (s) {
    case TGW_OK: return "ok";
    case TGW_ERR_INVALID_ARG: return "invalid argument";
    case TGW_ERR_SHAPE: return "inconsistent shape";
    case TGW_ERR_RANK_DEFICIENT: return "covariates rank deficient";
    case TGW_ERR_NONFINITE: return "non-finite input";
    case TGW_ERR_DEVICE: return "device error";
    case TGW_ERR_OUT_OF_MEMORY: return "out of memory";
    case TGW_ERR_UNSUPPORTED: return "unsupported";
    case TGW_ERR_TAIL_OVERFLOW: return "tail list overflow";
  }
  return "unknown status";
}

extern "C" const char* tgw_last_error(void) { return g_err.c_str(); }
extern "C" int32_t tgw_abi_version(void) { return TGW_ABI_VERSION; }

static void static_state_init(int dev);  // tgw_scan_static's per-device state

extern "C" tgw_status tgw_init(void) {
  TGW_GUARD_BEGIN
  int dev = 0;
  tgw_status st = device_info(&dev, nullptr);
  if (st == TGW_OK) static_state_init(dev);
  return st;
  TGW_GUARD_END
}

extern "C" tgw_status tgw_tile_shape(int32_t idx, int32_t* tile_markers, int32_t* tile_cols, int32_t* waves) {
  if (idx < 0 || idx >= n_tile_shapes()) return fail(TGW_ERR_INVALID_ARG, "tile index out of range");
  const TileShape s = tile_shape(idx);
  if (tile_markers) *tile_markers = s.tm();
  if (tile_cols) *tile_cols = s.tp();
  if (waves) *waves = s.waves;
  return TGW_OK;
}

// ---------------------------------------------------------------------------
// covariates
// ---------------------------------------------------------------------------
extern "C" void tgw_covariates_free(tgw_covariates* cov) {
  if (!cov) return;
  dev_release_begin(cov->mem);
  dev_free(cov->mem, cov->Q, nullptr);
  dev_free(cov->mem, cov->wop_fp32, nullptr);
  for (int k = 0; k < kNumPrec; ++k) dev_free(cov->mem, cov->wop_hl[k], nullptr);
  delete cov;
}

extern "C" tgw_status tgw_fit_covariates(int64_t n_samples, int32_t n_cov, const double* d_C, int64_t ldc,
                                         void* stream, tgw_covariates** out) {
  TGW_GUARD_BEGIN
  if (!out) return fail(TGW_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n_cov < 0 || n_cov > kMaxCov) return fail(TGW_ERR_SHAPE, "n_cov must be in [0, 31]");
  if (n_samples < (int64_t)n_cov + 3) return fail(TGW_ERR_SHAPE, "n_samples must be >= n_cov + 3");
  if (n_cov > 0 && !d_C) return fail(TGW_ERR_INVALID_ARG, "d_C is NULL");
  if (n_cov > 0 && ldc < n_samples) return fail(TGW_ERR_SHAPE, "ldc < n_samples");
  int dev;
  tgw_status st = device_info(&dev, nullptr);
  if (st != TGW_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  auto* cov = new tgw_covariates();
  cov->mem = current_allocator();
  cov->device = dev;
  cov->n = n_samples;
  cov->n_pad = round_up(n_samples, kChunk);
  cov->q = n_cov + 1;
  cov->n_chunks = (int)(cov->n_pad / kChunk);
  double *X = nullptr, *rdiag = nullptr, *qrs = nullptr;
  int32_t* flags = nullptr;
  const DevAllocator& A = cov->mem;
  auto cleanup = [&]() {  // after the stream has been synchronized
    dev_free(A, X, s);
    dev_free(A, rdiag, s);
    dev_free(A, qrs, s);
    dev_free(A, flags, s);
  };
  hipError_t e = dmalloc(A, &cov->Q, (size_t)cov->q * cov->n_pad, s);
  if (e == hipSuccess) e = dmalloc(A, &X, (size_t)cov->q * cov->n_pad, s);
  if (e == hipSuccess) e = dmalloc(A, &rdiag, (size_t)cov->q, s);
  if (e == hipSuccess) e = dmalloc(A, &qrs, (size_t)kQrScratch, s);
  if (e == hipSuccess) e = dmalloc(A, &flags, 2, s);
  if (e == hipSuccess) e = dev_alloc(A, &cov->wop_fp32, (size_t)cov->n_chunks * kBlockBytes, s);
  for (int k : {(int)kSplit, (int)kSplit16})
    if (e == hipSuccess) e = dev_alloc(A, &cov->wop_hl[k], (size_t)hl_blocks(cov->q) * cov->n_chunks * kBlockBytes, s);
  if (e == hipSuccess) e = hipMemsetAsync(flags, 0, 2 * sizeof(int32_t), s);
  if (e == hipSuccess) e = launch_qr(d_C, ldc, n_samples, cov->n_pad, cov->q, X, cov->Q, rdiag, qrs, flags, s);
  if (e == hipSuccess)
    e = launch_cov_operands(cov->Q, n_samples, cov->n_pad, cov->q, cov->wop_fp32, cov->wop_hl, s);
  int32_t hf[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) (void)hipStreamSynchronize(s);  // nothing enqueued may still use the temporaries
  cleanup();
  if (e != hipSuccess) {
    tgw_covariates_free(cov);
    return hip_fail(e, "tgw_fit_covariates");
  }
  if (hf[0]) {
    tgw_covariates_free(cov);
    return fail(TGW_ERR_NONFINITE, "covariates contain NaN or Inf");
  }
  if (hf[1]) {
    tgw_covariates_free(cov);
    return fail(TGW_ERR_RANK_DEFICIENT, "[1 | C] is rank deficient");
  }
  *out = cov;
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" tgw_status tgw_covariates_q(const tgw_covariates* cov, double* d_Q, int64_t ldq, void* stream) {
  TGW_GUARD_BEGIN
  if (!cov || !d_Q) return fail(TGW_ERR_INVALID_ARG, "NULL argument");
  if (ldq < cov->n) return fail(TGW_ERR_SHAPE, "ldq < n");
  HIP_TRY(hipMemcpy2DAsync(d_Q, ldq * sizeof(double), cov->Q, cov->n_pad * sizeof(double),
                           cov->n * sizeof(double), cov->q, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return TGW_OK;
  TGW_GUARD_END
}

// ---------------------------------------------------------------------------
// panels
// ---------------------------------------------------------------------------
extern "C" void tgw_panel_free(tgw_panel* p) {
  if (!p) return;
  dev_release_begin(p->mem);
  dev_free(p->mem, p->yop, nullptr);
  dev_free(p->mem, p->scale, nullptr);
  dev_free(p->mem, p->invny, nullptr);
  dev_free(p->mem, p->cw, nullptr);
  dev_free(p->mem, p->table, nullptr);
  dev_free(p->mem, p->lscale, nullptr);
  dev_free(p->mem, p->d_dev, nullptr);
  delete p;
}

extern "C" tgw_status tgw_prepare_phenotypes(const tgw_covariates* cov, int64_t n_pheno, const void* d_Y,
                                             int32_t y_is_fp64, int64_t ldy, tgw_precision prec, void* stream,
                                             tgw_panel** out) {
  TGW_GUARD_BEGIN
  if (!out) return fail(TGW_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!cov || !d_Y) return fail(TGW_ERR_INVALID_ARG, "NULL argument");
  if (prec != TGW_PREC_FP32 && prec != TGW_PREC_SPLIT && prec != TGW_PREC_SPLIT_F16 && prec != TGW_PREC_SPLIT_F8)
    return fail(TGW_ERR_INVALID_ARG, "bad precision");
  if (y_is_fp64 != 0 && y_is_fp64 != 1) return fail(TGW_ERR_INVALID_ARG, "y_is_fp64 must be 0 or 1");
  if (n_pheno < 1) return fail(TGW_ERR_SHAPE, "n_pheno must be >= 1");
  if (ldy < cov->n) return fail(TGW_ERR_SHAPE, "ldy < n_samples");
  int dev;
  tgw_status st = device_info(&dev, nullptr);
  if (st != TGW_OK) return st;
  if (dev != cov->device) return fail(TGW_ERR_INVALID_ARG, "covariates live on another device");
  hipStream_t s = (hipStream_t)stream;
  auto* p = new tgw_panel();
  p->mem = current_allocator();
  p->cov = cov;
  p->P = n_pheno;
  p->P_pad = round_up(n_pheno, kColBlock);
  p->prec = prec == TGW_PREC_SPLIT       ? kSplit
            : prec == TGW_PREC_SPLIT_F16 ? kSplit16
            : prec == TGW_PREC_SPLIT_F8  ? kSplit8
                                         : kFP32;
  p->df = cov->n - cov->q - 1;
  int32_t* flags = nullptr;
  const size_t op_bytes = (size_t)(p->P_pad / kColBlock) * cov->n_chunks * block_bytes(p->prec);
  const DevAllocator& A = p->mem;
  hipError_t e = dev_alloc(A, &p->yop, op_bytes, s);
  if (e == hipSuccess) e = dmalloc(A, &p->lscale, p->P_pad, s);
  if (e == hipSuccess) e = hipMemsetAsync(p->lscale, 127, p->P_pad, s);
  if (e == hipSuccess) e = dmalloc(A, &p->scale, p->P_pad, s);
  if (e == hipSuccess) e = dmalloc(A, &p->invny, p->P_pad, s);
  if (e == hipSuccess) e = dmalloc(A, &p->cw, (size_t)p->P_pad * kSlots, s);
  if (e == hipSuccess) e = dmalloc(A, &p->table, kTabIntervals, s);
  if (e == hipSuccess) e = dmalloc(A, &flags, 1, s);
  if (e == hipSuccess) e = dmalloc(A, &p->d_dev, 1, s);
  if (e == hipSuccess) e = hipMemsetAsync(p->yop, 0, op_bytes, s);
  if (e == hipSuccess) e = hipMemsetAsync(p->scale, 0, p->P_pad * sizeof(float), s);
  if (e == hipSuccess) e = hipMemsetAsync(p->invny, 0, p->P_pad * sizeof(float), s);
  if (e == hipSuccess) e = hipMemsetAsync(p->cw, 0, p->P_pad * kSlots * sizeof(float), s);
  if (e == hipSuccess) e = hipMemsetAsync(flags, 0, sizeof(int32_t), s);
  if (e == hipSuccess)
    e = launch_prep(d_Y, y_is_fp64, ldy, cov->n, cov->n_pad, n_pheno, cov->Q, cov->q, p->prec, p->yop, p->scale,
                    p->invny, p->cw, p->lscale, flags, s);
  if (e == hipSuccess) e = launch_table(p->table, (double)p->df, s);
  const PanelDev pd = panel_dev(p);
  if (e == hipSuccess) e = hipMemcpyAsync(p->d_dev, &pd, sizeof(pd), hipMemcpyHostToDevice, s);
  int32_t hf = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) (void)hipStreamSynchronize(s);  // nothing enqueued may still use flags
  dev_free(A, flags, s);
  if (e != hipSuccess) {
    tgw_panel_free(p);
    return hip_fail(e, "tgw_prepare_phenotypes");
  }
  if (hf) {
    tgw_panel_free(p);
    return fail(TGW_ERR_NONFINITE, "phenotypes contain NaN or Inf");
  }
  *out = p;
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" tgw_status tgw_panel_info(const tgw_panel* p, int64_t* n, int64_t* np, int32_t* q, int64_t* df) {
  if (!p) return fail(TGW_ERR_INVALID_ARG, "panel is NULL");
  if (n) *n = p->cov->n;
  if (np) *np = p->P;
  if (q) *q = p->cov->q;
  if (df) *df = p->df;
  return TGW_OK;
}

extern "C" tgw_status tgw_debug_set_operand(tgw_panel* p, const float* d_V, int64_t ldv, void* stream) {
  TGW_GUARD_BEGIN
  if (!p || !d_V) return fail(TGW_ERR_INVALID_ARG, "NULL argument");
  if (ldv < p->cov->n) return fail(TGW_ERR_SHAPE, "ldv < n");
  HIP_TRY(launch_set_operand(d_V, ldv, p->cov->n, p->cov->n_pad, p->P, p->prec, p->yop, p->lscale,
                             (hipStream_t)stream));
  return TGW_OK;
  TGW_GUARD_END
}

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
// the FP8 lo pass's integer centring needs the last correction slot free in
// every panel (the markers' operand tables are shared by the plan's panels)
static bool lo_int_for(int prec, const tgw_panel* const* panels, int n_panels) {
  if (prec != kSplit8) return false;
  for (int j = 0; j < n_panels; ++j)
    if (panels[j]->cov->q > kLoSlot) return false;
  return true;
}

extern "C" void tgw_plan_free(tgw_plan* pl) {
  if (!pl) return;
  for (auto& ev : pl->prof_events) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  const DevAllocator& A = pl->mem;
  dev_release_begin(A);
  dev_free(A, pl->d_cb_main, nullptr);
  dev_free(A, pl->d_cb_w, nullptr);
  dev_free(A, pl->d_panels, nullptr);
  dev_free(A, pl->d_outs, nullptr);
  dev_free(A, pl->mlut, nullptr);
  dev_free(A, pl->mstat, nullptr);
  dev_free(A, pl->wws, nullptr);
  dev_free(A, pl->invh, nullptr);
  dev_free(A, pl->redo_entries, nullptr);
  dev_free(A, pl->redo_count, nullptr);
  dev_free(A, pl->tail_entries, nullptr);
  dev_free(A, pl->tail_count, nullptr);
  delete pl;
}

static std::string tune_key(const tgw_plan* pl) {
  char buf[160];
  snprintf(buf, sizeof(buf), "%s/npad%lld/cb%d/np%d/prec%d", pl->arch.c_str(), (long long)pl->n_pad, pl->n_cb,
           pl->n_panels, pl->prec);
  return buf;
}

static std::string tune_cache_path() {
  const char* env = getenv("TGW_TUNE_CACHE");
  if (env && *env) return env;
  const char* home = getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/tgw/tune.json";
}

// the cache is a flat JSON object {"key": tile, ...}
static std::map<std::string, int> tune_cache_read() {
  std::map<std::string, int> m;
  FILE* f = fopen(tune_cache_path().c_str(), "r");
  if (!f) return m;
  std::string s;
  char buf[4096];
  size_t k;
  while ((k = fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, k);
  fclose(f);
  size_t pos = 0;
  while (true) {
    size_t a = s.find('"', pos);
    if (a == std::string::npos) break;
    size_t b = s.find('"', a + 1);
    if (b == std::string::npos) break;
    size_t c = s.find(':', b);
    if (c == std::string::npos) break;
    m[s.substr(a + 1, b - a - 1)] = atoi(s.c_str() + c + 1);
    pos = c + 1;
  }
  return m;
}

static void tune_cache_write(const std::string& key, int tile) {
  auto m = tune_cache_read();
  m[key] = tile;
  const std::string path = tune_cache_path();
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') mkdir(path.substr(0, i).c_str(), 0755);
  const std::string tmp = path + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fputs("{\n", f);
  size_t i = 0;
  for (auto& kv : m) fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < m.size() ? "," : "");
  fputs("}\n", f);
  fclose(f);
  rename(tmp.c_str(), path.c_str());
}

extern "C" tgw_status tgw_plan_create(const tgw_panel* const* panels, int32_t n_panels,
                                      const tgw_plan_options* opts, tgw_plan** out) {
  TGW_GUARD_BEGIN
  if (!out) return fail(TGW_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!panels || n_panels < 1) return fail(TGW_ERR_INVALID_ARG, "need at least one panel");
  for (int j = 0; j < n_panels; ++j)
    if (!panels[j]) return fail(TGW_ERR_INVALID_ARG, "NULL panel");
  const tgw_panel* p0 = panels[0];
  for (int j = 1; j < n_panels; ++j) {
    if (panels[j]->cov->n != p0->cov->n) return fail(TGW_ERR_SHAPE, "panels differ in n_samples");
    if (panels[j]->prec != p0->prec) return fail(TGW_ERR_INVALID_ARG, "panels differ in precision");
    if (panels[j]->cov->device != p0->cov->device) return fail(TGW_ERR_INVALID_ARG, "panels on different devices");
  }
  int dev;
  DevInfo info;
  tgw_status st = device_info(&dev, &info);
  if (st != TGW_OK) return st;
  if (dev != p0->cov->device) return fail(TGW_ERR_INVALID_ARG, "current device differs from the panels'");
  tgw_plan_options o{};
  if (opts) o = *opts;
  if (o.block_markers < 0 || o.tail_capacity < 0) return fail(TGW_ERR_INVALID_ARG, "negative option");
  if (o.tile >= n_tile_shapes()) return fail(TGW_ERR_INVALID_ARG, "tile index out of range");

  auto* pl = new tgw_plan();
  pl->mem = current_allocator();
  pl->panels.assign(panels, panels + n_panels);
  pl->device = dev;
  pl->n_cu = info.n_cu;
  pl->arch = info.arch;
  pl->prec = p0->prec;
  pl->n = p0->cov->n;
  pl->n_pad = p0->cov->n_pad;
  pl->n_chunks = p0->cov->n_chunks;
  pl->n_panels = n_panels;

  std::vector<ColBlock> cbm, cbw;
  std::vector<PanelDev> pdv;
  const bool hl = wprec(pl->prec) != kFP32;
  pl->w_mode = hl ? kRawHL : kRaw;
  for (int j = 0; j < n_panels; ++j) {
    const tgw_panel* p = panels[j];
    const int64_t nb = p->P_pad / kColBlock;
    for (int64_t b = 0; b < nb; ++b) {
      ColBlock c{};
      c.op = (const char*)p->yop + (size_t)b * pl->n_chunks * block_bytes(pl->prec);
      c.panel = j;
      c.col0 = (int32_t)(b * kColBlock);
      c.ncol = (int32_t)std::min<int64_t>(kColBlock, p->P - b * kColBlock);
      cbm.push_back(c);
    }
    if (hl) {  // slots 16 b .. 16 b + 15 from packed block b
      const int nb = hl_blocks(p->cov->q);
      for (int b = 0; b < nb; ++b) {
        ColBlock w{};
        w.op = (const char*)p->cov->wop_hl[wprec(pl->prec)] + (size_t)b * pl->n_chunks * kBlockBytes;
        w.panel = j;
        w.col0 = j * kSlots + b * kHLSlots;
        w.ncol = nb == 1 ? kSlots : kHLSlots;
        cbw.push_back(w);
      }
    } else {
      ColBlock w{};
      w.op = (const char*)p->cov->wop_fp32;
      w.panel = j;
      w.col0 = j * kSlots;
      w.ncol = kSlots;
      cbw.push_back(w);
    }
    pl->max_chunks = std::max<int>(pl->max_chunks, (int)((p->P + kRedoCols - 1) / kRedoCols));
    pdv.push_back(panel_dev(p));
  }
  pl->n_cb = (int)cbm.size();
  pl->n_cb_w = (int)cbw.size();
  pl->lo_int = lo_int_for(pl->prec, panels, n_panels);
  const int64_t per_marker = (int64_t)sizeof(uint4) + sizeof(MarkerStat) + (int64_t)n_panels * (kSlots + 3) * 4;
  int64_t MB = o.block_markers;
  if (MB == 0) MB = std::max<int64_t>(4096, std::min<int64_t>(1 << 20, (2ll << 30) / per_marker));
  MB = round_up(MB, 512);
  pl->MB = MB;
  pl->tail_cap = o.tail_capacity ? o.tail_capacity : (1 << 20);

  hipError_t e = dmalloc(pl->mem, &pl->d_cb_main, cbm.size());
  if (e == hipSuccess) e = dmalloc(pl->mem, &pl->d_cb_w, cbw.size());
  if (e == hipSuccess) e = dmalloc(pl->mem, &pl->d_panels, pdv.size());
  if (e == hipSuccess) e = dmalloc(pl->mem, &pl->d_outs, (size_t)n_panels);
  if (e == hipSuccess) e = dmalloc(pl->mem, &pl->mlut, (size_t)MB);
  if (e == hipSuccess) e = dmalloc(pl->mem, &pl->mstat, (size_t)MB);
  if (e == hipSuccess) e = dmalloc(pl->mem, &pl->wws, (size_t)MB * n_panels * kSlots);
  if (e == hipSuccess) e = dmalloc(pl->mem, &pl->invh, (size_t)MB * n_panels);
  if (e == hipSuccess) e = dmalloc(pl->mem, &pl->redo_entries, (size_t)MB * n_panels);
  if (e == hipSuccess) e = dmalloc(pl->mem, &pl->redo_count, (size_t)n_panels);
  if (e == hipSuccess) e = dmalloc(pl->mem, &pl->tail_entries, (size_t)pl->tail_cap);
  if (e == hipSuccess) e = dmalloc(pl->mem, &pl->tail_count, 1);
  if (e == hipSuccess) e = hipMemcpy(pl->d_cb_main, cbm.data(), cbm.size() * sizeof(ColBlock), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(pl->d_cb_w, cbw.data(), cbw.size() * sizeof(ColBlock), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(pl->d_panels, pdv.data(), pdv.size() * sizeof(PanelDev), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(pl->d_outs, 0, n_panels * sizeof(OutDev));
  if (e == hipSuccess) e = hipMemset(pl->tail_count, 0, sizeof(unsigned long long));
  if (e != hipSuccess) {
    tgw_plan_free(pl);
    return hip_fail(e, "tgw_plan_create");
  }
  for (int i = 0; i < n_tile_shapes(); ++i) pl->grid_main.push_back(gemm_grid(i, pl->prec, kTest, pl->n_cu));
  pl->grid_w = gemm_grid(wgemm_tile(), wprec(pl->prec), pl->w_mode, pl->n_cu);
  if (g8_supported(pl->prec)) {
    for (int i = 0; i < n_tile_shapes(); ++i) pl->grid_main8.push_back(gemm_grid(i, pl->prec, kTest, pl->n_cu, true));
    pl->grid_w8 = gemm_grid(wgemm_tile(), wprec(pl->prec), pl->w_mode, pl->n_cu, true);
    if (o.tile < 0) {
      auto cache8 = tune_cache_read();
      auto it8 = cache8.find(tune_key(pl) + "/g8");
      if (it8 != cache8.end() && it8->second >= 0 && it8->second < n_tile_shapes()) pl->tile8 = it8->second;
    }
  }
  if (o.tile >= 0) {
    pl->tile = o.tile;
    pl->tile8 = o.tile;  // the wide shapes run shape 2 for 8-bit dosages
  } else {
    auto cache = tune_cache_read();
    auto it = cache.find(tune_key(pl));
    pl->tile = (it != cache.end() && it->second >= 0 && it->second < n_tile_shapes()) ? it->second : 0;
  }
  *out = pl;
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" tgw_status tgw_plan_info(const tgw_plan* pl, int32_t* tile, int32_t* n_tiles, int64_t* block_markers) {
  if (!pl) return fail(TGW_ERR_INVALID_ARG, "plan is NULL");
  if (tile) *tile = pl->tile;
  if (n_tiles) *n_tiles = n_tile_shapes();
  if (block_markers) *block_markers = pl->MB;
  return TGW_OK;
}

// ---------------------------------------------------------------------------
// the scan
// ---------------------------------------------------------------------------
int64_t tgw::plan_samples(const tgw_plan* pl) { return pl->n; }

tgw_status tgw::check_call(const tgw_plan* pl, const ScanCall& c, bool need_outs) {
  if (!pl) return fail(TGW_ERR_INVALID_ARG, "plan is NULL");
  if (!c.geno) return fail(TGW_ERR_INVALID_ARG, "d_geno is NULL");
  if (((uintptr_t)c.geno & 15) != 0) return fail(TGW_ERR_SHAPE, "d_geno must be 16-byte aligned");
  if (c.code != TGW_CODE_DOSAGE && c.code != TGW_CODE_PLINK_BED && c.code != TGW_CODE_DOSAGE8)
    return fail(TGW_ERR_INVALID_ARG, "bad code");
  if (c.row_bytes <= 0 || c.row_bytes % 16 != 0) return fail(TGW_ERR_SHAPE, "row_bytes must be a positive multiple of 16");
  if (c.code == TGW_CODE_DOSAGE8) {
    if (!g8_supported(pl->prec))
      return fail(TGW_ERR_UNSUPPORTED, "8-bit dosages need TGW_PREC_FP32 or TGW_PREC_SPLIT_F16");
    if (c.row_bytes < pl->n_pad) return fail(TGW_ERR_SHAPE, "row_bytes < 64 * ceil(n_samples / 64) for 8-bit dosages");
  } else if (c.row_bytes < pl->n_pad / 4) {
    return fail(TGW_ERR_SHAPE, "row_bytes < 16 * ceil(n_samples / 64)");
  }
  if (c.n_markers < 0 || c.m_begin < 0 || c.m_begin > c.m_end || c.m_end > c.n_markers)
    return fail(TGW_ERR_SHAPE, "need 0 <= m_begin <= m_end <= n_markers");
  if (need_outs) {
    if (!c.outs) return fail(TGW_ERR_INVALID_ARG, "outs is NULL");
    for (int j = 0; j < pl->n_panels; ++j) {
      const tgw_outputs& o = c.outs[j];
      const bool dense = o.r || o.beta || o.se || o.t || o.nlog10p;
      if (dense && o.ld < pl->panels[j]->P) return fail(TGW_ERR_SHAPE, "outs[j].ld < n_pheno of panel j");
      if (dense && o.ld > kMaxOutLd) return fail(TGW_ERR_SHAPE, "outs[j].ld above 2^22 elements");
      if ((o.best || o.topk) && c.m_end > 0xffffffffll)
        return fail(TGW_ERR_SHAPE, "best and topk need marker indices below 2^32");
      if (o.topk && (o.topk_k < 1 || o.topk_k > kTopKMax)) return fail(TGW_ERR_SHAPE, "topk_k must be in [1, 64]");
    }
  }
  return TGW_OK;
}

static GemmArgs base_args(const tgw_plan* pl, const ScanCall& c, int64_t m0, int64_t nm) {
  GemmArgs a{};
  a.geno = c.geno;
  a.row_bytes = c.row_bytes;
  a.m0 = m0 - c.geno_row0;
  a.nm = nm;
  a.out_row0 = m0 - c.m_begin;
  a.n_chunks = pl->n_chunks;
  a.n_panels = pl->n_panels;
  a.panels = pl->d_panels;
  a.outs = pl->d_outs;
  a.mlut = pl->mlut;
  a.wws = pl->wws;
  a.invh = pl->invh;
  a.tail.entries = pl->tail_entries;
  a.tail.count = pl->tail_count;
  a.tail.capacity = pl->tail_cap;
  a.hits = pl->hits;
  a.m_begin = c.m_begin;
  a.gunit = c.code == TGW_CODE_DOSAGE8 ? kDosage8Unit : 1.0f;
  return a;
}

// per-block preamble: integer stats, Q^T g, ||g_res||
static hipError_t enqueue_block_stats(tgw_plan* pl, const ScanCall& c, int64_t m0, int64_t nm, hipStream_t s) {
  StatsArgs sa{};
  sa.geno = c.geno;
  sa.row_bytes = c.row_bytes;
  sa.m0 = m0 - c.geno_row0;
  sa.nm = nm;
  sa.n = pl->n;
  sa.code = c.code;
  sa.prec = pl->prec;
  sa.mlut = pl->mlut;
  sa.mstat = pl->mstat;
  sa.redo_count = pl->redo_count;
  sa.n_panels = pl->n_panels;
  sa.lo_int = pl->lo_int ? 1 : 0;
  hipError_t e = launch_stats(sa, s);
  if (e != hipSuccess) return e;
  GemmArgs a = base_args(pl, c, m0, nm);
  const TileShape ws = tile_shape(wgemm_tile());
  a.cblocks = pl->d_cb_w;
  a.n_cblocks = pl->n_cb_w;
  a.n_ctiles = (int)((pl->n_cb_w + ws.wn_frags - 1) / ws.wn_frags);
  a.n_mtiles = (int)((nm + ws.tm() - 1) / ws.tm());
  a.raw_out = pl->wws;
  a.raw_ld = (int64_t)pl->n_panels * kSlots;
  const bool g8 = c.code == TGW_CODE_DOSAGE8;
  e = launch_gemm(wgemm_tile(), wprec(pl->prec), pl->w_mode, a, g8 ? pl->grid_w8 : pl->grid_w, s, g8);
  if (e != hipSuccess) return e;
  return launch_finalize(pl->mstat, pl->wws, pl->invh, nm, pl->n_panels,
                         f16_scaled(pl->prec) ? 1.0f / kF16Scale : 1.0f, pl->lo_int ? 1 : 0,
                         RedoDev{pl->redo_entries, pl->redo_count, pl->MB}, s);
}

// the FP64 path of the block's covariate-collinear markers (after the main kernel)
static hipError_t enqueue_redo(tgw_plan* pl, const ScanCall& c, int64_t m0, hipStream_t s) {
  RedoArgs r{};
  r.geno = c.geno;
  r.row_bytes = c.row_bytes;
  r.m0 = m0 - c.geno_row0;
  r.n = pl->n;
  r.n_pad = pl->n_pad;
  r.n_chunks = pl->n_chunks;
  r.code = c.code;
  r.prec = pl->prec;
  r.n_panels = pl->n_panels;
  r.max_chunks = pl->max_chunks;
  r.gunit = c.code == TGW_CODE_DOSAGE8 ? kDosage8Unit : 1.0f;
  r.out_row0 = m0 - c.m_begin;
  r.m_begin = c.m_begin;
  r.mstat = pl->mstat;
  r.panels = pl->d_panels;
  r.outs = pl->d_outs;
  r.hits = pl->hits;
  r.redo = RedoDev{pl->redo_entries, pl->redo_count, pl->MB};
  return launch_redo(r, pl->n_cu, s);
}

static hipError_t enqueue_main(tgw_plan* pl, const ScanCall& c, int64_t m0, int64_t nm, int tile, hipStream_t s) {
  GemmArgs a = base_args(pl, c, m0, nm);
  const bool g8 = c.code == TGW_CODE_DOSAGE8;
  const TileShape ts = tile_shape_for(tile, pl->prec, g8);
  const int grid = g8 ? pl->grid_main8[tile] : pl->grid_main[tile];
  a.cblocks = pl->d_cb_main;
  a.n_cblocks = pl->n_cb;
  a.n_ctiles = (pl->n_cb + ts.wn_frags - 1) / ts.wn_frags;
  a.n_mtiles = (int)((nm + ts.tm() - 1) / ts.tm());
  if (!pl->profile) return launch_gemm(tile, pl->prec, kTest, a, grid, s, g8);
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  pl->prof_events.emplace_back(e0, e1);
  e = hipEventRecord(e0, s);
  if (e == hipSuccess) e = launch_gemm(tile, pl->prec, kTest, a, grid, s, g8);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  return e;
}

static hipError_t enqueue_bind(tgw_plan* pl, const tgw_outputs* outs, hipStream_t s) {
  for (int j0 = 0; j0 < pl->n_panels; j0 += kMaxPanelsPerBind) {
    BindArgs b{};
    b.dst = pl->d_outs;
    b.first = j0;
    b.count = std::min(kMaxPanelsPerBind, pl->n_panels - j0);
    for (int i = 0; i < b.count; ++i) {
      const tgw_outputs& o = outs[j0 + i];
      b.outs[i] = OutDev{o.r, o.beta, o.se, o.t, o.nlog10p, o.ld, o.best, o.topk, o.topk ? o.topk_k : 0, 0};
    }
    hipError_t e = launch_bind(b, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t tgw::enqueue_scan_begin(tgw_plan* pl, const tgw_outputs* outs, hipStream_t s) {
  hipError_t e = enqueue_bind(pl, outs, s);
  if (e == hipSuccess) e = launch_tail_reset(TailDev{pl->tail_entries, pl->tail_count, pl->tail_cap}, s);
  return e;
}

hipError_t tgw::enqueue_scan_rows(tgw_plan* pl, const ScanCall& c, int64_t m_lo, int64_t m_hi, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (int64_t m0 = m_lo; e == hipSuccess && m0 < m_hi; m0 += pl->MB) {
    const int64_t nm = std::min(pl->MB, m_hi - m0);
    e = enqueue_block_stats(pl, c, m0, nm, s);
    if (e == hipSuccess) e = enqueue_main(pl, c, m0, nm, c.code == TGW_CODE_DOSAGE8 ? pl->tile8 : pl->tile, s);
    if (e == hipSuccess) e = enqueue_redo(pl, c, m0, s);
  }
  return e;
}

hipError_t tgw::enqueue_scan_end(tgw_plan* pl, int64_t m_begin, hipStream_t s) {
  return launch_tail(TailDev{pl->tail_entries, pl->tail_count, pl->tail_cap}, pl->d_panels, pl->d_outs, pl->hits,
                     m_begin, s);
}

static hipError_t enqueue_scan(tgw_plan* pl, const ScanCall& c, hipStream_t s) {
  hipError_t e = enqueue_scan_begin(pl, c.outs, s);
  if (e == hipSuccess) e = enqueue_scan_rows(pl, c, c.m_begin, c.m_end, s);
  if (e == hipSuccess) e = enqueue_scan_end(pl, c.m_begin, s);
  return e;
}

extern "C" tgw_status tgw_plan_set_hits(tgw_plan* pl, tgw_hit* d_hits, int64_t capacity,
                                        unsigned long long* d_count, float threshold) {
  if (!pl) return fail(TGW_ERR_INVALID_ARG, "plan is NULL");
  if (!d_hits) {
    pl->hits = HitDev{};
    return TGW_OK;
  }
  if (!d_count) return fail(TGW_ERR_INVALID_ARG, "d_count is NULL");
  if (capacity < 0) return fail(TGW_ERR_INVALID_ARG, "negative capacity");
  if (!(threshold == threshold)) return fail(TGW_ERR_INVALID_ARG, "threshold is NaN");
  static_assert(sizeof(tgw_hit) == sizeof(Hit), "tgw_hit layout");
  // |t| below which -log10 p < threshold at every df: the normal tail is
  // lighter than Student's t, so -log10(erfc(|t|/sqrt 2)) bounds -log10 p
  // from above; bisection, then a small safety margin
  double lo = 0.0, hi = (double)kTMax;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double nl = -std::log10(std::erfc(mid / std::sqrt(2.0)));
    if (nl < (double)threshold)
      lo = mid;
    else
      hi = mid;
  }
  const float t_floor = (float)(lo * (1.0 - 1e-3));
  pl->hits = HitDev{(Hit*)d_hits, d_count, capacity, threshold, t_floor};
  return TGW_OK;
}

extern "C" tgw_status tgw_scan(tgw_plan* pl, const uint8_t* d_geno, int64_t n_markers, int64_t row_bytes,
                               tgw_geno_code code, int64_t m_begin, int64_t m_end, const tgw_outputs* outs,
                               void* stream) {
  TGW_GUARD_BEGIN
  ScanCall c{d_geno, n_markers, row_bytes, (int)code, m_begin, m_end, outs, 0};
  tgw_status st = check_call(pl, c, true);
  if (st != TGW_OK) return st;
  if (m_begin == m_end) return TGW_OK;
  HIP_TRY(enqueue_scan(pl, c, (hipStream_t)stream));
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" tgw_status tgw_topk_read(const tgw_panel* panel, const unsigned long long* d_words, int32_t k,
                                    float* d_nlog10p, int64_t* d_marker, void* stream) {
  TGW_GUARD_BEGIN
  if (!panel || !d_words) return fail(TGW_ERR_INVALID_ARG, "NULL argument");
  if (k < 1 || k > kTopKMax) return fail(TGW_ERR_SHAPE, "k must be in [1, 64]");
  HIP_TRY(launch_topk_read(d_words, panel->P * (int64_t)k, k, (double)panel->df, d_nlog10p, d_marker,
                           (hipStream_t)stream));
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" tgw_status tgw_plan_check(tgw_plan* pl, void* stream, int64_t* n_tail) {
  TGW_GUARD_BEGIN
  if (!pl) return fail(TGW_ERR_INVALID_ARG, "plan is NULL");
  hipStream_t s = (hipStream_t)stream;
  unsigned long long cnt = 0;
  HIP_TRY(hipMemcpyAsync(&cnt, pl->tail_count, sizeof(cnt), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (n_tail) *n_tail = (int64_t)cnt;
  if ((int64_t)cnt > pl->tail_cap) return fail(TGW_ERR_TAIL_OVERFLOW, "tail list overflow");
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" tgw_status tgw_plan_autotune(tgw_plan* pl, const uint8_t* d_geno, int64_t n_markers, int64_t row_bytes,
                                        tgw_geno_code code, int64_t m_begin, int64_t m_end,
                                        const tgw_outputs* outs, void* stream, double* best_ms) {
  TGW_GUARD_BEGIN
  ScanCall c{d_geno, n_markers, row_bytes, (int)code, m_begin, m_end, outs, 0};
  tgw_status st = check_call(pl, c, true);
  if (st != TGW_OK) return st;
  if (m_begin == m_end) return fail(TGW_ERR_SHAPE, "autotune needs at least one marker");
  hipStream_t s = (hipStream_t)stream;
  const int64_t nm = std::min(pl->MB, m_end - m_begin);
  HIP_TRY(enqueue_bind(pl, outs, s));
  HIP_TRY(launch_tail_reset(TailDev{pl->tail_entries, pl->tail_count, pl->tail_cap}, s));
  HIP_TRY(enqueue_block_stats(pl, c, m_begin, nm, s));
  const HitDev saved_hits = pl->hits;  // repeated timing runs must not append hits
  pl->hits = HitDev{};
  struct Restore {
    tgw_plan* p;
    HitDev h;
    ~Restore() { p->hits = h; }
  } restore{pl, saved_hits};
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const bool g8 = code == TGW_CODE_DOSAGE8;
  int best = g8 ? pl->tile8 : pl->tile;
  double best_t = 1e300;
  hipError_t err = hipSuccess;
  for (int t = 0; t < n_tile_shapes() && err == hipSuccess; ++t) {
    if (tile_alias(t, pl->prec, g8) != t) continue;  // same kernel as an earlier shape
    err = enqueue_main(pl, c, m_begin, nm, t, s);  // warm-up
    if (err != hipSuccess) break;
    const int reps = 3;
    err = hipEventRecord(e0, s);
    for (int r = 0; r < reps && err == hipSuccess; ++r) err = enqueue_main(pl, c, m_begin, nm, t, s);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && ms / reps < best_t) {
      best_t = ms / reps;
      best = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return hip_fail(err, "tgw_plan_autotune");
  if (g8) {
    pl->tile8 = best;
    tune_cache_write(tune_key(pl) + "/g8", best);
  } else {
    pl->tile = best;
    tune_cache_write(tune_key(pl), best);
  }
  if (best_ms) *best_ms = best_t;
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" tgw_status tgw_plan_profile(tgw_plan* pl, int32_t enable) {
  if (!pl) return fail(TGW_ERR_INVALID_ARG, "plan is NULL");
  pl->profile = enable != 0;
  return TGW_OK;
}

extern "C" tgw_status tgw_plan_profile_read(tgw_plan* pl, void* stream, double* main_ms, int64_t* launches) {
  TGW_GUARD_BEGIN
  if (!pl) return fail(TGW_ERR_INVALID_ARG, "plan is NULL");
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  double tot = 0.0;
  hipError_t err = hipSuccess;
  for (auto& ev : pl->prof_events) {
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, ev.first, ev.second);
    tot += ms;
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  const int64_t n = (int64_t)pl->prof_events.size();
  pl->prof_events.clear();
  if (err != hipSuccess) return hip_fail(err, "tgw_plan_profile_read");
  if (main_ms) *main_ms = tot;
  if (launches) *launches = n;
  return TGW_OK;
  TGW_GUARD_END
}

// ---------------------------------------------------------------------------
// graphs
// ---------------------------------------------------------------------------
extern "C" tgw_status tgw_graph_create(tgw_plan* pl, const uint8_t* d_geno, int64_t n_markers, int64_t row_bytes,
                                       tgw_geno_code code, int64_t m_begin, int64_t m_end, const tgw_outputs* outs,
                                       tgw_graph** out) {
  TGW_GUARD_BEGIN
  if (!out) return fail(TGW_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ScanCall c{d_geno, n_markers, row_bytes, (int)code, m_begin, m_end, outs, 0};
  tgw_status st = check_call(pl, c, true);
  if (st != TGW_OK) return st;
  hipStream_t s;
  HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t e2 = m_begin < m_end ? enqueue_scan(pl, c, s) : hipSuccess;
    e = hipStreamEndCapture(s, &g);
    if (e2 != hipSuccess) e = e2;
  }
  hipGraphExec_t ex = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipStreamDestroy(s);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(e, "tgw_graph_create");
  }
  auto* gr = new tgw_graph();
  gr->graph = g;
  gr->exec = ex;
  *out = gr;
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" tgw_status tgw_graph_launch(tgw_graph* g, void* stream) {
  TGW_GUARD_BEGIN
  if (!g) return fail(TGW_ERR_INVALID_ARG, "graph is NULL");
  HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" void tgw_graph_free(tgw_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

// ---------------------------------------------------------------------------
// allocation-free scan: tgw_scan_static keeps everything tgw_scan keeps in a
// plan (column-block tables, per-panel constants, output table, per-block
// workspace, FP64 lists, tail list) in `scratch`, a static device array that
// every GPU the library runs on holds until the process ends.  Host code
// never uses the array's name as an address: each device's address comes
// from hipGetSymbolAddress (device_info, once per device) and is kept in
// DevInfo.  Calls on one GPU share the array: a call leaves its contents
// behind, everything a call reads it writes first (the tables and the tail
// count by static_setup_kernel, the FP64 list counts by the stats kernel of
// each block), and calls that overlap on one GPU race.
// ---------------------------------------------------------------------------
constexpr size_t kStaticBytes = size_t(64) << 20;
constexpr int kStaticPanels = kMaxPanelsPerBind;  // 32
constexpr int kStaticColBlocks = 32768;           // 2^20 phenotype columns in all
constexpr int kStaticTail = 1 << 16;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

static hipError_t static_scratch_address(char** p) {
  void* a = nullptr;
  const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
  *p = e == hipSuccess ? (char*)a : nullptr;
  return e;
}

namespace {
struct StaticSetupArgs {
  const PanelDev* pd[kStaticPanels];  // each panel's device copy
  OutDev outs[kStaticPanels];
  int32_t cb_off[kStaticPanels + 1];  // main column blocks before panel j
  int32_t w_off[kStaticPanels + 1];   // Q^T g column blocks before panel j
  int32_t n_panels, n_chunks, prec, hl;
  ColBlock* cb_main;
  ColBlock* cb_w;
  PanelDev* panels;
  OutDev* outs_dev;
  unsigned long long* tail_count;
};
static_assert(sizeof(StaticSetupArgs) <= 4096, "kernel argument size");

// the tables tgw_plan_create builds on the host, built here from the
// panels' device constants; also clears the tail count
__global__ void static_setup_kernel(StaticSetupArgs a) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nt = gridDim.x * blockDim.x;
  if (tid == 0) a.tail_count[0] = 0ull;
  for (int j = tid; j < a.n_panels; j += nt) {
    const PanelDev pd = *a.pd[j];
    a.panels[j] = pd;
    a.outs_dev[j] = a.outs[j];
    const int nb = a.w_off[j + 1] - a.w_off[j];
    for (int b = 0; b < nb; ++b) {
      ColBlock w{};
      w.op = (const char*)pd.wop + (size_t)b * a.n_chunks * kBlockBytes;
      w.panel = j;
      w.col0 = j * kSlots + b * kHLSlots;
      w.ncol = (a.hl && nb > 1) ? kHLSlots : kSlots;
      a.cb_w[a.w_off[j] + b] = w;
    }
  }
  for (int k = tid; k < a.cb_off[a.n_panels]; k += nt) {
    int j = 0;
    while (k >= a.cb_off[j + 1]) ++j;
    const int b = k - a.cb_off[j];
    const PanelDev* pd = a.pd[j];
    ColBlock c{};
    c.op = (const char*)pd->yop + (size_t)b * a.n_chunks * block_bytes(a.prec);
    c.panel = j;
    c.col0 = b * kColBlock;
    c.ncol = (int32_t)std::min<int64_t>(kColBlock, pd->n_pheno - (int64_t)b * kColBlock);
    a.cb_main[k] = c;
  }
}

__global__ void static_tail_count_kernel(unsigned long long* dst, const unsigned long long* src) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

// the plan tgw_scan_static runs through, per device; its buffers point into
// that device's scratch (made once, with room for kStaticPanels panels, so
// that filling it in allocates nothing)
struct StaticState {
  std::mutex mu;
  tgw_plan plan;
};
std::mutex g_static_mu;
std::map<int, StaticState*> g_static;  // never freed: lives as long as the scratch

// made by tgw_init (or by the first tgw_scan_static on the device), so that
// later calls find it without allocating
StaticState* static_state(int dev) {
  std::lock_guard<std::mutex> lk(g_static_mu);
  auto it = g_static.find(dev);
  if (it != g_static.end()) return it->second;
  auto* s = new StaticState();
  s->plan.panels.reserve(kStaticPanels);
  s->plan.grid_main.reserve(16);
  s->plan.grid_main8.reserve(16);
  g_static.emplace(dev, s);
  return s;
}
}  // namespace

static void static_state_init(int dev) { (void)static_state(dev); }

extern "C" tgw_status tgw_scan_static(const tgw_panel* const* panels, int32_t n_panels, const uint8_t* d_geno,
                                      int64_t n_markers, int64_t row_bytes, tgw_geno_code code, int64_t m_begin,
                                      int64_t m_end, const tgw_outputs* outs, int32_t tile,
                                      unsigned long long* d_n_tail, void* stream) {
  TGW_GUARD_BEGIN
  if (!panels || n_panels < 1) return fail(TGW_ERR_INVALID_ARG, "need at least one panel");
  if (n_panels > kStaticPanels) return fail(TGW_ERR_SHAPE, "tgw_scan_static takes at most 32 panels");
  for (int j = 0; j < n_panels; ++j)
    if (!panels[j]) return fail(TGW_ERR_INVALID_ARG, "NULL panel");
  const tgw_panel* p0 = panels[0];
  for (int j = 1; j < n_panels; ++j) {
    if (panels[j]->cov->n != p0->cov->n) return fail(TGW_ERR_SHAPE, "panels differ in n_samples");
    if (panels[j]->prec != p0->prec) return fail(TGW_ERR_INVALID_ARG, "panels differ in precision");
    if (panels[j]->cov->device != p0->cov->device) return fail(TGW_ERR_INVALID_ARG, "panels on different devices");
  }
  if (tile >= n_tile_shapes()) return fail(TGW_ERR_INVALID_ARG, "tile index out of range");
  int dev = 0, n_cu = 0;
  char* base = nullptr;
  tgw_status st = device_basics(&dev, &n_cu, &base);
  if (st != TGW_OK) return st;
  if (dev != p0->cov->device) return fail(TGW_ERR_INVALID_ARG, "current device differs from the panels'");
  if (!base) return fail(TGW_ERR_DEVICE, "no static scratch on this device");

  // tables: sizes and offsets
  const int prec = p0->prec;
  const bool hl = wprec(prec) != kFP32;
  StaticSetupArgs sa{};
  int n_cb = 0, n_cbw = 0, max_chunks = 0;
  for (int j = 0; j < n_panels; ++j) {
    const tgw_panel* p = panels[j];
    sa.pd[j] = p->d_dev;
    sa.cb_off[j] = n_cb;
    sa.w_off[j] = n_cbw;
    n_cb += (int)std::min<int64_t>(p->P_pad / kColBlock, kStaticColBlocks + 1);
    n_cbw += hl ? hl_blocks(p->cov->q) : 1;
    max_chunks = std::max<int>(max_chunks, (int)((p->P + kRedoCols - 1) / kRedoCols));
    if (n_cb > kStaticColBlocks)
      return fail(TGW_ERR_SHAPE, "tgw_scan_static takes at most 2^20 phenotype columns in all");
  }
  sa.cb_off[n_panels] = n_cb;
  sa.w_off[n_panels] = n_cbw;

  // carve the scratch: tables and tail list, then the largest marker block
  // (a multiple of 512) whose workspace fits in the rest
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~size_t(255);
    char* q = base + off;
    off += bytes;
    return q;
  };
  ColBlock* cb_main = (ColBlock*)take(sizeof(ColBlock) * kStaticColBlocks);
  ColBlock* cb_w = (ColBlock*)take(sizeof(ColBlock) * 2 * kStaticPanels);
  PanelDev* pdev = (PanelDev*)take(sizeof(PanelDev) * kStaticPanels);
  OutDev* odev = (OutDev*)take(sizeof(OutDev) * kStaticPanels);
  unsigned long long* tail_count = (unsigned long long*)take(sizeof(unsigned long long));
  TailEntry* tail = (TailEntry*)take(sizeof(TailEntry) * kStaticTail);
  uint32_t* redo_count = (uint32_t*)take(sizeof(uint32_t) * kStaticPanels);
  const size_t per_marker = sizeof(uint4) + sizeof(MarkerStat) + (size_t)n_panels * (kSlots + 3) * 4;
  const size_t avail = kStaticBytes - off - 6 * 256;
  const int64_t MB = (int64_t)(avail / per_marker) / 512 * 512;
  if (MB < 512) return fail(TGW_ERR_SHAPE, "static scratch too small");
  uint4* mlut = (uint4*)take(sizeof(uint4) * MB);
  MarkerStat* mstat = (MarkerStat*)take(sizeof(MarkerStat) * MB);
  float* wws = (float*)take(sizeof(float) * MB * n_panels * kSlots);
  float2* invh = (float2*)take(sizeof(float2) * MB * n_panels);
  int32_t* redo_entries = (int32_t*)take(sizeof(int32_t) * MB * n_panels);
  if (off > kStaticBytes) return fail(TGW_ERR_SHAPE, "static scratch too small");

  StaticState* S = static_state(dev);
  std::lock_guard<std::mutex> lk(S->mu);
  tgw_plan& pl = S->plan;
  pl.panels.assign(panels, panels + n_panels);  // capacity reserved: no allocation
  pl.device = dev;
  pl.prec = prec;
  pl.n_cu = n_cu;
  pl.n = p0->cov->n;
  pl.n_pad = p0->cov->n_pad;
  pl.n_chunks = p0->cov->n_chunks;
  pl.n_panels = n_panels;
  pl.n_cb = n_cb;
  pl.n_cb_w = n_cbw;
  pl.MB = MB;
  pl.d_cb_main = cb_main;
  pl.d_cb_w = cb_w;
  pl.d_panels = pdev;
  pl.d_outs = odev;
  pl.mlut = mlut;
  pl.mstat = mstat;
  pl.wws = wws;
  pl.invh = invh;
  pl.redo_entries = redo_entries;
  pl.redo_count = redo_count;
  pl.max_chunks = max_chunks;
  pl.tail_entries = tail;
  pl.tail_count = tail_count;
  pl.tail_cap = kStaticTail;
  pl.hits = HitDev{};
  pl.w_mode = hl ? kRawHL : kRaw;
  pl.lo_int = lo_int_for(prec, panels, n_panels);
  pl.profile = false;
  pl.tile = tile >= 0 ? tile : 0;
  pl.tile8 = tile >= 0 ? tile : 2;
  pl.grid_main.clear();
  pl.grid_main8.clear();
  for (int i = 0; i < n_tile_shapes(); ++i) pl.grid_main.push_back(gemm_grid(i, prec, kTest, n_cu));
  pl.grid_w = gemm_grid(wgemm_tile(), wprec(prec), pl.w_mode, n_cu);
  if (g8_supported(prec)) {
    for (int i = 0; i < n_tile_shapes(); ++i) pl.grid_main8.push_back(gemm_grid(i, prec, kTest, n_cu, true));
    pl.grid_w8 = gemm_grid(wgemm_tile(), wprec(prec), pl.w_mode, n_cu, true);
  }

  ScanCall c{d_geno, n_markers, row_bytes, (int)code, m_begin, m_end, outs, 0};
  st = check_call(&pl, c, true);
  if (st != TGW_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  for (int j = 0; j < n_panels; ++j) {
    const tgw_outputs& o = outs[j];
    sa.outs[j] = OutDev{o.r, o.beta, o.se, o.t, o.nlog10p, o.ld, o.best, o.topk, o.topk ? o.topk_k : 0, 0};
  }
  sa.n_panels = n_panels;
  sa.n_chunks = pl.n_chunks;
  sa.prec = prec;
  sa.hl = hl ? 1 : 0;
  sa.cb_main = cb_main;
  sa.cb_w = cb_w;
  sa.panels = pdev;
  sa.outs_dev = odev;
  sa.tail_count = tail_count;
  hipLaunchKernelGGL(static_setup_kernel, dim3((unsigned)std::max(1, std::min(64, (n_cb + 255) / 256))), dim3(256),
                     0, s, sa);
  HIP_TRY(hipGetLastError());
  if (m_begin < m_end) {
    HIP_TRY(enqueue_scan_rows(&pl, c, m_begin, m_end, s));
    HIP_TRY(enqueue_scan_end(&pl, m_begin, s));
  }
  if (d_n_tail) {
    hipLaunchKernelGGL(static_tail_count_kernel, dim3(1), dim3(64), 0, s, d_n_tail, tail_count);
    HIP_TRY(hipGetLastError());
  }
  return TGW_OK;
  TGW_GUARD_END
}

// ---------------------------------------------------------------------------
// test hooks
// ---------------------------------------------------------------------------
extern "C" tgw_status tgw_debug_contract(tgw_plan* pl, const uint8_t* d_geno, int64_t n_markers, int64_t row_bytes,
                                         tgw_geno_code code, int64_t m_begin, int64_t m_end, float* d_S, int64_t lds,
                                         void* stream) {
  TGW_GUARD_BEGIN
  ScanCall c{d_geno, n_markers, row_bytes, (int)code, m_begin, m_end, nullptr, 0};
  tgw_status st = check_call(pl, c, false);
  if (st != TGW_OK) return st;
  if (pl->n_panels != 1) return fail(TGW_ERR_INVALID_ARG, "debug contraction needs a one-panel plan");
  if (!d_S) return fail(TGW_ERR_INVALID_ARG, "d_S is NULL");
  if (lds < pl->panels[0]->P) return fail(TGW_ERR_SHAPE, "lds < n_pheno");
  hipStream_t s = (hipStream_t)stream;
  for (int64_t m0 = m_begin; m0 < m_end; m0 += pl->MB) {
    const int64_t nm = std::min(pl->MB, m_end - m0);
    StatsArgs sa{};
    sa.geno = d_geno;
    sa.row_bytes = row_bytes;
    sa.m0 = m0;
    sa.nm = nm;
    sa.n = pl->n;
    sa.code = (int)code;
    sa.prec = pl->prec;
    sa.mlut = pl->mlut;
    sa.mstat = pl->mstat;
    sa.lo_int = pl->lo_int ? 1 : 0;
    HIP_TRY(launch_stats(sa, s));
    GemmArgs a = base_args(pl, c, m0, nm);
    const bool g8 = code == TGW_CODE_DOSAGE8;
    const int tile = g8 ? pl->tile8 : pl->tile;
    const TileShape ts = tile_shape_for(tile, pl->prec, g8);
    a.cblocks = pl->d_cb_main;
    a.n_cblocks = pl->n_cb;
    a.n_ctiles = (pl->n_cb + ts.wn_frags - 1) / ts.wn_frags;
    a.n_mtiles = (int)((nm + ts.tm() - 1) / ts.tm());
    a.raw_out = d_S + (m0 - m_begin) * lds;
    a.raw_ld = lds;
    HIP_TRY(launch_gemm(tile, pl->prec, kRaw, a, g8 ? pl->grid_main8[tile] : pl->grid_main[tile], s, g8));
  }
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" tgw_status tgw_debug_marker_stats(tgw_plan* pl, const uint8_t* d_geno, int64_t n_markers,
                                             int64_t row_bytes, tgw_geno_code code, int64_t m_begin, int64_t m_end,
                                             double* d_shift, double* d_mean, double* d_scale, void* stream) {
  TGW_GUARD_BEGIN
  ScanCall c{d_geno, n_markers, row_bytes, (int)code, m_begin, m_end, nullptr, 0};
  tgw_status st = check_call(pl, c, false);
  if (st != TGW_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  for (int64_t m0 = m_begin; m0 < m_end; m0 += pl->MB) {
    const int64_t nm = std::min(pl->MB, m_end - m0);
    StatsArgs sa{};
    sa.geno = d_geno;
    sa.row_bytes = row_bytes;
    sa.m0 = m0;
    sa.nm = nm;
    sa.n = pl->n;
    sa.code = (int)code;
    sa.prec = pl->prec;
    sa.mlut = pl->mlut;
    sa.mstat = pl->mstat;
    sa.lo_int = pl->lo_int ? 1 : 0;
    HIP_TRY(launch_stats(sa, s));
    HIP_TRY(launch_debug_stats(pl->mstat, nm, d_shift ? d_shift + (m0 - m_begin) : nullptr,
                               d_mean ? d_mean + (m0 - m_begin) : nullptr,
                               d_scale ? d_scale + (m0 - m_begin) : nullptr, s));
  }
  return TGW_OK;
  TGW_GUARD_END
}
