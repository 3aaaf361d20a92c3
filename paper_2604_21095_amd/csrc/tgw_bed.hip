// PLINK 1 binary genotype files behind the C ABI: the variant-major .bed
// reader, sample-table (.fam) matching, and a scan streamed from the file.
//
// The streamed scan overlaps three stages over marker blocks, with two
// buffer slots:
//   host threads : pread of block k into pinned slot k % 2
//   copy stream  : one host-to-device copy of the raw rows of block k
//   scan stream  : gather of the selected samples into scan rows
//                  (bed_repack_kernel), then the scan of block k
// so that reading block k runs while the device copies and scans block k - 1.
#include "tgw_host.h"
#include "tgw_internal.h"

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace tgw;

namespace {

constexpr uint8_t kMagic[3] = {0x6c, 0x1b, 0x01};  // PLINK 1 .bed, variant-major
constexpr int kRepackRows = 16;
constexpr int64_t kDefaultBlock = 65536;
constexpr int kMaxThreads = 64;

// ---------------------------------------------------------------------------
// raw .bed rows -> scan rows with a sample selection (HBM-bound gather)
//
// raw: nm rows of raw_bytes in file order (sample s at bits 2(s & 3) of byte
// s >> 2); sel: n_sel file sample indexes, each < 4 raw_bytes; dst: nm rows
// of row_bytes (a multiple of 16), output sample j at bits 2(j & 3) of byte
// j >> 2, code 01 (missing in PLINK coding) for j >= n_sel.  One thread per
// output dword (16 samples) and kRepackRows markers, so the 16 indexes are
// loaded once per kRepackRows rows; the stores of a wave are contiguous.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void bed_repack_kernel(const uint8_t* __restrict__ raw, int64_t raw_bytes,
                                                         const int32_t* __restrict__ sel, int64_t n_sel,
                                                         uint8_t* __restrict__ dst, int64_t row_bytes, int64_t nm) {
  const int64_t nd = row_bytes / 4;
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= nd) return;
  int32_t src[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t j = 16 * d + k;
    src[k] = j < n_sel ? sel[j] : -1;
  }
  for (int64_t m0 = (int64_t)blockIdx.y * kRepackRows; m0 < nm; m0 += (int64_t)gridDim.y * kRepackRows) {
    const int64_t m1 = m0 + kRepackRows < nm ? m0 + kRepackRows : nm;
    for (int64_t m = m0; m < m1; ++m) {
      const uint8_t* r = raw + m * raw_bytes;
      uint32_t w = 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const uint32_t code = src[k] >= 0 ? (r[src[k] >> 2] >> (2 * (src[k] & 3))) & 3u : 1u;
        w |= code << (2 * k);
      }
      reinterpret_cast<uint32_t*>(dst + m * row_bytes)[d] = w;
    }
  }
}

hipError_t launch_bed_repack(const uint8_t* raw, int64_t raw_bytes, const int32_t* sel, int64_t n_sel, uint8_t* dst,
                             int64_t row_bytes, int64_t nm, hipStream_t s) {
  if (nm <= 0) return hipSuccess;
  const int64_t nd = row_bytes / 4;
  const int64_t gy = std::min<int64_t>((nm + kRepackRows - 1) / kRepackRows, 65535);
  hipLaunchKernelGGL(bed_repack_kernel, dim3((unsigned)((nd + 255) / 256), (unsigned)gy), dim3(256), 0, s, raw,
                     raw_bytes, sel, n_sel, dst, row_bytes, nm);
  return hipGetLastError();
}

// read exactly `len` bytes at `off`
bool pread_all(int fd, uint8_t* dst, int64_t len, int64_t off) {
  while (len > 0) {
    const ssize_t got = ::pread(fd, dst, (size_t)std::min<int64_t>(len, 1ll << 30), (off_t)off);
    if (got < 0) {
      if (errno == EINTR) continue;
      return false;
    }
    if (got == 0) return false;
    dst += got;
    off += got;
    len -= got;
  }
  return true;
}

// read `len` bytes at `off` with up to n_threads threads on disjoint ranges
bool pread_parallel(int fd, uint8_t* dst, int64_t len, int64_t off, int n_threads) {
  const int64_t min_part = 8ll << 20;
  const int t = (int)std::max<int64_t>(1, std::min<int64_t>(n_threads, len / min_part));
  if (t == 1) return pread_all(fd, dst, len, off);
  std::vector<std::thread> th;
  std::vector<char> ok(t, 0);
  const int64_t part = (len + t - 1) / t;
  for (int i = 0; i < t; ++i) {
    const int64_t a = i * part, b = std::min(len, a + part);
    th.emplace_back([=, &ok] { ok[i] = a >= b || pread_all(fd, dst + a, b - a, off + a); });
  }
  for (auto& x : th) x.join();
  return std::all_of(ok.begin(), ok.end(), [](char c) { return c != 0; });
}

}  // namespace

struct tgw_bed {
  DevAllocator mem;  // the allocator of its device buffers (registered at the first tgw_scan_bed)
  int fd = -1;
  int64_t n_file = 0, n_markers = 0, raw_bytes = 0;
  std::vector<int32_t> sel;  // file sample of each scan sample, in scan order
  // streaming state, made by the first tgw_scan_bed (or when its shape changes)
  struct Slot {
    uint8_t* host = nullptr;   // pinned, block_markers x raw_bytes
    uint8_t* draw = nullptr;   // device, block_markers x raw_bytes
    uint8_t* dpack = nullptr;  // device, block_markers x row_bytes
    hipEvent_t copied = nullptr, used = nullptr;
    bool pending = false;
  };
  Slot slot[2];
  int device = -1;
  int64_t block = 0, row_bytes = 0;
  hipStream_t copy = nullptr;
  int32_t* d_sel = nullptr;
  bool sel_dirty = true;
};

static void release_stream_state(tgw_bed* b) {
  dev_release_begin(b->mem);
  for (auto& s : b->slot) {
    if (s.pending) {
      (void)hipEventSynchronize(s.copied);
      (void)hipEventSynchronize(s.used);
    }
    if (s.host) (void)hipHostFree(s.host);
    dev_free(b->mem, s.draw, nullptr);
    dev_free(b->mem, s.dpack, nullptr);
    if (s.copied) (void)hipEventDestroy(s.copied);
    if (s.used) (void)hipEventDestroy(s.used);
    s = tgw_bed::Slot{};
  }
  if (b->copy) (void)hipStreamDestroy(b->copy);
  dev_free(b->mem, b->d_sel, nullptr);
  b->copy = nullptr;
  b->d_sel = nullptr;
  b->sel_dirty = true;
  b->device = -1;
  b->block = 0;
  b->row_bytes = 0;
}

extern "C" tgw_status tgw_bed_open(const char* path, int64_t n_samples, tgw_bed** out) {
  TGW_GUARD_BEGIN
  if (!out) return fail(TGW_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!path) return fail(TGW_ERR_INVALID_ARG, "path is NULL");
  if (n_samples < 1 || n_samples > 0x7fffffffll) return fail(TGW_ERR_SHAPE, "need 1 <= n_samples < 2^31");
  const int fd = ::open(path, O_RDONLY | O_CLOEXEC);
  if (fd < 0) return fail(TGW_ERR_INVALID_ARG, std::string("cannot open ") + path + ": " + std::strerror(errno));
  struct stat st;
  uint8_t head[3] = {0, 0, 0};
  const bool ok = ::fstat(fd, &st) == 0 && st.st_size >= 3 && pread_all(fd, head, 3, 0);
  if (!ok || std::memcmp(head, kMagic, 3) != 0) {
    ::close(fd);
    return fail(TGW_ERR_INVALID_ARG, std::string(path) + " is not a variant-major PLINK 1 .bed file");
  }
  const int64_t raw_bytes = (n_samples + 3) / 4;
  const int64_t body = (int64_t)st.st_size - 3;
  if (body % raw_bytes != 0) {
    ::close(fd);
    return fail(TGW_ERR_SHAPE, "file size is not 3 + n_markers * ceil(n_samples / 4)");
  }
  auto* b = new tgw_bed();
  b->fd = fd;
  b->n_file = n_samples;
  b->n_markers = body / raw_bytes;
  b->raw_bytes = raw_bytes;
  b->sel.resize((size_t)n_samples);
  for (int64_t i = 0; i < n_samples; ++i) b->sel[(size_t)i] = (int32_t)i;
  *out = b;
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" void tgw_bed_close(tgw_bed* b) {
  if (!b) return;
  release_stream_state(b);
  if (b->fd >= 0) ::close(b->fd);
  delete b;
}

extern "C" tgw_status tgw_bed_info(const tgw_bed* b, int64_t* n_file_samples, int64_t* n_markers,
                                   int64_t* n_selected) {
  if (!b) return fail(TGW_ERR_INVALID_ARG, "bed is NULL");
  if (n_file_samples) *n_file_samples = b->n_file;
  if (n_markers) *n_markers = b->n_markers;
  if (n_selected) *n_selected = (int64_t)b->sel.size();
  return TGW_OK;
}

extern "C" tgw_status tgw_bed_select(tgw_bed* b, const int64_t* idx, int64_t n) {
  TGW_GUARD_BEGIN
  if (!b) return fail(TGW_ERR_INVALID_ARG, "bed is NULL");
  std::vector<int32_t> sel;
  if (!idx) {
    sel.resize((size_t)b->n_file);
    for (int64_t i = 0; i < b->n_file; ++i) sel[(size_t)i] = (int32_t)i;
  } else {
    if (n < 1) return fail(TGW_ERR_SHAPE, "need at least one selected sample");
    std::vector<char> seen((size_t)b->n_file, 0);
    sel.resize((size_t)n);
    for (int64_t j = 0; j < n; ++j) {
      const int64_t s = idx[j];
      if (s < 0 || s >= b->n_file) return fail(TGW_ERR_SHAPE, "selected sample index out of range");
      if (seen[(size_t)s]) return fail(TGW_ERR_INVALID_ARG, "a file sample is selected twice");
      seen[(size_t)s] = 1;
      sel[(size_t)j] = (int32_t)s;
    }
  }
  b->sel.swap(sel);
  b->sel_dirty = true;
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" tgw_status tgw_bed_read(const tgw_bed* b, int64_t m_begin, int64_t m_end, uint8_t* dst,
                                   int64_t row_bytes) {
  TGW_GUARD_BEGIN
  if (!b) return fail(TGW_ERR_INVALID_ARG, "bed is NULL");
  if (m_begin < 0 || m_begin > m_end || m_end > b->n_markers)
    return fail(TGW_ERR_SHAPE, "need 0 <= m_begin <= m_end <= n_markers");
  const int64_t n_sel = (int64_t)b->sel.size();
  if (row_bytes < (n_sel + 3) / 4) return fail(TGW_ERR_SHAPE, "row_bytes < ceil(n_selected / 4)");
  if (m_begin == m_end) return TGW_OK;
  if (!dst) return fail(TGW_ERR_INVALID_ARG, "dst is NULL");
  std::vector<uint8_t> raw((size_t)b->raw_bytes);
  for (int64_t m = m_begin; m < m_end; ++m) {
    if (!pread_all(b->fd, raw.data(), b->raw_bytes, 3 + m * b->raw_bytes))
      return fail(TGW_ERR_INVALID_ARG, std::string("read failed: ") + std::strerror(errno));
    uint8_t* row = dst + (m - m_begin) * row_bytes;
    std::memset(row, 0x55, (size_t)row_bytes);  // code 01 = missing
    for (int64_t j = 0; j < n_sel; ++j) {
      const int32_t s = b->sel[(size_t)j];
      const unsigned code = (raw[(size_t)(s >> 2)] >> (2 * (s & 3))) & 3u;
      uint8_t& o = row[j >> 2];
      o = (uint8_t)((o & ~(3u << (2 * (j & 3)))) | (code << (2 * (j & 3))));
    }
  }
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" tgw_status tgw_fam_match(const char* fam_path, const char* const* ids, int64_t n_ids, int64_t* idx,
                                    int64_t* n_file_samples, int64_t* n_found) {
  TGW_GUARD_BEGIN
  if (!fam_path) return fail(TGW_ERR_INVALID_ARG, "fam_path is NULL");
  if (n_ids < 0) return fail(TGW_ERR_INVALID_ARG, "negative n_ids");
  if (n_ids > 0 && (!ids || !idx)) return fail(TGW_ERR_INVALID_ARG, "ids / idx is NULL");
  std::ifstream in(fam_path);
  if (!in) return fail(TGW_ERR_INVALID_ARG, std::string("cannot open ") + fam_path);
  std::unordered_map<std::string, int64_t> where;  // IID -> line; -2 when it occurs twice
  std::string line;
  int64_t n = 0;
  while (std::getline(in, line)) {
    std::istringstream ss(line);
    std::string fid, iid;
    if (!(ss >> fid)) continue;  // blank line
    if (!(ss >> iid)) return fail(TGW_ERR_INVALID_ARG, "sample table line " + std::to_string(n + 1) + " has no IID");
    auto it = where.find(iid);
    if (it == where.end())
      where.emplace(iid, n);
    else
      it->second = -2;
    ++n;
  }
  std::unordered_map<std::string, int64_t> asked;
  int64_t found = 0;
  for (int64_t i = 0; i < n_ids; ++i) {
    if (!ids[i]) return fail(TGW_ERR_INVALID_ARG, "NULL id");
    const std::string id(ids[i]);
    if (!asked.emplace(id, i).second) return fail(TGW_ERR_INVALID_ARG, "id " + id + " is requested twice");
    auto it = where.find(id);
    if (it != where.end() && it->second == -2)
      return fail(TGW_ERR_INVALID_ARG, "id " + id + " occurs more than once in the sample table");
    idx[i] = it == where.end() ? -1 : it->second;
    found += idx[i] >= 0;
  }
  if (n_file_samples) *n_file_samples = n;
  if (n_found) *n_found = found;
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" tgw_status tgw_scan_bed(tgw_plan* pl, tgw_bed* b, int64_t m_begin, int64_t m_end, const tgw_outputs* outs,
                                   int64_t block_markers, int32_t n_threads, void* stream) {
  TGW_GUARD_BEGIN
  if (!pl) return fail(TGW_ERR_INVALID_ARG, "plan is NULL");
  if (!b) return fail(TGW_ERR_INVALID_ARG, "bed is NULL");
  if (block_markers < 0 || n_threads < 0) return fail(TGW_ERR_INVALID_ARG, "negative option");
  const int64_t n_sel = (int64_t)b->sel.size();
  if (plan_samples(pl) != n_sel) return fail(TGW_ERR_SHAPE, "plan's n_samples differs from the selected samples");
  if (m_begin < 0 || m_begin > m_end || m_end > b->n_markers)
    return fail(TGW_ERR_SHAPE, "need 0 <= m_begin <= m_end <= n_markers");
  const int64_t B = block_markers ? block_markers : kDefaultBlock;
  const int threads = n_threads ? std::min<int>(n_threads, kMaxThreads) : 4;
  const int64_t row_bytes = (n_sel + 63) / 64 * 16;  // 16 * ceil(n / 64): the scan's minimum
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));

  // streaming buffers
  if (b->device != dev || b->block != B || b->row_bytes != row_bytes) {
    release_stream_state(b);
    b->mem = current_allocator();
    b->device = dev;
    b->block = B;
    b->row_bytes = row_bytes;
    hipError_t e = hipStreamCreateWithFlags(&b->copy, hipStreamNonBlocking);
    for (auto& sl : b->slot) {
      if (e == hipSuccess) e = hipHostMalloc((void**)&sl.host, (size_t)(B * b->raw_bytes), hipHostMallocDefault);
      if (e == hipSuccess) e = dev_alloc(b->mem, (void**)&sl.draw, (size_t)(B * b->raw_bytes), nullptr);
      if (e == hipSuccess) e = dev_alloc(b->mem, (void**)&sl.dpack, (size_t)(B * row_bytes), nullptr);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.copied, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.used, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      release_stream_state(b);
      return hip_fail(e, "tgw_scan_bed buffers");
    }
  }
  if (b->sel_dirty) {
    for (auto& sl : b->slot)
      if (sl.pending) HIP_TRY(hipEventSynchronize(sl.used));  // the old selection may still be read
    dev_release_begin(b->mem);
    dev_free(b->mem, b->d_sel, nullptr);
    b->d_sel = nullptr;
    HIP_TRY(dev_alloc(b->mem, (void**)&b->d_sel, (size_t)n_sel * sizeof(int32_t), nullptr));
    HIP_TRY(hipMemcpy(b->d_sel, b->sel.data(), (size_t)n_sel * sizeof(int32_t), hipMemcpyHostToDevice));
    b->sel_dirty = false;
  }

  ScanCall c{b->slot[0].dpack, b->n_markers, row_bytes, TGW_CODE_PLINK_BED, m_begin, m_end, outs, 0};
  tgw_status st = check_call(pl, c, true);
  if (st != TGW_OK) return st;
  if (m_begin == m_end) return TGW_OK;

  HIP_TRY(enqueue_scan_begin(pl, outs, s));
  int k = 0;
  for (int64_t m0 = m_begin; m0 < m_end; m0 += B, ++k) {
    const int64_t m1 = std::min(m_end, m0 + B), nm = m1 - m0;
    tgw_bed::Slot& sl = b->slot[k & 1];
    if (sl.pending) HIP_TRY(hipEventSynchronize(sl.copied));  // the pinned slot is free again
    if (!pread_parallel(b->fd, sl.host, nm * b->raw_bytes, 3 + m0 * b->raw_bytes, threads)) {
      (void)hipStreamSynchronize(b->copy);
      return fail(TGW_ERR_INVALID_ARG, std::string("read failed: ") + std::strerror(errno));
    }
    if (sl.pending) HIP_TRY(hipStreamWaitEvent(b->copy, sl.used, 0));  // device slot no longer read
    HIP_TRY(hipMemcpyAsync(sl.draw, sl.host, (size_t)(nm * b->raw_bytes), hipMemcpyHostToDevice, b->copy));
    HIP_TRY(hipEventRecord(sl.copied, b->copy));
    HIP_TRY(hipStreamWaitEvent(s, sl.copied, 0));
    HIP_TRY(launch_bed_repack(sl.draw, b->raw_bytes, b->d_sel, n_sel, sl.dpack, row_bytes, nm, s));
    ScanCall cb = c;
    cb.geno = sl.dpack;
    cb.geno_row0 = m0;
    HIP_TRY(enqueue_scan_rows(pl, cb, m0, m1, s));
    HIP_TRY(hipEventRecord(sl.used, s));
    sl.pending = true;
  }
  HIP_TRY(enqueue_scan_end(pl, m_begin, s));
  HIP_TRY(hipStreamSynchronize(b->copy));  // every pinned slot is idle on return
  return TGW_OK;
  TGW_GUARD_END
}
