// Host-side plumbing shared by the runtime's translation units (the scan
// runtime and the PLINK .bed streamer): error reporting and the pieces of
// the scan launch sequence.
#pragma once

#include "../../include/tgw.h"
#include "../../include/tgw_debug.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace tgw {

tgw_status fail(tgw_status s, const std::string& msg);
tgw_status hip_fail(hipError_t e, const char* what);

// Device memory of the handles: the allocator registered with
// tgw_set_allocator when a handle is made (alloc NULL: hipMalloc / hipFree).
// A handle keeps the one it was made with and frees through it.
struct DevAllocator {
  tgw_alloc_fn alloc = nullptr;
  tgw_free_fn free = nullptr;
  void* ctx = nullptr;
};
DevAllocator current_allocator();
hipError_t dev_alloc(const DevAllocator& a, void** p, size_t bytes, hipStream_t s);
void dev_free(const DevAllocator& a, void* p, hipStream_t s);
// before a custom allocator gets memory back: no enqueued work may still use
// it (hipFree waits for the device by itself)
void dev_release_begin(const DevAllocator& a);

// One scan request.  geno points at the packed row of marker geno_row0
// (0 for a caller's whole genotype matrix, the block's first marker for a
// streamed block); rows [m0 - geno_row0, m1 - geno_row0) are read for the
// markers [m0, m1).  Output row of marker m: m - m_begin.
struct ScanCall {
  const uint8_t* geno;
  int64_t n_markers, row_bytes;
  int code;
  int64_t m_begin, m_end;
  const tgw_outputs* outs;
  int64_t geno_row0;
};

tgw_status check_call(const tgw_plan* pl, const ScanCall& c, bool need_outs);
int64_t plan_samples(const tgw_plan* pl);
// bind the outputs and clear the tail list
hipError_t enqueue_scan_begin(tgw_plan* pl, const tgw_outputs* outs, hipStream_t s);
// markers [m0, m1) of the call, in the plan's marker blocks
hipError_t enqueue_scan_rows(tgw_plan* pl, const ScanCall& c, int64_t m0, int64_t m1, hipStream_t s);
// FP64 tail of every test the call flagged
hipError_t enqueue_scan_end(tgw_plan* pl, int64_t m_begin, hipStream_t s);

}  // namespace tgw

#define HIP_TRY(expr)                                       \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return tgw::hip_fail(_e, #expr);  \
  } while (0)

#define TGW_GUARD_BEGIN try {
#define TGW_GUARD_END                                                              \
  }                                                                                \
  catch (const std::bad_alloc&) {                                                  \
    return tgw::fail(TGW_ERR_OUT_OF_MEMORY, "host allocation failed");             \
  }                                                                                \
  catch (const std::exception& ex) {                                               \
    return tgw::fail(TGW_ERR_DEVICE, std::string("internal error: ") + ex.what()); \
  }                                                                                \
  catch (...) {                                                                    \
    return tgw::fail(TGW_ERR_DEVICE, "internal error");                            \
  }
