// A sub-allocator over one caller-owned device buffer, shaped to be the
// registered device allocator (tgw_alloc_fn / tgw_free_fn with the arena as
// ctx).  A framework that owns the device memory (a torch tensor, say) hands
// the library one buffer up front; every handle then takes its memory from
// that buffer and gives it back there.
//
// Host bookkeeping only: the arena never reads or writes the buffer, so it
// works the same whether or not a device is present.  Blocks are multiples
// of 256 bytes at 256-byte offsets from a 256-byte-aligned base.  Allocation
// is best fit (the smallest free range that holds the request, the lowest
// address among equals), so the layout depends only on the sequence of calls.
// Freed ranges merge with free neighbours at once.  Streams are not looked
// at: the library gives memory back only after the device has finished with
// it, so a freed range can be handed out again on any stream.
#include "tgw_host.h"

#include <map>
#include <mutex>

using namespace tgw;

struct tgw_arena {
  uintptr_t base = 0;
  size_t capacity = 0;
  std::mutex mu;
  std::map<size_t, size_t> free_at;  // offset -> length of each free range
  std::map<size_t, size_t> used_at;  // offset -> length of each block handed out
  size_t in_use = 0, peak = 0;
  int64_t n_failed = 0, n_bad_free = 0;
};

namespace {
constexpr size_t kGrain = 256;
}

extern "C" tgw_status tgw_arena_create(void* d_base, size_t bytes, tgw_arena** out) {
  TGW_GUARD_BEGIN
  if (!out) return fail(TGW_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!d_base) return fail(TGW_ERR_INVALID_ARG, "d_base is NULL");
  if ((uintptr_t)d_base % kGrain) return fail(TGW_ERR_SHAPE, "d_base must be 256-byte aligned");
  if (bytes < kGrain) return fail(TGW_ERR_SHAPE, "the buffer must hold at least 256 bytes");
  auto* a = new tgw_arena();
  a->base = (uintptr_t)d_base;
  a->capacity = bytes / kGrain * kGrain;
  a->free_at[0] = a->capacity;
  *out = a;
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" void* tgw_arena_alloc(size_t bytes, void* stream, void* ctx) {
  (void)stream;
  auto* a = (tgw_arena*)ctx;
  if (!a) return nullptr;
  std::lock_guard<std::mutex> lk(a->mu);
  if (bytes > a->capacity) {
    ++a->n_failed;
    return nullptr;
  }
  const size_t need = bytes == 0 ? kGrain : (bytes + kGrain - 1) / kGrain * kGrain;
  auto best = a->free_at.end();
  for (auto it = a->free_at.begin(); it != a->free_at.end(); ++it)
    if (it->second >= need && (best == a->free_at.end() || it->second < best->second)) best = it;
  if (best == a->free_at.end()) {
    ++a->n_failed;
    return nullptr;
  }
  const size_t off = best->first, len = best->second;
  a->free_at.erase(best);
  if (len > need) a->free_at[off + need] = len - need;
  a->used_at[off] = need;
  a->in_use += need;
  if (a->in_use > a->peak) a->peak = a->in_use;
  return (void*)(a->base + off);
}

extern "C" void tgw_arena_free(void* ptr, void* stream, void* ctx) {
  (void)stream;
  auto* a = (tgw_arena*)ctx;
  if (!a || !ptr) return;
  std::lock_guard<std::mutex> lk(a->mu);
  const uintptr_t p = (uintptr_t)ptr;
  auto u = p >= a->base ? a->used_at.find((size_t)(p - a->base)) : a->used_at.end();
  if (u == a->used_at.end()) {  // not a block of this arena, or freed twice
    ++a->n_bad_free;
    return;
  }
  size_t off = u->first, len = u->second;
  a->used_at.erase(u);
  a->in_use -= len;
  auto next = a->free_at.lower_bound(off);
  if (next != a->free_at.end() && next->first == off + len) {
    len += next->second;
    next = a->free_at.erase(next);
  }
  if (next != a->free_at.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      off = prev->first;
      len += prev->second;
      a->free_at.erase(prev);
    }
  }
  a->free_at[off] = len;
}

extern "C" tgw_status tgw_arena_info(tgw_arena* a, tgw_arena_stats* out) {
  TGW_GUARD_BEGIN
  if (!a || !out) return fail(TGW_ERR_INVALID_ARG, "arena or out is NULL");
  std::lock_guard<std::mutex> lk(a->mu);
  out->capacity = a->capacity;
  out->in_use = a->in_use;
  out->peak = a->peak;
  out->largest_free = 0;
  for (const auto& f : a->free_at)
    if (f.second > out->largest_free) out->largest_free = f.second;
  out->n_blocks = (int64_t)a->used_at.size();
  out->n_free_ranges = (int64_t)a->free_at.size();
  out->n_failed = a->n_failed;
  out->n_bad_free = a->n_bad_free;
  return TGW_OK;
  TGW_GUARD_END
}

extern "C" tgw_status tgw_arena_destroy(tgw_arena* a) {
  TGW_GUARD_BEGIN
  if (!a) return TGW_OK;
  {
    std::lock_guard<std::mutex> lk(a->mu);
    if (!a->used_at.empty())
      return fail(TGW_ERR_INVALID_ARG, "the arena still has blocks in use (free the handles made under it first)");
  }
  delete a;
  return TGW_OK;
  TGW_GUARD_END
}
