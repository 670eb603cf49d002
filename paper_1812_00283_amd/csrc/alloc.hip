// Caching device allocator for the library's buffers.
//
// A build allocates and frees some eighty buffers and a count a few more;
// through the stream-ordered pool each call costs tens to hundreds of
// microseconds of host time, enough to leave the GPU idle between kernels.
// Here a freed block goes to a per-device free list together with the stream
// it was freed on and an event recorded there.  A later request of the same
// size class takes it when it comes from that stream (stream order puts the
// new work after the old) or once the event has completed; otherwise the
// block stays cached and a new one is allocated.  Memory is returned to the
// driver only when an allocation fails (blocks whose events have completed
// are freed and the allocation is retried).
//
// The blocks themselves come from hipMalloc, or from the functions the caller
// installs with bfc_set_allocator (for example a framework's caching
// allocator, so that the library's memory is counted in its pool).  Every
// block remembers the functions that made it and goes back through them.
#include "internal.hpp"

#include <map>
#include <unordered_map>

namespace bfc {

namespace {

// Where blocks come from: hipMalloc / hipFree when alloc is null.
struct Source {
  bfc_alloc_fn alloc = nullptr;
  bfc_free_fn free = nullptr;
  void* ctx = nullptr;
};

struct Block {
  size_t size = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  bool pending = false;  // ev marks the end of the work queued before the free
  Source src;            // the allocator that made the block
};

std::mutex g_mu;
Source g_src;  // the allocator for new blocks (guarded by g_mu)
std::unordered_map<void*, Block> g_live;
std::multimap<std::pair<int, size_t>, std::pair<void*, Block>> g_free;  // (device, size) -> block

// Rounds to 8 classes per power of two (at most 12.5% slack), 256 B minimum.
size_t size_class(size_t n) {
  if (n <= 256) return 256;
  int lg = 63 - __builtin_clzll((unsigned long long)(n - 1));  // n - 1 < 2^(lg + 1)
  const size_t step = lg >= 3 ? (size_t)1 << (lg - 2) : 1;
  return (n + step - 1) / step * step;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

void release_block(void* p, const Block& b) {
  if (b.src.free) b.src.free(p, b.stream, b.src.ctx);
  else (void)hipFree(p);
}

// Frees cached blocks of `device` (every device when device < 0) whose work
// has completed (caller holds g_mu).  Returns the number of bytes freed.
int64_t trim_locked(int device) {
  int64_t freed = 0;
  for (auto it = g_free.begin(); it != g_free.end();) {
    Block& b = it->second.second;
    if ((device < 0 || b.device == device) && (!b.pending || hipEventQuery(b.ev) == hipSuccess)) {
      if (b.ev) (void)hipEventDestroy(b.ev);
      int cur = -1;
      (void)hipGetDevice(&cur);
      if (cur != b.device) (void)hipSetDevice(b.device);
      release_block(it->second.first, b);
      if (cur >= 0 && cur != b.device) (void)hipSetDevice(cur);
      freed += (int64_t)b.size;
      it = g_free.erase(it);
    } else {
      ++it;
    }
  }
  return freed;
}

// One new block from the current source; null when it has no memory.
void* new_block(size_t size, hipStream_t s, const Source& src) {
  if (src.alloc) return src.alloc(size, s, src.ctx);
  void* p = nullptr;
  if (hipMalloc(&p, size) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

}  // namespace

void* cache_alloc(size_t bytes, hipStream_t s) {
  if (capturing(s)) throw Error{BFC_ERR_INVALID_ARGUMENT, "device allocation while the stream is being captured"};
  int device = 0;
  BFC_HIP(hipGetDevice(&device));
  const size_t size = size_class(bytes);
  {
    std::lock_guard<std::mutex> hold(g_mu);
    auto range = g_free.equal_range({device, size});
    for (auto it = range.first; it != range.second; ++it) {
      Block& b = it->second.second;
      if (b.pending && b.stream != s && hipEventQuery(b.ev) != hipSuccess) continue;
      void* p = it->second.first;
      Block nb = b;
      nb.pending = false;
      g_free.erase(it);
      g_live[p] = nb;
      return p;
    }
  }
  Source src;
  {
    std::lock_guard<std::mutex> hold(g_mu);
    src = g_src;
  }
  void* p = new_block(size, s, src);
  if (!p) {
    {
      std::lock_guard<std::mutex> hold(g_mu);
      trim_locked(device);
    }
    p = new_block(size, s, src);
    if (!p)
      throw Error{BFC_ERR_OUT_OF_MEMORY,
                  "device allocation of " + std::to_string(size) + " bytes failed" +
                      (src.alloc ? " (installed allocator returned null)" : "")};
  }
  std::lock_guard<std::mutex> hold(g_mu);
  Block b;
  b.size = size;
  b.device = device;
  b.stream = s;
  b.src = src;
  g_live[p] = b;
  return p;
}

void set_allocator(bfc_alloc_fn alloc_fn, bfc_free_fn free_fn, void* ctx) {
  std::lock_guard<std::mutex> hold(g_mu);
  // idle blocks go back to the allocator that made them before the switch
  trim_locked(-1);
  g_src.alloc = alloc_fn;
  g_src.free = free_fn;
  g_src.ctx = ctx;
}

int64_t trim_cache() {
  std::lock_guard<std::mutex> hold(g_mu);
  return trim_locked(-1);
}

int64_t cached_bytes() {
  std::lock_guard<std::mutex> hold(g_mu);
  int64_t b = 0;
  for (auto& kv : g_free) b += (int64_t)kv.second.second.size;
  return b;
}

void cache_free(void* p, hipStream_t s) {
  if (!p) return;
  std::lock_guard<std::mutex> hold(g_mu);
  auto it = g_live.find(p);
  if (it == g_live.end()) return;
  Block b = it->second;
  g_live.erase(it);
  // a block freed inside a stream capture is never reused: the captured work
  // that uses it runs at replay time
  if (capturing(s)) return;
  b.stream = s;
  b.pending = false;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur == b.device) {
    if (!b.ev) (void)hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
    b.pending = b.ev && hipEventRecord(b.ev, s) == hipSuccess;
  }
  if (!b.pending) {
    // no event on the block's device: wait for that device's work instead
    (void)hipSetDevice(b.device);
    (void)hipDeviceSynchronize();
    (void)hipSetDevice(cur);
  }
  g_free.emplace(std::make_pair(b.device, b.size), std::make_pair(p, b));
}

void cache_free_idle(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> hold(g_mu);
  auto it = g_live.find(p);
  if (it == g_live.end()) return;
  Block b = it->second;
  g_live.erase(it);
  b.stream = nullptr;
  b.pending = false;
  g_free.emplace(std::make_pair(b.device, b.size), std::make_pair(p, b));
}

// Per-thread pinned host buffer for small device-to-host read-backs: a copy
// into pinned memory is one transfer, where a pageable destination adds a
// staged copy and a wait of its own.  Grown on demand, kept until the
// process ends (a few KB per calling thread).
void* pinned_stage(size_t bytes) {
  thread_local void* buf = nullptr;
  thread_local size_t cap = 0;
  if (bytes > cap) {
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    cap = 0;
    const size_t want = bytes < 4096 ? 4096 : bytes;
    BFC_HIP(hipHostMalloc(&buf, want, hipHostMallocDefault));
    cap = want;
  }
  return buf;
}

}  // namespace bfc
