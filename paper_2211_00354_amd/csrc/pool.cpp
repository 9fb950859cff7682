// Error plumbing and the caching device allocator.
#include <map>
#include <memory>
#include <mutex>

#include "lens_internal.h"

namespace lensfmm {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
const std::string &last_error() { return g_last_error; }

void fail(lens_status st, const std::string &msg) { throw LensError{st, msg}; }

void check_hip(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    lens_status st = (e == hipErrorOutOfMemory) ? LENS_ENOMEM : LENS_EDEVICE;
    fail(st, std::string(what) + ": " + hipGetErrorString(e));
  }
}

namespace {

// One event per release batch, shared by the batch's blocks and destroyed
// with the last of them.
struct ReleaseEvent {
  hipEvent_t ev = nullptr;
  ~ReleaseEvent() {
    if (ev) (void)hipEventDestroy(ev);
  }
};

struct FreeBlock {
  void *ptr;
  size_t bytes;
  hipStream_t stream;                  // stream of the last use
  std::shared_ptr<ReleaseEvent> ev;    // recorded at release on `stream`
};

struct DevicePool {
  std::mutex mu;
  std::multimap<size_t, FreeBlock> free_list;
};

std::mutex g_pools_mu;
std::map<int, DevicePool *> g_pools;

DevicePool &pool_for(int dev) {
  std::lock_guard<std::mutex> lk(g_pools_mu);
  auto it = g_pools.find(dev);
  if (it != g_pools.end()) return *it->second;
  auto *p = new DevicePool();  // lives until process exit
  g_pools[dev] = p;
  return *p;
}

size_t round_bytes(size_t b) {
  const size_t g = (b < (size_t(1) << 20)) ? 4096 : (size_t(1) << 20);
  return (b + g - 1) / g * g;
}

}  // namespace

DevBuf pool_get(size_t bytes, hipStream_t stream) {
  int dev = 0;
  LENS_HIP(hipGetDevice(&dev));
  DevBuf out;
  out.device = dev;
  out.bytes = round_bytes(bytes == 0 ? 1 : bytes);
  DevicePool &pool = pool_for(dev);
  {
    std::lock_guard<std::mutex> lk(pool.mu);
    auto it = pool.free_list.lower_bound(out.bytes);
    if (it != pool.free_list.end() && it->first <= out.bytes * 2) {
      FreeBlock fb = it->second;
      pool.free_list.erase(it);
      if (fb.stream != stream) LENS_HIP(hipStreamWaitEvent(stream, fb.ev->ev, 0));
      out.ptr = fb.ptr;
      out.bytes = fb.bytes;
      return out;
    }
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, out.bytes);
  if (e == hipErrorOutOfMemory) {
    // give cached blocks back and retry once
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(pool.mu);
    for (auto &kv : pool.free_list) {
      (void)hipEventSynchronize(kv.second.ev->ev);
      (void)hipFree(kv.second.ptr);
    }
    pool.free_list.clear();
    e = hipMalloc(&p, out.bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(LENS_ENOMEM, "device allocation of " + std::to_string(out.bytes) + " bytes failed");
  }
  out.ptr = p;
  return out;
}

void pool_put_batch(DevBuf *const *bufs, size_t n, hipStream_t stream) {
  size_t live = 0;
  for (size_t i = 0; i < n; ++i) live += bufs[i]->ptr != nullptr;
  if (live == 0) return;
  auto ev = std::make_shared<ReleaseEvent>();
  if (hipEventCreateWithFlags(&ev->ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ev->ev, stream) != hipSuccess) {
    // cannot order the reuse: wait for the stream and free outright
    (void)hipGetLastError();
    (void)hipStreamSynchronize(stream);
    for (size_t i = 0; i < n; ++i) {
      if (bufs[i]->ptr) (void)hipFree(bufs[i]->ptr);
      bufs[i]->ptr = nullptr;
    }
    return;
  }
  for (size_t i = 0; i < n; ++i) {
    DevBuf &b = *bufs[i];
    if (!b.ptr) continue;
    DevicePool &pool = pool_for(b.device);
    std::lock_guard<std::mutex> lk(pool.mu);
    pool.free_list.emplace(b.bytes, FreeBlock{b.ptr, b.bytes, stream, ev});
    b.ptr = nullptr;
  }
}

void pool_put(DevBuf &b, hipStream_t stream) {
  DevBuf *p = &b;
  pool_put_batch(&p, 1, stream);
}

}  // namespace lensfmm
