// Error plumbing and the caching device allocator.
#include <map>
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

struct FreeBlock {
  void *ptr;
  size_t bytes;
  hipStream_t stream;   // stream of the last use
  hipEvent_t ev;        // recorded at release on `stream`
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
      if (fb.stream != stream) LENS_HIP(hipStreamWaitEvent(stream, fb.ev, 0));
      LENS_HIP(hipEventDestroy(fb.ev));
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
      (void)hipEventSynchronize(kv.second.ev);
      (void)hipEventDestroy(kv.second.ev);
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

void pool_put(DevBuf &b, hipStream_t stream) {
  if (!b.ptr) return;
  DevicePool &pool = pool_for(b.device);
  FreeBlock fb{b.ptr, b.bytes, stream, nullptr};
  if (hipEventCreateWithFlags(&fb.ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(fb.ev, stream) != hipSuccess) {
    // cannot order the reuse: wait for the stream and free outright
    (void)hipGetLastError();
    (void)hipStreamSynchronize(stream);
    if (fb.ev) (void)hipEventDestroy(fb.ev);
    (void)hipFree(b.ptr);
    b.ptr = nullptr;
    return;
  }
  std::lock_guard<std::mutex> lk(pool.mu);
  pool.free_list.emplace(fb.bytes, fb);
  b.ptr = nullptr;
}

}  // namespace lensfmm
