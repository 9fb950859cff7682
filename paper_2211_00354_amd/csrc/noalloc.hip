// Allocation-free grid deflection (lens_deflect_noalloc): the per-call
// buffers of lens_deflect live in a static device array instead of the
// library's pool, for callers that cannot allocate device memory.
//
// The array's device address differs per GPU and is not its host-side name:
// it is looked up once per device with hipGetSymbolAddress, on the device's
// first call, and only that address is handed to the kernels.
#include <mutex>
#include <vector>

#include "lens_internal.h"

static __device__ __align__(256) unsigned char scratch[LENS_NOALLOC_SCRATCH_BYTES];

namespace lensfmm {
namespace {

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // index = device

// The current device's address of `scratch` (looked up on first use).
char *scratch_on_device() {
  int dev = 0;
  LENS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      fail(LENS_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = ptr;
  }
  return static_cast<char *>(g_scratch_ptr[dev]);
}

}  // namespace
}  // namespace lensfmm

extern "C" LENS_API lens_status lens_deflect_noalloc(lens_plan *plan, const lens_field *field,
                                                     const lens_grid *grid, double *y_out,
                                                     const lens_opts *opts, void *stream) {
  using namespace lensfmm;
  try {
    char *region = scratch_on_device();
    deflect_grid_no_alloc(plan, field, grid, y_out, opts, region, LENS_NOALLOC_SCRATCH_BYTES,
                          (hipStream_t)stream);
    return LENS_OK;
  } catch (const LensError &e) {
    set_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return LENS_ENOMEM;
  } catch (...) {
    set_error("unexpected internal error");
    return LENS_EDEVICE;
  }
}
