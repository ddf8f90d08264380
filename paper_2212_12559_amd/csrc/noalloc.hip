// mg_apply_dslash_noalloc: mg_apply_dslash with its work batch in a static
// device array instead of the context's scratch workspace, for callers that
// cannot allocate device memory at all.
//
// The array is a file-scope __device__ symbol: every GPU the library runs on
// holds its own copy (kNoallocScratchBytes) until the process ends.  Host code
// never passes the symbol itself to a kernel (on the host it only names a
// stand-in): its device address is looked up once per device with
// hipGetSymbolAddress, at mg_setup or at the first call on a device, and
// that address is what the kernels receive.
#include <mutex>

#include "mg.hpp"

namespace {

constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_lock;
void* g_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up once)
mg_status scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return mg::set_last_error(MG_E_HIP, "hipGetDevice failed or device index out of range");
  std::lock_guard<std::mutex> g(g_lock);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return mg::set_last_error(MG_E_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return MG_OK;
}

}  // namespace

mg_status mg::noalloc_init_current_device() {
  void* p = nullptr;
  return scratch_ptr(&p);
}

extern "C" {

size_t mg_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

mg_status mg_apply_dslash_noalloc(mg_ctx ctx, int32_t op, double mass, int32_t dtype, const void* in, void* out,
                                  int32_t nrhs, void* stream) {
  if (!ctx) return mg::set_last_error(MG_E_ARG, "null context");
  if (dtype != MG_C128 && dtype != MG_C64) return mg::set_last_error(MG_E_ARG, "dtype must be MG_C128 or MG_C64");
  if (nrhs < 1) return mg::set_last_error(MG_E_ARG, "nrhs must be >= 1");
  // ops 1, 3 and 4 stage one intermediate fine vector per rhs
  const size_t need = (op == 1 || op == 3 || op == 4)
                          ? (size_t)nrhs * (size_t)ctx->c.g0.V * 3 * (dtype == MG_C128 ? 16 : 8)
                          : 0;
  if (need > kNoallocScratchBytes)
    return mg::set_last_error(MG_E_ARG, "nrhs x fine vector exceeds the 64 MiB static work array");
  void* p = nullptr;
  const mg_status s = scratch_ptr(&p);
  if (s != MG_OK) return s;
  return mg::apply_dslash_with(ctx->c, op, mass, dtype, in, out, nrhs, stream, p);
}

}  // extern "C"
