// Entry points that allocate nothing and take no workspace: their scratch
// memory is a fixed device array of this library, one per GPU, held until the
// process ends.  For callers that cannot allocate device memory (code under
// stream capture, tight serving loops).
//
// The array below is a device symbol: in host code its name is not a device
// address.  Its address on the current device is looked up once per device
// with hipGetSymbolAddress and every kernel argument uses that address.
#include <mutex>

#include "lqcd_internal.h"

using namespace lqcd;

namespace {

// meson partials of the largest supported lattice (see lqcd.h)
static __device__ __align__(256) double2 scratch[LQCD_NOALLOC_SCRATCH_BYTES / sizeof(double2)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// address of `scratch` on the current device (looked up on the first call per
// device, with that device current); nullptr and the last error set on failure
void* scratch_on_current_device(const char* who) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    fail(LQCD_EDEVICE, "%s: hipGetDevice: %s", who, hipGetErrorString(e));
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    fail(LQCD_EDEVICE, "%s: device %d beyond the %d this library tracks", who, dev, kMaxDevices);
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      fail(LQCD_EDEVICE, "%s: hipGetSymbolAddress(scratch) on device %d: %s", who, dev, hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" size_t lqcd_noalloc_scratch_bytes(void) { return (size_t)LQCD_NOALLOC_SCRATCH_BYTES; }

extern "C" int lqcd_meson_noalloc(const lqcd_geom_t* g, const void* psi, int npairs, const int32_t* pairs, void* C,
                                  void* G, void* stream) {
  const int rc = meson_check("lqcd_meson_noalloc", g, psi, npairs, pairs, C, G);
  if (rc) return rc;
  const size_t need = meson_scratch_bytes(g);
  if (need > (size_t)LQCD_NOALLOC_SCRATCH_BYTES)
    return fail(LQCD_EINVAL, "lqcd_meson_noalloc: lattice needs %zu scratch bytes, above the fixed %zu", need,
                (size_t)LQCD_NOALLOC_SCRATCH_BYTES);
  double2* s = static_cast<double2*>(scratch_on_current_device("lqcd_meson_noalloc"));
  if (!s) return LQCD_EDEVICE;
  double2* outs[kMaxMesonPairs];
  for (int p = 0; p < npairs; ++p) outs[p] = (double2*)C + (size_t)p * g->desc.L[3];
  // every partial the reduction reads is written first by the same call: no
  // clearing needed
  LQCD_HIP(launch_meson(g->kg, (const double2*)psi, npairs, pairs, outs, 1.0, (double2*)G, s, (hipStream_t)stream));
  return LQCD_OK;
}
