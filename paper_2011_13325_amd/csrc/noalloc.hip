// eamg_vcycle_noalloc: the V-cycle of eamg_vcycle for callers that cannot allocate device
// memory or synchronize (code under HIP graph capture, tight serving loops).  Its per-call
// scratch -- the colour-major copies of r and z -- lives in a file-scope device array of fixed
// size instead of the hierarchy's own buffers; everything else it touches (level matrices and
// vectors, the coarsest inverse, the dense tail) was allocated by eamg_setup.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hierarchy.hpp"

namespace {

// 32 MiB: the two staging vectors of a level 0 with up to 2M dofs.
constexpr size_t kScratchDoubles = size_t(4) << 20;
static __device__ __align__(256) double scratch[kScratchDoubles];

// The array's device address on each device (the host-side name is only a stand-in), looked up
// once per device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

double *scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) eamg::fail(EAMG_ERR_INVALID_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    eamg::hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) eamg::fail(EAMG_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch[dev] = static_cast<double *>(p);
  }
  return g_scratch[dev];
}

}  // namespace

extern "C" eamg_status eamg_vcycle_noalloc(eamg_hierarchy *h, const double *r_dev, double *z_dev,
                                           int32_t precision, void *stream) {
  return eamg::guarded([&] {
    if (!h || !r_dev || !z_dev) eamg::fail(EAMG_ERR_INVALID_ARG, "NULL argument");
    eamg::reject_fused(h);
    if (precision != EAMG_PRECOND_VCYCLE && precision != EAMG_PRECOND_VCYCLE_FP32)
      eamg::fail(EAMG_ERR_INVALID_ARG, "precision must be EAMG_PRECOND_VCYCLE or EAMG_PRECOND_VCYCLE_FP32");
    if (precision == EAMG_PRECOND_VCYCLE_FP32 && !h->prm.vcycle_fp32)
      eamg::fail(EAMG_ERR_INVALID_ARG, "FP32 V-cycle needs setup with vcycle_fp32 = 1");
    if (h->prof_on) eamg::fail(EAMG_ERR_INVALID_ARG, "the profiler allocates events: disable it first");
    const size_t N = size_t(h->lv[0].n) * size_t(h->lv[0].bs);
    if (2 * N > kScratchDoubles)
      eamg::fail(EAMG_ERR_INVALID_ARG, "level 0 has " + std::to_string(N) +
                                           " dofs; the no-allocation V-cycle takes at most " +
                                           std::to_string(kScratchDoubles / 2));
    int dev = -1;
    eamg::hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev != h->device) eamg::fail(EAMG_ERR_INVALID_ARG, "the hierarchy lives on another device");
    double *sc = scratch_on(dev);
    // every entry of both staging vectors is written before it is read: nothing to clear
    eamg::vcycle_staged(h, r_dev, z_dev, precision == EAMG_PRECOND_VCYCLE_FP32, sc, sc + N,
                        static_cast<hipStream_t>(stream));
  });
}
