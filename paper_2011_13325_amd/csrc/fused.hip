// Kernels of the fused multi-system solve (fused.cpp): segmented CG vector operations with one
// set of CG scalars per system (the systems' dense operators are applied by the multi-part
// symmetric product of coarse.hip).
// Every sum has a fixed order (a block tree per block, then a system's blocks in order), so
// results are bitwise reproducible; no atomics.
#include "fused.hpp"

#include <cmath>

#include "panel.hpp"

namespace eamg {
namespace {

constexpr int kFB = 256;   // threads per block of the segmented kernels

inline int64_t cdiv64f(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Sum of v over the block's threads, fixed tree order; the result is valid in thread 0.
__device__ inline double block_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kFB / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

__global__ __launch_bounds__(kFB) void k_sdot(const int64_t *__restrict__ d0,
                                             const int64_t *__restrict__ d1,
                                             const double *__restrict__ a,
                                             const double *__restrict__ b, double *part) {
  __shared__ double sh[kFB];
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int64_t i = d0[k] + threadIdx.x; i < d1[k]; i += kFB) acc = fma(a[i], b[i], acc);
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[k] = t;
}

__global__ __launch_bounds__(kFB) void k_supdate_xr(int nsys, const int *__restrict__ sys,
                                                   const int64_t *__restrict__ d0,
                                                   const int64_t *__restrict__ d1,
                                                   const double *__restrict__ scal, double *x,
                                                   double *r, const double *__restrict__ p,
                                                   const double *__restrict__ q, double *part) {
  __shared__ double sh[kFB];
  const int k = blockIdx.x;
  const int m = sys[k];
  const bool active = scal[PS_ACTIVE * nsys + m] != 0.0;
  const double alpha = scal[PS_ALPHA * nsys + m];
  double acc = 0.0;
  for (int64_t i = d0[k] + threadIdx.x; i < d1[k]; i += kFB) {
    double ri = r[i];
    if (active) {
      x[i] = fma(alpha, p[i], x[i]);
      ri = fma(-alpha, q[i], ri);
      r[i] = ri;
    }
    acc = fma(ri, ri, acc);
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[k] = t;
}

__global__ __launch_bounds__(kFB) void k_supdate_p(int nsys, const int *__restrict__ sys,
                                                  const int64_t *__restrict__ d0,
                                                  const int64_t *__restrict__ d1,
                                                  const double *__restrict__ scal,
                                                  const double *__restrict__ z, double *p) {
  const int k = blockIdx.x;
  const int m = sys[k];
  if (scal[PS_ACTIVE * nsys + m] == 0.0) return;
  const double beta = scal[PS_BETA * nsys + m];
  for (int64_t i = d0[k] + threadIdx.x; i < d1[k]; i += kFB) p[i] = fma(beta, p[i], z[i]);
}

__global__ __launch_bounds__(kFB) void k_sfinite(int nsys, const int *__restrict__ sys,
                                                const int64_t *__restrict__ d0,
                                                const int64_t *__restrict__ d1,
                                                const double *__restrict__ a, double *scal) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const int k = blockIdx.x;
  for (int64_t i = d0[k] + threadIdx.x; i < d1[k]; i += kFB)
    if (!isfinite(a[i])) bad = 1;
  __syncthreads();
  // every block of the system that sees a bad entry stores the same value
  if (threadIdx.x == 0 && bad) scal[PS_NONFINITE * nsys + sys[k]] = 1.0;
}

// One thread per system: its blocks' partials in block order, then the CG bookkeeping of `op`
// (the same rules as the block-panel reduction, one system per column).
__global__ __launch_bounds__(kFB) void k_sreduce(int nsys, const int *__restrict__ bptr,
                                                const double *__restrict__ part, double *scal,
                                                int slot, int op) {
  const int m = int(blockIdx.x) * kFB + int(threadIdx.x);
  if (m >= nsys) return;
  double t = 0.0;
  for (int k = bptr[m]; k < bptr[m + 1]; ++k) t += part[k];
  auto at = [&](int sl) -> double & { return scal[sl * nsys + m]; };
  at(slot) = t;
  const bool active = at(PS_ACTIVE) != 0.0;
  auto stop_bad = [&]() {
    at(PS_BAD) = 1.0;
    at(PS_ACTIVE) = 0.0;
  };
  switch (op) {
    case PRED_INIT: {
      const bool finite = at(PS_NONFINITE) == 0.0 && isfinite(t);
      at(PS_ACTIVE) = (finite && t > 0.0) ? 1.0 : 0.0;
      at(PS_CONV) = (finite && t == 0.0) ? 1.0 : 0.0;
      at(PS_BAD) = finite ? 0.0 : 1.0;
      break;
    }
    case PRED_RHO0:
      if (active && !(t > 0.0 && isfinite(t))) {
        at(PS_ACTIVE) = 0.0;
        if (at(PS_RR0) == 0.0)
          at(PS_CONV) = 1.0;
        else
          at(PS_BAD) = 1.0;
      }
      break;
    case PRED_ALPHA:
      if (active) {
        if (!(t > 0.0) || !isfinite(t)) {
          stop_bad();
          at(PS_ALPHA) = 0.0;
        } else {
          at(PS_ALPHA) = at(PS_RHO) / t;
        }
      }
      break;
    case PRED_BETA:
      if (active) {
        if (!(t > 0.0) || !isfinite(t)) {
          stop_bad();
        } else {
          at(PS_BETA) = t / at(PS_RHO);
          at(PS_RHO) = t;
        }
      }
      break;
    case PRED_RR:
      if (active) {
        at(PS_ITS) += 1.0;
        if (!isfinite(t)) {
          stop_bad();
        } else if (sqrt(t) <= at(PS_RTOL) * sqrt(at(PS_BB))) {
          at(PS_CONV) = 1.0;
          at(PS_ACTIVE) = 0.0;
        } else if (at(PS_ITS) >= at(PS_MAXIT)) {
          at(PS_ACTIVE) = 0.0;
        }
      }
      break;
    default:
      break;
  }
}

__global__ void k_sinit(int nsys, double rtol, double max_it, double *scal) {
  const int i = int(blockIdx.x) * kFB + int(threadIdx.x);
  if (i >= PS_COUNT * nsys) return;
  const int slot = i / nsys;
  scal[i] = slot == PS_RTOL ? rtol : slot == PS_MAXIT ? max_it : 0.0;
}

__global__ void k_scatter_in(int n, int bs, const int *__restrict__ map,
                             const uint8_t *__restrict__ mask, const double *__restrict__ in,
                             double *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * kFB + threadIdx.x;
  if (i >= int64_t(n) * bs) return;
  const int64_t v = i / bs;
  const int c = int(i - v * bs);
  out[int64_t(map[v]) * bs + c] = (mask && mask[v]) ? 0.0 : in[i];
}

__global__ void k_gather_out(int n, int bs, const int *__restrict__ map,
                             const double *__restrict__ in, double *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * kFB + threadIdx.x;
  if (i >= int64_t(n) * bs) return;
  const int64_t v = i / bs;
  const int c = int(i - v * bs);
  out[i] = in[int64_t(map[v]) * bs + c];
}

}  // namespace

hipError_t launch_sdot(const SegTable &T, const double *a, const double *b, double *part,
                       hipStream_t s) {
  if (T.nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sdot, dim3(T.nblk), dim3(kFB), 0, s, T.d0, T.d1, a, b, part);
  return hipGetLastError();
}

hipError_t launch_sreduce(const SegTable &T, const double *part, double *scal, int slot, int op,
                          hipStream_t s) {
  if (T.nsys == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sreduce, dim3(unsigned(cdiv64f(T.nsys, kFB))), dim3(kFB), 0, s, T.nsys,
                     T.bptr, part, scal, slot, op);
  return hipGetLastError();
}

hipError_t launch_supdate_xr(const SegTable &T, const double *scal, double *x, double *r,
                             const double *p, const double *q, double *part, hipStream_t s) {
  if (T.nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_supdate_xr, dim3(T.nblk), dim3(kFB), 0, s, T.nsys, T.sys, T.d0, T.d1, scal,
                     x, r, p, q, part);
  return hipGetLastError();
}

hipError_t launch_supdate_p(const SegTable &T, const double *scal, const double *z, double *p,
                            hipStream_t s) {
  if (T.nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_supdate_p, dim3(T.nblk), dim3(kFB), 0, s, T.nsys, T.sys, T.d0, T.d1, scal,
                     z, p);
  return hipGetLastError();
}

hipError_t launch_sfinite(const SegTable &T, const double *a, double *scal, hipStream_t s) {
  if (T.nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sfinite, dim3(T.nblk), dim3(kFB), 0, s, T.nsys, T.sys, T.d0, T.d1, a, scal);
  return hipGetLastError();
}

hipError_t launch_sinit(int nsys, double rtol, int max_it, double *scal, hipStream_t s) {
  if (nsys < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sinit, dim3(unsigned(cdiv64f(int64_t(PS_COUNT) * nsys, kFB))), dim3(kFB), 0,
                     s, nsys, rtol, double(max_it), scal);
  return hipGetLastError();
}

hipError_t launch_scatter_in(int n, int bs, const int *map, const uint8_t *mask, const double *in,
                             double *out, hipStream_t s) {
  const int64_t nn = int64_t(n) * bs;
  if (nn == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_in, dim3(unsigned(cdiv64f(nn, kFB))), dim3(kFB), 0, s, n, bs, map,
                     mask, in, out);
  return hipGetLastError();
}

hipError_t launch_gather_out(int n, int bs, const int *map, const double *in, double *out,
                             hipStream_t s) {
  const int64_t nn = int64_t(n) * bs;
  if (nn == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_out, dim3(unsigned(cdiv64f(nn, kFB))), dim3(kFB), 0, s, n, bs, map,
                     in, out);
  return hipGetLastError();
}

}  // namespace eamg
