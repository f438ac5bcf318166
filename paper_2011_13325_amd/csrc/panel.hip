// Block-panel kernels for gfx950: K right-hand sides per launch (layout and lane mapping in
// panel.hpp).  The V-cycle kernels are templated on the value type T of matrices and vectors
// (double, or float for the FP32 V-cycle) and accumulate in T; the CG kernels are FP64.
#include <hip/hip_runtime.h>

#include <cmath>

#include "panel.hpp"

namespace eamg {
namespace {

constexpr int kPB = 256;   // threads per workgroup; a multiple of every panel width K

inline unsigned pgrid(int64_t items, int per_block) {
  return unsigned((items + per_block - 1) / per_block);
}

template <class T>
const T *pvals(const SoaMat &M);
template <>
const double *pvals<double>(const SoaMat &M) {
  return M.val;
}
template <>
const float *pvals<float>(const SoaMat &M) {
  return M.val32;
}

// acc[r] += sum over blocks p in [p0, p1) of M_p X_col(p), column k.  The block's entries are
// the same address for the K lanes of the team; the X loads are K-wide contiguous.
template <class T, int BR, int BC>
__device__ inline void pteam_accumulate(int p0, int p1, int k, int K, const int *__restrict__ col,
                                        const T *__restrict__ val, int64_t nnz,
                                        const T *__restrict__ x, T (&acc)[BR]) {
#pragma unroll 2
  for (int p = p0; p < p1; ++p) {
    const int64_t c = col[p];
    T xv[BC];
#pragma unroll
    for (int cc = 0; cc < BC; ++cc) xv[cc] = x[(c * BC + cc) * K + k];
#pragma unroll
    for (int r = 0; r < BR; ++r)
#pragma unroll
      for (int cc = 0; cc < BC; ++cc) acc[r] = fma(val[int64_t(r * BC + cc) * nnz + p], xv[cc], acc[r]);
  }
}

// One colour of the symmetric block Gauss-Seidel sweep for K columns (see launch_pgs_fwd /
// launch_pgs_bwd).  The row's D^+ block and right-hand side are loaded before the row's blocks
// so their latency overlaps the block stream.
template <class T, int B, bool FWD>
__global__ __launch_bounds__(kPB) void k_pgs_color(int r0, int r1, int K, const int *__restrict__ rp,
                                                   const int *__restrict__ col,
                                                   const int *__restrict__ diag,
                                                   const T *__restrict__ val, int64_t nnz,
                                                   const T *__restrict__ Dinv,
                                                   const T *__restrict__ b, T *x, T *r) {
  const int k = threadIdx.x & (K - 1);
  const int row = r0 + blockIdx.x * (kPB / K) + threadIdx.x / K;
  if (row >= r1) return;
  const int p0 = rp[row];
  const int dp = diag[row];
  const int p1 = FWD ? dp : rp[row + 1];
  T bq[B], D[B][B];
#pragma unroll
  for (int q = 0; q < B; ++q) {
    bq[q] = b[(int64_t(row) * B + q) * K + k];
#pragma unroll
    for (int c = 0; c < B; ++c) D[q][c] = Dinv[(int64_t(row) * B + q) * B + c];
  }
  T acc[B];
#pragma unroll
  for (int q = 0; q < B; ++q) acc[q] = T(0);
  pteam_accumulate<T, B, B>(p0, p1, k, K, col, val, nnz, x, acc);
  T t[B], xi[B];
#pragma unroll
  for (int q = 0; q < B; ++q) t[q] = bq[q] - acc[q];
#pragma unroll
  for (int q = 0; q < B; ++q) {
    T v = T(0);
#pragma unroll
    for (int c = 0; c < B; ++c) v = fma(D[q][c], t[c], v);
    xi[q] = v;
  }
  if (FWD) {
#pragma unroll
    for (int q = 0; q < B; ++q) {
      T v = t[q];
#pragma unroll
      for (int c = 0; c < B; ++c) v = fma(-val[int64_t(q * B + c) * nnz + dp], xi[c], v);
      x[(int64_t(row) * B + q) * K + k] = xi[q];
      r[(int64_t(row) * B + q) * K + k] = v;
    }
  } else {
#pragma unroll
    for (int q = 0; q < B; ++q) x[(int64_t(row) * B + q) * K + k] += xi[q];
  }
}

template <class T, int B>
__global__ __launch_bounds__(kPB) void k_presid_upper(int n_rows, int K, const int *__restrict__ rp,
                                                      const int *__restrict__ col,
                                                      const int *__restrict__ diag,
                                                      const T *__restrict__ val, int64_t nnz,
                                                      const T *__restrict__ x, T *__restrict__ r) {
  const int k = threadIdx.x & (K - 1);
  const int row = blockIdx.x * (kPB / K) + threadIdx.x / K;
  if (row >= n_rows) return;
  T rq[B], acc[B];
#pragma unroll
  for (int q = 0; q < B; ++q) {
    rq[q] = r[(int64_t(row) * B + q) * K + k];
    acc[q] = T(0);
  }
  pteam_accumulate<T, B, B>(diag[row] + 1, rp[row + 1], k, K, col, val, nnz, x, acc);
#pragma unroll
  for (int q = 0; q < B; ++q) r[(int64_t(row) * B + q) * K + k] = rq[q] - acc[q];
}

template <class T, int BR, int BC>
__global__ __launch_bounds__(kPB) void k_prect(int n_rows, int K, const int *__restrict__ rp,
                                               const int *__restrict__ col,
                                               const T *__restrict__ val, int64_t nnz,
                                               const T *__restrict__ x, T *__restrict__ y,
                                               int accumulate) {
  const int k = threadIdx.x & (K - 1);
  const int row = blockIdx.x * (kPB / K) + threadIdx.x / K;
  if (row >= n_rows) return;
  T acc[BR];
#pragma unroll
  for (int q = 0; q < BR; ++q) acc[q] = accumulate ? y[(int64_t(row) * BR + q) * K + k] : T(0);
  pteam_accumulate<T, BR, BC>(rp[row], rp[row + 1], k, K, col, val, nnz, x, acc);
#pragma unroll
  for (int q = 0; q < BR; ++q) y[(int64_t(row) * BR + q) * K + k] = acc[q];
}

// Y = D X: team of K lanes per row of D, FP64 accumulation.
template <class T>
__global__ __launch_bounds__(kPB) void k_pdense(int n, int K, const double *__restrict__ D,
                                                const T *__restrict__ x, T *__restrict__ y) {
  const int k = threadIdx.x & (K - 1);
  const int row = blockIdx.x * (kPB / K) + threadIdx.x / K;
  if (row >= n) return;
  double acc = 0.0;
  const double *Dr = D + int64_t(row) * n;
#pragma unroll 4
  for (int c = 0; c < n; ++c) acc = fma(Dr[c], double(x[int64_t(c) * K + k]), acc);
  y[int64_t(row) * K + k] = T(acc);
}

// Reduce v over the threads of a workgroup that share t mod K; the sums end in threads t < K.
__device__ inline double pcol_sum(double v, int K, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kPB / 2; s >= K; s >>= 1) {
    if (int(threadIdx.x) < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[threadIdx.x];
}

template <int B>
__global__ __launch_bounds__(kPB) void k_pspmv(int n_rows, int K, const int *__restrict__ rp,
                                               const int *__restrict__ col,
                                               const double *__restrict__ val, int64_t nnz,
                                               const double *__restrict__ x, double *__restrict__ y,
                                               double *part) {
  __shared__ double sh[kPB];
  const int k = threadIdx.x & (K - 1);
  const int row = blockIdx.x * (kPB / K) + threadIdx.x / K;
  double d = 0.0;
  if (row < n_rows) {
    double acc[B];
#pragma unroll
    for (int q = 0; q < B; ++q) acc[q] = 0.0;
    pteam_accumulate<double, B, B>(rp[row], rp[row + 1], k, K, col, val, nnz, x, acc);
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int64_t e = (int64_t(row) * B + q) * K + k;
      y[e] = acc[q];
      d = fma(x[e], acc[q], d);
    }
  }
  if (part) {
    const double s = pcol_sum(d, K, sh);
    if (int(threadIdx.x) < K) part[int64_t(blockIdx.x) * K + threadIdx.x] = s;
  }
}

// ---- panel CG vectors -------------------------------------------------------------------------
// Entry e of a panel vector belongs to column e mod K; grid strides are multiples of K, so a
// thread always meets the same column.

constexpr int kPDotMax = 1024;

__global__ __launch_bounds__(kPB) void k_pdot(int64_t n, int K, const double *__restrict__ a,
                                              const double *__restrict__ b, double *part) {
  __shared__ double sh[kPB];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kPB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kPB)
    s = fma(a[i], b[i], s);
  const double t = pcol_sum(s, K, sh);
  if (int(threadIdx.x) < K) part[int64_t(blockIdx.x) * K + threadIdx.x] = t;
}

__global__ __launch_bounds__(kPB) void k_preduce(int nparts, int K, const double *__restrict__ part,
                                                 double *scal, int slot, int op) {
  __shared__ double sh[kPB];
  const int k = threadIdx.x & (K - 1);
  double s = 0.0;
  for (int j = threadIdx.x / K; j < nparts; j += kPB / K) s += part[int64_t(j) * K + k];
  const double t = pcol_sum(s, K, sh);
  if (int(threadIdx.x) >= K) return;
  double *S = scal;
  auto at = [&](int sl) -> double & { return S[sl * K + k]; };
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
          at(PS_ACTIVE) = 0.0;
          at(PS_CONV) = 1.0;
        } else if (at(PS_ITS) >= at(PS_MAXIT)) {
          at(PS_ACTIVE) = 0.0;
        }
      }
      break;
    default: break;
  }
}

__global__ __launch_bounds__(kPB) void k_pupdate_xr(int64_t n, int K, const double *__restrict__ scal,
                                                    double *x, double *r, const double *__restrict__ p,
                                                    const double *__restrict__ q, double *part) {
  __shared__ double sh[kPB];
  const int k = threadIdx.x & (K - 1);
  const bool active = scal[PS_ACTIVE * K + k] != 0.0;
  const double alpha = scal[PS_ALPHA * K + k];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kPB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kPB) {
    double ri = r[i];
    if (active) {
      x[i] = fma(alpha, p[i], x[i]);
      ri = fma(-alpha, q[i], ri);
      r[i] = ri;
    }
    s = fma(ri, ri, s);
  }
  const double t = pcol_sum(s, K, sh);
  if (int(threadIdx.x) < K) part[int64_t(blockIdx.x) * K + threadIdx.x] = t;
}

__global__ __launch_bounds__(kPB) void k_pupdate_p(int64_t n, int K, const double *__restrict__ scal,
                                                   const double *__restrict__ z, double *p) {
  const int k = threadIdx.x & (K - 1);
  if (scal[PS_ACTIVE * K + k] == 0.0) return;
  const double beta = scal[PS_BETA * K + k];
  for (int64_t i = int64_t(blockIdx.x) * kPB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kPB)
    p[i] = fma(beta, p[i], z[i]);
}

__global__ void k_pinit_scal(int K, double rtol, double max_it, double *scal) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= PS_COUNT * K) return;
  const int slot = i / K;
  scal[i] = slot == PS_RTOL ? rtol : slot == PS_MAXIT ? max_it : 0.0;
}

__global__ void k_pfinite(int64_t n, int K, const double *a, double *scal) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(a[i])) scal[PS_NONFINITE * K + int(i % K)] = 1.0;
}

__global__ void k_pzero_unstarted(int64_t n, int K, const double *scal, double *x) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = int(i % K);
  if (scal[PS_BB * K + k] == 0.0 || scal[PS_NONFINITE * K + k] != 0.0) x[i] = 0.0;
}

__global__ void k_ppack(int n, int bs, int K, int nrhs, const int *perm, const uint8_t *mask,
                        const double *in, int64_t ld, double *out) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= int64_t(n) * bs * K) return;
  const int k = int(gid % K);
  const int64_t d = gid / K;
  const int64_t r = d / bs;
  const int c = int(d % bs);
  const int o = perm[r];
  out[gid] = (k >= nrhs || (mask && mask[o])) ? 0.0 : in[int64_t(k) * ld + int64_t(o) * bs + c];
}

__global__ void k_punpack(int n, int bs, int K, int nrhs, const int *perm, const double *in,
                          double *out, int64_t ld) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= int64_t(n) * bs * K) return;
  const int k = int(gid % K);
  if (k >= nrhs) return;
  const int64_t d = gid / K;
  const int64_t r = d / bs;
  const int c = int(d % bs);
  out[int64_t(k) * ld + int64_t(perm[r]) * bs + c] = in[gid];
}

bool valid_k(int K) { return K >= 1 && K <= 64 && (K & (K - 1)) == 0; }

}  // namespace

#define EAMG_PCHECK() return hipGetLastError()

template <class T>
hipError_t launch_pgs_fwd(const SoaMat &A, const T *Dinv, int r0, int r1, int K, const T *b, T *x,
                          T *r, hipStream_t s) {
  if (r1 <= r0) return hipSuccess;
  const T *val = pvals<T>(A);
  if (!val || !valid_k(K) || !A.diag) return hipErrorInvalidValue;
  const dim3 grid(pgrid(r1 - r0, kPB / K));
  switch (A.br) {
    case 1: hipLaunchKernelGGL((k_pgs_color<T, 1, true>), grid, dim3(kPB), 0, s, r0, r1, K, A.rp, A.col, A.diag, val, A.nnz, Dinv, b, x, r); break;
    case 3: hipLaunchKernelGGL((k_pgs_color<T, 3, true>), grid, dim3(kPB), 0, s, r0, r1, K, A.rp, A.col, A.diag, val, A.nnz, Dinv, b, x, r); break;
    case 6: hipLaunchKernelGGL((k_pgs_color<T, 6, true>), grid, dim3(kPB), 0, s, r0, r1, K, A.rp, A.col, A.diag, val, A.nnz, Dinv, b, x, r); break;
    default: return hipErrorInvalidValue;
  }
  EAMG_PCHECK();
}

template <class T>
hipError_t launch_pgs_bwd(const SoaMat &A, const T *Dinv, int r0, int r1, int K, const T *b, T *x,
                          hipStream_t s) {
  if (r1 <= r0) return hipSuccess;
  const T *val = pvals<T>(A);
  if (!val || !valid_k(K) || !A.diag) return hipErrorInvalidValue;
  const dim3 grid(pgrid(r1 - r0, kPB / K));
  T *none = nullptr;
  switch (A.br) {
    case 1: hipLaunchKernelGGL((k_pgs_color<T, 1, false>), grid, dim3(kPB), 0, s, r0, r1, K, A.rp, A.col, A.diag, val, A.nnz, Dinv, b, x, none); break;
    case 3: hipLaunchKernelGGL((k_pgs_color<T, 3, false>), grid, dim3(kPB), 0, s, r0, r1, K, A.rp, A.col, A.diag, val, A.nnz, Dinv, b, x, none); break;
    case 6: hipLaunchKernelGGL((k_pgs_color<T, 6, false>), grid, dim3(kPB), 0, s, r0, r1, K, A.rp, A.col, A.diag, val, A.nnz, Dinv, b, x, none); break;
    default: return hipErrorInvalidValue;
  }
  EAMG_PCHECK();
}

template <class T>
hipError_t launch_presid_upper(const SoaMat &A, int K, const T *x, T *r, hipStream_t s) {
  if (A.n_rows == 0) return hipSuccess;
  const T *val = pvals<T>(A);
  if (!val || !valid_k(K) || !A.diag) return hipErrorInvalidValue;
  const dim3 grid(pgrid(A.n_rows, kPB / K));
  switch (A.br) {
    case 1: hipLaunchKernelGGL((k_presid_upper<T, 1>), grid, dim3(kPB), 0, s, A.n_rows, K, A.rp, A.col, A.diag, val, A.nnz, x, r); break;
    case 3: hipLaunchKernelGGL((k_presid_upper<T, 3>), grid, dim3(kPB), 0, s, A.n_rows, K, A.rp, A.col, A.diag, val, A.nnz, x, r); break;
    case 6: hipLaunchKernelGGL((k_presid_upper<T, 6>), grid, dim3(kPB), 0, s, A.n_rows, K, A.rp, A.col, A.diag, val, A.nnz, x, r); break;
    default: return hipErrorInvalidValue;
  }
  EAMG_PCHECK();
}

template <class T>
hipError_t launch_prect(const SoaMat &M, int K, const T *x, T *y, bool accumulate, hipStream_t s) {
  if (M.n_rows == 0) return hipSuccess;
  const T *val = pvals<T>(M);
  if (!val || !valid_k(K)) return hipErrorInvalidValue;
  const dim3 grid(pgrid(M.n_rows, kPB / K));
  const int accf = accumulate ? 1 : 0;
#define EAMG_PRECT(BR_, BC_)                                                                   \
  hipLaunchKernelGGL((k_prect<T, BR_, BC_>), grid, dim3(kPB), 0, s, M.n_rows, K, M.rp, M.col, \
                     val, M.nnz, x, y, accf)
  if (M.br == 1 && M.bc == 1) EAMG_PRECT(1, 1);
  else if (M.br == 3 && M.bc == 6) EAMG_PRECT(3, 6);
  else if (M.br == 6 && M.bc == 3) EAMG_PRECT(6, 3);
  else if (M.br == 6 && M.bc == 6) EAMG_PRECT(6, 6);
  else return hipErrorInvalidValue;
#undef EAMG_PRECT
  EAMG_PCHECK();
}

template <class T>
hipError_t launch_pdense(int n, int K, const double *D, const T *x, T *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (!valid_k(K)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pdense<T>, dim3(pgrid(n, kPB / K)), dim3(kPB), 0, s, n, K, D, x, y);
  EAMG_PCHECK();
}

int pspmv_blocks(const SoaMat &A, int K) { return int(pgrid(A.n_rows, kPB / K)); }

hipError_t launch_pspmv(const SoaMat &A, int K, const double *x, double *y, double *part,
                        hipStream_t s) {
  if (A.n_rows == 0) return hipSuccess;
  if (!valid_k(K) || A.br != A.bc) return hipErrorInvalidValue;
  const dim3 grid(pgrid(A.n_rows, kPB / K));
  switch (A.br) {
    case 1: hipLaunchKernelGGL((k_pspmv<1>), grid, dim3(kPB), 0, s, A.n_rows, K, A.rp, A.col, A.val, A.nnz, x, y, part); break;
    case 3: hipLaunchKernelGGL((k_pspmv<3>), grid, dim3(kPB), 0, s, A.n_rows, K, A.rp, A.col, A.val, A.nnz, x, y, part); break;
    case 6: hipLaunchKernelGGL((k_pspmv<6>), grid, dim3(kPB), 0, s, A.n_rows, K, A.rp, A.col, A.val, A.nnz, x, y, part); break;
    default: return hipErrorInvalidValue;
  }
  EAMG_PCHECK();
}

int pdot_blocks(int64_t n) {
  const int64_t b = (n + kPB - 1) / kPB;
  return int(b < kPDotMax ? (b < 1 ? 1 : b) : kPDotMax);
}

hipError_t launch_pdot(int64_t n, int K, const double *a, const double *b, double *part,
                       hipStream_t s) {
  if (!valid_k(K)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pdot, dim3(pdot_blocks(n)), dim3(kPB), 0, s, n, K, a, b, part);
  EAMG_PCHECK();
}

hipError_t launch_preduce(int nparts, int K, const double *part, double *scal, int slot, int op,
                          hipStream_t s) {
  if (!valid_k(K)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_preduce, dim3(1), dim3(kPB), 0, s, nparts, K, part, scal, slot, op);
  EAMG_PCHECK();
}

hipError_t launch_pupdate_xr(int64_t n, int K, const double *scal, double *x, double *r,
                             const double *p, const double *q, double *part, hipStream_t s) {
  if (!valid_k(K)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pupdate_xr, dim3(pdot_blocks(n)), dim3(kPB), 0, s, n, K, scal, x, r, p, q, part);
  EAMG_PCHECK();
}

hipError_t launch_pupdate_p(int64_t n, int K, const double *scal, const double *z, double *p,
                            hipStream_t s) {
  if (!valid_k(K)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pupdate_p, dim3(pdot_blocks(n)), dim3(kPB), 0, s, n, K, scal, z, p);
  EAMG_PCHECK();
}

hipError_t launch_pinit_scal(int K, double rtol, int max_it, double *scal, hipStream_t s) {
  if (!valid_k(K)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pinit_scal, dim3(pgrid(PS_COUNT * K, kPB)), dim3(kPB), 0, s, K, rtol,
                     double(max_it), scal);
  EAMG_PCHECK();
}

hipError_t launch_pfinite(int64_t n, int K, const double *a, double *scal, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pfinite, dim3(pgrid(n, kPB)), dim3(kPB), 0, s, n, K, a, scal);
  EAMG_PCHECK();
}

hipError_t launch_pzero_unstarted(int64_t n, int K, const double *scal, double *x, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pzero_unstarted, dim3(pgrid(n, kPB)), dim3(kPB), 0, s, n, K, scal, x);
  EAMG_PCHECK();
}

hipError_t launch_ppack(int n, int bs, int K, int nrhs, const int *perm, const uint8_t *mask,
                        const double *in, int64_t ld, double *out, hipStream_t s) {
  const int64_t tot = int64_t(n) * bs * K;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ppack, dim3(pgrid(tot, kPB)), dim3(kPB), 0, s, n, bs, K, nrhs, perm, mask,
                     in, ld, out);
  EAMG_PCHECK();
}

hipError_t launch_punpack(int n, int bs, int K, int nrhs, const int *perm, const double *in,
                          double *out, int64_t ld, hipStream_t s) {
  const int64_t tot = int64_t(n) * bs * K;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_punpack, dim3(pgrid(tot, kPB)), dim3(kPB), 0, s, n, bs, K, nrhs, perm, in,
                     out, ld);
  EAMG_PCHECK();
}

template hipError_t launch_pgs_fwd<double>(const SoaMat &, const double *, int, int, int, const double *, double *, double *, hipStream_t);
template hipError_t launch_pgs_fwd<float>(const SoaMat &, const float *, int, int, int, const float *, float *, float *, hipStream_t);
template hipError_t launch_pgs_bwd<double>(const SoaMat &, const double *, int, int, int, const double *, double *, hipStream_t);
template hipError_t launch_pgs_bwd<float>(const SoaMat &, const float *, int, int, int, const float *, float *, hipStream_t);
template hipError_t launch_presid_upper<double>(const SoaMat &, int, const double *, double *, hipStream_t);
template hipError_t launch_presid_upper<float>(const SoaMat &, int, const float *, float *, hipStream_t);
template hipError_t launch_prect<double>(const SoaMat &, int, const double *, double *, bool, hipStream_t);
template hipError_t launch_prect<float>(const SoaMat &, int, const float *, float *, bool, hipStream_t);
template hipError_t launch_pdense<double>(int, int, const double *, const double *, double *, hipStream_t);
template hipError_t launch_pdense<float>(int, int, const double *, const float *, float *, hipStream_t);

}  // namespace eamg
