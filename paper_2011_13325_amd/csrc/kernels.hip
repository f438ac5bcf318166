// gfx950 kernels of the edge-matrix AMG-PCG library.  See kernels.hpp for the data layouts.
//
// Every floating point reduction has a fixed order (per-lane strided sums, then a fixed
// butterfly / tree), so results are bitwise reproducible run to run; no floating point
// atomics are used anywhere.
#include "kernels.hpp"

#include <cmath>
#include <cstdlib>
#include <type_traits>

namespace eamg {

namespace {


inline int cdiv64(int64_t a, int64_t b) { return int((a + b - 1) / b); }

// Workgroups are dispatched round-robin over the eight XCDs (workgroup b to XCD b mod 8), each
// XCD with its own L2.  The colour sweeps use this logical workgroup index instead of
// blockIdx.x: XCD x gets one contiguous run of logical workgroups (the first nb mod 8 XCDs one
// more), so the rows of a colour that one XCD updates are neighbours in the numbering and share
// their gathered x blocks in that XCD's L2 (sweeps 3 % faster at 64^3).  A bijection on
// [0, gridDim.x), so results do not change.  Not used where row lengths drift along the
// numbering: the residual update over all colour-major rows (upper blocks only, long rows first)
// would load one XCD with the longest rows (+33 % measured).
__device__ inline int xcd_block() {
  const int nb = int(gridDim.x), b = int(blockIdx.x);
  const int x = b & 7, q = nb >> 3, rem = nb & 7;
  return x * q + min(x, rem) + (b >> 3);
}

// ---- small dense helpers (one thread) ----------------------------------------------------

__device__ inline void dev_skew_q(const double *t, int k, double *Q) {
  for (int i = 0; i < k * k; ++i) Q[i] = 0.0;
  for (int i = 0; i < k; ++i) Q[i * k + i] = 1.0;
  if (k == 6) {
    // upper right block Skew(t): Skew(t) r = t x r
    Q[0 * 6 + 4] = -t[2];
    Q[0 * 6 + 5] = t[1];
    Q[1 * 6 + 3] = t[2];
    Q[1 * 6 + 5] = -t[0];
    Q[2 * 6 + 3] = -t[1];
    Q[2 * 6 + 4] = t[0];
  }
}

// C (m x p) = A (m x n) * B (n x p)
__device__ inline void dev_mm(int m, int n, int p, const double *A, const double *B, double *C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < p; ++j) {
      double s = 0.0;
      for (int l = 0; l < n; ++l) s += A[i * n + l] * B[l * p + j];
      C[i * p + j] = s;
    }
}

// C (m x p) = A^T * B with A (n x m)
__device__ inline void dev_tmm(int m, int n, int p, const double *A, const double *B, double *C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < p; ++j) {
      double s = 0.0;
      for (int l = 0; l < n; ++l) s += A[l * m + i] * B[l * p + j];
      C[i * p + j] = s;
    }
}

// Symmetric pseudo-inverse by cyclic Jacobi; eigenvalues <= tau * max(lambda_max, 0) dropped.
__device__ void dev_pinv(int n, const double *X, double *P, double tau) {
  double A[36], V[36], w[6];
  double fro2 = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      A[i * n + j] = 0.5 * (X[i * n + j] + X[j * n + i]);
      V[i * n + j] = i == j ? 1.0 : 0.0;
      fro2 += A[i * n + j] * A[i * n + j];
    }
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off <= 1e-40 * fro2 || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = cs * akp - sn * akq;
          A[k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = cs * apk - sn * aqk;
          A[q * n + k] = sn * apk + cs * aqk;
        }
        A[p * n + q] = 0.0;
        A[q * n + p] = 0.0;
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = cs * vkp - sn * vkq;
          V[k * n + q] = sn * vkp + cs * vkq;
        }
      }
  }
  double lmax = A[0];
  for (int i = 0; i < n; ++i) {
    w[i] = A[i * n + i];
    lmax = w[i] > lmax ? w[i] : lmax;
  }
  for (int i = 0; i < n * n; ++i) P[i] = 0.0;
  if (!(lmax > 0.0)) return;
  for (int k = 0; k < n; ++k) {
    if (!(w[k] > tau * lmax)) continue;
    const double inv = 1.0 / w[k];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) P[i * n + j] += V[i * n + k] * inv * V[j * n + k];
  }
}

// ---- setup kernels --------------------------------------------------------------------------

__global__ void k_dirichlet(int n, int bs, const int64_t *rp, const int *col, double *val,
                            const uint8_t *dir) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int bsz = bs * bs;
  for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
    const int j = col[p];
    if (!(dir[i] || dir[j])) continue;
    for (int e = 0; e < bsz; ++e)
      val[p * bsz + e] = (i == j && dir[i] && (e / bs == e % bs)) ? 1.0 : 0.0;
  }
}

__global__ void k_diag_pinv(int n, int bs, const int64_t *rp, const int *col, const double *val,
                            double *Dinv, double tau) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int bsz = bs * bs;
  double blk[36], P[36];
  for (int e = 0; e < bsz; ++e) blk[e] = 0.0;
  for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
    if (col[p] == i) {
      for (int e = 0; e < bsz; ++e) blk[e] = val[p * bsz + e];
      break;
    }
  dev_pinv(bs, blk, P, tau);
  for (int e = 0; e < bsz; ++e) Dinv[int64_t(i) * bsz + e] = P[e];
}

// Tentative block P_iJ = Q^{J->i} restricted to its first bs rows (bs x k).
__device__ inline void dev_tentative(int k, int bs, const double *xf, const double *xcJ, double *out) {
  double t[3] = {xf[0] - xcJ[0], xf[1] - xcJ[1], xf[2] - xcJ[2]};
  double Q[36];
  dev_skew_q(t, k, Q);
  for (int e = 0; e < bs * k; ++e) out[e] = Q[e];
}

// One fine row of the auxiliary smoothed prolongation (Def. def:aux_sp).
__global__ void k_ps_numeric(PsArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int type = a.type[i];
  if (type == 2) return;  // dropped row: no entries
  const int k = a.k, bs = a.bs, Ji = a.agg[i];
  const double *xi = a.x + 3 * int64_t(i);
  double Dp[36], acc[36], tmp[36], T[36];
  if (type == 0) {
    // real-matrix row: P_i - omega pinv(A_ii) sum_j A_ij P_j
    double Aii[36];
    for (int e = 0; e < bs * bs; ++e) Aii[e] = 0.0;
    for (int64_t p = a.Arp[i]; p < a.Arp[i + 1]; ++p)
      if (a.Acol[p] == i) {
        for (int e = 0; e < bs * bs; ++e) Aii[e] = a.Aval[p * bs * bs + e];
        break;
      }
    dev_pinv(bs, Aii, Dp, a.tau);
    for (int64_t q = a.Prp[i]; q < a.Prp[i + 1]; ++q) {
      const int J = a.Pcol[q];
      for (int e = 0; e < bs * k; ++e) acc[e] = 0.0;
      for (int64_t p = a.Arp[i]; p < a.Arp[i + 1]; ++p) {
        const int j = a.Acol[p];
        if (a.agg[j] != J) continue;
        dev_tentative(k, bs, a.x + 3 * int64_t(j), a.xc + 3 * int64_t(J), T);
        dev_mm(bs, bs, k, a.Aval + p * bs * bs, T, tmp);
        for (int e = 0; e < bs * k; ++e) acc[e] += tmp[e];
      }
      dev_mm(bs, bs, k, Dp, acc, tmp);
      double *out = a.Pval + q * bs * k;
      if (J == Ji) {
        dev_tentative(k, bs, xi, a.xc + 3 * int64_t(J), T);
        for (int e = 0; e < bs * k; ++e) out[e] = T[e] - a.omega * tmp[e];
      } else {
        for (int e = 0; e < bs * k; ++e) out[e] = -a.omega * tmp[e];
      }
    }
    return;
  }
  // edge-matrix row: P_i - omega pinv(Dhat0_ii) (Dhat0_ii P_i + sum_{l in F} Ahat0_il P_l)
  double Dh[36], Qa[36], Qb[36], Ee[36];
  for (int e = 0; e < k * k; ++e) Dh[e] = 0.0;
  for (int64_t f = a.Fptr[i]; f < a.Fptr[i + 1]; ++f) {
    const double *xl = a.x + 3 * int64_t(a.Fvtx[f]);
    const double th[3] = {0.5 * (xl[0] - xi[0]), 0.5 * (xl[1] - xi[1]), 0.5 * (xl[2] - xi[2])};
    dev_skew_q(th, k, Qa);  // Q^{il}
    const double *Ef = a.E + int64_t(a.Fedge[f]) * k * k;
    dev_tmm(k, k, k, Qa, Ef, tmp);
    dev_mm(k, k, k, tmp, Qa, Ee);
    for (int e = 0; e < k * k; ++e) Dh[e] += Ee[e];
  }
  dev_pinv(k, Dh, Dp, a.tau);
  double Pi[36];
  {
    const double *xJ = a.xc + 3 * int64_t(Ji);
    const double t[3] = {xi[0] - xJ[0], xi[1] - xJ[1], xi[2] - xJ[2]};
    dev_skew_q(t, k, Pi);  // Q^{J->i}, full k x k
  }
  for (int64_t q = a.Prp[i]; q < a.Prp[i + 1]; ++q) {
    const int J = a.Pcol[q];
    if (J == Ji)
      dev_mm(k, k, k, Dh, Pi, acc);
    else
      for (int e = 0; e < k * k; ++e) acc[e] = 0.0;
    for (int64_t f = a.Fptr[i]; f < a.Fptr[i + 1]; ++f) {
      const int l = a.Fvtx[f];
      if (a.agg[l] != J) continue;
      const double *xl = a.x + 3 * int64_t(l);
      const double th[3] = {0.5 * (xl[0] - xi[0]), 0.5 * (xl[1] - xi[1]), 0.5 * (xl[2] - xi[2])};
      const double mh[3] = {-th[0], -th[1], -th[2]};
      dev_skew_q(th, k, Qa);  // Q^{il}
      dev_skew_q(mh, k, Qb);  // Q^{li}
      const double *Ef = a.E + int64_t(a.Fedge[f]) * k * k;
      dev_tmm(k, k, k, Qa, Ef, tmp);
      dev_mm(k, k, k, tmp, Qb, Ee);  // Q^{il,T} E Q^{li}
      const double *xJ = a.xc + 3 * int64_t(J);
      const double t[3] = {xl[0] - xJ[0], xl[1] - xJ[1], xl[2] - xJ[2]};
      dev_skew_q(t, k, T);   // Q^{J->l}
      dev_mm(k, k, k, Ee, T, tmp);
      for (int e = 0; e < k * k; ++e) acc[e] -= tmp[e];
    }
    dev_mm(k, k, k, Dp, acc, tmp);
    double *out = a.Pval + q * bs * k;
    for (int r = 0; r < bs; ++r)
      for (int c = 0; c < k; ++c)
        out[r * k + c] = (J == Ji ? Pi[r * k + c] : 0.0) - a.omega * tmp[r * k + c];
  }
}

__global__ void k_spgemm_numeric(int64_t nnzC, int ra, int ca, int cb, const int *crow,
                                 const int *Ccol, const int64_t *Arp, const int *Acol,
                                 const double *Aval, const int64_t *Brp, const int *Bcol,
                                 const double *Bval, double *Cval) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= nnzC * ra) return;
  const int64_t q = gid / ra;
  const int r = int(gid % ra);
  const int i = crow[q], J = Ccol[q];
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t p = Arp[i]; p < Arp[i + 1]; ++p) {
    const int kk = Acol[p];
    int64_t lo = Brp[kk], hi = Brp[kk + 1];
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (Bcol[mid] < J)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo == Brp[kk + 1] || Bcol[lo] != J) continue;
    const double *Ab = Aval + p * ra * ca + r * ca;
    const double *Bb = Bval + lo * ca * cb;
    for (int c = 0; c < cb; ++c) {
      double s = 0.0;
      for (int t = 0; t < ca; ++t) s += Ab[t] * Bb[t * cb + c];
      acc[c] += s;
    }
  }
  for (int c = 0; c < cb; ++c) Cval[q * ra * cb + r * cb + c] = acc[c];
}

__global__ void k_transpose_blocks(int64_t nnz, int r, int c, const int64_t *src, const double *in,
                                   double *out) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int bsz = r * c;
  if (gid >= nnz * bsz) return;
  const int64_t q = gid / bsz;
  const int e = int(gid % bsz);
  const int oi = e / r, oj = e % r;   // out block is c x r: (oi, oj) = in (oj, oi)
  out[q * bsz + e] = in[src[q] * bsz + oj * c + oi];
}

// Block q of out := block src[q] of in (blocks of bsz values).
__global__ void k_gather_blocks(int64_t nnz, int bsz, const int64_t *src, const double *in, double *out) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= nnz * bsz) return;
  const int64_t q = gid / bsz;
  const int e = int(gid % bsz);
  out[gid] = in[src[q] * bsz + e];
}

__global__ void k_gather_rows(int n, int bsz, const int *perm, const double *in, double *out) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= int64_t(n) * bsz) return;
  const int64_t r = gid / bsz;
  const int e = int(gid % bsz);
  out[gid] = in[int64_t(perm[r]) * bsz + e];
}

// ---- solve kernels ---------------------------------------------------------------------------

__device__ inline double block_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// The solve-phase kernels below are templated on the value type T of the matrices and vectors
// they stream (double, or float for the FP32 V-cycle); they accumulate in T.

template <class T, int BR>
__device__ inline void group_reduce(T (&acc)[BR], int G) {
  for (int off = G >> 1; off > 0; off >>= 1)
#pragma unroll
    for (int r = 0; r < BR; ++r) acc[r] += __shfl_xor(acc[r], off, G);
}

// A row team of W wavefronts (64 W lanes, "wide"; kBlock / (64 W) rows per workgroup):
// butterfly within each wavefront, then the W wavefront sums of the row added in wavefront order
// through LDS; every lane of the row gets the total.  sh: kBlock / 64 * BR values.
template <class T, int BR, int W>
__device__ inline void wide_reduce(T (&acc)[BR], T *sh) {
  group_reduce<T, BR>(acc, 64);
  const int wv = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int r = 0; r < BR; ++r) sh[wv * BR + r] = acc[r];
  __syncthreads();
  const int w0 = wv - wv % W;   // first wavefront of this row
#pragma unroll
  for (int r = 0; r < BR; ++r) {
    T v = sh[w0 * BR + r];
    for (int w = 1; w < W; ++w) v += sh[(w0 + w) * BR + r];
    acc[r] = v;
  }
}

// xv = the BC entries of block column c of x.  Six-entry blocks start at a multiple of 24 (FP32)
// or 48 (FP64) bytes, so they are gathered as three 8- or 16-byte pairs: half the load
// instructions of a scattered gather (every lane of it touches its own cache line).
template <class T, int BC>
__device__ inline void gather_block(const T *x, int64_t c, T (&xv)[BC]) {
  if constexpr (BC % 2 == 0) {
    using T2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
    const T2 *x2 = reinterpret_cast<const T2 *>(x + c * BC);
#pragma unroll
    for (int h = 0; h < BC / 2; ++h) {
      const T2 v = x2[h];
      xv[2 * h] = v.x;
      xv[2 * h + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int cc = 0; cc < BC; ++cc) xv[cc] = x[c * BC + cc];
  }
}

// acc[r] += sum over blocks p in [p0, p1) (strided by G) of A_p x_col(p)
template <class T, int BR, int BC>
__device__ inline void row_accumulate(int p0, int p1, int lane, int G, const int *__restrict__ col,
                                      const T *__restrict__ val, int64_t nnz, const T *x,
                                      T (&acc)[BR]) {
  for (int p = p0 + lane; p < p1; p += G) {
    const int64_t c = col[p];
    T v[BR * BC];
#pragma unroll
    for (int e = 0; e < BR * BC; ++e) v[e] = val[int64_t(p) * (BR * BC) + e];
    // every value load is issued before the gathers of x, which wait for the column index
    __builtin_amdgcn_sched_barrier(0);
    T xv[BC];
    gather_block<T, BC>(x, c, xv);
#pragma unroll
    for (int r = 0; r < BR; ++r)
#pragma unroll
      for (int cc = 0; cc < BC; ++cc) acc[r] = fma(v[r * BC + cc], xv[cc], acc[r]);
  }
}

template <int BR, int BC>
__global__ __launch_bounds__(kBlock) void k_spmv(int n_rows, int G, const int *__restrict__ rp,
                                                const int *__restrict__ col,
                                                const double *__restrict__ val, int64_t nnz,
                                                const double *__restrict__ x, double *__restrict__ y,
                                                double *part) {
  __shared__ double sh[kBlock];
  const int lane = threadIdx.x & (G - 1);
  const int wg = xcd_block();
  const int row = wg * (kBlock / G) + threadIdx.x / G;
  double acc[BR];
#pragma unroll
  for (int r = 0; r < BR; ++r) acc[r] = 0.0;
  if (row < n_rows) row_accumulate<double, BR, BC>(rp[row], rp[row + 1], lane, G, col, val, nnz, x, acc);
  group_reduce<double, BR>(acc, G);
  double d = 0.0;
  if (row < n_rows && lane == 0) {
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      y[int64_t(row) * BR + r] = acc[r];
      d += x[int64_t(row) * BR + r] * acc[r];
    }
  }
  if (part) {
    const double s = block_sum(d, sh);
    if (threadIdx.x == 0) part[wg] = s;
  }
}

template <class T, int B>
__device__ inline T pick(const T (&v)[B], int i) {
  T out = T(0);
#pragma unroll
  for (int q = 0; q < B; ++q) out = (q == i) ? v[q] : out;
  return out;
}

// One row of a multicolour block Gauss-Seidel sweep, computed by the G lanes of a row group.
// FWD: x = 0 before the sweep, so only the blocks left of the diagonal (lower colours) are read
// (rp, col, val: the lower part) and A_ii is block `row` of dval;
// also writes r_i = t - A_ii x_i.  BWD: x_i += Dinv_i (b_i - sum_j A_ij x_j) over the whole row
// (rp, col, val: the full matrix).
// Lane q < B owns component q: it prefetches b_i[q], row q of Dinv_i and (FWD) row q of A_ii,
// (BWD) x_i[q], together with the row's blocks, so a row costs one round of row loads plus the
// x gathers; a butterfly all-reduce leaves the row sum on every lane.  No other row of the
// colour writes x_i, so the prefetched x_i[q] is the value the gathers see.
template <class T, int B, bool FWD, int W>
__device__ inline void gs_row(int row, bool valid, int lane, int G, const int *__restrict__ rp,
                              const int *__restrict__ col, const T *__restrict__ val, int64_t nnz,
                              const T *__restrict__ dval, int64_t nd, const T *__restrict__ Dinv,
                              const T *__restrict__ b, T *x, T *r, T *sh) {
  const bool own = valid && lane < B;
  int p0 = 0, p1 = 0;
  if (valid) {
    p0 = rp[row];
    p1 = rp[row + 1];
  }
  T bq = T(0), xo = T(0), Dq[B], Aq[B];
#pragma unroll
  for (int c = 0; c < B; ++c) {
    Dq[c] = T(0);
    Aq[c] = T(0);
  }
  if (own) {
    bq = b[int64_t(row) * B + lane];
    if (!FWD) xo = x[int64_t(row) * B + lane];
#pragma unroll
    for (int c = 0; c < B; ++c) {
      Dq[c] = Dinv[int64_t(row) * B * B + lane * B + c];
      if (FWD) Aq[c] = dval[int64_t(row) * (B * B) + lane * B + c];
    }
  }
  T acc[B];
#pragma unroll
  for (int q = 0; q < B; ++q) acc[q] = T(0);
  if (valid) row_accumulate<T, B, B>(p0, p1, lane, G, col, val, nnz, x, acc);
  if (W > 1)
    wide_reduce<T, B, W>(acc, sh);
  else
    group_reduce<T, B>(acc, G);
  // wide teams: the owning lanes (< B) are in the row's first wavefront; shuffles stay within
  // wavefronts
  const int GS = W > 1 ? 64 : G;
  const T tq = bq - pick<T, B>(acc, lane);   // t component of this lane (lanes < B)
  T t[B];
#pragma unroll
  for (int c = 0; c < B; ++c) t[c] = __shfl(tq, c, GS);
  T xq = T(0);
#pragma unroll
  for (int c = 0; c < B; ++c) xq = fma(Dq[c], t[c], xq);
  if (FWD) {
    T xi[B];
#pragma unroll
    for (int c = 0; c < B; ++c) xi[c] = __shfl(xq, c, GS);
    T rq = tq;
#pragma unroll
    for (int c = 0; c < B; ++c) rq = fma(-Aq[c], xi[c], rq);
    if (own) {
      x[int64_t(row) * B + lane] = xq;
      r[int64_t(row) * B + lane] = rq;
    }
  } else {
    if (own) x[int64_t(row) * B + lane] = xo + xq;
  }
}

// r_i -= sum_{j > i} A_ij x_j for one row (rp, col, val: the blocks right of the diagonal).
template <class T, int B, int W>
__device__ inline void resid_row(int row, bool valid, int lane, int G, const int *__restrict__ rp,
                                 const int *__restrict__ col, const T *__restrict__ val,
                                 int64_t nnz, const T *x, T *r, T *sh) {
  T rq = T(0);
  int p0 = 0, p1 = 0;
  if (valid) {
    p0 = rp[row];
    p1 = rp[row + 1];
    if (lane < B) rq = r[int64_t(row) * B + lane];
  }
  T acc[B];
#pragma unroll
  for (int a = 0; a < B; ++a) acc[a] = T(0);
  if (valid) row_accumulate<T, B, B>(p0, p1, lane, G, col, val, nnz, x, acc);
  if (W > 1)
    wide_reduce<T, B, W>(acc, sh);
  else
    group_reduce<T, B>(acc, G);
  if (valid && lane < B) r[int64_t(row) * B + lane] = rq - pick<T, B>(acc, lane);
}

// One colour (rows [r0, r1)) per launch, kBlock / G rows per workgroup.  G = 64 W lanes per
// row with W = 2 or 4 wavefronts ("wide", W = 4: one row per workgroup) for levels whose rows
// are long; else G <= 64 (W = 1).
template <class T, int B, bool FWD, int W>
__global__ __launch_bounds__(kBlock) void k_gs_color(int r0, int r1, int G, const int *__restrict__ rp,
                                                    const int *__restrict__ col,
                                                    const T *__restrict__ val, int64_t nnz,
                                                    const T *__restrict__ dval, int64_t nd,
                                                    const T *__restrict__ Dinv,
                                                    const T *__restrict__ b, T *x, T *r) {
  __shared__ T sh[W > 1 ? (kBlock / 64) * B : 1];
  const int lane = threadIdx.x & (G - 1);
  const int row = r0 + xcd_block() * (kBlock / G) + threadIdx.x / G;
  gs_row<T, B, FWD, W>(row, row < r1, lane, G, rp, col, val, nnz, dval, nd, Dinv, b, x, r, sh);
}

template <class T, int B, int W>
__global__ __launch_bounds__(kBlock) void k_resid_upper(int r0, int r1, int G, const int *__restrict__ rp,
                                                       const int *__restrict__ col,
                                                       const T *__restrict__ val, int64_t nnz,
                                                       const T *x, T *r) {
  __shared__ T sh[W > 1 ? (kBlock / 64) * B : 1];
  const int lane = threadIdx.x & (G - 1);
  const int row = r0 + int(blockIdx.x) * (kBlock / G) + int(threadIdx.x) / G;
  resid_row<T, B, W>(row, row < r1, lane, G, rp, col, val, nnz, x, r, sh);
}

template <class T, int BR, int BC>
__global__ __launch_bounds__(kBlock) void k_rect(int n_rows, int G, const int *__restrict__ rp,
                                                const int *__restrict__ col,
                                                const T *__restrict__ val, int64_t nnz,
                                                const T *__restrict__ x, T *__restrict__ y,
                                                int accumulate) {
  const int lane = threadIdx.x & (G - 1);
  const int row = xcd_block() * (kBlock / G) + threadIdx.x / G;
  // the old y_i is read with the row's first loads, not after the reduction
  T acc[BR], yo[BR];
#pragma unroll
  for (int r = 0; r < BR; ++r) {
    acc[r] = T(0);
    yo[r] = T(0);
  }
  if (accumulate && row < n_rows && lane == 0)
#pragma unroll
    for (int r = 0; r < BR; ++r) yo[r] = y[int64_t(row) * BR + r];
  if (row < n_rows) row_accumulate<T, BR, BC>(rp[row], rp[row + 1], lane, G, col, val, nnz, x, acc);
  group_reduce<T, BR>(acc, G);
  if (row < n_rows && lane == 0) {
#pragma unroll
    for (int r = 0; r < BR; ++r) y[int64_t(row) * BR + r] = accumulate ? yo[r] + acc[r] : acc[r];
  }
}

template <class S, class D>
__global__ void k_convert(int64_t n, const S *__restrict__ in, D *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = D(in[i]);
}

__global__ void k_gather_blocks_f32(int64_t nnz, int bsz, const int64_t *src, const double *in, float *out) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= nnz * bsz) return;
  const int64_t q = gid / bsz;
  const int e = int(gid % bsz);
  out[gid] = float(in[src[q] * bsz + e]);
}

// b in double, or the FP32 V-cycle's output read as it is (each value converted exactly)
template <class TB>
__global__ __launch_bounds__(kBlock) void k_dot(int64_t n, const double *__restrict__ a,
                                               const TB *__restrict__ b, double *part) {
  __shared__ double sh[kBlock];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    s = fma(a[i], double(b[i]), s);
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_reduce(int nparts, const double *__restrict__ part,
                                                  double *scal, int slot, int op) {
  __shared__ double sh[kBlock];
  double s = 0.0;
  // unrolled so that the loads are in flight together (the CG SpMV leaves one partial per
  // workgroup: hundreds of thousands on a large level); the sum keeps its order
#pragma unroll 16
  for (int i = threadIdx.x; i < nparts; i += kBlock) s += part[i];
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) {
    scal[slot] = t;
    if (op == RED_ALPHA) {
      if (!(t > 0.0) || !isfinite(t)) scal[SC_BAD] = 1.0;
      scal[SC_ALPHA] = scal[SC_RHO] / t;
    } else if (op == RED_BETA) {
      if (!(t > 0.0) || !isfinite(t)) scal[SC_BAD] = 1.0;
      scal[SC_BETA] = t / scal[SC_RHO];
      scal[SC_RHO] = t;
    }
  }
}

// r32 (optional): the FP32 copy of the new r, the next FP32 V-cycle's right-hand side.
__global__ __launch_bounds__(kBlock) void k_update_xr(int64_t n, const double *scal, double *x,
                                                     double *r, const double *__restrict__ p,
                                                     const double *__restrict__ q, double *part,
                                                     float *__restrict__ r32) {
  __shared__ double sh[kBlock];
  const double alpha = scal[SC_ALPHA];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    x[i] = fma(alpha, p[i], x[i]);
    const double ri = fma(-alpha, q[i], r[i]);
    r[i] = ri;
    if (r32) r32[i] = float(ri);
    s = fma(ri, ri, s);
  }
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <class TZ>
__global__ __launch_bounds__(kBlock) void k_update_p(int64_t n, const double *scal,
                                                    const TZ *__restrict__ z, double *p) {
  const double beta = scal[SC_BETA];
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    p[i] = fma(beta, p[i], double(z[i]));
}

__global__ void k_sub(int64_t n, const double *a, const double *b, double *y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] - b[i];
}

__global__ void k_copy(int64_t n, const double *a, double *y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i];
}

__global__ void k_fill(int64_t n, double v, double *a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_perm_in(int n, int bs, const int *perm, const uint8_t *mask, const double *in,
                          double *out) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= int64_t(n) * bs) return;
  const int64_t r = gid / bs;
  const int c = int(gid % bs);
  const int o = perm[r];
  out[gid] = (mask && mask[o]) ? 0.0 : in[int64_t(o) * bs + c];
}

__global__ void k_perm_out(int n, int bs, const int *perm, const double *in, double *out) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= int64_t(n) * bs) return;
  const int64_t r = gid / bs;
  const int c = int(gid % bs);
  out[int64_t(perm[r]) * bs + c] = in[gid];
}

__global__ void k_finite_check(int64_t n, const double *a, double *scal, int slot) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(a[i])) scal[slot] = 1.0;
}

int groups_for(int G) { return kBlock / G; }

}  // namespace

// ---- launchers ---------------------------------------------------------------------------------

#define EAMG_LAUNCH_CHECK() return hipGetLastError()

hipError_t launch_dirichlet(int n, int bs, const int64_t *rp, const int *col, double *val,
                            const uint8_t *dir, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dirichlet, dim3(cdiv64(n, 128)), dim3(128), 0, s, n, bs, rp, col, val, dir);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_diag_pinv(int n, int bs, const int64_t *rp, const int *col, const double *val,
                            double *Dinv, double tau, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_pinv, dim3(cdiv64(n, 64)), dim3(64), 0, s, n, bs, rp, col, val, Dinv, tau);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_ps_numeric(const PsArgs &a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ps_numeric, dim3(cdiv64(a.n, 64)), dim3(64), 0, s, a);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_spgemm_numeric(int64_t nnzC, int ra, int ca, int cb, const int *crow,
                                 const int *Ccol, const int64_t *Arp, const int *Acol,
                                 const double *Aval, const int64_t *Brp, const int *Bcol,
                                 const double *Bval, double *Cval, hipStream_t s) {
  if (nnzC == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spgemm_numeric, dim3(cdiv64(nnzC * ra, 256)), dim3(256), 0, s, nnzC, ra, ca,
                     cb, crow, Ccol, Arp, Acol, Aval, Brp, Bcol, Bval, Cval);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_transpose_blocks(int64_t nnz, int r, int c, const int64_t *src, const double *in,
                                   double *out, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_blocks, dim3(cdiv64(nnz * r * c, 256)), dim3(256), 0, s, nnz, r, c,
                     src, in, out);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_gather_blocks(int64_t nnz, int bsz, const int64_t *src, const double *in, double *out,
                             hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_blocks, dim3(cdiv64(nnz * bsz, 256)), dim3(256), 0, s, nnz, bsz, src, in,
                     out);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_gather_rows(int n, int bsz, const int *perm, const double *in, double *out,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3(cdiv64(int64_t(n) * bsz, 256)), dim3(256), 0, s, n, bsz,
                     perm, in, out);
  EAMG_LAUNCH_CHECK();
}

#define EAMG_DISPATCH_SQ(B, KERNEL, ...)                                                        \
  switch (B) {                                                                                  \
    case 1: hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__); break;                                  \
    case 3: hipLaunchKernelGGL(KERNEL<3>, __VA_ARGS__); break;                                  \
    case 6: hipLaunchKernelGGL(KERNEL<6>, __VA_ARGS__); break;                                  \
    default: return hipErrorInvalidValue;                                                       \
  }

// k_spmv reduces within wavefronts: a matrix with one row per workgroup runs it with 64 lanes
// per row.
inline int spmv_group(const SolveMat &A) { return A.group > 64 ? 64 : A.group; }

int spmv_blocks(const SolveMat &A) { return int(cdiv64(A.n_rows, groups_for(spmv_group(A)))); }

hipError_t launch_spmv(const SolveMat &A, const double *x, double *y, double *part, hipStream_t s) {
  if (A.n_rows == 0) return hipSuccess;
  const int G = spmv_group(A);
  const dim3 grid(spmv_blocks(A));
  if (A.br != A.bc) return hipErrorInvalidValue;
  switch (A.br) {
    case 1: hipLaunchKernelGGL((k_spmv<1, 1>), grid, dim3(kBlock), 0, s, A.n_rows, G, A.rp, A.col, A.val, A.nnz, x, y, part); break;
    case 3: hipLaunchKernelGGL((k_spmv<3, 3>), grid, dim3(kBlock), 0, s, A.n_rows, G, A.rp, A.col, A.val, A.nnz, x, y, part); break;
    case 6: hipLaunchKernelGGL((k_spmv<6, 6>), grid, dim3(kBlock), 0, s, A.n_rows, G, A.rp, A.col, A.val, A.nnz, x, y, part); break;
    default: return hipErrorInvalidValue;
  }
  EAMG_LAUNCH_CHECK();
}

template <class T>
const T *solve_vals(const SolveMat &M);
template <>
const double *solve_vals<double>(const SolveMat &M) {
  return M.val;
}
template <>
const float *solve_vals<float>(const SolveMat &M) {
  return M.val32;
}

// Wavefronts per row team for G lanes per row: 4 (kBlock), 2 (128) or 1 (<= 64).
#define EAMG_GS_W(W_, ...)                                                                       \
  if (G == kBlock) { constexpr int W_ = 4; __VA_ARGS__; }                                       \
  else if (G == 128) { constexpr int W_ = 2; __VA_ARGS__; }                                     \
  else { constexpr int W_ = 1; __VA_ARGS__; }

template <class T>
hipError_t launch_gs_fwd(const SolveMat &A, const T *Dinv, int r0, int r1, const T *b, T *x, T *r,
                         hipStream_t s) {
  if (r1 <= r0) return hipSuccess;
  const T *lo = sizeof(T) == 4 ? reinterpret_cast<const T *>(A.lo_val32) : reinterpret_cast<const T *>(A.lo_val);
  const T *dg = sizeof(T) == 4 ? reinterpret_cast<const T *>(A.dg_val32) : reinterpret_cast<const T *>(A.dg_val);
  if (!lo || !dg || !A.lo_rp || r0 < 0 || r1 > A.n_rows) return hipErrorInvalidValue;
  const int G = A.group;
  const dim3 grid(cdiv64(r1 - r0, groups_for(G)));
  const int64_t nd = A.n_rows;
  switch (A.br) {
    case 1: EAMG_GS_W(W_, hipLaunchKernelGGL((k_gs_color<T, 1, true, W_>), grid, dim3(kBlock), 0, s, r0, r1, G, A.lo_rp, A.lo_col, lo, A.lo_nnz, dg, nd, Dinv, b, x, r)); break;
    case 3: EAMG_GS_W(W_, hipLaunchKernelGGL((k_gs_color<T, 3, true, W_>), grid, dim3(kBlock), 0, s, r0, r1, G, A.lo_rp, A.lo_col, lo, A.lo_nnz, dg, nd, Dinv, b, x, r)); break;
    case 6: EAMG_GS_W(W_, hipLaunchKernelGGL((k_gs_color<T, 6, true, W_>), grid, dim3(kBlock), 0, s, r0, r1, G, A.lo_rp, A.lo_col, lo, A.lo_nnz, dg, nd, Dinv, b, x, r)); break;
    default: return hipErrorInvalidValue;
  }
  EAMG_LAUNCH_CHECK();
}

template <class T>
hipError_t launch_gs_bwd(const SolveMat &A, const T *Dinv, int r0, int r1, const T *b, T *x,
                         hipStream_t s) {
  if (r1 <= r0) return hipSuccess;
  const T *val = solve_vals<T>(A);
  if (!val) return hipErrorInvalidValue;
  const int G = A.group_bwd ? A.group_bwd : A.group;
  const dim3 grid(cdiv64(r1 - r0, groups_for(G)));
  T *none = nullptr;
  const T *none_c = nullptr;
  switch (A.br) {
    case 1: EAMG_GS_W(W_, hipLaunchKernelGGL((k_gs_color<T, 1, false, W_>), grid, dim3(kBlock), 0, s, r0, r1, G, A.rp, A.col, val, A.nnz, none_c, int64_t(0), Dinv, b, x, none)); break;
    case 3: EAMG_GS_W(W_, hipLaunchKernelGGL((k_gs_color<T, 3, false, W_>), grid, dim3(kBlock), 0, s, r0, r1, G, A.rp, A.col, val, A.nnz, none_c, int64_t(0), Dinv, b, x, none)); break;
    case 6: EAMG_GS_W(W_, hipLaunchKernelGGL((k_gs_color<T, 6, false, W_>), grid, dim3(kBlock), 0, s, r0, r1, G, A.rp, A.col, val, A.nnz, none_c, int64_t(0), Dinv, b, x, none)); break;
    default: return hipErrorInvalidValue;
  }
  EAMG_LAUNCH_CHECK();
}

template <class T>
hipError_t launch_resid_upper(const SolveMat &A, int r0, int r1, const T *x, T *r, hipStream_t s) {
  if (r0 < 0 || r1 > A.n_rows) return hipErrorInvalidValue;
  if (r1 <= r0) return hipSuccess;
  const T *up = sizeof(T) == 4 ? reinterpret_cast<const T *>(A.up_val32) : reinterpret_cast<const T *>(A.up_val);
  if (!up || !A.up_rp) return hipErrorInvalidValue;
  const int G = A.group;
  const dim3 grid(cdiv64(r1 - r0, groups_for(G)));
  switch (A.br) {
    case 1: EAMG_GS_W(W_, hipLaunchKernelGGL((k_resid_upper<T, 1, W_>), grid, dim3(kBlock), 0, s, r0, r1, G, A.up_rp, A.up_col, up, A.up_nnz, x, r)); break;
    case 3: EAMG_GS_W(W_, hipLaunchKernelGGL((k_resid_upper<T, 3, W_>), grid, dim3(kBlock), 0, s, r0, r1, G, A.up_rp, A.up_col, up, A.up_nnz, x, r)); break;
    case 6: EAMG_GS_W(W_, hipLaunchKernelGGL((k_resid_upper<T, 6, W_>), grid, dim3(kBlock), 0, s, r0, r1, G, A.up_rp, A.up_col, up, A.up_nnz, x, r)); break;
    default: return hipErrorInvalidValue;
  }
  EAMG_LAUNCH_CHECK();
}

template <class T>
hipError_t launch_rect(const SolveMat &M, const T *x, T *y, bool accumulate, hipStream_t s) {
  if (M.n_rows == 0) return hipSuccess;
  const T *val = solve_vals<T>(M);
  if (!val) return hipErrorInvalidValue;
  const dim3 grid(cdiv64(M.n_rows, groups_for(M.group)));
  const int accf = accumulate ? 1 : 0;
#define EAMG_RECT(BR_, BC_)                                                                          \
  hipLaunchKernelGGL((k_rect<T, BR_, BC_>), grid, dim3(kBlock), 0, s, M.n_rows, M.group, M.rp, M.col, \
                     val, M.nnz, x, y, accf)
  if (M.br == 1 && M.bc == 1) EAMG_RECT(1, 1);
  else if (M.br == 3 && M.bc == 6) EAMG_RECT(3, 6);
  else if (M.br == 6 && M.bc == 3) EAMG_RECT(6, 3);
  else if (M.br == 6 && M.bc == 6) EAMG_RECT(6, 6);
  else return hipErrorInvalidValue;
#undef EAMG_RECT
  EAMG_LAUNCH_CHECK();
}

template <class S, class D>
hipError_t launch_convert(int64_t n, const S *in, D *out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_convert<S, D>), dim3(cdiv64(n, 256)), dim3(256), 0, s, n, in, out);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_gather_blocks_f32(int64_t nnz, int bsz, const int64_t *src, const double *in,
                                 float *out, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_blocks_f32, dim3(cdiv64(nnz * bsz, 256)), dim3(256), 0, s, nnz, bsz, src,
                     in, out);
  EAMG_LAUNCH_CHECK();
}

template hipError_t launch_gs_fwd<double>(const SolveMat &, const double *, int, int, const double *, double *, double *, hipStream_t);
template hipError_t launch_gs_fwd<float>(const SolveMat &, const float *, int, int, const float *, float *, float *, hipStream_t);
template hipError_t launch_gs_bwd<double>(const SolveMat &, const double *, int, int, const double *, double *, hipStream_t);
template hipError_t launch_gs_bwd<float>(const SolveMat &, const float *, int, int, const float *, float *, hipStream_t);
template hipError_t launch_resid_upper<double>(const SolveMat &, int, int, const double *, double *, hipStream_t);
template hipError_t launch_resid_upper<float>(const SolveMat &, int, int, const float *, float *, hipStream_t);
template hipError_t launch_rect<double>(const SolveMat &, const double *, double *, bool, hipStream_t);
template hipError_t launch_rect<float>(const SolveMat &, const float *, float *, bool, hipStream_t);
template hipError_t launch_convert<double, float>(int64_t, const double *, float *, hipStream_t);
template hipError_t launch_convert<float, double>(int64_t, const float *, double *, hipStream_t);

int dot_blocks(int64_t n) {
  const int64_t b = (n + kBlock - 1) / kBlock;
  return int(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

hipError_t launch_dot(int64_t n, const double *a, const double *b, double *part, hipStream_t s) {
  hipLaunchKernelGGL(k_dot<double>, dim3(dot_blocks(n)), dim3(kBlock), 0, s, n, a, b, part);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_dot(int64_t n, const double *a, const float *b, double *part, hipStream_t s) {
  hipLaunchKernelGGL(k_dot<float>, dim3(dot_blocks(n)), dim3(kBlock), 0, s, n, a, b, part);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_reduce(int nparts, const double *part, double *scal, int slot, int op,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, nparts, part, scal, slot, op);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_update_xr(int64_t n, const double *scal, double *x, double *r, const double *p,
                            const double *q, double *part, hipStream_t s, float *r32) {
  hipLaunchKernelGGL(k_update_xr, dim3(dot_blocks(n)), dim3(kBlock), 0, s, n, scal, x, r, p, q, part, r32);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_update_p(int64_t n, const double *scal, const double *z, double *p, hipStream_t s) {
  hipLaunchKernelGGL(k_update_p<double>, dim3(dot_blocks(n)), dim3(kBlock), 0, s, n, scal, z, p);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_update_p(int64_t n, const double *scal, const float *z, double *p, hipStream_t s) {
  hipLaunchKernelGGL(k_update_p<float>, dim3(dot_blocks(n)), dim3(kBlock), 0, s, n, scal, z, p);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_sub(int64_t n, const double *a, const double *b, double *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sub, dim3(cdiv64(n, 256)), dim3(256), 0, s, n, a, b, y);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_copy(int64_t n, const double *a, double *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(cdiv64(n, 256)), dim3(256), 0, s, n, a, y);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_fill(int64_t n, double v, double *a, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(cdiv64(n, 256)), dim3(256), 0, s, n, v, a);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_perm_in(int n, int bs, const int *perm, const uint8_t *mask, const double *in,
                          double *out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_perm_in, dim3(cdiv64(int64_t(n) * bs, 256)), dim3(256), 0, s, n, bs, perm,
                     mask, in, out);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_perm_out(int n, int bs, const int *perm, const double *in, double *out,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_perm_out, dim3(cdiv64(int64_t(n) * bs, 256)), dim3(256), 0, s, n, bs, perm,
                     in, out);
  EAMG_LAUNCH_CHECK();
}

hipError_t launch_finite_check(int64_t n, const double *a, double *scal, int slot, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finite_check, dim3(cdiv64(n, 256)), dim3(256), 0, s, n, a, scal, slot);
  EAMG_LAUNCH_CHECK();
}

}  // namespace eamg
