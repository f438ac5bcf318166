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

// Logical workgroup index of the colour sweeps: workgroup b runs on XCD b mod 8 (round-robin
// dispatch, one L2 per XCD); XCD x takes one contiguous run of logical workgroups so that the
// rows it updates are neighbours and share their gathered x panel blocks in its L2.  A
// bijection on [0, gridDim.x): results do not change.
__device__ inline int xcd_block() {
  const int nb = int(gridDim.x), b = int(blockIdx.x);
  const int x = b & 7, q = nb >> 3, rem = nb & 7;
  return x * q + min(x, rem) + (b >> 3);
}

template <class T>
const T *pvals(const SolveMat &M);
template <>
const double *pvals<double>(const SolveMat &M) {
  return M.val;
}
template <>
const float *pvals<float>(const SolveMat &M) {
  return M.val32;
}

// A block row belongs to a team of 64 W lanes (W = 1: one wavefront per row, four rows per
// workgroup; W = 4: the whole workgroup on one row, for levels of few long rows).  A lane owns C
// consecutive columns (register blocking: every matrix value it loads serves C columns, and the
// C values of one dof are one vector load); the K / C lanes covering a panel form a sub-team,
// and the S = 64 W C / K sub-teams of the team take the row's blocks in turn: sub-team s reads
// blocks p0 + s, p0 + s + S, ...  At every step the S sub-teams read S consecutive blocks (one
// contiguous run of memory), and the column index of a sub-team's next block is
// fetched one step ahead, so a step waits for one round of gathers only.  The row sums of
// column group g end in lane g of the team (sub-team 0).
constexpr int kWave = 64;

template <class T, int C>
struct PVec {
  T v[C];
};

// X entries of one dof for columns g C .. g C + C - 1 (C-aligned, contiguous).
template <class T, int C>
__device__ inline PVec<T, C> pload(const T *p) {
  PVec<T, C> out;
  if constexpr (C == 1) {
    out.v[0] = p[0];
  } else {
    typedef T vec_t __attribute__((ext_vector_type(C)));
    const vec_t w = *reinterpret_cast<const vec_t *>(p);
#pragma unroll
    for (int i = 0; i < C; ++i) out.v[i] = w[i];
  }
  return out;
}

template <class T, int C>
__device__ inline void pstore(T *p, const T (&v)[C]) {
  if constexpr (C == 1) {
    p[0] = v[0];
  } else {
    typedef T vec_t __attribute__((ext_vector_type(C)));
    vec_t w;
#pragma unroll
    for (int i = 0; i < C; ++i) w[i] = v[i];
    *reinterpret_cast<vec_t *>(p) = w;
  }
}

// Where a thread sits in a row team of 64 W lanes for K columns, C per lane.
template <int C, int W>
struct PTeam {
  int row_in_wg;   // which of the kPB / (64 W) rows of the workgroup
  int t;           // lane within the row team
  int lg;          // log2(K / C)
  int g;           // column group (columns g C .. g C + C - 1)
  int s;           // sub-team
  int S;           // sub-teams per row
  __device__ PTeam(int K) {
    row_in_wg = threadIdx.x / (kWave * W);
    t = threadIdx.x % (kWave * W);
    lg = __builtin_ctz(K / C);
    g = t & ((K / C) - 1);
    s = t >> lg;
    S = (kWave * W) >> lg;
  }
  __device__ bool lead() const { return t < (1 << lg); }
};

// Column groups per sub-team are at most 64 / 4 (K <= 64 with C = 4 for K >= 4).
constexpr int kMaxGroups = 16;

// acc[r][i] = sum over blocks p in [p0, p1) of M_p X_col(p), column g C + i, in the lead lanes.
// red: W > 1 only, kPB / (64 W) * W * kMaxGroups * BR * C values of LDS.
template <class T, int BR, int BC, int C, int W>
__device__ inline void pteam_accumulate(int p0, int p1, int K, const PTeam<C, W> &tm,
                                        const int *__restrict__ col, const T *__restrict__ val,
                                        int64_t nnz, const T *__restrict__ x, T (&acc)[BR][C],
                                        T *red) {
  int p = p0 + tm.s;
  int cn = p < p1 ? col[p] : 0;
  for (; p < p1; p += tm.S) {
    const int64_t c = cn;
    const int pn = p + tm.S;
    cn = pn < p1 ? col[pn] : 0;
    T a[BR * BC];
#pragma unroll
    for (int e = 0; e < BR * BC; ++e) a[e] = val[int64_t(p) * (BR * BC) + e];
    PVec<T, C> xv[BC];
#pragma unroll
    for (int cc = 0; cc < BC; ++cc) xv[cc] = pload<T, C>(x + (c * BC + cc) * K + tm.g * C);
#pragma unroll
    for (int r = 0; r < BR; ++r)
#pragma unroll
      for (int cc = 0; cc < BC; ++cc)
#pragma unroll
        for (int i = 0; i < C; ++i) acc[r][i] = fma(a[r * BC + cc], xv[cc].v[i], acc[r][i]);
  }
  // sub-teams of one wavefront: butterfly over the lane bits above the column group
  for (int off = K / C; off < kWave; off <<= 1)
#pragma unroll
    for (int r = 0; r < BR; ++r)
#pragma unroll
      for (int i = 0; i < C; ++i) acc[r][i] += __shfl_xor(acc[r][i], off, kWave);
  if constexpr (W > 1) {
    // wavefronts of the team: through LDS, summed in wavefront order by the lead lanes
    const int wv = tm.t / kWave, ln = tm.t % kWave;
    T *rr = red + tm.row_in_wg * (W * kMaxGroups * BR * C);
    if (ln < (K / C))
#pragma unroll
      for (int r = 0; r < BR; ++r)
#pragma unroll
        for (int i = 0; i < C; ++i) rr[((wv * kMaxGroups + ln) * BR + r) * C + i] = acc[r][i];
    __syncthreads();
    if (tm.lead())
#pragma unroll
      for (int r = 0; r < BR; ++r)
#pragma unroll
        for (int i = 0; i < C; ++i) {
          T v = rr[(tm.t * BR + r) * C + i];
#pragma unroll
          for (int w = 1; w < W; ++w) v += rr[((w * kMaxGroups + tm.t) * BR + r) * C + i];
          acc[r][i] = v;
        }
  }
}

// LDS for the cross-wavefront reduction of a W = 4 team (one row per workgroup).
template <class T, int BR, int C, int W>
struct PRed {
  static constexpr int n = W > 1 ? (kPB / (kWave * W)) * W * kMaxGroups * BR * C : 1;
};

// One colour of the symmetric block Gauss-Seidel sweep for K columns (see launch_pgs_fwd /
// launch_pgs_bwd).  The row's D^+ block and right-hand side are loaded before the row's blocks
// so their latency overlaps the block stream; the lead lanes finish the row.
// FWD: rp, col, val hold the blocks left of the diagonal and dval the diagonal blocks (block i
// for row i); BWD: rp, col, val hold whole rows.
template <class T, int B, bool FWD, int C, int W>
__global__ __launch_bounds__(kPB) void k_pgs_color(int r0, int r1, int K, const int *__restrict__ rp,
                                                   const int *__restrict__ col,
                                                   const T *__restrict__ val, int64_t nnz,
                                                   const T *__restrict__ dval, int64_t nd,
                                                   const T *__restrict__ Dinv,
                                                   const T *__restrict__ b, T *x, T *r) {
  __shared__ T red[PRed<T, B, C, W>::n];
  const PTeam<C, W> tm(K);
  const int row = r0 + xcd_block() * (kPB / (kWave * W)) + tm.row_in_wg;
  if (row >= r1) return;   // W = 4: the whole workgroup leaves together
  const int p0 = rp[row];
  const int p1 = rp[row + 1];
  PVec<T, C> bq[B];
  T D[B][B];
  const int64_t rb = int64_t(row) * B;
  // every lane loads (valid addresses); only the lead lanes use them
#pragma unroll
  for (int q = 0; q < B; ++q) {
    bq[q] = pload<T, C>(b + (rb + q) * K + tm.g * C);
#pragma unroll
    for (int c = 0; c < B; ++c) D[q][c] = Dinv[(rb + q) * B + c];
  }
  T acc[B][C];
#pragma unroll
  for (int q = 0; q < B; ++q)
#pragma unroll
    for (int i = 0; i < C; ++i) acc[q][i] = T(0);
  pteam_accumulate<T, B, B, C, W>(p0, p1, K, tm, col, val, nnz, x, acc, red);
  if (!tm.lead()) return;
  // forward: the diagonal block, loaded after the row stream to keep registers for it
  T Ad[B][B];
#pragma unroll
  for (int q = 0; q < B; ++q)
#pragma unroll
    for (int c = 0; c < B; ++c) Ad[q][c] = FWD ? dval[int64_t(row) * (B * B) + q * B + c] : T(0);
  T xo[B][C];
#pragma unroll
  for (int i = 0; i < C; ++i) {
    T t[B];
#pragma unroll
    for (int q = 0; q < B; ++q) t[q] = bq[q].v[i] - acc[q][i];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      T v = T(0);
#pragma unroll
      for (int c = 0; c < B; ++c) v = fma(D[q][c], t[c], v);
      xo[q][i] = v;
    }
    if (FWD) {
      // r = t - A_ii x_i, kept in acc
#pragma unroll
      for (int q = 0; q < B; ++q) {
        T v = t[q];
#pragma unroll
        for (int c = 0; c < B; ++c) v = fma(-Ad[q][c], xo[c][i], v);
        acc[q][i] = v;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < B; ++q) {
    T *xq = x + (rb + q) * K + tm.g * C;
    if (FWD) {
      pstore<T, C>(xq, xo[q]);
      pstore<T, C>(r + (rb + q) * K + tm.g * C, acc[q]);
    } else {
      const PVec<T, C> old = pload<T, C>(xq);
      T nv[C];
#pragma unroll
      for (int i = 0; i < C; ++i) nv[i] = old.v[i] + xo[q][i];
      pstore<T, C>(xq, nv);
    }
  }
}

// rp, col, val: the blocks right of the diagonal.
template <class T, int B, int C, int W>
__global__ __launch_bounds__(kPB) void k_presid_upper(int n_rows, int K, const int *__restrict__ rp,
                                                      const int *__restrict__ col,
                                                      const T *__restrict__ val, int64_t nnz,
                                                      const T *__restrict__ x, T *__restrict__ r) {
  __shared__ T red[PRed<T, B, C, W>::n];
  const PTeam<C, W> tm(K);
  const int row = blockIdx.x * (kPB / (kWave * W)) + tm.row_in_wg;
  if (row >= n_rows) return;
  const int64_t rb = int64_t(row) * B;
  PVec<T, C> rq[B];
  T acc[B][C];
#pragma unroll
  for (int q = 0; q < B; ++q) {
    rq[q] = pload<T, C>(r + (rb + q) * K + tm.g * C);
#pragma unroll
    for (int i = 0; i < C; ++i) acc[q][i] = T(0);
  }
  pteam_accumulate<T, B, B, C, W>(rp[row], rp[row + 1], K, tm, col, val, nnz, x, acc, red);
  if (!tm.lead()) return;
#pragma unroll
  for (int q = 0; q < B; ++q) {
    T v[C];
#pragma unroll
    for (int i = 0; i < C; ++i) v[i] = rq[q].v[i] - acc[q][i];
    pstore<T, C>(r + (rb + q) * K + tm.g * C, v);
  }
}

template <class T, int BR, int BC, int C, int W>
__global__ __launch_bounds__(kPB) void k_prect(int n_rows, int K, const int *__restrict__ rp,
                                               const int *__restrict__ col,
                                               const T *__restrict__ val, int64_t nnz,
                                               const T *__restrict__ x, T *__restrict__ y,
                                               int accumulate) {
  __shared__ T red[PRed<T, BR, C, W>::n];
  const PTeam<C, W> tm(K);
  const int row = blockIdx.x * (kPB / (kWave * W)) + tm.row_in_wg;
  if (row >= n_rows) return;
  T acc[BR][C];
#pragma unroll
  for (int q = 0; q < BR; ++q)
#pragma unroll
    for (int i = 0; i < C; ++i) acc[q][i] = T(0);
  pteam_accumulate<T, BR, BC, C, W>(rp[row], rp[row + 1], K, tm, col, val, nnz, x, acc, red);
  if (!tm.lead()) return;
#pragma unroll
  for (int q = 0; q < BR; ++q) {
    T *yq = y + (int64_t(row) * BR + q) * K + tm.g * C;
    T v[C];
    if (accumulate) {
      const PVec<T, C> old = pload<T, C>(yq);
#pragma unroll
      for (int i = 0; i < C; ++i) v[i] = old.v[i] + acc[q][i];
    } else {
#pragma unroll
      for (int i = 0; i < C; ++i) v[i] = acc[q][i];
    }
    pstore<T, C>(yq, v);
  }
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

// Y = A X (W = 1 teams), the workgroups striding over groups of four rows so that the
// per-column partial sums of X.Y come in at most kPSpmvMax workgroups.
constexpr int kPSpmvMax = 2048;

template <int B, int C>
__global__ __launch_bounds__(kPB) void k_pspmv(int n_rows, int K, const int *__restrict__ rp,
                                               const int *__restrict__ col,
                                               const double *__restrict__ val, int64_t nnz,
                                               const double *__restrict__ x, double *__restrict__ y,
                                               double *part) {
  __shared__ double sh[kPB][C];
  const PTeam<C, 1> tm(K);
  constexpr int rows_pb = kPB / kWave;
  double d[C];
#pragma unroll
  for (int i = 0; i < C; ++i) d[i] = 0.0;
  for (int row0 = blockIdx.x * rows_pb; row0 < n_rows; row0 += gridDim.x * rows_pb) {
    const int row = row0 + tm.row_in_wg;
    if (row >= n_rows) continue;   // whole wavefronts; no workgroup barrier inside
    double acc[B][C];
#pragma unroll
    for (int q = 0; q < B; ++q)
#pragma unroll
      for (int i = 0; i < C; ++i) acc[q][i] = 0.0;
    pteam_accumulate<double, B, B, C, 1>(rp[row], rp[row + 1], K, tm, col, val, nnz, x, acc, nullptr);
    if (tm.lead()) {
#pragma unroll
      for (int q = 0; q < B; ++q) {
        const int64_t e = (int64_t(row) * B + q) * K + tm.g * C;
        const PVec<double, C> xv = pload<double, C>(x + e);
        pstore<double, C>(y + e, acc[q]);
#pragma unroll
        for (int i = 0; i < C; ++i) d[i] = fma(xv.v[i], acc[q][i], d[i]);
      }
    }
  }
  if (part) {
    // per-column sums over the workgroup: thread t holds columns (t mod (K / C)) C + i
#pragma unroll
    for (int i = 0; i < C; ++i) sh[threadIdx.x][i] = tm.lead() ? d[i] : 0.0;
    __syncthreads();
    const int KL = K / C;
    for (int st = kPB / 2; st >= KL; st >>= 1) {
      if (int(threadIdx.x) < st)
#pragma unroll
        for (int i = 0; i < C; ++i) sh[threadIdx.x][i] += sh[threadIdx.x + st][i];
      __syncthreads();
    }
    if (int(threadIdx.x) < KL)
#pragma unroll
      for (int i = 0; i < C; ++i) part[int64_t(blockIdx.x) * K + threadIdx.x * C + i] = sh[threadIdx.x][i];
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
  // unrolled so that the loads are in flight together; the sum keeps its order
#pragma unroll 16
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

// Columns per lane: 4 when the panel is at least 4 wide.
inline int pcols(int K) { return K >= 4 ? 4 : K; }

// Team width: a whole workgroup per row when its 64 * 4 * C / K sub-teams still find a block
// each in an average row, else one wavefront per row.
inline int pwaves(const SolveMat &M, int K) {
  if (M.panel_waves == 1 || M.panel_waves == 4) return M.panel_waves;   // tuned
  const double avg = M.n_rows ? double(M.nnz) / M.n_rows : 0.0;
  return (kWave * 4.0 * pcols(K) / K <= avg) ? 4 : 1;
}

inline unsigned pteam_grid(int rows, int W) { return pgrid(rows, kPB / (kWave * W)); }

#define EAMG_PCOLS(C_, ...)                                     \
  switch (pcols(K)) {                                           \
    case 1: { constexpr int C_ = 1; __VA_ARGS__; } break;       \
    case 2: { constexpr int C_ = 2; __VA_ARGS__; } break;       \
    default: { constexpr int C_ = 4; __VA_ARGS__; } break;      \
  }
#define EAMG_PTEAM(W_, M_, ...)                                 \
  if (pwaves(M_, K) == 4) { constexpr int W_ = 4; __VA_ARGS__; } \
  else { constexpr int W_ = 1; __VA_ARGS__; }

template <class T, bool FWD>
hipError_t launch_pgs(const SolveMat &A, const T *Dinv, int r0, int r1, int K, const T *b, T *x, T *r,
                      hipStream_t s) {
  if (r1 <= r0) return hipSuccess;
  const bool f32 = sizeof(T) == 4;
  const T *val = FWD ? reinterpret_cast<const T *>(f32 ? (const void *)A.lo_val32 : (const void *)A.lo_val)
                     : pvals<T>(A);
  const T *dval = FWD ? reinterpret_cast<const T *>(f32 ? (const void *)A.dg_val32 : (const void *)A.dg_val)
                      : nullptr;
  const int *rp = FWD ? A.lo_rp : A.rp;
  const int *col = FWD ? A.lo_col : A.col;
  const int64_t nnz = FWD ? A.lo_nnz : A.nnz;
  const int64_t nd = A.n_rows;
  if (!val || !rp || !valid_k(K) || (FWD && !dval) || r0 < 0 || r1 > A.n_rows) return hipErrorInvalidValue;
#define EAMG_PGS(B_)                                                                                \
  EAMG_PTEAM(W, A, EAMG_PCOLS(C, hipLaunchKernelGGL((k_pgs_color<T, B_, FWD, C, W>),               \
                                                    dim3(pteam_grid(r1 - r0, W)), dim3(kPB), 0, s, \
                                                    r0, r1, K, rp, col, val, nnz, dval, nd,        \
                                                    Dinv, b, x, r)))
  switch (A.br) {
    case 1: EAMG_PGS(1); break;
    case 3: EAMG_PGS(3); break;
    case 6: EAMG_PGS(6); break;
    default: return hipErrorInvalidValue;
  }
#undef EAMG_PGS
  EAMG_PCHECK();
}

template <class T>
hipError_t launch_pgs_fwd(const SolveMat &A, const T *Dinv, int r0, int r1, int K, const T *b, T *x,
                          T *r, hipStream_t s) {
  return launch_pgs<T, true>(A, Dinv, r0, r1, K, b, x, r, s);
}

template <class T>
hipError_t launch_pgs_bwd(const SolveMat &A, const T *Dinv, int r0, int r1, int K, const T *b, T *x,
                          hipStream_t s) {
  return launch_pgs<T, false>(A, Dinv, r0, r1, K, b, x, nullptr, s);
}

template <class T>
hipError_t launch_presid_upper(const SolveMat &A, int K, const T *x, T *r, hipStream_t s) {
  if (A.n_rows == 0) return hipSuccess;
  const T *val = reinterpret_cast<const T *>(sizeof(T) == 4 ? (const void *)A.up_val32 : (const void *)A.up_val);
  if (!val || !A.up_rp || !valid_k(K)) return hipErrorInvalidValue;
#define EAMG_PRES(B_)                                                                             \
  EAMG_PTEAM(W, A, EAMG_PCOLS(C, hipLaunchKernelGGL((k_presid_upper<T, B_, C, W>),               \
                                                    dim3(pteam_grid(A.n_rows, W)), dim3(kPB), 0, \
                                                    s, A.n_rows, K, A.up_rp, A.up_col, val,      \
                                                    A.up_nnz, x, r)))
  switch (A.br) {
    case 1: EAMG_PRES(1); break;
    case 3: EAMG_PRES(3); break;
    case 6: EAMG_PRES(6); break;
    default: return hipErrorInvalidValue;
  }
#undef EAMG_PRES
  EAMG_PCHECK();
}

template <class T>
hipError_t launch_prect(const SolveMat &M, int K, const T *x, T *y, bool accumulate, hipStream_t s) {
  if (M.n_rows == 0) return hipSuccess;
  const T *val = pvals<T>(M);
  if (!val || !valid_k(K)) return hipErrorInvalidValue;
  const int accf = accumulate ? 1 : 0;
#define EAMG_PRECT(BR_, BC_)                                                                      \
  EAMG_PTEAM(W, M, EAMG_PCOLS(C, hipLaunchKernelGGL((k_prect<T, BR_, BC_, C, W>),                \
                                                    dim3(pteam_grid(M.n_rows, W)), dim3(kPB), 0, \
                                                    s, M.n_rows, K, M.rp, M.col, val, M.nnz, x,  \
                                                    y, accf)))
  if (M.br == 1 && M.bc == 1) { EAMG_PRECT(1, 1); }
  else if (M.br == 3 && M.bc == 6) { EAMG_PRECT(3, 6); }
  else if (M.br == 6 && M.bc == 3) { EAMG_PRECT(6, 3); }
  else if (M.br == 6 && M.bc == 6) { EAMG_PRECT(6, 6); }
  else return hipErrorInvalidValue;
#undef EAMG_PRECT
  EAMG_PCHECK();
}

int pspmv_blocks(const SolveMat &A, int K) {
  const int g = K > 0 ? int(pgrid(A.n_rows, kPB / kWave)) : 0;
  return g < kPSpmvMax ? (g < 1 ? 1 : g) : kPSpmvMax;
}

hipError_t launch_pspmv(const SolveMat &A, int K, const double *x, double *y, double *part,
                        hipStream_t s) {
  if (A.n_rows == 0) return hipSuccess;
  if (!valid_k(K) || A.br != A.bc) return hipErrorInvalidValue;
  const dim3 grid(pspmv_blocks(A, K));
  switch (A.br) {
    case 1: EAMG_PCOLS(C, hipLaunchKernelGGL((k_pspmv<1, C>), grid, dim3(kPB), 0, s, A.n_rows, K, A.rp, A.col, A.val, A.nnz, x, y, part)); break;
    case 3: EAMG_PCOLS(C, hipLaunchKernelGGL((k_pspmv<3, C>), grid, dim3(kPB), 0, s, A.n_rows, K, A.rp, A.col, A.val, A.nnz, x, y, part)); break;
    case 6: EAMG_PCOLS(C, hipLaunchKernelGGL((k_pspmv<6, C>), grid, dim3(kPB), 0, s, A.n_rows, K, A.rp, A.col, A.val, A.nnz, x, y, part)); break;
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

template hipError_t launch_pgs_fwd<double>(const SolveMat &, const double *, int, int, int, const double *, double *, double *, hipStream_t);
template hipError_t launch_pgs_fwd<float>(const SolveMat &, const float *, int, int, int, const float *, float *, float *, hipStream_t);
template hipError_t launch_pgs_bwd<double>(const SolveMat &, const double *, int, int, int, const double *, double *, hipStream_t);
template hipError_t launch_pgs_bwd<float>(const SolveMat &, const float *, int, int, int, const float *, float *, hipStream_t);
template hipError_t launch_presid_upper<double>(const SolveMat &, int, const double *, double *, hipStream_t);
template hipError_t launch_presid_upper<float>(const SolveMat &, int, const float *, float *, hipStream_t);
template hipError_t launch_prect<double>(const SolveMat &, int, const double *, double *, bool, hipStream_t);
template hipError_t launch_prect<float>(const SolveMat &, int, const float *, float *, bool, hipStream_t);

}  // namespace eamg
