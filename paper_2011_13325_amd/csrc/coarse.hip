// Coarsest-level direct solve: device assembly of the dense regularized matrix, its in-place
// blocked Gauss-Jordan inversion, and the dense products that apply the inverse and the dense
// V-cycle tails: full matrix times a vector or a panel, and the packed symmetric product
// (coarse.hpp).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "coarse.hpp"

namespace eamg {

namespace {

constexpr int T64 = kDenseTile;
constexpr int kThreads = 256;

inline int cdiv(int64_t a, int64_t b) { return int((a + b - 1) / b); }

// ---- assembly ------------------------------------------------------------------------------

// One thread per dof row (i, a): row i * bs + a of D gets the blocks of block row i of the
// block CSR matrix (AoS bs x bs blocks), plus reg_i on the diagonal block.  D is zero on entry.
__global__ void k_dense_assemble(int n, int bs, const int64_t *__restrict__ rp,
                                 const int *__restrict__ col, const double *__restrict__ val,
                                 const double *__restrict__ reg, int ld, double *__restrict__ D) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(n) * bs) return;
  const int i = int(t / bs), a = int(t % bs);
  double *Dr = D + size_t(t) * ld;
  for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
    const int j = col[q];
    for (int c = 0; c < bs; ++c) {
      double v = val[size_t(q) * bs * bs + a * bs + c];
      if (j == i) v += reg[size_t(i) * bs * bs + a * bs + c];
      Dr[size_t(j) * bs + c] = v;
    }
  }
}

__global__ void k_dense_pad_identity(int N, int ld, double *D) {
  const int i = N + int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < ld) D[size_t(i) * ld + i] = 1.0;
}

// ---- Gauss-Jordan inversion ----------------------------------------------------------------
// Block step K with P = A_KK^{-1}:  A_KJ := P A_KJ (J != K),  A_IK := -A_IK P (I != K),
// A_IJ := A_IJ - A_IK P A_KJ (I, J != K),  A_KK := P.  Without pivoting this needs every pivot
// block (a Schur complement of A) to be invertible, which holds for SPD A.

// P = A_KK^{-1} by unblocked Gauss-Jordan on the tile in LDS (the same step with scalars).
__global__ __launch_bounds__(kThreads) void k_gj_pivot(int ld, int K, const double *__restrict__ A,
                                                      double *__restrict__ P, int *flag) {
  __shared__ double M[T64][T64 + 1];
  __shared__ double rowk[T64], colk[T64];
  const int t = threadIdx.x;
  const double *Akk = A + size_t(K) * T64 * ld + size_t(K) * T64;
  for (int e = t; e < T64 * T64; e += kThreads) M[e / T64][e % T64] = Akk[size_t(e / T64) * ld + e % T64];
  __syncthreads();
  bool bad = false;
  for (int k = 0; k < T64; ++k) {
    double piv = M[k][k];
    if (!(piv > 0.0) || !isfinite(piv)) {   // the same value on every thread: a uniform branch
      bad = true;
      piv = 1.0;
    }
    if (t < T64) {
      rowk[t] = (t == k ? 1.0 : M[k][t]) / piv;
      colk[t] = M[t][k];
    }
    __syncthreads();
    // rows i != k only: row k and column k are read from rowk / colk
    for (int e = t; e < T64 * T64; e += kThreads) {
      const int i = e / T64, j = e % T64;
      if (i != k) M[i][j] = (j == k ? 0.0 : M[i][j]) - colk[i] * rowk[j];
    }
    if (t < T64) M[k][t] = rowk[t];
    __syncthreads();
  }
  for (int e = t; e < T64 * T64; e += kThreads) P[e] = M[e / T64][e % T64];
  if (bad && t == 0) *flag = 1;
}

// Row panel R_J = P A_KJ (J != K), R_K = P; saved column panel C_J = A_JK (J != K).
// One workgroup per tile J; thread (ty, tx) computes rows 4 ty + p, columns tx + 16 q.
__global__ __launch_bounds__(kThreads) void k_gj_panels(int ld, int K, const double *__restrict__ A,
                                                       const double *__restrict__ P,
                                                       double *__restrict__ R,
                                                       double *__restrict__ C) {
  __shared__ double Ps[T64][T64 + 1], Bs[T64][T64 + 1];
  const int J = blockIdx.x, t = threadIdx.x;
  double *Rj = R + size_t(J) * T64 * T64;
  if (J == K) {
    for (int e = t; e < T64 * T64; e += kThreads) Rj[e] = P[e];
    return;
  }
  const double *Akj = A + size_t(K) * T64 * ld + size_t(J) * T64;
  const double *Ajk = A + size_t(J) * T64 * ld + size_t(K) * T64;
  double *Cj = C + size_t(J) * T64 * T64;
  for (int e = t; e < T64 * T64; e += kThreads) {
    const int i = e / T64, j = e % T64;
    Ps[i][j] = P[e];
    Bs[i][j] = Akj[size_t(i) * ld + j];
    Cj[e] = Ajk[size_t(i) * ld + j];
  }
  __syncthreads();
  const int ty = t / 16, tx = t % 16;
  double acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
  for (int k = 0; k < T64; ++k) {
    double a[4], b[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) a[p] = Ps[ty * 4 + p][k];
#pragma unroll
    for (int q = 0; q < 4; ++q) b[q] = Bs[k][tx + 16 * q];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) Rj[(ty * 4 + p) * T64 + tx + 16 * q] = acc[p][q];
}

// Tile (I, J): I == K: A_KJ := R_J; else A_IJ := [J != K] A_IJ - C_I R_J.
__global__ __launch_bounds__(kThreads) void k_gj_update(int ld, int K, double *__restrict__ A,
                                                       const double *__restrict__ R,
                                                       const double *__restrict__ C) {
  __shared__ double Cs[T64][T64 + 1], Rs[T64][T64 + 1];
  const int J = blockIdx.x, I = blockIdx.y, t = threadIdx.x;
  double *Aij = A + size_t(I) * T64 * ld + size_t(J) * T64;
  const double *Rj = R + size_t(J) * T64 * T64;
  if (I == K) {
    for (int e = t; e < T64 * T64; e += kThreads) Aij[size_t(e / T64) * ld + e % T64] = Rj[e];
    return;
  }
  const double *Ci = C + size_t(I) * T64 * T64;
  for (int e = t; e < T64 * T64; e += kThreads) {
    Cs[e / T64][e % T64] = Ci[e];
    Rs[e / T64][e % T64] = Rj[e];
  }
  const int ty = t / 16, tx = t % 16;
  double acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      acc[p][q] = (J == K) ? 0.0 : Aij[size_t(ty * 4 + p) * ld + tx + 16 * q];
  __syncthreads();
  for (int k = 0; k < T64; ++k) {
    double a[4], b[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) a[p] = Cs[ty * 4 + p][k];
#pragma unroll
    for (int q = 0; q < 4; ++q) b[q] = Rs[k][tx + 16 * q];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[p][q] = fma(-a[p], b[q], acc[p][q]);
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) Aij[size_t(ty * 4 + p) * ld + tx + 16 * q] = acc[p][q];
}

// A := (A + A^T) / 2; each unordered pair {i, j} belongs to one thread.
__global__ void k_symmetrize(int ld, double *A) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(ld) * ld) return;
  const int i = int(e / ld), j = int(e % ld);
  if (i >= j) return;
  const double v = 0.5 * (A[size_t(i) * ld + j] + A[size_t(j) * ld + i]);
  A[size_t(i) * ld + j] = v;
  A[size_t(j) * ld + i] = v;
}

// ---- application -----------------------------------------------------------------------------

// y = D x: one wavefront per row; lane l reads columns 128 c + 2 l, 128 c + 1 + 2 l (one 16-byte
// load) for every chunk c, four chunks in flight; the padding columns (>= n) are zero in D and
// read as zero from x.
template <class T>
__global__ __launch_bounds__(kThreads) void k_dense_gemv(int n, int ld, const double *__restrict__ D,
                                                        const T *__restrict__ x, T *__restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int row = int(blockIdx.x) * (kThreads / 64) + int(threadIdx.x) / 64;
  if (row >= n) return;   // whole wavefronts
  const double2 *Dr = reinterpret_cast<const double2 *>(D + size_t(row) * ld);
  const int nc = ld / 128;
  double acc0 = 0.0, acc1 = 0.0;
  int c = 0;
  for (; c + 4 <= nc; c += 4) {
    double2 d[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) d[u] = Dr[(c + u) * 64 + lane];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = (c + u) * 128 + 2 * lane;
      const double x0 = j < n ? double(x[j]) : 0.0;
      const double x1 = j + 1 < n ? double(x[j + 1]) : 0.0;
      acc0 = fma(d[u].x, x0, acc0);
      acc1 = fma(d[u].y, x1, acc1);
    }
  }
  for (; c < nc; ++c) {
    const double2 d = Dr[c * 64 + lane];
    const int j = c * 128 + 2 * lane;
    const double x0 = j < n ? double(x[j]) : 0.0;
    const double x1 = j + 1 < n ? double(x[j + 1]) : 0.0;
    acc0 = fma(d.x, x0, acc0);
    acc1 = fma(d.y, x1, acc1);
  }
  double acc = acc0 + acc1;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) y[row] = T(acc);
}

// ---- symmetric packed product ----------------------------------------------------------------

// Tile (i, j) of the upper block triangle from its packed index t (row by row: tile (i, j) has
// index i * nb - i * (i - 1) / 2 + j - i).  Uniform over the workgroup.
__device__ inline void sym_tile_of(int t, int nb, int &i, int &j) {
  int r = t, a = 0;
  while (r >= nb - a) {
    r -= nb - a;
    ++a;
  }
  i = a;
  j = a + r;
}

// S (packed, TM) := the upper tiles of (D + D^T) / 2 for the first n rows and columns of D
// (leading dimension ld), zero elsewhere.  Grid: (entries per tile / 256, tiles).
template <class TM>
__global__ void k_pack_sym(int n, int ld, int nb, const double *__restrict__ D, TM *__restrict__ S) {
  int i, j;
  sym_tile_of(int(blockIdx.y), nb, i, j);
  const int e = int(blockIdx.x) * blockDim.x + threadIdx.x;   // < kSymTile^2
  const int a = i * kSymTile + e / kSymTile, b = j * kSymTile + e % kSymTile;
  double v = 0.0;
  if (a < n && b < n) v = 0.5 * (D[size_t(a) * ld + b] + D[size_t(b) * ld + a]);
  S[size_t(blockIdx.y) * kSymTile * kSymTile + e] = TM(v);
}

__device__ inline double2 load_pair(const double *p) { return *reinterpret_cast<const double2 *>(p); }
__device__ inline double2 load_pair(const float *p) {
  const float2 v = *reinterpret_cast<const float2 *>(p);
  return make_double2(double(v.x), double(v.y));
}

// One halving exchange of the row sums: p[k] of lane l is its part of row k (k < 2 H); the lane
// keeps the half of its rows that matches lane bit 2 H, summed with its partner's (H a constant,
// so p stays in registers).
template <int H>
__device__ __forceinline__ void halve_rows(double (&p)[32], int lane) {
  const bool up = (lane & (2 * H)) != 0;
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const double send = up ? p[k] : p[k + H];
    const double keep = up ? p[k + H] : p[k];
    p[k] = keep + __shfl_xor(send, 2 * H, 64);
  }
}

// Tile t (packed index) of y = S x for one workgroup of four wavefronts (S, x and W of one
// matrix).  Wavefront w takes rows 32 w .. 32 w + 31 of the tile, lane l columns 2 l and 2 l + 1
// (one 16- or 8-byte load per row).  Row sums (the tile's part of y_i) are reduced across the
// lanes by halving exchanges; column sums (the part of y_j that the mirrored tile (j, i) would
// give, i < j) accumulate per lane and meet across the wavefronts in LDS.  Both go to W[b][q]
// (128 doubles: the part of output block b from source block q); every (b, q) is written exactly
// once.
template <class TM, class TV>
__device__ __forceinline__ void symv_tile(int n, int nb, int t, const TM *__restrict__ S,
                                          const TV *__restrict__ x, double *__restrict__ W,
                                          double (&colp)[4][kSymTile]) {
  int i, j;
  sym_tile_of(t, nb, i, j);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * w;
  const TM *T = S + size_t(t) * kSymTile * kSymTile + size_t(r0) * kSymTile + 2 * lane;
  // the three x loads of a lane at clamped indices (no branch between them), zero past n; x of
  // the wavefront's 32 rows is loaded once per lane (lanes l and l + 32 alike) and read out of
  // lane r for row r, so the loop has no load of x and no wait
  const int cj = j * kSymTile + 2 * lane;
  const int ri = i * kSymTile + r0 + (lane & 31);
  const double xj0r = double(x[min(cj, n - 1)]);
  const double xj1r = double(x[min(cj + 1, n - 1)]);
  const double xlr = double(x[min(ri, n - 1)]);
  const double xj0 = cj < n ? xj0r : 0.0;
  const double xj1 = cj + 1 < n ? xj1r : 0.0;
  const double xl = ri < n ? xlr : 0.0;
  const int xl_lo = __double2loint(xl), xl_hi = __double2hiint(xl);
  double p[32];
  double c0 = 0.0, c1 = 0.0;
#pragma unroll
  for (int r = 0; r < 32; ++r) {
    const double2 v = load_pair(T + r * kSymTile);
    const double xi = __hiloint2double(__builtin_amdgcn_readlane(xl_hi, r), __builtin_amdgcn_readlane(xl_lo, r));
    p[r] = fma(v.y, xj1, v.x * xj0);
    c0 = fma(v.x, xi, c0);
    c1 = fma(v.y, xi, c1);
  }
  // exchanges over lane bits 32, 16, .., 2
  halve_rows<16>(p, lane);
  halve_rows<8>(p, lane);
  halve_rows<4>(p, lane);
  halve_rows<2>(p, lane);
  halve_rows<1>(p, lane);
  const double rs = p[0] + __shfl_xor(p[0], 1, 64);   // row (lane >> 1) of this wavefront
  if ((lane & 1) == 0) W[(size_t(i) * nb + j) * kSymTile + r0 + (lane >> 1)] = rs;
  if (i != j) {
    colp[w][2 * lane] = c0;
    colp[w][2 * lane + 1] = c1;
    __syncthreads();
    if (threadIdx.x < kSymTile) {
      const int k = threadIdx.x;
      W[(size_t(j) * nb + i) * kSymTile + k] = ((colp[0][k] + colp[1][k]) + colp[2][k]) + colp[3][k];
    }
  }
}

// Row i of y from the partial sums W of its matrix: sum over q of W[i / 128][q][i % 128], q
// ascending.
__device__ inline double symv_row_sum(int nb, int i, const double *__restrict__ W) {
  const double *w = W + size_t(i / kSymTile) * nb * kSymTile + i % kSymTile;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int q = 0;
  for (; q + 4 <= nb; q += 4) {
    a0 += w[size_t(q) * kSymTile];
    a1 += w[size_t(q + 1) * kSymTile];
    a2 += w[size_t(q + 2) * kSymTile];
    a3 += w[size_t(q + 3) * kSymTile];
  }
  for (; q < nb; ++q) a0 += w[size_t(q) * kSymTile];
  return (a0 + a1) + (a2 + a3);
}

template <class TM, class TV>
__global__ __launch_bounds__(256) void k_dense_symv(int n, int nb, const TM *__restrict__ S,
                                                    const TV *__restrict__ x, double *__restrict__ W) {
  __shared__ double colp[4][kSymTile];
  symv_tile<TM, TV>(n, nb, int(blockIdx.x), S, x, W, colp);
}

template <class TV>
__global__ void k_dense_symv_sum(int n, int nb, const double *__restrict__ W, TV *__restrict__ y) {
  const int g = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= n) return;
  y[g] = TV(symv_row_sum(nb, g, W));
}

// The last part whose first tile (by_tile) or first row is at most t.
__device__ inline int sym_part_of(int nparts, const SymPart *__restrict__ parts, int t, bool by_tile) {
  int lo = 0, hi = nparts - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((by_tile ? parts[mid].t0 : parts[mid].row0) <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// One stored tile of any part per workgroup; parts whose system has stopped are skipped.
template <class TM, class TV>
__global__ __launch_bounds__(256) void k_dense_symv_multi(int nparts, const SymPart *__restrict__ parts,
                                                          const double *__restrict__ active,
                                                          const TV *__restrict__ x, double *__restrict__ W) {
  __shared__ double colp[4][kSymTile];
  const int t = int(blockIdx.x);
  const SymPart P = parts[sym_part_of(nparts, parts, t, true)];
  if (active && active[P.sys] == 0.0) return;   // the whole workgroup
  symv_tile<TM, TV>(P.n, P.nb, t - P.t0, static_cast<const TM *>(P.S), x + P.off, W + P.woff, colp);
}

template <class TV>
__global__ void k_dense_symv_sum_multi(int nparts, const SymPart *__restrict__ parts, int rows,
                                       const double *__restrict__ active, const double *__restrict__ W,
                                       TV *__restrict__ y) {
  const int g = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= rows) return;
  const SymPart P = parts[sym_part_of(nparts, parts, g, false)];
  if (active && active[P.sys] == 0.0) return;
  const int i = g - P.row0;
  y[P.off + i] = TV(symv_row_sum(P.nb, i, W + P.woff));
}

// Panel of K columns (entry (dof, k) at dof * K + k) holding columns j0 .. j0 + K - 1 of the
// n x n identity (zero where j0 + k >= n).
__global__ void k_identity_panel(int n, int K, int j0, double *__restrict__ B) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(n) * K) return;
  const int d = int(t / K), k = int(t % K);
  B[t] = (d == j0 + k) ? 1.0 : 0.0;
}

// Columns j0 .. j0 + ncols - 1 of the row-major matrix D (leading dimension ld, first n rows)
// := the first ncols columns of the panel X (n x K).
__global__ void k_scatter_panel(int n, int K, int j0, int ncols, const double *__restrict__ X, int ld,
                                double *__restrict__ D) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(n) * ncols) return;
  const int d = int(t / ncols), k = int(t % ncols);
  D[size_t(d) * ld + j0 + k] = X[size_t(d) * K + k];
}

// Y = D X for a panel of K columns on the matrix cores (v_mfma_f64_16x16x4): a dense FP64
// contraction, n x n by n x K.  One wavefront per 16-row tile of D and slice of the inner
// dimension (the slices give the chip enough wavefronts).  The inner indices go in blocks of 16:
// in step s (0..3) of a block, lane l supplies A[l % 16][l / 16] = D(row, kb + 4 (l / 16) + s) and,
// for each 16-column tile of the panel, B[l / 16][l % 16] = X(kb + 4 (l / 16) + s, column), so a
// lane's four D operands of a block are one contiguous 32-byte load (a row's 16 values of the
// block are one 128-byte line).  Lane l accumulates rows l / 16 + 4 v (v = 0..3) of column l % 16.
// D is read once in all; the partial products of the slices go to P (slice-major) and are summed
// in slice order by k_dense_panel_sum, so the result is deterministic.  NCT: 16-column tiles.
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <class T, int NCT>
__global__ __launch_bounds__(64) void k_dense_panel_mfma(int n, int ld, int K, int S,
                                                         const double *__restrict__ D,
                                                         const T *__restrict__ X,
                                                         double *__restrict__ P) {
  const int l = threadIdx.x;
  const int r0 = int(blockIdx.x) * 16, sl = int(blockIdx.y);
  const int blocks = (n + 15) / 16;                  // inner blocks of 16
  const int per = (blocks + S - 1) / S;
  const int k_begin = sl * per * 16;
  const int k_end = min(n, (sl + 1) * per * 16);
  const int ko = l >> 4, cl = l & 15;
  // rows r0..r0+15 are below ld (16-row tiles of n, ld a multiple of 128 >= n); rows >= n hold
  // the identity padding and their products are not stored.  Row starts are 1 KiB aligned and
  // kb + 4 ko is a multiple of 4, so the 32-byte loads are aligned.
  const double *Drow = D + size_t(r0 + cl) * ld;
  dbl4 acc[NCT];
#pragma unroll
  for (int t = 0; t < NCT; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int kb = k_begin; kb < k_end; kb += 16) {
    const int kq = kb + 4 * ko;
    dbl4 a4;
    if (kq + 4 <= k_end) {
      a4 = *reinterpret_cast<const dbl4 *>(Drow + kq);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) a4[q] = kq + q < k_end ? Drow[kq + q] : 0.0;
    }
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = kq + st;
      const bool kin = k < k_end;
#pragma unroll
      for (int t = 0; t < NCT; ++t) {
        const int col = 16 * t + cl;
        const double bv = (kin && col < K) ? double(X[size_t(k) * K + col]) : 0.0;
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a4[st], bv, acc[t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NCT; ++t) {
    const int col = 16 * t + cl;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = r0 + ko + 4 * v;
      if (row < n && col < K) P[(size_t(sl) * n + row) * K + col] = acc[t][v];
    }
  }
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_dense_panel_sum(int64_t nk, int S,
                                                              const double *__restrict__ P,
                                                              T *__restrict__ Y) {
  const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= nk) return;
  double v = P[i];
  for (int sl = 1; sl < S; ++sl) v += P[int64_t(sl) * nk + i];
  Y[i] = T(v);
}

}  // namespace

hipError_t launch_dense_assemble(int n, int bs, const int64_t *rp, const int *col,
                                 const double *val, const double *reg, int ld, double *D,
                                 hipStream_t s) {
  const int N = n * bs;
  if (N > ld) return hipErrorInvalidValue;
  hipError_t e = hipMemsetAsync(D, 0, sizeof(double) * size_t(ld) * ld, s);
  if (e != hipSuccess) return e;
  if (N > 0) hipLaunchKernelGGL(k_dense_assemble, dim3(cdiv(N, 256)), dim3(256), 0, s, n, bs, rp, col, val, reg, ld, D);
  if (ld > N) hipLaunchKernelGGL(k_dense_pad_identity, dim3(cdiv(ld - N, 256)), dim3(256), 0, s, N, ld, D);
  return hipGetLastError();
}

hipError_t launch_gj_invert(int ld, double *A, double *work, int *flag, hipStream_t s) {
  if (ld <= 0 || ld % 128 != 0) return hipErrorInvalidValue;
  const int nt = ld / T64;
  double *P = work;
  double *R = P + T64 * T64;
  double *C = R + size_t(nt) * T64 * T64;
  for (int K = 0; K < nt; ++K) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(kThreads), 0, s, ld, K, A, P, flag);
    hipLaunchKernelGGL(k_gj_panels, dim3(nt), dim3(kThreads), 0, s, ld, K, A, P, R, C);
    hipLaunchKernelGGL(k_gj_update, dim3(nt, nt), dim3(kThreads), 0, s, ld, K, A, R, C);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_symmetrize, dim3(cdiv(int64_t(ld) * ld, 256)), dim3(256), 0, s, ld, A);
  return hipGetLastError();
}

template <class T>
hipError_t launch_dense_gemv(int n, int ld, const double *D, const T *x, T *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (ld < n || ld % 128 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dense_gemv<T>, dim3(cdiv(n, kThreads / 64)), dim3(kThreads), 0, s, n, ld, D, x, y);
  return hipGetLastError();
}

hipError_t launch_identity_panel(int n, int K, int j0, double *B, hipStream_t s) {
  const int64_t nk = int64_t(n) * K;
  if (nk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_identity_panel, dim3(cdiv(nk, kThreads)), dim3(kThreads), 0, s, n, K, j0, B);
  return hipGetLastError();
}

hipError_t launch_scatter_panel(int n, int K, int j0, int ncols, const double *X, int ld, double *D,
                                hipStream_t s) {
  if (ncols < 1 || ncols > K || j0 + ncols > ld) return hipErrorInvalidValue;
  const int64_t nk = int64_t(n) * ncols;
  if (nk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_panel, dim3(cdiv(nk, kThreads)), dim3(kThreads), 0, s, n, K, j0, ncols,
                     X, ld, D);
  return hipGetLastError();
}

int dense_panel_splits(int n) {
  const int tiles = (n + 15) / 16;
  const int S = tiles > 0 ? (4096 + tiles - 1) / tiles : 1;
  return S < 1 ? 1 : (S > 32 ? 32 : S);
}

size_t dense_panel_work_doubles(int n, int K) { return size_t(dense_panel_splits(n)) * n * K; }

template <class T>
hipError_t launch_dense_panel(int n, int ld, int K, const double *D, const T *X, T *Y,
                              double *work, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (ld < n || ld % 128 != 0 || K < 1 || K > 64 || (K & (K - 1)) || !work)
    return hipErrorInvalidValue;
  const int S = dense_panel_splits(n);
  const dim3 grid(cdiv(n, 16), S);
  if (K <= 16)
    hipLaunchKernelGGL((k_dense_panel_mfma<T, 1>), grid, dim3(64), 0, s, n, ld, K, S, D, X, work);
  else if (K == 32)
    hipLaunchKernelGGL((k_dense_panel_mfma<T, 2>), grid, dim3(64), 0, s, n, ld, K, S, D, X, work);
  else
    hipLaunchKernelGGL((k_dense_panel_mfma<T, 4>), grid, dim3(64), 0, s, n, ld, K, S, D, X, work);
  const int64_t nk = int64_t(n) * K;
  hipLaunchKernelGGL(k_dense_panel_sum<T>, dim3(unsigned((nk + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, nk, S, work, Y);
  return hipGetLastError();
}

template <class TM>
hipError_t launch_pack_sym(int n, int ld, const double *D, TM *S, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (ld < n || ld % kSymTile != 0) return hipErrorInvalidValue;
  const int nb = sym_blocks(n);
  hipLaunchKernelGGL(k_pack_sym<TM>, dim3(kSymTile * kSymTile / 256, unsigned(sym_tiles(nb))), dim3(256), 0, s,
                     n, ld, nb, D, S);
  return hipGetLastError();
}

template <class TM, class TV>
hipError_t launch_dense_symv(int n, const TM *S, const TV *x, TV *y, double *W, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (!S || !W) return hipErrorInvalidValue;
  const int nb = sym_blocks(n);
  hipLaunchKernelGGL((k_dense_symv<TM, TV>), dim3(unsigned(sym_tiles(nb))), dim3(256), 0, s, n, nb, S, x, W);
  hipLaunchKernelGGL(k_dense_symv_sum<TV>, dim3(cdiv(n, kThreads)), dim3(kThreads), 0, s, n, nb, W, y);
  return hipGetLastError();
}

template <class TM, class TV>
hipError_t launch_dense_symv_multi(int nparts, const SymPart *parts, int tiles, int rows,
                                   const double *active, const TV *x, TV *y, double *W, hipStream_t s) {
  if (nparts == 0 || rows == 0) return hipSuccess;
  if (!parts || !W || tiles < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_dense_symv_multi<TM, TV>), dim3(unsigned(tiles)), dim3(256), 0, s, nparts, parts,
                     active, x, W);
  hipLaunchKernelGGL(k_dense_symv_sum_multi<TV>, dim3(cdiv(rows, kThreads)), dim3(kThreads), 0, s, nparts,
                     parts, rows, active, W, y);
  return hipGetLastError();
}

template hipError_t launch_pack_sym<double>(int, int, const double *, double *, hipStream_t);
template hipError_t launch_pack_sym<float>(int, int, const double *, float *, hipStream_t);
template hipError_t launch_dense_symv<double, double>(int, const double *, const double *, double *, double *, hipStream_t);
template hipError_t launch_dense_symv<double, float>(int, const double *, const float *, float *, double *, hipStream_t);
template hipError_t launch_dense_symv<float, float>(int, const float *, const float *, float *, double *, hipStream_t);
template hipError_t launch_dense_symv_multi<double, double>(int, const SymPart *, int, int, const double *,
                                                            const double *, double *, double *, hipStream_t);
template hipError_t launch_dense_symv_multi<double, float>(int, const SymPart *, int, int, const double *,
                                                           const float *, float *, double *, hipStream_t);
template hipError_t launch_dense_symv_multi<float, float>(int, const SymPart *, int, int, const double *,
                                                          const float *, float *, double *, hipStream_t);
template hipError_t launch_dense_gemv<double>(int, int, const double *, const double *, double *, hipStream_t);
template hipError_t launch_dense_gemv<float>(int, int, const double *, const float *, float *, hipStream_t);
template hipError_t launch_dense_panel<double>(int, int, int, const double *, const double *, double *, double *, hipStream_t);
template hipError_t launch_dense_panel<float>(int, int, int, const double *, const float *, float *, double *, hipStream_t);

}  // namespace eamg
