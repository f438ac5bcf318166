// Batched exact coarsening criteria on the device (Lemma thm:mu2, Thm thm:mu1).
//
// Both kernels perform the arithmetic of crit_core.hpp in FP64, compiled with -ffp-contract=off
// like the host, so every value equals the host's bit for bit.  This is latency-bound work on
// small matrices (k x k blocks, k <= 6, and union matrices up to 24 x 24), not a dense
// contraction: neither HBM nor MFMA bounds it, the chain of dependent operations per pair does.
//
//  * mu_b: one thread per pair, the shared routine itself.  A pair's chain is short; batches of
//    thousands of pairs fill the chip.
//  * mu_g: one wavefront per union.  The chain of a union (two cyclic Jacobi solves of order up
//    to 24, about 2000 rotations each) is far too long for one thread, so the wavefront spreads
//    the independent entries of every step over its lanes with the matrices in LDS.  Each entry
//    still sees the host's operations in the host's order: block products accumulate in the same
//    index order with the same zero skips, a rotation updates column and row entries with the
//    same formulas, sums of squares run sequentially in the same order on every lane, and the
//    eigenvalue sort applies the host's stable insertion sort as a permutation.
#include "criteria.hpp"
#include "hierarchy.hpp"

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

namespace eamg {
namespace {

constexpr int kCritBlock = 64;

__global__ __launch_bounds__(kCritBlock) void k_mu_b(LevelView w, const Sq *D, int np,
                                                     const int *pairs, double tau, double *out) {
  const int stride = gridDim.x * kCritBlock;
  for (int u = blockIdx.x * kCritBlock + threadIdx.x; u < np; u += stride)
    out[u] = crit::mu_b(w, D, pairs[2 * u], pairs[2 * u + 1], tau);
}

// ---- mu_g, one wavefront (one 64-lane workgroup) per union ---------------------------------

constexpr int kWLd = crit::kMaxUnionDim;   // leading dimension of the union matrices
constexpr int kWMat = kWLd * kWLd;
constexpr int kWOut = 192;                 // outside-neighbour entries held (NaN beyond)
constexpr int kMaxGWaves = 256 * 8;        // mu_g grid (grid-stride over the unions)

// small k x k matrices (row-major, leading dimension k) in LDS
enum {
  S_Y = 0,            // Y[a] = D_a Q^{H->a}, kMaxUnion slots
  S_Z = 4, S_ZP, S_YZ, S_S, S_T1, S_Q1, S_Q2, S_EE, S_X,
  S_KCC,              // kMaxUnion slots
  S_KCW = S_KCC + 4,  // kMaxUnion slots
  S_KWW = S_KCW + 4, S_WP, S_KW, S_A6, S_V6, S_P6T,
  S_COUNT
};

struct WShared {
  double L[kWMat], R[kWMat], U[kWMat], G[kWMat];
  double w[kWLd];
  double sm[S_COUNT][36];
  double w6[6];
  int ol[kWOut], oa[kWOut], oe[kWOut];   // outside entries in encounter order
  int sl[kWOut], sa[kWOut], se[kWOut];   // the same, sorted by neighbour (stable)
  int perm[kWLd];
};

__device__ __forceinline__ void wsync() { __syncthreads(); }

// the value every lane holds, as a wave-uniform value (all lanes hold the same)
__device__ __forceinline__ double uni(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane(int(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane(int(b >> 32));
  return __longlong_as_double(static_cast<long long>(static_cast<unsigned>(lo)) |
                              (static_cast<long long>(hi) << 32));
}

// C = A B, C = A^T B, C = A B^T (crit::mul with tr() operands): entry (i, j) accumulates over l
// ascending from 0.0, skipping zero entries of the left factor.
__device__ void w_mul(double *C, const double *A, const double *B, int k) {
  const int t = threadIdx.x;
  if (t < k * k) {
    const int i = t / k, j = t - i * k;
    double c = 0.0;
    for (int l = 0; l < k; ++l) {
      const double a = A[i * k + l];
      if (a == 0.0) continue;
      c += a * B[l * k + j];
    }
    C[t] = c;
  }
  wsync();
}
__device__ void w_mul_tA(double *C, const double *A, const double *B, int k) {
  const int t = threadIdx.x;
  if (t < k * k) {
    const int i = t / k, j = t - i * k;
    double c = 0.0;
    for (int l = 0; l < k; ++l) {
      const double a = A[l * k + i];
      if (a == 0.0) continue;
      c += a * B[l * k + j];
    }
    C[t] = c;
  }
  wsync();
}
__device__ void w_mul_tB(double *C, const double *A, const double *B, int k) {
  const int t = threadIdx.x;
  if (t < k * k) {
    const int i = t / k, j = t - i * k;
    double c = 0.0;
    for (int l = 0; l < k; ++l) {
      const double a = A[i * k + l];
      if (a == 0.0) continue;
      c += a * B[j * k + l];
    }
    C[t] = c;
  }
  wsync();
}
// out = A^T B C (crit::t3), tmp a scratch slot
__device__ void w_t3(double *out, const double *A, const double *B, const double *C, double *tmp,
                     int k) {
  w_mul_tA(tmp, A, B, k);
  w_mul(out, tmp, C, k);
}
// Q(t) of crit::q
__device__ void w_q(double *Q, const double *tv, int k) {
  const int t = threadIdx.x;
  if (t < k * k) {
    const int i = t / k, j = t - i * k;
    double v = i == j ? 1.0 : 0.0;
    if (k == 6) {
      if (i == 0 && j == 4) v = -tv[2];
      if (i == 0 && j == 5) v = tv[1];
      if (i == 1 && j == 3) v = tv[2];
      if (i == 1 && j == 5) v = -tv[0];
      if (i == 2 && j == 3) v = -tv[1];
      if (i == 2 && j == 4) v = tv[0];
    }
    Q[t] = v;
  }
  wsync();
}
__device__ void w_qtrans(double *Q, const double *xa, const double *xb, int k) {
  const double tv[3] = {xb[0] - xa[0], xb[1] - xa[1], xb[2] - xa[2]};
  w_q(Q, tv, k);
}
__device__ void w_qhalf(double *Q, const double *xa, const double *xb, int k) {
  const double tv[3] = {0.5 * (xb[0] - xa[0]), 0.5 * (xb[1] - xa[1]), 0.5 * (xb[2] - xa[2])};
  w_q(Q, tv, k);
}
__device__ void w_load(double *S, const double *src, int k) {
  if (int(threadIdx.x) < k * k) S[threadIdx.x] = src[threadIdx.x];
  wsync();
}
__device__ void w_zero(double *S, int k) {
  if (int(threadIdx.x) < k * k) S[threadIdx.x] = 0.0;
  wsync();
}
// Y += s X (crit::axpy)
__device__ void w_axpy(double *Y, double s, const double *X, int k) {
  if (int(threadIdx.x) < k * k) Y[threadIdx.x] += s * X[threadIdx.x];
  wsync();
}
__device__ void w_neg(double *Y, int k) {
  if (int(threadIdx.x) < k * k) Y[threadIdx.x] = -Y[threadIdx.x];
  wsync();
}
// block (a, b) of X (leading dimension ld) += s S, or s S^T (crit::put)
__device__ void w_put(double *X, int k, int a, int b, const double *S, double s, bool trans) {
  const int t = threadIdx.x;
  if (t < k * k) {
    const int u = t / k, v = t - u * k;
    X[(a * k + u) * kWLd + b * k + v] += s * (trans ? S[v * k + u] : S[t]);
  }
  wsync();
}

// crit::jacobi on the n x n matrix A (leading dimension ld) in LDS.  Rotations: lanes 0..n-1 own
// row / column entries of A, lanes 32..32+n-1 the entries of V.  tmp (n x n, ld) and perm are
// scratch for the final column permutation.
__device__ void w_jacobi(double *A, int n, int ld, double *w, double *V, double *tmp, int *perm) {
  const int t = threadIdx.x;
  if (V)
    for (int idx = t; idx < n * n; idx += kCritBlock) {
      const int i = idx / n, j = idx - i * n;
      V[i * ld + j] = i == j ? 1.0 : 0.0;
    }
  wsync();
  double fro2 = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) fro2 += A[i * ld + j] * A[i * ld + j];
  fro2 = uni(fro2);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * ld + q] * A[p * ld + q];
    off = uni(off);
    if (off <= 1e-40 * fro2 || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = uni(A[p * ld + q]);
        if (apq == 0.0) continue;
        const double theta = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
        const double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double cs = 1.0 / sqrt(tt * tt + 1.0), sn = tt * cs;
        // columns p, q of A
        if (t < n) {
          const double x = A[t * ld + p], y = A[t * ld + q];
          A[t * ld + p] = cs * x - sn * y;
          A[t * ld + q] = sn * x + cs * y;
        }
        wsync();
        // rows p, q of A (lanes < n) and columns p, q of V (lanes 32..)
        double *px = nullptr, *py = nullptr;
        if (t < n) {
          px = &A[p * ld + t];
          py = &A[q * ld + t];
        } else if (V && t >= 32 && t < 32 + n) {
          px = &V[(t - 32) * ld + p];
          py = &V[(t - 32) * ld + q];
        }
        if (px) {
          const double x = *px, y = *py;
          *px = cs * x - sn * y;
          *py = sn * x + cs * y;
        }
        wsync();
        if (t == 0) {
          A[p * ld + q] = 0.0;
          A[q * ld + p] = 0.0;
        }
        wsync();
      }
  }
  // eigenvalues ascending by the host's stable insertion sort, applied to V as a permutation
  if (t == 0) {
    for (int i = 0; i < n; ++i) {
      w[i] = A[i * ld + i];
      perm[i] = i;
    }
    for (int i = 1; i < n; ++i)
      for (int j = i; j > 0 && w[j] < w[j - 1]; --j) {
        const double x = w[j];
        w[j] = w[j - 1];
        w[j - 1] = x;
        const int pj = perm[j];
        perm[j] = perm[j - 1];
        perm[j - 1] = pj;
      }
  }
  wsync();
  if (V) {
    for (int idx = t; idx < n * n; idx += kCritBlock) {
      const int r = idx / n, c = idx - r * n;
      tmp[r * ld + c] = V[r * ld + perm[c]];
    }
    wsync();
    for (int idx = t; idx < n * n; idx += kCritBlock) {
      const int r = idx / n, c = idx - r * n;
      V[r * ld + c] = tmp[r * ld + c];
    }
    wsync();
  }
}

// P = pinv(X, tau) of crit::pinv (6 x 6 slots)
__device__ void w_pinv(double *P, const double *X, int k, double tau, WShared &sh) {
  const int t = threadIdx.x;
  double *A = sh.sm[S_A6], *V = sh.sm[S_V6];
  if (t < k * k) {
    const int i = t / k, j = t - i * k;
    A[t] = 0.5 * (X[i * k + j] + X[j * k + i]);
  }
  wsync();
  w_jacobi(A, k, k, sh.w6, V, sh.sm[S_P6T], sh.perm);
  const double lmax = sh.w6[k - 1];
  if (t < k * k) {
    const int i = t / k, j = t - i * k;
    double pv = 0.0;
    if (lmax > 0.0)
      for (int m = 0; m < k; ++m) {
        if (!(sh.w6[m] > tau * lmax)) continue;
        const double inv = 1.0 / sh.w6[m];
        const double vi = V[i * k + m] * inv;
        pv += vi * V[j * k + m];
      }
    P[t] = pv;
  }
  wsync();
}

// crit::genmax_n on L, R (n x n, leading dimension kWLd); U, G and R's storage are scratch.
__device__ double w_genmax(int n, double tau, WShared &sh) {
  const int t = threadIdx.x, ld = kWLd;
  double *L = sh.L, *R = sh.R, *U = sh.U, *G = sh.G;
  for (int idx = t; idx < n * n; idx += kCritBlock) {
    const int i = idx / n, j = idx - i * n;
    if (i < j) {
      const double l = 0.5 * (L[i * ld + j] + L[j * ld + i]);
      L[i * ld + j] = L[j * ld + i] = l;
      const double r = 0.5 * (R[i * ld + j] + R[j * ld + i]);
      R[i * ld + j] = R[j * ld + i] = r;
    }
  }
  wsync();
  double nL = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) nL += L[i * ld + j] * L[i * ld + j];
  nL = uni(sqrt(nL));
  if (nL == 0.0) return 0.0;
  w_jacobi(R, n, ld, sh.w, U, G, sh.perm);
  const double lmax = sh.w[n - 1];
  int nk = 0, nd = 0;
  for (int m = 0; m < n; ++m) {
    if (lmax > 0.0 && sh.w[m] > tau * lmax)
      ++nk;
    else
      ++nd;
  }
  // T(i, b) = sum_j L(i, j) U(j, c0 + b) into R's storage (the host's inner sums, computed once
  // per (i, b) instead of once per (a, i, b): the same values)
  auto tcols = [&](int c0, int nc) {
    for (int idx = t; idx < n * nc; idx += kCritBlock) {
      const int i = idx / nc, b = idx - i * nc;
      double li = 0.0;
      for (int j = 0; j < n; ++j) li += L[i * ld + j] * U[j * ld + c0 + b];
      R[i * ld + b] = li;
    }
    wsync();
  };
  if (nd) {
    tcols(0, nd);
    for (int idx = t; idx < nd * nd; idx += kCritBlock) {
      const int a = idx / nd, b = idx - a * nd;
      double v = 0.0;
      for (int i = 0; i < n; ++i) v += U[i * ld + a] * R[i * ld + b];
      G[a * ld + b] = v;
    }
    wsync();
    double s = 0.0;
    for (int a = 0; a < nd; ++a)
      for (int b = 0; b < nd; ++b) s += G[a * ld + b] * G[a * ld + b];
    if (uni(sqrt(s)) > tau * nL) return crit::inf();
    wsync();
  }
  if (!nk) return 0.0;
  tcols(nd, nk);
  for (int idx = t; idx < nk * nk; idx += kCritBlock) {
    const int a = idx / nk, b = idx - a * nk;
    double v = 0.0;
    for (int i = 0; i < n; ++i) v += U[i * ld + nd + a] * R[i * ld + b];
    G[a * ld + b] = v / (sqrt(sh.w[nd + a]) * sqrt(sh.w[nd + b]));
  }
  wsync();
  for (int idx = t; idx < nk * nk; idx += kCritBlock) {
    const int a = idx / nk, b = idx - a * nk;
    if (a < b) {
      const double g = 0.5 * (G[a * ld + b] + G[b * ld + a]);
      G[a * ld + b] = G[b * ld + a] = g;
    }
  }
  wsync();
  w_jacobi(G, nk, ld, sh.w, nullptr, nullptr, sh.perm);
  return uni(sh.w[nk - 1]);
}

// crit::mu_g of the union mem[0..nC) (ascending) with the whole wavefront
__device__ double w_mu_g(const LevelView &lev, const Sq *D, const int *mem, int nC, double tau,
                         WShared &sh) {
  const int t = threadIdx.x, k = lev.k, n = nC * k, ld = kWLd;
  double xH[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < nC; ++a)
    for (int d = 0; d < 3; ++d) xH[d] = xH[d] + lev.x[int64_t(3) * mem[a] + d];
  for (int d = 0; d < 3; ++d) xH[d] = xH[d] / double(nC);
  double *Z = sh.sm[S_Z], *Zp = sh.sm[S_ZP], *YZ = sh.sm[S_YZ], *S = sh.sm[S_S];
  double *T1 = sh.sm[S_T1], *Q1 = sh.sm[S_Q1], *Q2 = sh.sm[S_Q2], *Ee = sh.sm[S_EE];
  double *X = sh.sm[S_X];
  // L = D_C - D_C P_C pinv(P_C^T D_C P_C) P_C^T D_C
  w_zero(Z, k);
  for (int a = 0; a < nC; ++a) {
    w_qtrans(Q1, xH, lev.xp(mem[a]), k);
    w_mul(sh.sm[S_Y + a], D[mem[a]].a, Q1, k);
    w_mul_tA(X, Q1, sh.sm[S_Y + a], k);
    w_axpy(Z, 1.0, X, k);
  }
  w_pinv(Zp, Z, k, tau, sh);
  for (int idx = t; idx < n * n; idx += kCritBlock) {
    const int i = idx / n, j = idx - i * n;
    sh.L[i * ld + j] = 0.0;
    sh.R[i * ld + j] = 0.0;
  }
  wsync();
  for (int a = 0; a < nC; ++a) {
    w_mul(YZ, sh.sm[S_Y + a], Zp, k);
    for (int b = 0; b < nC; ++b) {
      w_mul_tB(S, YZ, sh.sm[S_Y + b], k);
      w_put(sh.L, k, a, b, S, -1.0, false);
    }
    w_put(sh.L, k, a, a, D[mem[a]].a, 1.0, false);
    w_put(sh.R, k, a, a, lev.M + int64_t(mem[a]) * k * k, 1.0, false);
  }
  // edges inside C and, in encounter order, the edges to outside neighbours
  int no = 0;
  for (int a = 0; a < nC; ++a) {
    const int i = mem[a];
    for (int64_t p = lev.nb_ptr[i]; p < lev.nb_ptr[i + 1]; ++p) {
      const int l = lev.nb[p], e = lev.nb_e[p];
      int b = -1;
      for (int c = 0; c < nC; ++c)
        if (mem[c] == l) b = c;
      if (b >= 0) {
        if (i < l) {
          w_qhalf(Q1, lev.xp(i), lev.xp(l), k);
          w_qhalf(Q2, lev.xp(l), lev.xp(i), k);
          w_load(Ee, lev.E + int64_t(e) * k * k, k);
          w_t3(X, Q1, Ee, Q1, T1, k);
          w_put(sh.R, k, a, a, X, 1.0, false);
          w_t3(X, Q2, Ee, Q2, T1, k);
          w_put(sh.R, k, b, b, X, 1.0, false);
          w_t3(X, Q1, Ee, Q2, T1, k);
          w_put(sh.R, k, a, b, X, -1.0, false);
          w_t3(X, Q2, Ee, Q1, T1, k);
          w_put(sh.R, k, b, a, X, -1.0, false);
        }
      } else {
        if (no == kWOut) return __builtin_nan("");
        if (t == 0) {
          sh.ol[no] = l;
          sh.oa[no] = a;
          sh.oe[no] = e;
        }
        ++no;
      }
    }
  }
  wsync();
  // group by outside neighbour, ascending, keeping encounter order within a neighbour: the
  // host's stable insertion sort, as ranks
  for (int s0 = t; s0 < no; s0 += kCritBlock) {
    const int l = sh.ol[s0];
    int r = 0;
    for (int q = 0; q < no; ++q) r += (sh.ol[q] < l || (sh.ol[q] == l && q < s0)) ? 1 : 0;
    sh.sl[r] = l;
    sh.sa[r] = sh.oa[s0];
    sh.se[r] = sh.oe[s0];
  }
  wsync();
  for (int s0 = 0; s0 < no;) {
    int s1 = s0 + 1;
    while (s1 < no && sh.sl[s1] == sh.sl[s0]) ++s1;
    const int cnt = s1 - s0;
    if (cnt > crit::kMaxUnion) return __builtin_nan("");
    if (cnt >= 2) {
      const int l = sh.sl[s0];
      int am[crit::kMaxUnion];
      double *Kww = sh.sm[S_KWW];
      w_zero(Kww, k);
      for (int x = 0; x < cnt; ++x) {
        const int a = sh.sa[s0 + x], e = sh.se[s0 + x], i = mem[a];
        w_qhalf(Q1, lev.xp(i), lev.xp(l), k);
        w_qhalf(Q2, lev.xp(l), lev.xp(i), k);
        w_load(Ee, lev.E + int64_t(e) * k * k, k);
        am[x] = a;
        w_t3(sh.sm[S_KCC + x], Q1, Ee, Q1, T1, k);
        w_t3(sh.sm[S_KCW + x], Q1, Ee, Q2, T1, k);
        w_neg(sh.sm[S_KCW + x], k);
        w_t3(X, Q2, Ee, Q2, T1, k);
        w_axpy(Kww, 1.0, X, k);
      }
      double *Wp = sh.sm[S_WP], *KW = sh.sm[S_KW];
      w_pinv(Wp, Kww, k, tau, sh);
      for (int x = 0; x < cnt; ++x) {
        w_mul(KW, sh.sm[S_KCW + x], Wp, k);
        for (int y = 0; y < cnt; ++y) {
          w_mul_tB(S, KW, sh.sm[S_KCW + y], k);
          w_neg(S, k);
          if (x == y) w_axpy(S, 1.0, sh.sm[S_KCC + x], k);
          w_put(sh.R, k, am[x], am[y], S, 0.25, false);
          w_put(sh.R, k, am[y], am[x], S, 0.25, true);
        }
      }
    }
    s0 = s1;
  }
  return w_genmax(n, tau, sh);
}

__global__ __launch_bounds__(kCritBlock) void k_mu_g_wave(LevelView lev, const Sq *D, int nu,
                                                          const int *unions, double tau,
                                                          double *out) {
  __shared__ WShared sh;
  for (int u = blockIdx.x; u < nu; u += gridDim.x) {
    int mem[crit::kMaxUnion];
    int nC = 0;
    for (int a = 0; a < crit::kMaxUnion; ++a) mem[a] = unions[crit::kMaxUnion * u + a];
    while (nC < crit::kMaxUnion && mem[nC] >= 0) ++nC;
    const double v = w_mu_g(lev, D, mem, nC, tau, sh);
    if (threadIdx.x == 0) out[u] = v;
    wsync();
  }
}

// ---- coarse level weights (Thm thm:cemats), one thread per aggregate / coarse edge ------------

// M^I = sum over members i (ascending) of Q^T W_i Q, Q = Q^{I->i}, W_i = M^i + the edges from i
// to dropped vertices pulled to i
__global__ __launch_bounds__(kCritBlock) void k_coarse_M(LevelView f, int nc, const int *mptr,
                                                         const int *mem,
                                                         const unsigned char *dmask,
                                                         const double *cc, double *Mout) {
  const int k = f.k;
  const int stride = gridDim.x * kCritBlock;
  for (int I = blockIdx.x * kCritBlock + threadIdx.x; I < nc; I += stride) {
    Sq acc(k);
    for (int a = mptr[I]; a < mptr[I + 1]; ++a) {
      const int i = mem[a];
      Sq W = f.Mmat(i);
      for (int64_t p = f.nb_ptr[i]; p < f.nb_ptr[i + 1]; ++p)
        if (dmask[f.nb[p]]) {
          const Sq Q = crit::qhalf(f.xp(i), f.xp(f.nb[p]), k);
          crit::axpy(W, 1.0, crit::t3(Q, f.Emat(f.nb_e[p]), Q));
        }
      const Sq Q = crit::qtrans(cc + int64_t(3) * I, f.xp(i), k);
      crit::axpy(acc, 1.0, crit::t3(Q, W, Q));
    }
    for (int t = 0; t < k * k; ++t) Mout[int64_t(I) * k * k + t] = acc.a[t];
  }
}

// E^{IJ} = sum over the fine edges (i, j) of the group, in order, of T^T E^{ij} T with
// T = Q^{ij} Q^{I->i} Q^{JI}
__global__ __launch_bounds__(kCritBlock) void k_coarse_E(LevelView f, const int *e0, const int *e1,
                                                         const int *agg_of, const double *cc,
                                                         int64_t ne, const int64_t *start,
                                                         const int64_t *order, double *Eout) {
  const int k = f.k;
  const int64_t stride = int64_t(gridDim.x) * kCritBlock;
  for (int64_t g = int64_t(blockIdx.x) * kCritBlock + threadIdx.x; g < ne; g += stride) {
    Sq acc(k);
    for (int64_t q = start[g]; q < start[g + 1]; ++q) {
      const int64_t e = order[q];
      const int i = e0[e], j = e1[e];
      const int I = agg_of[i], J = agg_of[j];
      const double *cI = cc + int64_t(3) * I, *cJ = cc + int64_t(3) * J;
      const Sq T = crit::mul(crit::mul(crit::qhalf(f.xp(i), f.xp(j), k), crit::qtrans(cI, f.xp(i), k)),
                             crit::qhalf(cJ, cI, k));
      crit::axpy(acc, 1.0, crit::t3(T, f.Emat(e), T));
    }
    for (int t = 0; t < k * k; ++t) Eout[g * k * k + t] = acc.a[t];
  }
}

// Device buffer that only grows.
struct DBuf {
  void *p = nullptr;
  size_t cap = 0;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  ~DBuf() {
    if (p) (void)hipFree(p);
  }
  void *reserve(size_t bytes) {
    if (bytes == 0) bytes = 1;
    if (bytes > cap) {
      if (p) hip_check(hipFree(p), "hipFree");
      p = nullptr;
      cap = 0;
      hip_check(hipMalloc(&p, bytes), "hipMalloc");
      cap = bytes;
    }
    return p;
  }
  template <class T>
  T *put(const T *h, size_t count, hipStream_t s) {
    T *d = static_cast<T *>(reserve(count * sizeof(T)));
    hip_check(copy_h2d_sync(d, h, count * sizeof(T), s), "upload");
    return d;
  }
};

// Device copy of one auxiliary level and its D-hat blocks.
struct DevLevel {
  DBuf x, E, M, nb_ptr, nb, nb_e, D, e0b, e1b;
  LevelView v;
  const Sq *d = nullptr;
  const int *e0 = nullptr, *e1 = nullptr;
  int64_t m = 0;
  void upload(const AuxLevel &l, const std::vector<Sq> &Dh, hipStream_t s) {
    if (l.n > 0 && Dh.size() != size_t(l.n)) fail(EAMG_ERR_INVALID_ARG, "criteria: D-hat size");
    v.n = l.n;
    v.k = l.k;
    v.x = x.put(l.x.data(), l.x.size(), s);
    v.E = E.put(l.E.data(), l.E.size(), s);
    v.M = M.put(l.M.data(), l.M.size(), s);
    v.nb_ptr = nb_ptr.put(l.nb_ptr.data(), l.nb_ptr.size(), s);
    v.nb = nb.put(l.nb.data(), l.nb.size(), s);
    v.nb_e = nb_e.put(l.nb_e.data(), l.nb_e.size(), s);
    d = D.put(Dh.data(), Dh.size(), s);
    e0 = e0b.put(l.e0.data(), l.e0.size(), s);
    e1 = e1b.put(l.e1.data(), l.e1.size(), s);
    m = l.m();
    // the sources may change once this returns
    hip_check(hipStreamSynchronize(s), "sync");
  }
};

class DeviceCriteria final : public CritBatch {
 public:
  explicit DeviceCriteria(hipStream_t s) : s_(s) {}

  void level(const AuxLevel &lev, const std::vector<Sq> &D) override {
    lev_.upload(lev, D, s_);
    lev_src_ = &lev;
    work_ = &lev_;
    wrk_src_ = nullptr;
  }
  void work(const AuxLevel &w, const std::vector<Sq> &D) override {
    if (&w == lev_src_) {
      work_ = &lev_;
      return;
    }
    wrk_.upload(w, D, s_);
    work_ = &wrk_;
    wrk_src_ = &w;
  }
  bool coarse_weights(const AuxLevel &fine, const std::vector<std::vector<int>> &aggs,
                      const std::vector<int> &agg_of, const std::vector<char> &dmask,
                      const std::vector<double> &cc, const std::vector<int64_t> &order,
                      const std::vector<int64_t> &start, WeightVec &M,
                      WeightVec &E) override {
    const DevLevel *dl = nullptr;
    if (&fine == lev_src_)
      dl = &lev_;
    else if (&fine == wrk_src_ && work_ == &wrk_)
      dl = &wrk_;
    if (!dl || dl->v.n != fine.n || dl->m != fine.m() || dl->v.k != fine.k || fine.k > 6) return false;
    const auto t0 = std::chrono::steady_clock::now();
    const int k = fine.k, kk = k * k, nc = int(aggs.size());
    const int64_t ne = int64_t(start.size()) - 1;
    // host checks of everything the kernels index with
    if (int64_t(agg_of.size()) != fine.n || int64_t(dmask.size()) != fine.n ||
        int64_t(cc.size()) != int64_t(3) * nc || ne < 0 || start.front() != 0 ||
        start.back() != int64_t(order.size()))
      fail(EAMG_ERR_INVALID_ARG, "coarse weights: sizes");
    std::vector<int> mptr(size_t(nc) + 1, 0), mem;
    for (int I = 0; I < nc; ++I) {
      for (int i : aggs[I]) {
        if (i < 0 || i >= fine.n || agg_of[i] != I) fail(EAMG_ERR_INVALID_ARG, "coarse weights: member");
        mem.push_back(i);
      }
      mptr[I + 1] = int(mem.size());
    }
    for (int64_t e : order)
      if (e < 0 || e >= fine.m() || agg_of[fine.e0[e]] < 0 || agg_of[fine.e1[e]] < 0)
        fail(EAMG_ERR_INVALID_ARG, "coarse weights: edge");
    for (int64_t g = 0; g < ne; ++g)
      if (start[g] > start[g + 1]) fail(EAMG_ERR_INVALID_ARG, "coarse weights: groups");
    std::vector<unsigned char> dm(dmask.begin(), dmask.end());
    const int *d_mptr = cw_mptr_.put(mptr.data(), mptr.size(), s_);
    const int *d_mem = cw_mem_.put(mem.data(), mem.size(), s_);
    const unsigned char *d_dm = cw_dm_.put(dm.data(), dm.size(), s_);
    const double *d_cc = cw_cc_.put(cc.data(), cc.size(), s_);
    const int *d_agg = cw_agg_.put(agg_of.data(), agg_of.size(), s_);
    const int64_t *d_start = cw_start_.put(start.data(), start.size(), s_);
    const int64_t *d_order = cw_order_.put(order.data(), order.size(), s_);
    double *d_M = static_cast<double *>(cw_M_.reserve(size_t(nc) * kk * sizeof(double)));
    double *d_E = static_cast<double *>(cw_E_.reserve(size_t(ne) * kk * sizeof(double)));
    if (nc > 0) {
      const int grid = std::min((nc + kCritBlock - 1) / kCritBlock, 8192);
      hipLaunchKernelGGL(k_coarse_M, dim3(grid), dim3(kCritBlock), 0, s_, dl->v, nc, d_mptr, d_mem,
                         d_dm, d_cc, d_M);
      hip_check(hipGetLastError(), "k_coarse_M");
    }
    if (ne > 0) {
      const int grid = int(std::min<int64_t>((ne + kCritBlock - 1) / kCritBlock, 16384));
      hipLaunchKernelGGL(k_coarse_E, dim3(grid), dim3(kCritBlock), 0, s_, dl->v, dl->e0, dl->e1,
                         d_agg, d_cc, ne, d_start, d_order, d_E);
      hip_check(hipGetLastError(), "k_coarse_E");
    }
    M.resize(size_t(nc) * kk);   // every entry is downloaded below
    E.resize(size_t(ne) * kk);
    hip_check(copy_d2h_sync(M.data(), d_M, M.size() * sizeof(double), s_), "download");
    hip_check(copy_d2h_sync(E.data(), d_E, E.size() * sizeof(double), s_), "download");
    note("coarse weights", int(ne), t0);
    return true;
  }
  void mu_b(const std::vector<int32_t> &pairs, double tau, std::vector<double> &out) override {
    const int np = int(pairs.size() / 2);
    out.assign(size_t(np), 0.0);
    if (np == 0) return;
    if (!work_) fail(EAMG_ERR_INVALID_ARG, "criteria: no working level");
    // every pair must be an edge of the working level (the kernel reads its edge matrix)
    const AuxLevel *hw = work_ == &lev_ ? lev_src_ : wrk_src_;
    for (int u = 0; u < np; ++u) {
      const int i = pairs[2 * size_t(u)], j = pairs[2 * size_t(u) + 1];
      if (i < 0 || i >= work_->v.n || j < 0 || j >= work_->v.n || !hw || hw->edge_id(i, j) < 0)
        fail(EAMG_ERR_INVALID_ARG, "criteria: pair is not an edge of the working level");
    }
    const auto t0 = std::chrono::steady_clock::now();
    const int *dp = idx_.put(pairs.data(), pairs.size(), s_);
    double *dout = static_cast<double *>(res_.reserve(size_t(np) * sizeof(double)));
    const int grid = std::min((np + kCritBlock - 1) / kCritBlock, 4096);
    hipLaunchKernelGGL(k_mu_b, dim3(grid), dim3(kCritBlock), 0, s_, work_->v, work_->d, np, dp,
                       tau, dout);
    hip_check(hipGetLastError(), "k_mu_b");
    hip_check(copy_d2h_sync(out.data(), dout, size_t(np) * sizeof(double), s_), "download");
    note("mu_b", np, t0);
  }
  void mu_g(const std::vector<int32_t> &unions, double tau, std::vector<double> &out) override {
    const int nu = int(unions.size() / crit::kMaxUnion);
    out.assign(size_t(nu), 0.0);
    if (nu == 0) return;
    if (!lev_src_) fail(EAMG_ERR_INVALID_ARG, "criteria: no level");
    if (lev_.v.k > 6) fail(EAMG_ERR_INVALID_ARG, "criteria: k > 6");
    for (int u = 0; u < nu; ++u) {
      // members ascending and distinct, at least one, padding only at the end
      const int32_t *m = &unions[size_t(u) * crit::kMaxUnion];
      if (m[0] < 0) fail(EAMG_ERR_INVALID_ARG, "criteria: empty union");
      for (int a = 0; a < crit::kMaxUnion; ++a) {
        if (m[a] >= lev_.v.n) fail(EAMG_ERR_INVALID_ARG, "criteria: union member out of range");
        if (a > 0 && m[a] >= 0 && !(m[a - 1] >= 0 && m[a - 1] < m[a]))
          fail(EAMG_ERR_INVALID_ARG, "criteria: union not ascending");
      }
    }
    const auto t0 = std::chrono::steady_clock::now();
    const int *du = idx_.put(unions.data(), unions.size(), s_);
    double *dout = static_cast<double *>(res_.reserve(size_t(nu) * sizeof(double)));
    const int grid = std::min(nu, kMaxGWaves);
    hipLaunchKernelGGL(k_mu_g_wave, dim3(grid), dim3(kCritBlock), 0, s_, lev_.v, lev_.d, nu, du,
                       tau, dout);
    hip_check(hipGetLastError(), "k_mu_g");
    hip_check(copy_d2h_sync(out.data(), dout, size_t(nu) * sizeof(double), s_), "download");
    if (verbose_) {
      int nan = 0;
      for (double v : out) nan += std::isnan(v) ? 1 : 0;
      if (nan) std::fprintf(stderr, "[eamg]     device mu_g: %d unions beyond the device capacity\n", nan);
    }
    note("mu_g", nu, t0);
  }

 private:
  void note(const char *what, int count, std::chrono::steady_clock::time_point t0) const {
    if (!verbose_) return;
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::fprintf(stderr, "[eamg]     device %s: %d in %.4f s\n", what, count, dt);
  }
  const bool verbose_ = std::getenv("EAMG_VERBOSE") != nullptr;
  hipStream_t s_;
  DevLevel lev_, wrk_;
  const AuxLevel *lev_src_ = nullptr, *wrk_src_ = nullptr;
  const DevLevel *work_ = nullptr;
  DBuf idx_, res_;
  DBuf cw_mptr_, cw_mem_, cw_dm_, cw_cc_, cw_agg_, cw_start_, cw_order_, cw_M_, cw_E_;
};

}  // namespace

std::unique_ptr<CritBatch> make_device_criteria(hipStream_t s) {
  return std::unique_ptr<CritBatch>(new DeviceCriteria(s));
}

}  // namespace eamg
