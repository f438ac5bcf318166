// Coarsening criteria mu_b (Lemma thm:mu2) and mu_g (Thm thm:mu1, unions of up to four vertices),
// written once for the host walk (coarsen.cpp) and the batched device evaluation (criteria.hip):
// the same operations in the same order on both, so both give the same values.
//
// Small square matrices are k x k with k <= 6 (Sq, row-major); the union matrices of mu_g are at
// most 24 x 24 (fixed capacity).  Symmetric eigenproblems use cyclic Jacobi (eigenvalues
// ascending).  Pseudo-inverses and the generalized largest eigenvalue drop eigenvalues
// <= tau * lambda_max.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#define EAMG_HD __host__ __device__

namespace eamg {

// Small square matrix, k <= 6, row-major.
struct Sq {
  int k = 0;
  double a[36];
  EAMG_HD Sq() {}
  EAMG_HD explicit Sq(int k_) : k(k_) {
    for (int i = 0; i < 36; ++i) a[i] = 0.0;
  }
  EAMG_HD double &operator()(int i, int j) { return a[i * k + j]; }
  EAMG_HD double operator()(int i, int j) const { return a[i * k + j]; }
};

// Raw view of one auxiliary level (AuxLevel's arrays, host or device memory): positions n x 3,
// edge matrices m x k x k, vertex matrices n x k x k, adjacency sorted by neighbour id.
struct LevelView {
  int n = 0, k = 6;
  const double *x = nullptr, *E = nullptr, *M = nullptr;
  const int64_t *nb_ptr = nullptr;
  const int *nb = nullptr, *nb_e = nullptr;

  EAMG_HD const double *xp(int i) const { return x + int64_t(3) * i; }
  EAMG_HD int edge_id(int i, int j) const {
    int64_t lo = nb_ptr[i], hi = nb_ptr[i + 1];
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (nb[mid] < j)
        lo = mid + 1;
      else
        hi = mid;
    }
    return (lo < nb_ptr[i + 1] && nb[lo] == j) ? nb_e[lo] : -1;
  }
  EAMG_HD Sq Emat(int64_t e) const {
    Sq S(k);
    const double *p = E + e * k * k;
    for (int i = 0; i < k * k; ++i) S.a[i] = p[i];
    return S;
  }
  EAMG_HD Sq Mmat(int i) const {
    Sq S(k);
    const double *p = M + int64_t(i) * k * k;
    for (int j = 0; j < k * k; ++j) S.a[j] = p[j];
    return S;
  }
};

namespace crit {

EAMG_HD inline double inf() { return __builtin_huge_val(); }

EAMG_HD inline Sq mul(const Sq &A, const Sq &B) {
  const int k = A.k;
  Sq C(k);
  for (int i = 0; i < k; ++i)
    for (int l = 0; l < k; ++l) {
      const double ail = A(i, l);
      if (ail == 0.0) continue;
      for (int j = 0; j < k; ++j) C(i, j) += ail * B(l, j);
    }
  return C;
}

EAMG_HD inline Sq tr(const Sq &A) {
  Sq T(A.k);
  for (int i = 0; i < A.k; ++i)
    for (int j = 0; j < A.k; ++j) T(j, i) = A(i, j);
  return T;
}

// A^T B C
EAMG_HD inline Sq t3(const Sq &A, const Sq &B, const Sq &C) { return mul(mul(tr(A), B), C); }

EAMG_HD inline void axpy(Sq &Y, double s, const Sq &X) {
  for (int i = 0; i < Y.k * Y.k; ++i) Y.a[i] += s * X.a[i];
}

EAMG_HD inline Sq sym(const Sq &X) {
  Sq S(X.k);
  for (int i = 0; i < X.k; ++i)
    for (int j = 0; j < X.k; ++j) S(i, j) = 0.5 * (X(i, j) + X(j, i));
  return S;
}

EAMG_HD inline double frob(const Sq &X) {
  double s = 0.0;
  for (int i = 0; i < X.k * X.k; ++i) s += X.a[i] * X.a[i];
  return sqrt(s);
}

EAMG_HD inline double trace(const Sq &X) {
  double s = 0.0;
  for (int i = 0; i < X.k; ++i) s += X(i, i);
  return s;
}

// Cyclic Jacobi on the n x n row-major matrix A (overwritten), leading dimension ld; eigenvalues
// ascending into w and, when V is not null, the eigenvectors as columns of V (ld x ld).  Ties keep
// their index order.
EAMG_HD inline void jacobi(double *A, int n, int ld, double *w, double *V) {
  if (V)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) V[i * ld + j] = i == j ? 1.0 : 0.0;
  double fro2 = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) fro2 += A[i * ld + j] * A[i * ld + j];
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * ld + q] * A[p * ld + q];
    if (off <= 1e-40 * fro2 || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * ld + q];
        if (apq == 0.0) continue;
        const double theta = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * ld + p], akq = A[k * ld + q];
          A[k * ld + p] = cs * akp - sn * akq;
          A[k * ld + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * ld + k], aqk = A[q * ld + k];
          A[p * ld + k] = cs * apk - sn * aqk;
          A[q * ld + k] = sn * apk + cs * aqk;
        }
        A[p * ld + q] = 0.0;
        A[q * ld + p] = 0.0;
        if (V)
          for (int k = 0; k < n; ++k) {
            const double vkp = V[k * ld + p], vkq = V[k * ld + q];
            V[k * ld + p] = cs * vkp - sn * vkq;
            V[k * ld + q] = sn * vkp + cs * vkq;
          }
      }
  }
  // stable insertion sort of the eigenvalues (and their vectors) ascending
  for (int i = 0; i < n; ++i) w[i] = A[i * ld + i];
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && w[j] < w[j - 1]; --j) {
      const double t = w[j];
      w[j] = w[j - 1];
      w[j - 1] = t;
      if (V)
        for (int r = 0; r < n; ++r) {
          const double v = V[r * ld + j];
          V[r * ld + j] = V[r * ld + j - 1];
          V[r * ld + j - 1] = v;
        }
    }
}

EAMG_HD inline void eigh(const Sq &Ain, double *w, Sq &V) {
  Sq A = Ain;
  V = Sq(Ain.k);
  jacobi(A.a, Ain.k, Ain.k, w, V.a);
}

EAMG_HD inline Sq pinv(const Sq &X, double tau) {
  const int n = X.k;
  double w[6];
  Sq V;
  eigh(sym(X), w, V);
  Sq P(n);
  const double lmax = w[n - 1];
  if (lmax <= 0.0) return P;
  for (int k = 0; k < n; ++k) {
    if (!(w[k] > tau * lmax)) continue;
    const double inv = 1.0 / w[k];
    for (int i = 0; i < n; ++i) {
      const double vi = V(i, k) * inv;
      for (int j = 0; j < n; ++j) P(i, j) += vi * V(j, k);
    }
  }
  return P;
}

// Harmonic mean H(A, B) = A (A + B)^+ B, symmetrized.
EAMG_HD inline Sq harmonic(const Sq &A, const Sq &B, double tau) {
  Sq S = A;
  axpy(S, 1.0, B);
  return sym(mul(mul(A, pinv(S, tau)), B));
}

// Smallest mu with L <= mu R on PSD pencils of order n (row-major, leading dimension ld, both
// overwritten): +inf when L is positive on a tau-null direction of R, 0 when L = 0.  U and G are
// scratch of ld x ld, w of ld.
EAMG_HD inline double genmax_n(double *L, double *R, int n, int ld, double tau, double *U, double *G,
                               double *w) {
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double l = 0.5 * (L[i * ld + j] + L[j * ld + i]);
      L[i * ld + j] = L[j * ld + i] = l;
      const double r = 0.5 * (R[i * ld + j] + R[j * ld + i]);
      R[i * ld + j] = R[j * ld + i] = r;
    }
  double nL = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) nL += L[i * ld + j] * L[i * ld + j];
  nL = sqrt(nL);
  if (nL == 0.0) return 0.0;
  jacobi(R, n, ld, w, U);
  const double lmax = w[n - 1];
  int nk = 0, nd = 0;
  for (int k = 0; k < n; ++k) {
    if (lmax > 0.0 && w[k] > tau * lmax)
      ++nk;
    else
      ++nd;
  }
  // eigenvalues are ascending: the dropped ones come first
  if (nd) {
    double s = 0.0;
    for (int a = 0; a < nd; ++a)
      for (int b = 0; b < nd; ++b) {
        double v = 0.0;
        for (int i = 0; i < n; ++i) {
          double li = 0.0;
          for (int j = 0; j < n; ++j) li += L[i * ld + j] * U[j * ld + b];
          v += U[i * ld + a] * li;
        }
        s += v * v;
      }
    if (sqrt(s) > tau * nL) return inf();
  }
  if (!nk) return 0.0;
  for (int a = 0; a < nk; ++a)
    for (int b = 0; b < nk; ++b) {
      double v = 0.0;
      for (int i = 0; i < n; ++i) {
        double li = 0.0;
        for (int j = 0; j < n; ++j) li += L[i * ld + j] * U[j * ld + nd + b];
        v += U[i * ld + nd + a] * li;
      }
      G[a * ld + b] = v / (sqrt(w[nd + a]) * sqrt(w[nd + b]));
    }
  for (int a = 0; a < nk; ++a)
    for (int b = a + 1; b < nk; ++b) {
      const double g = 0.5 * (G[a * ld + b] + G[b * ld + a]);
      G[a * ld + b] = G[b * ld + a] = g;
    }
  jacobi(G, nk, ld, w, nullptr);
  return w[nk - 1];
}

EAMG_HD inline double genmax(const Sq &Lin, const Sq &Rin, double tau) {
  Sq L = Lin, R = Rin, U, G;
  double w[6];
  return genmax_n(L.a, R.a, Lin.k, Lin.k, tau, U.a, G.a, w);
}

// Q(t) = [[I, Skew(t)], [0, I]] (k = 6; Skew(t) r = t x r) or [[1]] (k = 1).
EAMG_HD inline Sq q(const double *t, int k) {
  Sq Q(k);
  for (int i = 0; i < k; ++i) Q(i, i) = 1.0;
  if (k == 6) {
    Q(0, 4) = -t[2];
    Q(0, 5) = t[1];
    Q(1, 3) = t[2];
    Q(1, 5) = -t[0];
    Q(2, 3) = -t[1];
    Q(2, 4) = t[0];
  }
  return Q;
}

// Q^{a->b} = Q(x_b - x_a)
EAMG_HD inline Sq qtrans(const double *xa, const double *xb, int k) {
  const double t[3] = {xb[0] - xa[0], xb[1] - xa[1], xb[2] - xa[2]};
  return q(t, k);
}

// Q^{ab} = Q((x_b - x_a) / 2)
EAMG_HD inline Sq qhalf(const double *xa, const double *xb, int k) {
  const double t[3] = {0.5 * (xb[0] - xa[0]), 0.5 * (xb[1] - xa[1]), 0.5 * (xb[2] - xa[2])};
  return q(t, k);
}

// mu_b of pair (i, j) of level w with D-hat blocks D (Lemma thm:mu2, delta = 1).
EAMG_HD inline double mu_b(const LevelView &w, const Sq *D, int i, int j, double tau) {
  const int k = w.k;
  const double *xi = w.xp(i), *xj = w.xp(j);
  const Sq Qij = qhalf(xi, xj, k), Qji = qhalf(xj, xi, k);
  const Sq L = harmonic(t3(Qji, D[i], Qji), t3(Qij, D[j], Qij), tau);
  Sq R = w.Emat(w.edge_id(i, j));
  for (int64_t p = w.nb_ptr[i]; p < w.nb_ptr[i + 1]; ++p) {
    const int l = w.nb[p];
    if (l == j) continue;
    const int ejl = w.edge_id(j, l);
    if (ejl < 0) continue;
    const int eil = w.nb_e[p];
    const double *xl = w.xp(l);
    const Sq Qli = qhalf(xl, xi, k), Qlj = qhalf(xl, xj, k);
    const Sq Hl = harmonic(t3(Qli, w.Emat(eil), Qli), t3(Qlj, w.Emat(ejl), Qlj), tau);
    const Sq T = mul(qtrans(xi, xl, k), Qji);
    axpy(R, 0.5, t3(T, Hl, T));
  }
  return genmax(L, R, tau);
}

// mu_g of a union C of up to kMaxUnion vertices (Thm thm:mu1, delta = 1), members sorted
// ascending.  Scratch: GScratch.  Returns NaN when the union's outside neighbours exceed the
// scratch capacity (the caller then evaluates it elsewhere).
constexpr int kMaxUnion = 4;
constexpr int kMaxUnionDim = kMaxUnion * 6;
constexpr int kMaxOutside = 384;

struct GScratch {
  double L[kMaxUnionDim * kMaxUnionDim], R[kMaxUnionDim * kMaxUnionDim];
  double U[kMaxUnionDim * kMaxUnionDim], G[kMaxUnionDim * kMaxUnionDim];
  double w[kMaxUnionDim];
  int ol[kMaxOutside], oa[kMaxOutside], oe[kMaxOutside];   // outside neighbour, member, edge
};

EAMG_HD inline void put(double *X, int ld, int k, int a, int b, const Sq &S, double s) {
  for (int u = 0; u < k; ++u)
    for (int v = 0; v < k; ++v) X[(a * k + u) * ld + b * k + v] += s * S(u, v);
}

EAMG_HD inline double mu_g(const LevelView &lev, const Sq *D, const int *mem, int nC, double tau,
                           GScratch &g) {
  const int k = lev.k, n = nC * k, ld = kMaxUnionDim;
  double xH[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < nC; ++a)
    for (int d = 0; d < 3; ++d) xH[d] = xH[d] + lev.x[int64_t(3) * mem[a] + d];
  for (int d = 0; d < 3; ++d) xH[d] = xH[d] / double(nC);
  // L = D_C - D_C P_C pinv(P_C^T D_C P_C) P_C^T D_C with P_C = [Q^{H->i}]
  Sq Y[kMaxUnion];
  Sq Z(k);
  for (int a = 0; a < nC; ++a) {
    const Sq Q = qtrans(xH, lev.xp(mem[a]), k);
    Y[a] = mul(D[mem[a]], Q);
    axpy(Z, 1.0, mul(tr(Q), Y[a]));
  }
  const Sq Zp = pinv(Z, tau);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) g.L[i * ld + j] = g.R[i * ld + j] = 0.0;
  for (int a = 0; a < nC; ++a) {
    const Sq YZ = mul(Y[a], Zp);
    for (int b = 0; b < nC; ++b) put(g.L, ld, k, a, b, mul(YZ, tr(Y[b])), -1.0);
    put(g.L, ld, k, a, a, D[mem[a]], 1.0);
    put(g.R, ld, k, a, a, lev.Mmat(mem[a]), 1.0);
  }
  // edges inside C (eq. auxa) and, in encounter order, the edges to outside neighbours
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
          const Sq Qil = qhalf(lev.xp(i), lev.xp(l), k), Qli = qhalf(lev.xp(l), lev.xp(i), k);
          const Sq Ee = lev.Emat(e);
          put(g.R, ld, k, a, a, t3(Qil, Ee, Qil), 1.0);
          put(g.R, ld, k, b, b, t3(Qli, Ee, Qli), 1.0);
          put(g.R, ld, k, a, b, t3(Qil, Ee, Qli), -1.0);
          put(g.R, ld, k, b, a, t3(Qli, Ee, Qil), -1.0);
        }
      } else {
        if (no == kMaxOutside) return __builtin_nan("");
        g.ol[no] = l;
        g.oa[no] = a;
        g.oe[no] = e;
        ++no;
      }
    }
  }
  // group by outside neighbour, ascending, keeping encounter order within a neighbour
  for (int s = 1; s < no; ++s)
    for (int t = s; t > 0 && g.ol[t] < g.ol[t - 1]; --t) {
      const int l = g.ol[t], a = g.oa[t], e = g.oe[t];
      g.ol[t] = g.ol[t - 1];
      g.oa[t] = g.oa[t - 1];
      g.oe[t] = g.oe[t - 1];
      g.ol[t - 1] = l;
      g.oa[t - 1] = a;
      g.oe[t - 1] = e;
    }
  for (int s0 = 0; s0 < no;) {
    int s1 = s0 + 1;
    while (s1 < no && g.ol[s1] == g.ol[s0]) ++s1;
    const int cnt = s1 - s0;
    if (cnt > kMaxUnion) return __builtin_nan("");   // repeated adjacency entries
    if (cnt >= 2) {
      // local assembly of the edges (i, l), i in C, with unknowns (v_C, w); Schur complement on
      // v_C.  An outside neighbour meets at most kMaxUnion members (one edge each).
      const int l = g.ol[s0];
      Sq Kcw[kMaxUnion], Kcc[kMaxUnion];
      int am[kMaxUnion];
      Sq Kww(k);
      for (int x = 0; x < cnt; ++x) {
        const int a = g.oa[s0 + x], e = g.oe[s0 + x], i = mem[a];
        const Sq Qil = qhalf(lev.xp(i), lev.xp(l), k), Qli = qhalf(lev.xp(l), lev.xp(i), k);
        const Sq Ee = lev.Emat(e);
        am[x] = a;
        Kcc[x] = t3(Qil, Ee, Qil);
        Sq X = t3(Qil, Ee, Qli);
        for (int q2 = 0; q2 < k * k; ++q2) X.a[q2] = -X.a[q2];
        Kcw[x] = X;
        axpy(Kww, 1.0, t3(Qli, Ee, Qli));
      }
      const Sq Wp = pinv(Kww, tau);
      for (int x = 0; x < cnt; ++x) {
        const Sq KW = mul(Kcw[x], Wp);
        for (int y = 0; y < cnt; ++y) {
          Sq S = mul(KW, tr(Kcw[y]));
          for (int q2 = 0; q2 < k * k; ++q2) S.a[q2] = -S.a[q2];
          if (x == y) axpy(S, 1.0, Kcc[x]);
          // 1/2 sym(S_l): add half of the block and half of its mirror
          put(g.R, ld, k, am[x], am[y], S, 0.25);
          put(g.R, ld, k, am[y], am[x], tr(S), 0.25);
        }
      }
    }
    s0 = s1;
  }
  return genmax_n(g.L, g.R, n, ld, tau, g.U, g.G, g.w);
}

}  // namespace crit

}  // namespace eamg
