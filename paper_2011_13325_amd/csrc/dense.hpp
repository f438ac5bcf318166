// Small dense linear algebra for the host-side setup (coarsening criteria, pseudo-inverses,
// coarsest level factorization).  All FP64.  Matrices are row-major std::vector backed.
//
// Symmetric eigenproblems use the cyclic Jacobi method (rotations chosen to annihilate one
// off-diagonal pair at a time, Golub & Van Loan section 8.5) up to 8 x 8 and Householder
// tridiagonalization + implicit QL above; both are accurate to a few ulps of the matrix norm.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <vector>

namespace eamg {

struct Mat {
  int r = 0, c = 0;
  std::vector<double> a;
  Mat() = default;
  Mat(int r_, int c_) : r(r_), c(c_), a(size_t(r_) * c_, 0.0) {}
  double &operator()(int i, int j) { return a[size_t(i) * c + j]; }
  double operator()(int i, int j) const { return a[size_t(i) * c + j]; }
  static Mat eye(int n) {
    Mat m(n, n);
    for (int i = 0; i < n; ++i) m(i, i) = 1.0;
    return m;
  }
  static Mat from(int r_, int c_, const double *p) {
    Mat m(r_, c_);
    std::copy(p, p + size_t(r_) * c_, m.a.begin());
    return m;
  }
};

inline Mat matmul(const Mat &A, const Mat &B) {
  Mat C(A.r, B.c);
  for (int i = 0; i < A.r; ++i)
    for (int k = 0; k < A.c; ++k) {
      const double aik = A(i, k);
      if (aik == 0.0) continue;
      for (int j = 0; j < B.c; ++j) C(i, j) += aik * B(k, j);
    }
  return C;
}

inline Mat transpose(const Mat &A) {
  Mat T(A.c, A.r);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < A.c; ++j) T(j, i) = A(i, j);
  return T;
}

// A^T B C
inline Mat tmul3(const Mat &A, const Mat &B, const Mat &C) { return matmul(matmul(transpose(A), B), C); }

inline void axpy_mat(Mat &Y, double s, const Mat &X) {
  for (size_t i = 0; i < Y.a.size(); ++i) Y.a[i] += s * X.a[i];
}

inline Mat sym(const Mat &X) {
  Mat S(X.r, X.c);
  for (int i = 0; i < X.r; ++i)
    for (int j = 0; j < X.c; ++j) S(i, j) = 0.5 * (X(i, j) + X(j, i));
  return S;
}

inline double frob(const Mat &X) {
  double s = 0.0;
  for (double v : X.a) s += v * v;
  return std::sqrt(s);
}

inline double trace(const Mat &X) {
  double s = 0.0;
  for (int i = 0; i < X.r; ++i) s += X(i, i);
  return s;
}

// Symmetric eigen-decomposition for larger matrices: Householder reduction to tridiagonal form
// (accumulating the reflections; Golub & Van Loan section 8.3.1), then the implicit QL
// iteration with shifts from the leading 2 x 2 block on the tridiagonal matrix, in the form of
// procedure tql2 of Bowdler, Martin, Reinsch and Wilkinson, "The QR and QL algorithms for
// symmetric matrices", Numer. Math. 11 (1968) 293-306 (Handbook for Automatic Computation
// vol. II, contribution II/3; the EISPACK routine TQL2): the sweep over the rotations, its
// variables and the premature-deflation exit follow that procedure.  w ascending, V columns
// are the eigenvectors.
inline void eigh_tridiag_ql(const Mat &Ain, std::vector<double> &w, Mat &V, bool vectors = true) {
  const int n = Ain.r;
  Mat A = Ain;
  V = vectors ? Mat::eye(n) : Mat();
  w.assign(n, 0.0);
  if (n == 0) return;
  std::vector<double> v(n), p(n), q(n), e(n, 0.0);
  for (int k = 0; k + 2 < n; ++k) {
    double alpha2 = 0.0;
    for (int i = k + 1; i < n; ++i) alpha2 += A(i, k) * A(i, k);
    const double x0 = A(k + 1, k);
    double tail2 = alpha2 - x0 * x0;
    if (tail2 <= 0.0) continue;  // column already tridiagonal
    const double alpha = std::sqrt(alpha2);
    const double sub = x0 >= 0.0 ? -alpha : alpha;  // new subdiagonal entry
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    v[k + 1] = x0 - sub;
    for (int i = k + 2; i < n; ++i) v[i] = A(i, k);
    double vn2 = 0.0;
    for (int i = k + 1; i < n; ++i) vn2 += v[i] * v[i];
    if (vn2 == 0.0) continue;
    const double beta = 2.0 / vn2;
    // A <- H A H on the trailing block, H = I - beta v v^T
    double K = 0.0;
    for (int i = k + 1; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += A(i, j) * v[j];
      p[i] = beta * s;
      K += p[i] * v[i];
    }
    K *= 0.5 * beta;
    for (int i = k + 1; i < n; ++i) q[i] = p[i] - K * v[i];
    for (int i = k + 1; i < n; ++i)
      for (int j = k + 1; j < n; ++j) A(i, j) -= v[i] * q[j] + q[i] * v[j];
    A(k + 1, k) = A(k, k + 1) = sub;
    for (int i = k + 2; i < n; ++i) A(i, k) = A(k, i) = 0.0;
    // V <- V H
    for (int r = 0; vectors && r < n; ++r) {
      double t = 0.0;
      for (int j = k + 1; j < n; ++j) t += V(r, j) * v[j];
      t *= beta;
      for (int j = k + 1; j < n; ++j) V(r, j) -= t * v[j];
    }
  }
  std::vector<double> d(n);
  for (int i = 0; i < n; ++i) d[i] = A(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = A(i + 1, i);
  e[n - 1] = 0.0;
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < n; ++l) {
    for (int iter = 0; iter < 100; ++iter) {
      int m = l;
      for (; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      // Wilkinson-type shift from the leading 2x2 block
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, pp = 0.0;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        double f = s * e[i];
        const double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {  // premature deflation
          d[i + 1] -= pp;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pp;
        r = (d[i] - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - b;
        for (int k = 0; vectors && k < n; ++k) {
          f = V(k, i + 1);
          V(k, i + 1) = s * V(k, i) + c * f;
          V(k, i) = c * V(k, i) - s * f;
        }
      }
      if (deflated) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int j = 0; j < n; ++j) w[j] = d[idx[j]];
  if (!vectors) return;
  Mat Vs(n, n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) Vs(i, j) = V(i, idx[j]);
  V = Vs;
}

// Symmetric eigen-decomposition: w ascending, V columns are the eigenvectors.  Cyclic Jacobi for
// small matrices, tridiagonal QL above 8 x 8.
inline void eigh_jacobi(const Mat &Ain, std::vector<double> &w, Mat &V);
inline void eigh(const Mat &Ain, std::vector<double> &w, Mat &V) {
  if (Ain.r > 8)
    eigh_tridiag_ql(Ain, w, V);
  else
    eigh_jacobi(Ain, w, V);
}

inline void eigh_jacobi(const Mat &Ain, std::vector<double> &w, Mat &V) {
  const int n = Ain.r;
  Mat A = Ain;
  V = Mat::eye(n);
  w.assign(n, 0.0);
  if (n == 0) return;
  double fro2 = 0.0;
  for (double v : A.a) fro2 += v * v;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A(p, q) * A(p, q);
    if (off <= 1e-40 * fro2 || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A(p, q);
        if (apq == 0.0) continue;
        const double app = A(p, p), aqq = A(q, q);
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {
          const double akp = A(k, p), akq = A(k, q);
          A(k, p) = cs * akp - sn * akq;
          A(k, q) = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A(p, k), aqk = A(q, k);
          A(p, k) = cs * apk - sn * aqk;
          A(q, k) = sn * apk + cs * aqk;
        }
        A(p, q) = 0.0;
        A(q, p) = 0.0;
        for (int k = 0; k < n; ++k) {
          const double vkp = V(k, p), vkq = V(k, q);
          V(k, p) = cs * vkp - sn * vkq;
          V(k, q) = sn * vkp + cs * vkq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return A(x, x) < A(y, y); });
  Mat Vs(n, n);
  for (int j = 0; j < n; ++j) {
    w[j] = A(idx[j], idx[j]);
    for (int i = 0; i < n; ++i) Vs(i, j) = V(i, idx[j]);
  }
  V = Vs;
}

// Symmetric pseudo-inverse: eigenvalues <= tau * max(lambda_max, 0) are treated as zero.
inline Mat pinv_tau(const Mat &X, double tau) {
  const int n = X.r;
  std::vector<double> w;
  Mat V;
  eigh(sym(X), w, V);
  Mat P(n, n);
  const double lmax = n ? w[n - 1] : 0.0;
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

// Orthonormal basis (columns) of the tau-kernel of symmetric X.
inline Mat kernel_basis(const Mat &X, double tau) {
  const int n = X.r;
  std::vector<double> w;
  Mat V;
  eigh(sym(X), w, V);
  const double lmax = n ? w[n - 1] : 0.0;
  std::vector<int> ks;
  for (int k = 0; k < n; ++k)
    if (lmax <= 0.0 || !(w[k] > tau * lmax)) ks.push_back(k);
  Mat U(n, int(ks.size()));
  for (int j = 0; j < int(ks.size()); ++j)
    for (int i = 0; i < n; ++i) U(i, j) = V(i, ks[j]);
  return U;
}

// Harmonic mean H(A, B) = A (A + B)^+ B, symmetrized.
inline Mat harmonic(const Mat &A, const Mat &B, double tau) {
  Mat S = A;
  axpy_mat(S, 1.0, B);
  return sym(matmul(matmul(A, pinv_tau(S, tau)), B));
}

// Smallest mu with L <= mu R on PSD pencils (largest generalized eigenvalue); +inf when L is
// positive on a null direction of R; 0 when L = 0.
inline double genmax(const Mat &Lin, const Mat &Rin, double tau) {
  const Mat L = sym(Lin), R = sym(Rin);
  const int n = L.r;
  const double nL = frob(L);
  if (nL == 0.0) return 0.0;
  std::vector<double> w;
  Mat U;
  eigh(R, w, U);
  const double lmax = w[n - 1];
  std::vector<int> keep, drop;
  for (int k = 0; k < n; ++k) {
    if (lmax > 0.0 && w[k] > tau * lmax)
      keep.push_back(k);
    else
      drop.push_back(k);
  }
  if (!drop.empty()) {
    Mat U0(n, int(drop.size()));
    for (int j = 0; j < int(drop.size()); ++j)
      for (int i = 0; i < n; ++i) U0(i, j) = U(i, drop[j]);
    if (frob(tmul3(U0, L, U0)) > tau * nL) return std::numeric_limits<double>::infinity();
  }
  if (keep.empty()) return 0.0;
  Mat W(n, int(keep.size()));
  for (int j = 0; j < int(keep.size()); ++j) {
    const double s = 1.0 / std::sqrt(w[keep[j]]);
    for (int i = 0; i < n; ++i) W(i, j) = U(i, keep[j]) * s;
  }
  std::vector<double> g;
  Mat G;
  const Mat S = sym(tmul3(W, L, W));
  if (S.r > 8)
    eigh_tridiag_ql(S, g, G, false);
  else
    eigh(S, g, G);
  return g.back();
}

// In-place lower Cholesky of an SPD matrix; returns false on a non-positive pivot.
inline bool cholesky(Mat &A) {
  const int n = A.r;
  for (int j = 0; j < n; ++j) {
    double d = A(j, j);
    for (int k = 0; k < j; ++k) d -= A(j, k) * A(j, k);
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    A(j, j) = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A(i, j);
      for (int k = 0; k < j; ++k) s -= A(i, k) * A(j, k);
      A(i, j) = s / d;
    }
    for (int k = j + 1; k < n; ++k) A(j, k) = 0.0;
  }
  return true;
}

// Skew(t): Skew(t) r = t x r.
inline void skew3(const double *t, double S[9]) {
  S[0] = 0.0;   S[1] = -t[2]; S[2] = t[1];
  S[3] = t[2];  S[4] = 0.0;   S[5] = -t[0];
  S[6] = -t[1]; S[7] = t[0];  S[8] = 0.0;
}

// Q(t) = [[I, Skew(t)], [0, I]] (k = 6) or [[1]] (k = 1).
inline Mat qmat(const double *t, int k) {
  Mat Q = Mat::eye(k);
  if (k == 6) {
    double S[9];
    skew3(t, S);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Q(i, 3 + j) = S[3 * i + j];
  }
  return Q;
}

// Q^{a->b} = Q(x_b - x_a)
inline Mat q_transport(const double *xa, const double *xb, int k) {
  const double t[3] = {xb[0] - xa[0], xb[1] - xa[1], xb[2] - xa[2]};
  return qmat(t, k);
}

// Q^{ab} = Q((x_b - x_a) / 2)
inline Mat q_half(const double *xa, const double *xb, int k) {
  const double t[3] = {0.5 * (xb[0] - xa[0]), 0.5 * (xb[1] - xa[1]), 0.5 * (xb[2] - xa[2])};
  return qmat(t, k);
}

}  // namespace eamg
