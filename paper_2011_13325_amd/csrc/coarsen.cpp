// Host-side auxiliary topology, coarsening criteria and successive matching.
// See coarsen.hpp for the passages each part follows.
#include "coarsen.hpp"

#include <algorithm>
#include <atomic>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <future>
#include <limits>
#include <memory>
#include <unordered_map>

namespace eamg {

namespace {

const double kInf = std::numeric_limits<double>::infinity();


// ---- small square matrices (crit_core.hpp, shared with the device criteria) ---------------

Sq sq_mul(const Sq &A, const Sq &B) { return crit::mul(A, B); }
Sq sq_t(const Sq &A) { return crit::tr(A); }
Sq sq_t3(const Sq &A, const Sq &B, const Sq &C) { return crit::t3(A, B, C); }
void sq_axpy(Sq &Y, double s, const Sq &X) { crit::axpy(Y, s, X); }
Sq sq_sym(const Sq &X) { return crit::sym(X); }
double sq_frob(const Sq &X) { return crit::frob(X); }
double sq_trace(const Sq &X) { return crit::trace(X); }
void sq_eigh(const Sq &A, double *w, Sq &V) { crit::eigh(A, w, V); }
Sq sq_pinv(const Sq &X, double tau) { return crit::pinv(X, tau); }
Sq sq_harmonic(const Sq &A, const Sq &B, double tau) { return crit::harmonic(A, B, tau); }
double sq_genmax(const Sq &L, const Sq &R, double tau) { return crit::genmax(L, R, tau); }
Sq sq_qtrans(const double *xa, const double *xb, int k) { return crit::qtrans(xa, xb, k); }
Sq sq_qhalf(const double *xa, const double *xb, int k) { return crit::qhalf(xa, xb, k); }

void mean_pos(const AuxLevel &lev, const std::vector<int> &members, double *out) {
  std::vector<int> s = members;
  std::sort(s.begin(), s.end());
  double acc[3] = {0.0, 0.0, 0.0};
  for (int i : s)
    for (int d = 0; d < 3; ++d) acc[d] = acc[d] + lev.x[size_t(3) * i + d];
  for (int d = 0; d < 3; ++d) out[d] = acc[d] / double(s.size());
}

// Q^{ab,T} E Q^{ab} of edge e seen from endpoint `at`.
Sq pulled(const AuxLevel &lev, int64_t e, int at) {
  const int other = lev.e0[e] == at ? lev.e1[e] : lev.e0[e];
  const Sq Q = sq_qhalf(lev.xp(at), lev.xp(other), lev.k);
  return sq_t3(Q, lev.Emat(e), Q);
}

}  // namespace

// ---- AuxLevel -----------------------------------------------------------------------------

void AuxLevel::build_adjacency() {
  const int64_t mm = m();
  nb_ptr.assign(size_t(n) + 1, 0);
  for (int64_t e = 0; e < mm; ++e) {
    nb_ptr[e0[e] + 1]++;
    nb_ptr[e1[e] + 1]++;
  }
  for (int i = 0; i < n; ++i) nb_ptr[i + 1] += nb_ptr[i];
  nb.assign(size_t(2 * mm), 0);
  nb_e.assign(size_t(2 * mm), 0);
  std::vector<int64_t> fill(nb_ptr.begin(), nb_ptr.end() - 1);
  for (int64_t e = 0; e < mm; ++e) {
    nb[fill[e0[e]]] = e1[e];
    nb_e[fill[e0[e]]++] = int(e);
    nb[fill[e1[e]]] = e0[e];
    nb_e[fill[e1[e]]++] = int(e);
  }
  parallel_for(n, [&](int64_t i) {
    const int64_t s = nb_ptr[i], t = nb_ptr[i + 1];
    std::vector<std::pair<int, int>> tmp;
    tmp.reserve(size_t(t - s));
    for (int64_t p = s; p < t; ++p) tmp.emplace_back(nb[p], nb_e[p]);
    std::sort(tmp.begin(), tmp.end());
    for (int64_t p = s; p < t; ++p) {
      nb[p] = tmp[p - s].first;
      nb_e[p] = tmp[p - s].second;
    }
  });
}

int AuxLevel::edge_id(int i, int j) const {
  const int *b = nb.data() + nb_ptr[i], *e = nb.data() + nb_ptr[i + 1];
  const int *p = std::lower_bound(b, e, j);
  if (p == e || *p != j) return -1;
  return nb_e[size_t(p - nb.data())];
}

Sq AuxLevel::Emat(int64_t e) const {
  Sq S(k);
  const double *p = &E[size_t(e) * k * k];
  for (int i = 0; i < k * k; ++i) S.a[i] = p[i];
  return S;
}

Sq AuxLevel::Mmat(int i) const {
  Sq S(k);
  const double *p = &M[size_t(i) * k * k];
  for (int j = 0; j < k * k; ++j) S.a[j] = p[j];
  return S;
}

// ---- finest level ---------------------------------------------------------------------------

bool finest_aux(int dim, int n, const double *coords, const int32_t *row_ptr, const int32_t *col,
                const double *vals, const int32_t *edges, int64_t n_edges, AuxLevel &out,
                std::string &err) {
  const int k = dim == 3 ? 6 : 1;
  const int bs2 = dim * dim;
  out = AuxLevel();
  out.n = n;
  out.k = k;
  out.x.assign(coords, coords + size_t(3) * n);
  auto find_block = [&](int i, int j) -> int64_t {
    const int32_t *b = col + row_ptr[i], *e = col + row_ptr[i + 1];
    const int32_t *p = std::lower_bound(b, e, j);
    if (p == e || *p != j) return -1;
    return int64_t(p - col);
  };
  std::vector<std::pair<int, int>> el;
  if (edges) {
    el.reserve(size_t(n_edges));
    for (int64_t e = 0; e < n_edges; ++e) {
      const int i = edges[2 * e], j = edges[2 * e + 1];
      if (i < 0 || j < 0 || i >= n || j >= n || i >= j) {
        err = "edges must satisfy 0 <= i < j < n_vertices";
        return false;
      }
      if (find_block(i, j) < 0) {
        err = "every edge must be an off-diagonal block position of A_N";
        return false;
      }
      el.emplace_back(i, j);
    }
    std::sort(el.begin(), el.end());
    if (std::adjacent_find(el.begin(), el.end()) != el.end()) {
      err = "duplicate edge";
      return false;
    }
  } else {
    for (int i = 0; i < n; ++i)
      for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
        if (col[p] > i) el.emplace_back(i, col[p]);
  }
  const int64_t m = int64_t(el.size());
  out.e0.resize(size_t(m));
  out.e1.resize(size_t(m));
  out.E.resize(size_t(m) * k * k);   // every entry written below
  out.M.resize(size_t(n) * k * k);
  parallel_for(int64_t(out.M.size()), [&](int64_t q) { out.M[q] = 0.0; });
  std::atomic<bool> same_pos{false};
  parallel_for(m, [&](int64_t e) {
    const int i = el[e].first, j = el[e].second;
    out.e0[e] = i;
    out.e1[e] = j;
    const double *blk = vals + size_t(find_block(i, j)) * bs2;
    double *Ee = &out.E[size_t(e) * k * k];
    for (int q = 0; q < k * k; ++q) Ee[q] = 0.0;
    if (dim == 3) {
      double c = 0.0;
      for (int q = 0; q < 9; ++q) c += std::fabs(blk[q]);
      c /= 9.0;
      double t[3] = {coords[3 * j] - coords[3 * i], coords[3 * j + 1] - coords[3 * i + 1],
                     coords[3 * j + 2] - coords[3 * i + 2]};
      const double nt = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
      if (!(nt > 0.0)) {
        same_pos = true;
        return;
      }
      for (double &v : t) v /= nt;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Ee[6 * a + b] = c * t[a] * t[b];
    } else {
      Ee[0] = std::fabs(blk[0]);
    }
  });
  if (same_pos) {
    err = "two vertices joined by an edge have the same position";
    return false;
  }
  if (dim == 1) {
    for (int i = 0; i < n; ++i) {
      double d = 0.0, off = 0.0;
      for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        if (col[p] == i)
          d = vals[p];
        else
          off += std::fabs(vals[p]);
      }
      out.M[i] = std::max(0.0, d - off);
    }
  }
  out.build_adjacency();
  return true;
}

// ---- coarse level (Thm thm:cemats) -------------------------------------------------------------

AuxLevel coarse_aux(const AuxLevel &lev, const std::vector<std::vector<int>> &aggs,
                    const std::vector<char> &dmask, const std::vector<double> &cc, CritBatch *dev) {
  const int k = lev.k, kk = k * k;
  const int nc = int(aggs.size());
  std::vector<int> agg_of(static_cast<size_t>(lev.n), -1);
  for (int I = 0; I < nc; ++I)
    for (int i : aggs[I]) agg_of[i] = I;
  AuxLevel out;
  out.n = nc;
  out.k = k;
  out.x = cc;
  // coarse edge key of every fine edge (-1: dropped); the fine edges of one key are summed in
  // ascending fine-edge order (stable sort), so the result does not depend on the threads
  const int64_t m = lev.m();
  std::vector<int64_t> key(static_cast<size_t>(m), -1);
  parallel_for(m, [&](int64_t e) {
    const int I = agg_of[lev.e0[e]], J = agg_of[lev.e1[e]];
    if (I < 0 || J < 0 || I == J) return;
    key[e] = int64_t(std::min(I, J)) * nc + std::max(I, J);
  });
  // stable sort by key = (I, J): counting sort by I keeps ascending e within an I bucket, then a
  // stable insertion sort by J inside each (small) bucket
  std::vector<int64_t> bucket(static_cast<size_t>(nc) + 1, 0);
  for (int64_t e = 0; e < m; ++e)
    if (key[e] >= 0) ++bucket[size_t(key[e] / nc) + 1];
  for (int I = 0; I < nc; ++I) bucket[I + 1] += bucket[I];
  std::vector<int64_t> order(static_cast<size_t>(bucket[nc]));
  {
    std::vector<int64_t> fill(bucket.begin(), bucket.end() - 1);
    for (int64_t e = 0; e < m; ++e)
      if (key[e] >= 0) order[size_t(fill[size_t(key[e] / nc)]++)] = e;
  }
  parallel_for(nc, [&](int64_t I) {
    for (int64_t a = bucket[I] + 1; a < bucket[I + 1]; ++a)
      for (int64_t b = a; b > bucket[I] && key[order[b]] < key[order[b - 1]]; --b)
        std::swap(order[b], order[b - 1]);
  });
  std::vector<int64_t> start;
  for (size_t q = 0; q < order.size(); ++q)
    if (q == 0 || key[order[q]] != key[order[q - 1]]) start.push_back(int64_t(q));
  const int64_t ne = int64_t(start.size());
  start.push_back(int64_t(order.size()));
  out.e0.resize(static_cast<size_t>(ne));
  out.e1.resize(static_cast<size_t>(ne));
  for (int64_t g = 0; g < ne; ++g) {
    const int64_t kk0 = key[order[start[g]]];
    out.e0[g] = int(kk0 / nc);
    out.e1[g] = int(kk0 % nc);
  }
  if (dev && k <= 6) {
    std::vector<std::vector<int>> sorted(aggs);
    for (auto &mem : sorted) std::sort(mem.begin(), mem.end());
    if (dev->coarse_weights(lev, sorted, agg_of, dmask, cc, order, start, out.M, out.E)) {
      out.build_adjacency();
      return out;
    }
  }
  out.M.resize(size_t(nc) * kk);   // every entry written below
  parallel_for(nc, [&](int64_t I) {
    std::vector<int> mem = aggs[I];
    std::sort(mem.begin(), mem.end());
    Sq acc(k);
    for (int i : mem) {
      Sq W = lev.Mmat(i);
      for (int64_t p = lev.nb_ptr[i]; p < lev.nb_ptr[i + 1]; ++p)
        if (dmask[lev.nb[p]]) sq_axpy(W, 1.0, pulled(lev, lev.nb_e[p], i));
      const Sq Q = sq_qtrans(&cc[size_t(3) * I], lev.xp(i), k);
      sq_axpy(acc, 1.0, sq_t3(Q, W, Q));
    }
    std::copy(acc.a, acc.a + kk, &out.M[size_t(I) * kk]);
  });
  out.E.resize(size_t(ne) * kk);   // every entry written below
  parallel_for(ne, [&](int64_t g) {
    Sq acc(k);
    for (int64_t q = start[g]; q < start[g + 1]; ++q) {
      const int64_t e = order[q];
      const int i = lev.e0[e], j = lev.e1[e];
      const int I = agg_of[i], J = agg_of[j];
      const Sq T = sq_mul(sq_mul(sq_qhalf(lev.xp(i), lev.xp(j), k),
                                 sq_qtrans(&cc[size_t(3) * I], lev.xp(i), k)),
                          sq_qhalf(&cc[size_t(3) * J], &cc[size_t(3) * I], k));
      sq_axpy(acc, 1.0, sq_t3(T, lev.Emat(e), T));
    }
    std::copy(acc.a, acc.a + kk, &out.E[size_t(g) * kk]);
  });
  out.build_adjacency();
  return out;
}

// ---- criteria ----------------------------------------------------------------------------------

void dhat_all(const AuxLevel &lev, std::vector<Sq> &D) {
  D.assign(size_t(lev.n), Sq(lev.k));
  parallel_for(lev.n, [&](int64_t i) {
    Sq d = lev.Mmat(int(i));
    for (int64_t p = lev.nb_ptr[i]; p < lev.nb_ptr[i + 1]; ++p) sq_axpy(d, 1.0, pulled(lev, lev.nb_e[p], int(i)));
    D[i] = d;
  });
}

void trace_strength(const AuxLevel &lev, std::vector<double> &m) {
  // m_i = max(tr M^i, tr E^il over the edges at i), raised only by a strictly larger trace: the
  // value does not depend on the order the edges are visited in
  m.assign(size_t(lev.n), 0.0);
  const int k = lev.k;
  parallel_for(lev.n, [&](int64_t i) {
    double v = sq_trace(lev.Mmat(int(i)));
    for (int64_t p = lev.nb_ptr[i]; p < lev.nb_ptr[i + 1]; ++p) {
      const double *E = &lev.E[size_t(lev.nb_e[p]) * k * k];
      double t = 0.0;
      for (int d = 0; d < k; ++d) t += E[d * k + d];   // summed as sq_trace does
      if (t > v) v = t;
    }
    m[i] = v;
  });
}

double mu_D(const AuxLevel &lev, int i, const std::vector<Sq> &D, double tau) {
  return sq_genmax(D[i], lev.Mmat(i), tau);
}

// mu_s of the pair (i, j) joined by edge e (-1: no edge)
static double mu_s_edge(const AuxLevel &lev, int i, int j, int64_t e, const std::vector<double> &mtr) {
  double t = 0.0;
  if (e >= 0) {
    const int k = lev.k;
    const double *E = &lev.E[size_t(e) * k * k];
    for (int d = 0; d < k; ++d) t += E[d * k + d];   // the trace, summed as sq_trace does
  }
  if (t == 0.0) return kInf;
  return std::sqrt(mtr[i] * mtr[j]) / t;
}

double mu_s(const AuxLevel &lev, int i, int j, const std::vector<double> &mtr) {
  return mu_s_edge(lev, i, j, lev.edge_id(i, j), mtr);
}

// Features of candidate pair (i, j) (edge e): log mu_s, the spectrum of sym(E^{ij}) / tr E^{ij}
// (descending, padded), log of the smaller and larger tr D-hat over tr E^{ij}, log(1 + sum of
// tr M / tr D-hat at both ends), the aggregate sizes / 4, |log| of the trace-strength ratio.
void pair_features(const AuxLevel &lev, int i, int j, int e, const std::vector<Sq> &D,
                   const std::vector<double> &mtr, int nmem_i, int nmem_j, float *f) {
  const Sq Ee = lev.Emat(e);
  const double t = sq_trace(Ee);
  double w[6] = {0, 0, 0, 0, 0, 0};
  Sq S = sq_sym(Ee);   // eigenvalues only: the rotations do not depend on the eigenvectors
  crit::jacobi(S.a, S.k, S.k, w, nullptr);
  for (int q = 0; q < kPairFeatures; ++q) f[q] = 0.0f;
  f[0] = float(std::log(std::sqrt(mtr[i] * mtr[j]) / t));
  for (int q = 0; q < lev.k && q < 6; ++q) f[1 + q] = float(w[lev.k - 1 - q] / t);
  const double di = sq_trace(D[i]), dj = sq_trace(D[j]);
  f[7] = float(std::log(std::min(di, dj) / t));
  f[8] = float(std::log(std::max(di, dj) / t));
  f[9] = float(std::log1p(sq_trace(lev.Mmat(i)) / di + sq_trace(lev.Mmat(j)) / dj));
  f[10] = float(double(nmem_i + nmem_j) / 4.0);
  f[11] = float(std::fabs(std::log(mtr[i] / mtr[j])));
}

double mu_b(const AuxLevel &lev, int i, int j, const std::vector<Sq> &D, double tau) {
  return crit::mu_b(lev.view(), D.data(), i, j, tau);
}

double mu_g(const AuxLevel &lev, const std::vector<int> &Cin, const std::vector<Sq> &D, double tau) {
  // Block form of Thm thm:mu1 (delta = 1): every matrix below is assembled from k x k blocks.
  const int k = lev.k;
  std::vector<int> mem = Cin;
  std::sort(mem.begin(), mem.end());
  const int nC = int(mem.size());
  // unions of up to four vertices: the fixed-capacity form shared with the device criteria
  if (nC <= crit::kMaxUnion && k <= 6) {
    auto g = std::make_unique<crit::GScratch>();
    const double v = crit::mu_g(lev.view(), D.data(), mem.data(), nC, tau, *g);
    if (!std::isnan(v)) return v;
  }
  double xH[3];
  mean_pos(lev, mem, xH);
  // L = D_C - D_C P_C pinv(P_C^T D_C P_C) P_C^T D_C with P_C = [Q^{H->i}]
  std::vector<Sq> Y(static_cast<size_t>(nC));
  Sq Z(k);
  for (int a = 0; a < nC; ++a) {
    const Sq Q = sq_qtrans(xH, lev.xp(mem[a]), k);
    Y[a] = sq_mul(D[mem[a]], Q);              // D_a Q_a
    sq_axpy(Z, 1.0, sq_mul(sq_t(Q), Y[a]));  // Q_a^T D_a Q_a
  }
  const Sq Zp = sq_pinv(Z, tau);
  Mat L(nC * k, nC * k), R(nC * k, nC * k);
  auto put = [&](Mat &X, int a, int b, const Sq &S, double s) {
    for (int u = 0; u < k; ++u)
      for (int v = 0; v < k; ++v) X(a * k + u, b * k + v) += s * S(u, v);
  };
  for (int a = 0; a < nC; ++a) {
    const Sq YZ = sq_mul(Y[a], Zp);
    for (int b = 0; b < nC; ++b) put(L, a, b, sq_mul(YZ, sq_t(Y[b])), -1.0);
    put(L, a, a, D[mem[a]], 1.0);
    put(R, a, a, lev.Mmat(mem[a]), 1.0);
  }
  // edges inside C (eq. auxa) and the outside neighbours
  std::vector<std::pair<int, std::vector<std::pair<int, int>>>> outside;  // l -> (a, e)
  std::unordered_map<int, size_t> opos;
  for (int a = 0; a < nC; ++a) {
    const int i = mem[a];
    for (int64_t p = lev.nb_ptr[i]; p < lev.nb_ptr[i + 1]; ++p) {
      const int l = lev.nb[p], e = lev.nb_e[p];
      const auto it = std::lower_bound(mem.begin(), mem.end(), l);
      if (it != mem.end() && *it == l) {
        if (i < l) {
          const int b = int(it - mem.begin());
          const Sq Qil = sq_qhalf(lev.xp(i), lev.xp(l), k), Qli = sq_qhalf(lev.xp(l), lev.xp(i), k);
          const Sq Ee = lev.Emat(e);
          put(R, a, a, sq_t3(Qil, Ee, Qil), 1.0);
          put(R, b, b, sq_t3(Qli, Ee, Qli), 1.0);
          put(R, a, b, sq_t3(Qil, Ee, Qli), -1.0);
          put(R, b, a, sq_t3(Qli, Ee, Qil), -1.0);
        }
      } else {
        auto f = opos.find(l);
        if (f == opos.end()) {
          opos.emplace(l, outside.size());
          outside.push_back({l, {{a, e}}});
        } else {
          outside[f->second].second.emplace_back(a, e);
        }
      }
    }
  }
  std::sort(outside.begin(), outside.end(),
            [](const auto &x, const auto &y) { return x.first < y.first; });
  std::vector<Sq> Kcw, Kcc;
  std::vector<int> am;
  for (const auto &ol : outside) {
    if (ol.second.size() < 2) continue;
    const int l = ol.first;
    // local assembly of the edges (i, l), i in C, with unknowns (v_C, w); Schur complement on v_C
    Kcw.clear();
    Kcc.clear();
    am.clear();
    Sq Kww(k);
    for (const auto &ae : ol.second) {
      const int a = ae.first, e = ae.second, i = mem[a];
      const Sq Qil = sq_qhalf(lev.xp(i), lev.xp(l), k), Qli = sq_qhalf(lev.xp(l), lev.xp(i), k);
      const Sq Ee = lev.Emat(e);
      am.push_back(a);
      Kcc.push_back(sq_t3(Qil, Ee, Qil));
      Sq X = sq_t3(Qil, Ee, Qli);
      for (int q = 0; q < k * k; ++q) X.a[q] = -X.a[q];
      Kcw.push_back(X);
      sq_axpy(Kww, 1.0, sq_t3(Qli, Ee, Qli));
    }
    const Sq Wp = sq_pinv(Kww, tau);
    for (size_t x = 0; x < am.size(); ++x) {
      const Sq KW = sq_mul(Kcw[x], Wp);
      for (size_t y = 0; y < am.size(); ++y) {
        Sq S = sq_mul(KW, sq_t(Kcw[y]));
        for (int q = 0; q < k * k; ++q) S.a[q] = -S.a[q];
        if (x == y) sq_axpy(S, 1.0, Kcc[x]);
        // 1/2 sym(S_l): add half of the block and half of its mirror
        put(R, am[x], am[y], S, 0.25);
        put(R, am[y], am[x], sq_t(S), 0.25);
      }
    }
  }
  return genmax(sym(L), sym(R), tau);
}

// ---- Algorithm alg:pwagg --------------------------------------------------------------------

std::vector<int> cuthill_mckee(const AuxLevel &lev, const std::vector<char> &free_mask) {
  const int n = lev.n;
  // the graph: edges of positive trace between free vertices, read through the level's
  // adjacency lists (the order of a vertex's neighbours does not matter: they are visited sorted
  // by (degree, id))
  std::vector<char> live(static_cast<size_t>(lev.m()));
  parallel_for(lev.m(), [&](int64_t e) {
    live[e] = sq_trace(lev.Emat(e)) > 0.0 && free_mask[lev.e0[e]] && free_mask[lev.e1[e]];
  });
  std::vector<int> deg(static_cast<size_t>(n));
  parallel_for(n, [&](int64_t v) {
    int d = 0;
    for (int64_t q = lev.nb_ptr[v]; q < lev.nb_ptr[v + 1]; ++q) d += live[lev.nb_e[q]];
    deg[v] = d;
  });
  std::vector<std::pair<int, int>> starts;
  for (int v = 0; v < n; ++v)
    if (free_mask[v]) starts.emplace_back(deg[v], v);
  std::sort(starts.begin(), starts.end());
  std::vector<char> visited(static_cast<size_t>(n), 0);
  std::vector<int> order;
  order.reserve(starts.size());
  size_t ptr = 0;
  std::deque<int> queue;
  std::vector<std::pair<int, int>> nbv;
  while (order.size() < starts.size()) {
    while (visited[starts[ptr].second]) ++ptr;
    const int s = starts[ptr].second;
    visited[s] = 1;
    queue.push_back(s);
    while (!queue.empty()) {
      const int v = queue.front();
      queue.pop_front();
      order.push_back(v);
      nbv.clear();
      for (int64_t q = lev.nb_ptr[v]; q < lev.nb_ptr[v + 1]; ++q) {
        const int u = lev.nb[q];
        if (live[lev.nb_e[q]] && !visited[u]) nbv.emplace_back(deg[u], u);
      }
      std::sort(nbv.begin(), nbv.end());
      for (const auto &du : nbv) {
        visited[du.second] = 1;
        queue.push_back(du.second);
      }
    }
  }
  return order;
}

MatchResult successive_matching(const AuxLevel &lev, const std::vector<char> &vd,
                                const MatchParams &prm) {
  const int n = lev.n;
  const double sigma = prm.sigma;
  MatchResult res;
  PhaseTimer tm;
  auto note = [&](double mu) {
    if (std::isfinite(mu)) res.min_margin = std::min(res.min_margin, std::fabs(mu - sigma) / sigma);
  };
  std::vector<Sq> Dhat;
  dhat_all(lev, Dhat);
  tm.mark("dhat");
  res.dmask.assign(static_cast<size_t>(n), 0);
  for (int i = 0; i < n; ++i) res.dmask[i] = vd.empty() ? 0 : vd[i];
  std::vector<double> md(static_cast<size_t>(n), 0.0);
  parallel_for(n, [&](int64_t i) {
    if (!res.dmask[i]) md[i] = mu_D(lev, int(i), Dhat, prm.tau);
  });
  for (int i = 0; i < n; ++i) {
    if (res.dmask[i]) continue;
    note(md[i]);
    if (md[i] < sigma) res.dmask[i] = 1;
  }
  std::vector<char> in_T(static_cast<size_t>(n));
  for (int i = 0; i < n; ++i) in_T[i] = !res.dmask[i];
  tm.mark("mu_D");
  // The walk order runs on a thread of its own while the first pass computes its per-edge data
  // (trace strengths, mu_s), which does not depend on it; it is joined before the first use.
  std::future<std::vector<int>> order_job =
      std::async(std::launch::async, [&lev, mask = in_T] { return cuthill_mckee(lev, mask); });
  std::vector<int> order;

  AuxLevel work_store;
  const AuxLevel *work = &lev;
  std::vector<Sq> wdhat_store;
  const std::vector<Sq> *wdhat = &Dhat;
  std::vector<std::vector<int>> members(static_cast<size_t>(n));
  for (int i = 0; i < n; ++i) members[i] = {i};
  std::vector<std::vector<int>> entries;
  std::vector<double> mtr;
  std::vector<int> pos;
  // Optimistic parallel walks.  mu_b and mu_g of a pair are functions of this pass's level data
  // only.  A walk that meets a pair whose criteria are not known yet records it and assumes it
  // passes; all pairs recorded by a walk are then evaluated in parallel and the walk is repeated,
  // until one walk needs no unknown pair.  That walk used exact criteria only, so it is the
  // sequential algorithm's walk, bit for bit.
  struct Crit {
    double mub, mug;   // mug NaN when not needed (mub >= sigma or a pair of single vertices)
  };
  // per working-level adjacency entry q (the pair (i, nb[q]), i the walking vertex): mu_s, the
  // criteria once evaluated, the learned acceptance probability
  std::vector<double> ms_q;
  std::vector<Crit> crit_q;
  std::vector<char> has_q;
  std::vector<float> prob_q;
  bool batch_level = false;
  for (int p = 1; p <= prm.rounds; ++p) {
    bool batch_work = false;
    trace_strength(*work, mtr);
    const size_t nq = work->nb.size();
    ms_q.assign(nq, 0.0);
    parallel_for(work->n, [&](int64_t i) {
      for (int64_t q = work->nb_ptr[i]; q < work->nb_ptr[i + 1]; ++q)
        ms_q[q] = mu_s_edge(*work, int(i), work->nb[q], work->nb_e[q], mtr);
    });
    if (p == 1) {
      order = order_job.get();
      tm.mark("cuthill-mckee (beside mu_s)");
    }
    pos.assign(size_t(work->n), 0);
    for (size_t a = 0; a < order.size(); ++a) pos[order[a]] = int(a);
    crit_q.assign(nq, Crit{0.0, 0.0});
    has_q.assign(nq, 0);
    // adjacency entry of j in the list of i (-1: not adjacent)
    auto qpos = [&](int i, int j) -> int64_t {
      const auto b = work->nb.begin() + work->nb_ptr[i], e = work->nb.begin() + work->nb_ptr[i + 1];
      const auto it = std::lower_bound(b, e, j);
      return (it != e && *it == j) ? int64_t(it - work->nb.begin()) : -1;
    };
    // candidate pairs of the pass (both ends free, mu_s < sigma), scored by the learned model
    const bool learned = bool(prm.scorer) && prm.skip > 0.0;
    PassSamples ps;
    std::vector<int64_t> ps_q;   // adjacency entries (i -> j, j -> i) of each candidate pair
    if (learned) prob_q.assign(nq, 1.0f);
    if (learned || prm.record) {
      ps.n = work->n;
      for (int i = 0; i < work->n; ++i) {
        if (!in_T[i]) continue;
        for (int64_t q = work->nb_ptr[i]; q < work->nb_ptr[i + 1]; ++q) {
          const int j = work->nb[q];
          if (j <= i || !in_T[j]) continue;
          if (!(ms_q[q] < sigma)) continue;
          ps.edges.push_back(i);
          ps.edges.push_back(j);
          ps_q.push_back(q);
          ps_q.push_back(qpos(j, i));
        }
      }
      const size_t np = ps.edges.size() / 2;
      ps.X.assign(np * kPairFeatures, 0.0f);
      parallel_for(int64_t(np), [&](int64_t q) {
        const int i = ps.edges[2 * q], j = ps.edges[2 * q + 1];
        pair_features(*work, i, j, work->edge_id(i, j), *wdhat, mtr, int(members[i].size()),
                      int(members[j].size()), &ps.X[size_t(q) * kPairFeatures]);
      });
      if (learned && np > 0) {
        std::vector<float> z;
        prm.scorer(ps, z);
        for (size_t q = 0; q < np; ++q) {
          const float pr = 1.0f / (1.0f + std::exp(-z[q]));
          prob_q[ps_q[2 * q]] = pr;
          if (ps_q[2 * q + 1] >= 0) prob_q[ps_q[2 * q + 1]] = pr;
        }
      }
    }
    tm.mark("candidate scores");
    int64_t w_eval = 0, w_eval_g = 0, w_skip = 0;
    std::vector<std::pair<int, int>> pairs;
    std::vector<int> singles;
    struct Unknown {
      int ci, cj;
      int64_t q;   // adjacency entry of (ci, cj)
    };
    std::vector<Unknown> unknown;
    int walks = 0;
    long n_eval = 0;
    double t_walk = 0.0, t_eval = 0.0;
    // Walk state; a walk resumes from the state just before the first vertex at which the
    // previous walk used an unknown pair (everything before it was already exact).
    struct WalkState {
      size_t a = 0;                  // position in `order`
      std::vector<char> inT;
      size_t npairs = 0, nsingles = 0;
      double min_margin = 1e300;
      int max_tie = 0;
      int64_t ev = 0, evg = 0, sk = 0;
    };
    WalkState ck;
    ck.inT = in_T;
    pairs.clear();
    singles.clear();
    for (;;) {
      ++walks;
      const auto tw0 = std::chrono::steady_clock::now();
      std::vector<char> inT = ck.inT;
      pairs.resize(ck.npairs);
      singles.resize(ck.nsingles);
      double min_margin = ck.min_margin;
      int max_tie = ck.max_tie;
      w_eval = ck.ev;
      w_eval_g = ck.evg;
      w_skip = ck.sk;
      unknown.clear();
      WalkState next;
      bool have_next = false;
      auto note_w = [&](double mu) {
        if (std::isfinite(mu)) min_margin = std::min(min_margin, std::fabs(mu - sigma) / sigma);
      };
      struct Cand {
        int cj;
        double ms;
        int64_t q;
      };
      std::vector<Cand> cands;
      for (size_t a = ck.a; a < order.size(); ++a) {
        const int ci = order[a];
        if (!inT[ci]) continue;
        // state before this vertex (scalars; inT is copied only if it becomes the next start)
        const size_t np0 = pairs.size(), ns0 = singles.size();
        const double mm0 = min_margin;
        const int mt0 = max_tie;
        const int64_t ev0 = w_eval, evg0 = w_eval_g, sk0 = w_skip;
        inT[ci] = 0;
        cands.clear();
        for (int64_t q = work->nb_ptr[ci]; q < work->nb_ptr[ci + 1]; ++q) {
          const int cj = work->nb[q];
          if (!inT[cj]) continue;
          const double ms = ms_q[q];
          note_w(ms);
          if (ms < sigma) cands.push_back(Cand{cj, ms, q});
        }
        int matched = -1;
        // the exact criteria for (ci, cj), or an optimistic pass when not known yet
        auto check = [&](int cj, int64_t q) {
          if (prm.mu_s_only) return true;
          ++w_eval;
          if (!has_q[q]) {
            if (!have_next) {
              have_next = true;
              next.a = a;
              next.inT = inT;
              next.inT[ci] = 1;
              next.npairs = np0;
              next.nsingles = ns0;
              next.min_margin = mm0;
              next.max_tie = mt0;
              next.ev = ev0;
              next.evg = evg0;
              next.sk = sk0;
            }
            unknown.push_back(Unknown{ci, cj, q});
            return true;   // optimistic
          }
          const Crit &c = crit_q[q];
          note_w(c.mub);
          bool ok = c.mub < sigma;
          if (ok && !std::isnan(c.mug)) {
            ++w_eval_g;
            note_w(c.mug);
            ok = c.mug < sigma;
          }
          return ok;
        };
        bool any_checked = false;
        int pass_over = -1;       // best scored candidate passed over
        int64_t pass_over_q = -1;
        float pass_over_p = -1.0f;
        while (!cands.empty()) {
          double mmin = cands[0].ms;
          for (const auto &c : cands) mmin = std::min(mmin, c.ms);
          int best = -1, ntie = 0;
          for (size_t c = 0; c < cands.size(); ++c)
            if (cands[c].ms <= mmin * (1.0 + prm.tie_rtol)) {
              ++ntie;
              if (best < 0 || pos[cands[c].cj] < pos[cands[best].cj]) best = int(c);
            }
          max_tie = std::max(max_tie, ntie);
          const int cj = cands[best].cj;
          const int64_t cq = cands[best].q;
          if (learned) {
            const float pr = prob_q[cq];
            if (pr < prm.skip) {
              ++w_skip;
              if (pr > pass_over_p) {
                pass_over_p = pr;
                pass_over = cj;
                pass_over_q = cq;
              }
              cands.erase(cands.begin() + best);
              continue;
            }
          }
          any_checked = true;
          if (check(cj, cq)) {
            matched = cj;
            break;
          }
          cands.erase(cands.begin() + best);
        }
        // fallback: every candidate was passed over -> the exact criteria decide the best scored
        if (matched < 0 && !any_checked && pass_over >= 0 && check(pass_over, pass_over_q))
          matched = pass_over;
        if (matched >= 0) {
          pairs.emplace_back(ci, matched);
          inT[matched] = 0;
        } else {
          singles.push_back(ci);
        }
      }
      t_walk += std::chrono::duration<double>(std::chrono::steady_clock::now() - tw0).count();
      if (unknown.empty()) {
        res.min_margin = std::min(res.min_margin, min_margin);
        res.max_tie = std::max(res.max_tie, max_tie);
        res.evaluated += w_eval;
        res.evaluated_g += w_eval_g;
        res.skipped += w_skip;
        in_T = inT;
        break;
      }
      ck = std::move(next);
      const auto te0 = std::chrono::steady_clock::now();
      std::vector<Crit> val(unknown.size());
      if (prm.batch) {
        // the batch evaluator takes mu_b of the unknown pairs when there are batch_min_pairs of
        // them, and mu_g of the unions of up to crit::kMaxUnion vertices whose mu_b passes when
        // there are batch_min_unions of them; host threads take the rest, larger unions and
        // unions the evaluator could not hold
        auto ensure_levels = [&] {
          if (!batch_level) {
            prm.batch->level(lev, Dhat);
            batch_level = true;
          }
          if (!batch_work) {
            prm.batch->work(*work, *wdhat);
            batch_work = true;
          }
        };
        std::vector<double> mub(unknown.size()), mug;
        if (unknown.size() >= size_t(std::max(1, prm.batch_min_pairs))) {
          ensure_levels();
          std::vector<int32_t> pr(2 * unknown.size());
          for (size_t u = 0; u < unknown.size(); ++u) {
            pr[2 * u] = unknown[u].ci;
            pr[2 * u + 1] = unknown[u].cj;
          }
          prm.batch->mu_b(pr, prm.tau, mub);
        } else {
          parallel_for_dynamic(int64_t(unknown.size()), [&](int64_t u) {
            mub[u] = mu_b(*work, unknown[u].ci, unknown[u].cj, *wdhat, prm.tau);
          }, 16);
        }
        std::vector<int32_t> un4;
        std::vector<size_t> on_dev, on_host;
        for (size_t u = 0; u < unknown.size(); ++u) {
          const int ci = unknown[u].ci, cj = unknown[u].cj;
          val[u] = Crit{mub[u], std::numeric_limits<double>::quiet_NaN()};
          const size_t nC = members[ci].size() + members[cj].size();
          if (!(mub[u] < sigma) || nC <= 2) continue;
          if (nC > size_t(crit::kMaxUnion) || lev.k > 6) {
            on_host.push_back(u);
            continue;
          }
          std::vector<int> un = members[ci];
          un.insert(un.end(), members[cj].begin(), members[cj].end());
          std::sort(un.begin(), un.end());
          for (int a2 = 0; a2 < crit::kMaxUnion; ++a2) un4.push_back(a2 < int(nC) ? un[a2] : -1);
          on_dev.push_back(u);
        }
        if (on_dev.size() >= size_t(std::max(1, prm.batch_min_unions))) {
          ensure_levels();
          prm.batch->mu_g(un4, prm.tau, mug);
          for (size_t q = 0; q < on_dev.size(); ++q) {
            if (std::isnan(mug[q]))
              on_host.push_back(on_dev[q]);
            else
              val[on_dev[q]].mug = mug[q];
          }
        } else {
          on_host.insert(on_host.end(), on_dev.begin(), on_dev.end());
        }
        parallel_for_dynamic(int64_t(on_host.size()), [&](int64_t q) {
          const size_t u = on_host[size_t(q)];
          const int ci = unknown[u].ci, cj = unknown[u].cj;
          std::vector<int> un = members[ci];
          un.insert(un.end(), members[cj].begin(), members[cj].end());
          val[u].mug = mu_g(lev, un, Dhat, prm.tau);
        }, 4);
      } else {
        parallel_for_dynamic(int64_t(unknown.size()), [&](int64_t u) {
          const int ci = unknown[u].ci, cj = unknown[u].cj;
          Crit c{mu_b(*work, ci, cj, *wdhat, prm.tau), std::numeric_limits<double>::quiet_NaN()};
          if (c.mub < sigma && members[ci].size() + members[cj].size() > 2) {
            std::vector<int> un = members[ci];
            un.insert(un.end(), members[cj].begin(), members[cj].end());
            c.mug = mu_g(lev, un, Dhat, prm.tau);
          }
          val[u] = c;
        }, 16);
      }
      for (size_t u = 0; u < unknown.size(); ++u) {
        crit_q[unknown[u].q] = val[u];
        has_q[unknown[u].q] = 1;
      }
      n_eval += long(unknown.size());
      t_eval += std::chrono::duration<double>(std::chrono::steady_clock::now() - te0).count();
    }
    if (tm.on)
      std::fprintf(stderr, "[eamg]   %d walks, %ld pairs evaluated in parallel, %zu pairs formed, %zu singles; "
                   "walk: %lld evaluations (%lld with mu_g), %lld passed over; walks %.3f s, "
                   "parallel criteria %.3f s\n",
                   walks, n_eval, pairs.size(), singles.size(), (long long)w_eval, (long long)w_eval_g,
                   (long long)w_skip, t_walk, t_eval);
    if (prm.record) {
      const size_t np = ps.edges.size() / 2;
      ps.y.assign(np, 0.0f);
      ps.w.assign(np, 0.0f);
      for (size_t q = 0; q < np; ++q) {
        int64_t at = ps_q[2 * q];
        if (!has_q[at]) at = ps_q[2 * q + 1];
        if (at < 0 || !has_q[at]) continue;
        const Crit &c = crit_q[at];
        const bool acc = c.mub < sigma && (std::isnan(c.mug) || c.mug < sigma);
        ps.y[q] = acc ? 1.0f : 0.0f;
        ps.w[q] = 1.0f;
      }
      res.samples.push_back(std::move(ps));
    }
    tm.mark("matching pass");
    std::vector<std::vector<int>> groups;
    for (const auto &pq : pairs) groups.push_back({pq.first, pq.second});
    for (int s : singles) groups.push_back({s});
    entries.clear();
    for (const auto &g : groups) {
      std::vector<int> m = members[g[0]];
      if (g.size() == 2) m.insert(m.end(), members[g[1]].begin(), members[g[1]].end());
      entries.push_back(m);
    }
    if (p < prm.rounds) {
      std::vector<double> ic(entries.size() * 3);
      for (size_t I = 0; I < entries.size(); ++I) mean_pos(lev, entries[I], &ic[3 * I]);
      std::vector<char> wmask = p == 1 ? res.dmask : std::vector<char>(size_t(work->n), 0);
      if (prm.batch) {
        if (!batch_level) {
          prm.batch->level(lev, Dhat);
          batch_level = true;
        }
        if (!batch_work) {
          prm.batch->work(*work, *wdhat);
          batch_work = true;
        }
      }
      AuxLevel next = coarse_aux(*work, groups, wmask, ic, prm.batch);
      work_store = std::move(next);
      work = &work_store;
      dhat_all(*work, wdhat_store);
      wdhat = &wdhat_store;
      tm.mark("intermediate weights");
      members = entries;
      in_T.assign(entries.size(), 1);
      order.resize(entries.size());
      for (size_t a = 0; a < entries.size(); ++a) order[a] = int(entries.size() - 1 - a);
    }
  }
  res.aggs = entries;
  for (auto &a : res.aggs) std::sort(a.begin(), a.end());
  res.ccoords.resize(res.aggs.size() * 3);
  for (size_t I = 0; I < res.aggs.size(); ++I) mean_pos(lev, res.aggs[I], &res.ccoords[3 * I]);
  if (prm.batch && !batch_level) {
    prm.batch->level(lev, Dhat);
    batch_level = true;
  }
  res.coarse = coarse_aux(lev, res.aggs, res.dmask, res.ccoords, prm.batch);
  tm.mark("coarse weights");
  return res;
}

}  // namespace eamg
