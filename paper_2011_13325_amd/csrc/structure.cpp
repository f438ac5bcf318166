#include "structure.hpp"

#include <algorithm>
#include <functional>
#include <map>
#include <queue>

namespace eamg {

namespace {

// Row chunks of a pattern pass: contiguous ranges, a count that depends on n only, so results
// that are concatenated in chunk order do not depend on the thread count.
inline int n_chunks(int n) { return std::max(1, std::min(64, n / 1024)); }
inline int chunk_lo(int n, int nch, int64_t c) { return int(int64_t(n) * c / nch); }

}  // namespace

ProlongPlan plan_prolongation(const Pattern &A, const AuxLevel &aux, const std::vector<int> &agg_of,
                              const std::vector<char> &dmask, int cap_S, int cap_A, double tie_rtol) {
  const int n = A.n_rows;
  const int k = aux.k;
  ProlongPlan pl;
  pl.type.assign(static_cast<size_t>(n), ROW_D);
  pl.P.n_rows = n;
  pl.P.rp.assign(size_t(n) + 1, 0);
  pl.F_ptr.assign(size_t(n) + 1, 0);
  int nc = 0;
  for (int v : agg_of) nc = std::max(nc, v + 1);
  pl.P.n_cols = nc;
  // per chunk: P columns and F entries of its rows, lengths in pl.P.rp / pl.F_ptr [i + 1]
  struct Part {
    std::vector<int> col, fv, fe;
  };
  const int nch = n_chunks(n);
  std::vector<Part> parts(static_cast<size_t>(nch));
  parallel_for_dynamic(nch, [&](int64_t c) {
    Part &pt = parts[size_t(c)];
    std::vector<int> cs;
    std::vector<std::pair<int, int>> F;         // (l, e)
    for (int i = chunk_lo(n, nch, c); i < chunk_lo(n, nch, c + 1); ++i) {
      if (dmask[i]) continue;
      cs.clear();
      cs.push_back(agg_of[i]);
      for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p) {
        const int j = A.col[p];
        if (!dmask[j]) cs.push_back(agg_of[j]);
      }
      std::sort(cs.begin(), cs.end());
      cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
      if (int(cs.size()) <= cap_S) {
        pl.type[i] = ROW_S;
        pt.col.insert(pt.col.end(), cs.begin(), cs.end());
        pl.P.rp[i + 1] = int64_t(cs.size());
        continue;
      }
      pl.type[i] = ROW_A;
      F.clear();
      std::map<int, double> ws;
      for (int64_t p = aux.nb_ptr[i]; p < aux.nb_ptr[i + 1]; ++p) {
        const int l = aux.nb[p];
        if (dmask[l]) continue;
        const int e = aux.nb_e[p];
        double tr = 0.0;
        for (int d = 0; d < k; ++d) tr += aux.E[size_t(e) * k * k + size_t(d) * k + d];
        ws[agg_of[l]] += tr;
      }
      const int own = agg_of[i];
      std::vector<std::pair<int, double>> others;   // ascending group id
      for (const auto &g : ws)
        if (g.first != own) others.emplace_back(g.first, g.second);
      std::vector<int> keep = {own};
      while (!others.empty() && int(keep.size()) < cap_A) {
        double wmax = others[0].second;
        for (const auto &g : others) wmax = std::max(wmax, g.second);
        size_t pick = 0;
        while (!(others[pick].second >= wmax * (1.0 - tie_rtol))) ++pick;   // smallest id in band
        keep.push_back(others[pick].first);
        others.erase(others.begin() + long(pick));
      }
      std::sort(keep.begin(), keep.end());
      for (int64_t p = aux.nb_ptr[i]; p < aux.nb_ptr[i + 1]; ++p) {
        const int l = aux.nb[p];
        if (dmask[l]) continue;
        if (std::binary_search(keep.begin(), keep.end(), agg_of[l])) F.emplace_back(l, aux.nb_e[p]);
      }
      std::sort(F.begin(), F.end());
      for (const auto &le : F) {
        pt.fv.push_back(le.first);
        pt.fe.push_back(le.second);
      }
      pl.F_ptr[i + 1] = int64_t(F.size());
      pt.col.insert(pt.col.end(), keep.begin(), keep.end());
      pl.P.rp[i + 1] = int64_t(keep.size());
    }
  }, 1);
  for (int i = 0; i < n; ++i) {
    pl.P.rp[i + 1] += pl.P.rp[i];
    pl.F_ptr[i + 1] += pl.F_ptr[i];
  }
  pl.P.col.reserve(size_t(pl.P.rp[n]));
  pl.F_vtx.reserve(size_t(pl.F_ptr[n]));
  pl.F_edge.reserve(size_t(pl.F_ptr[n]));
  for (const Part &pt : parts) {
    pl.P.col.insert(pl.P.col.end(), pt.col.begin(), pt.col.end());
    pl.F_vtx.insert(pl.F_vtx.end(), pt.fv.begin(), pt.fv.end());
    pl.F_edge.insert(pl.F_edge.end(), pt.fe.begin(), pt.fe.end());
  }
  return pl;
}

Pattern spgemm_symbolic(const Pattern &A, const Pattern &B) {
  Pattern C;
  const int n = A.n_rows;
  C.n_rows = n;
  C.n_cols = B.n_cols;
  C.rp.assign(size_t(n) + 1, 0);
  const int nch = n_chunks(n);
  std::vector<std::vector<int>> parts(static_cast<size_t>(nch));
  parallel_for_dynamic(nch, [&](int64_t c) {
    std::vector<int> &out = parts[size_t(c)];
    std::vector<int> mark(size_t(B.n_cols), -1);
    std::vector<int> row;
    for (int i = chunk_lo(n, nch, c); i < chunk_lo(n, nch, c + 1); ++i) {
      row.clear();
      for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p) {
        const int j = A.col[p];
        for (int64_t q = B.rp[j]; q < B.rp[j + 1]; ++q) {
          const int cc = B.col[q];
          if (mark[cc] != i) {
            mark[cc] = i;
            row.push_back(cc);
          }
        }
      }
      std::sort(row.begin(), row.end());
      out.insert(out.end(), row.begin(), row.end());
      C.rp[i + 1] = int64_t(row.size());
    }
  }, 1);
  for (int i = 0; i < n; ++i) C.rp[i + 1] += C.rp[i];
  C.col.reserve(size_t(C.rp[n]));
  for (const auto &pt : parts) C.col.insert(C.col.end(), pt.begin(), pt.end());
  return C;
}

Pattern transpose_pattern(const Pattern &P, std::vector<int64_t> &src) {
  Pattern T;
  T.n_rows = P.n_cols;
  T.n_cols = P.n_rows;
  T.rp.assign(size_t(P.n_cols) + 1, 0);
  for (int64_t q = 0; q < P.nnz(); ++q) T.rp[P.col[q] + 1]++;
  for (int c = 0; c < P.n_cols; ++c) T.rp[c + 1] += T.rp[c];
  T.col.resize(size_t(P.nnz()));
  src.resize(size_t(P.nnz()));
  std::vector<int64_t> fill(T.rp.begin(), T.rp.end() - 1);
  for (int i = 0; i < P.n_rows; ++i)
    for (int64_t q = P.rp[i]; q < P.rp[i + 1]; ++q) {
      const int64_t d = fill[P.col[q]]++;
      T.col[d] = i;
      src[d] = q;
    }
  return T;
}

std::vector<int> greedy_coloring(int n, const int64_t *rp, const int *col, int &n_colors) {
  // smallest-last order: remove a vertex of minimum remaining degree (lowest id on ties).
  // Indexed binary min-heap on the key (degree, id), one entry per vertex; a removal lowers
  // its neighbours' keys in place.
  std::vector<int64_t> key(static_cast<size_t>(n));
  for (int i = 0; i < n; ++i) {
    int64_t d = 0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
      if (col[p] != i) ++d;
    key[i] = (d << 32) | int64_t(i);
  }
  std::vector<int> heap(static_cast<size_t>(n)), where(static_cast<size_t>(n));
  for (int i = 0; i < n; ++i) heap[i] = where[i] = i;
  int size = n;
  auto swap_at = [&](int a, int b) {
    std::swap(heap[a], heap[b]);
    where[heap[a]] = a;
    where[heap[b]] = b;
  };
  auto sift_up = [&](int a) {
    while (a > 0) {
      const int par = (a - 1) / 2;
      if (key[heap[par]] <= key[heap[a]]) break;
      swap_at(a, par);
      a = par;
    }
  };
  auto sift_down = [&](int a) {
    for (;;) {
      const int l = 2 * a + 1, r = l + 1;
      int m = a;
      if (l < size && key[heap[l]] < key[heap[m]]) m = l;
      if (r < size && key[heap[r]] < key[heap[m]]) m = r;
      if (m == a) break;
      swap_at(a, m);
      a = m;
    }
  };
  for (int a = n / 2 - 1; a >= 0; --a) sift_down(a);
  std::vector<char> removed(static_cast<size_t>(n), 0);
  std::vector<int> seq;
  seq.reserve(static_cast<size_t>(n));
  while (size > 0) {
    const int v = heap[0];
    swap_at(0, size - 1);
    --size;
    sift_down(0);
    removed[v] = 1;
    seq.push_back(v);
    for (int64_t p = rp[v]; p < rp[v + 1]; ++p) {
      const int u = col[p];
      if (u == v || removed[u]) continue;
      key[u] -= int64_t(1) << 32;
      sift_up(where[u]);
    }
  }
  std::vector<int> color(static_cast<size_t>(n), -1);
  std::vector<int> used;
  n_colors = 0;
  for (auto it = seq.rbegin(); it != seq.rend(); ++it) {
    const int i = *it;
    used.clear();
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      const int j = col[p];
      if (j != i && color[j] >= 0) used.push_back(color[j]);
    }
    std::sort(used.begin(), used.end());
    int c = 0;
    for (int u : used) {
      if (u == c) ++c;
      else if (u > c) break;
    }
    color[i] = c;
    n_colors = std::max(n_colors, c + 1);
  }
  return color;
}

Pattern permute_pattern(const Pattern &A, const std::vector<int> &perm, const std::vector<int> &inv,
                        std::vector<int64_t> &src) {
  return permute_rect(A, perm, inv, src);
}

Pattern permute_rect(const Pattern &P, const std::vector<int> &perm_rows,
                     const std::vector<int> &inv_cols, std::vector<int64_t> &src) {
  Pattern R;
  R.n_rows = P.n_rows;
  R.n_cols = P.n_cols;
  R.rp.assign(size_t(P.n_rows) + 1, 0);
  R.col.resize(size_t(P.nnz()));
  src.resize(size_t(P.nnz()));
  for (int r = 0; r < P.n_rows; ++r) {
    const int o = perm_rows[r];
    R.rp[r + 1] = R.rp[r] + (P.rp[o + 1] - P.rp[o]);
  }
  const int n = P.n_rows, nch = n_chunks(n);
  parallel_for_dynamic(nch, [&](int64_t c) {
    std::vector<std::pair<int, int64_t>> row;
    for (int r = chunk_lo(n, nch, c); r < chunk_lo(n, nch, c + 1); ++r) {
      const int o = perm_rows[r];
      row.clear();
      for (int64_t q = P.rp[o]; q < P.rp[o + 1]; ++q) row.emplace_back(inv_cols[P.col[q]], q);
      std::sort(row.begin(), row.end());
      const int64_t base = R.rp[r];
      for (size_t t = 0; t < row.size(); ++t) {
        R.col[size_t(base) + t] = row[t].first;
        src[size_t(base) + t] = row[t].second;
      }
    }
  }, 1);
  return R;
}

}  // namespace eamg
