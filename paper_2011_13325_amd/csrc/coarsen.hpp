// Host-side auxiliary topology and coarsening (paper section "deng" and section "crs2").
//
//  * AuxLevel: vertices with k x k vertex weights M^i and edges (i < j) with k x k edge weights
//    E^ij that define the auxiliary matrix of Def. def:deng (eq. auxa).
//  * finest_aux: Thm thm:deng_elast (elasticity, E^ij = c^ij [[t t^T, 0], [0, 0]], M^i = 0, c^ij
//    the mean absolute entry of (A_N)_ij, t the unit edge direction) and the scalar M-matrix
//    splitting (E^ij = |A_ij|, M^i = max(0, A_ii - sum |A_ij|)).
//  * coarse_aux: Thm thm:cemats.
//  * mu_D / mu_s / mu_b / mu_g: Thm thm:mu1 (eqs. mu_a, mu_d), Lemma thm:mu2, Def. def:muc.
//  * successive_matching: Algorithm alg:pwagg.
#pragma once

#include <algorithm>
#include <cstdint>
#include <string>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <functional>
#include <thread>
#include <utility>
#include <vector>

#include "crit_core.hpp"

#include "dense.hpp"

namespace eamg {

// f(i) for i in [0, n) on up to 16 threads (contiguous chunks); f must not throw and must only
// write data owned by index i, so the result does not depend on the thread count.
template <class F>
void parallel_for(int64_t n, F &&f) {
  unsigned nt = std::thread::hardware_concurrency();
  nt = std::max(1u, std::min(nt, 16u));
  if (n < 2048 || nt == 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    const int64_t lo = int64_t(t) * chunk, hi = std::min(n, lo + chunk);
    if (lo >= hi) break;
    th.emplace_back([&f, lo, hi] {
      for (int64_t i = lo; i < hi; ++i) f(i);
    });
  }
  for (auto &x : th) x.join();
}


// Phase timing on stderr when EAMG_VERBOSE is set.
struct PhaseTimer {
  bool on;
  std::chrono::steady_clock::time_point t0;
  // when set, every phase's (name, seconds) is appended here
  std::vector<std::pair<std::string, double>> *sink = nullptr;
  PhaseTimer() : on(std::getenv("EAMG_VERBOSE") != nullptr), t0(std::chrono::steady_clock::now()) {}
  void mark(const char *what) {
    if (!on && !sink) return;
    const auto t1 = std::chrono::steady_clock::now();
    const double dt = std::chrono::duration<double>(t1 - t0).count();
    if (sink) sink->emplace_back(what, dt);
    if (on) std::fprintf(stderr, "[eamg] %-28s %8.3f s\n", what, dt);
    t0 = t1;
  }
};

// Parallel loop with dynamic chunks, for iterations of uneven cost.
template <class F>
void parallel_for_dynamic(int64_t n, F &&f, int64_t chunk = 64) {
  unsigned nt = std::thread::hardware_concurrency();
  nt = std::max(1u, std::min(nt, 16u));
  if (n < 2 * chunk || nt == 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&] {
      for (int64_t lo = next.fetch_add(chunk); lo < n; lo = next.fetch_add(chunk))
        for (int64_t i = lo; i < std::min(n, lo + chunk); ++i) f(i);
    });
  for (auto &x : th) x.join();
}

// Features of the candidate pairs of one matching pass (kPairFeatures per pair), for the
// learned walk and for training: pairs (i, j) of working-level vertices, the graph's node count,
// labels y (1: the exact criterion accepts) and weights w (1: the pair was evaluated).
constexpr int kPairFeatures = 12;
struct PassSamples {
  int n = 0;
  std::vector<int32_t> edges;   // 2 per pair
  std::vector<float> X;         // kPairFeatures per pair
  std::vector<float> y, w;
};

// Scores the candidate pairs of a pass: logits (one per pair) of "the exact criterion accepts".
using PairScorer = std::function<void(const PassSamples &, std::vector<float> &)>;

struct AuxLevel;

// Allocator that leaves new elements uninitialized on resize(), so that a large weight array is
// not written twice: every writer of an AuxLevel's E and M fills all their entries.
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U> &) {}
  template <class U>
  void construct(U *p) noexcept {
    ::new (static_cast<void *>(p)) U;
  }
  template <class U, class... Args>
  void construct(U *p, Args &&...args) {
    ::new (static_cast<void *>(p)) U(std::forward<Args>(args)...);
  }
};
using WeightVec = std::vector<double, NoInitAlloc<double>>;

// Batched evaluation of the exact criteria of a matching pass on another processor (the device
// implementation is in criteria.hip).  level(): the level being coarsened and its D-hat blocks
// (the data of mu_g); work(): the working level of the current pass and its D-hat blocks (the
// data of mu_b; may be the same objects as level()).  Both stay referenced until the next call.
// mu_b(): one value per pair (i, j) of working-level vertices (2 ints per pair).  mu_g(): one
// value per union of up to crit::kMaxUnion level vertices (ascending, padded with -1); NaN where
// the union could not be evaluated there (the caller evaluates it itself).  Values are those of
// the host criteria bit for bit.
struct CritBatch {
  virtual ~CritBatch() = default;
  virtual void level(const AuxLevel &lev, const std::vector<Sq> &D) = 0;
  virtual void work(const AuxLevel &w, const std::vector<Sq> &D) = 0;
  virtual void mu_b(const std::vector<int32_t> &pairs, double tau, std::vector<double> &out) = 0;
  virtual void mu_g(const std::vector<int32_t> &unions, double tau, std::vector<double> &out) = 0;
  // Weights of the coarse level (Thm thm:cemats) from the fine level `fine`, which must be the
  // object last handed to level() or work(); else false and nothing is computed.  aggs: sorted
  // members per aggregate; order / start: the fine edges of coarse edge g are order[start[g] ..
  // start[g + 1]) (ascending), summed in that order.  M: nc*k*k, E: (start.size() - 1)*k*k.
  virtual bool coarse_weights(const AuxLevel &fine, const std::vector<std::vector<int>> &aggs,
                              const std::vector<int> &agg_of, const std::vector<char> &dmask,
                              const std::vector<double> &cc, const std::vector<int64_t> &order,
                              const std::vector<int64_t> &start, WeightVec &M,
                              WeightVec &E) = 0;
};

struct MatchParams {
  double sigma = 20.0;
  int rounds = 2;
  double tie_rtol = 1e-12;
  double tau = 1e-10;
  // learned walk: candidates scored below `skip` (probability) are passed over without
  // evaluating the criteria; a vertex whose candidates were all passed over evaluates its best
  // scored one.  Every pair formed is accepted by the exact criteria.
  PairScorer scorer;
  double skip = 0.0;
  bool record = false;   // keep every pass's candidate pairs, features and labels
  // pair the candidate of smallest mu_s without evaluating mu_b / mu_g (the scalar-only
  // coarsening the paper contrasts the robust criteria with)
  bool mu_s_only = false;
  // evaluate the walks' unknown pairs through this batch evaluator instead of host threads:
  // batches of at least batch_min_pairs pairs (mu_b) and batch_min_unions unions (mu_g); smaller
  // ones, whose cost is the evaluator's latency rather than its throughput, stay on host threads
  CritBatch *batch = nullptr;
  int batch_min_pairs = 1, batch_min_unions = 1;
};

struct AuxLevel {
  int n = 0, k = 6;
  std::vector<double> x;          // n*3 positions
  std::vector<int> e0, e1;        // edges, e0 < e1, ascending (e0, e1)
  WeightVec E;                    // m*k*k
  WeightVec M;                    // n*k*k
  std::vector<int64_t> nb_ptr;    // adjacency sorted by neighbour id
  std::vector<int> nb, nb_e;

  int64_t m() const { return int64_t(e0.size()); }
  LevelView view() const {
    LevelView v;
    v.n = n;
    v.k = k;
    v.x = x.data();
    v.E = E.data();
    v.M = M.data();
    v.nb_ptr = nb_ptr.data();
    v.nb = nb.data();
    v.nb_e = nb_e.data();
    return v;
  }
  void build_adjacency();
  int edge_id(int i, int j) const;   // -1 if absent
  Sq Emat(int64_t e) const;
  Sq Mmat(int i) const;
  const double *xp(int i) const { return &x[size_t(3) * i]; }
};

struct MatchResult {
  std::vector<std::vector<int>> aggs;   // sorted members, coarse id = position
  std::vector<char> dmask;              // dropped set D
  std::vector<double> ccoords;          // nc*3
  AuxLevel coarse;
  double min_margin = 1e300;
  int max_tie = 0;
  // criteria evaluations the walk made (mu_b; mu_g among them) and candidates it passed over
  int64_t evaluated = 0, evaluated_g = 0, skipped = 0;
  std::vector<PassSamples> samples;
};

// Build the finest level.  Returns false with err set on malformed input.
bool finest_aux(int dim, int n, const double *coords, const int32_t *row_ptr, const int32_t *col,
                const double *vals, const int32_t *edges, int64_t n_edges, AuxLevel &out,
                std::string &err);

// dev: optional evaluator holding `lev` on the device, which then computes the weights
AuxLevel coarse_aux(const AuxLevel &lev, const std::vector<std::vector<int>> &aggs,
                    const std::vector<char> &dmask, const std::vector<double> &ccoords,
                    CritBatch *dev = nullptr);

void dhat_all(const AuxLevel &lev, std::vector<Sq> &D);
void trace_strength(const AuxLevel &lev, std::vector<double> &m);
double mu_D(const AuxLevel &lev, int i, const std::vector<Sq> &D, double tau);
double mu_s(const AuxLevel &lev, int i, int j, const std::vector<double> &mtr);
double mu_b(const AuxLevel &lev, int i, int j, const std::vector<Sq> &D, double tau);
double mu_g(const AuxLevel &lev, const std::vector<int> &C, const std::vector<Sq> &D, double tau);

std::vector<int> cuthill_mckee(const AuxLevel &lev, const std::vector<char> &free_mask);

MatchResult successive_matching(const AuxLevel &lev, const std::vector<char> &vd,
                                const MatchParams &prm);

}  // namespace eamg
