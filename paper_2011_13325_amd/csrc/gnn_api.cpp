// C ABI of the edge-scoring network (include/eamg.h: eamg_gnn_*): parameters on the device,
// graphs uploaded from host arrays, forward / gradient / Adam training on the GPU (gnn.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <memory>
#include <vector>

#include "gnn.hpp"
#include "gnn_host.hpp"
#include "hierarchy.hpp"

struct eamg_gnn {
  eamg::DevArena arena;
  float *master = nullptr, *used = nullptr, *m1 = nullptr, *m2 = nullptr, *grad = nullptr;
  float *loss = nullptr;
  int steps = 0;   // Adam steps taken
};

namespace eamg {

namespace {

// splitmix64: a counter-based generator for the initial weights
uint64_t splitmix(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

std::vector<float> init_params(uint64_t seed) {
  std::vector<float> p(size_t(kGnnParams), 0.0f);
  uint64_t s = seed;
  auto uni = [&](double lim) { return float((double(splitmix(s) >> 11) * 0x1.0p-53 * 2.0 - 1.0) * lim); };
  for (int j = kGnnOffW1; j < kGnnOffB1; ++j) p[j] = uni(std::sqrt(6.0 / kGnnF));
  for (int j = kGnnOffW2a; j < kGnnOffB2; ++j) p[j] = uni(std::sqrt(6.0 / kGnnH));
  for (int j = kGnnOffW3; j < kGnnOffB3; ++j) p[j] = uni(std::sqrt(6.0 / kGnnH));
  return p;
}

}  // namespace

DeviceGraph::DeviceGraph(int64_t m_, int n_, const float *X, const int32_t *edges, const float *y,
                         const float *w, hipStream_t s) {
  m = m_;
  n = n_;
  const size_t ms = static_cast<size_t>(m), ns = static_cast<size_t>(n);
  std::vector<int> eu(ms), ev(ms), ptr(ns + 1, 0), inc(2 * ms);
  for (int64_t e = 0; e < m; ++e) {
    eu[e] = edges[2 * e];
    ev[e] = edges[2 * e + 1];
    if (eu[e] < 0 || eu[e] >= n || ev[e] < 0 || ev[e] >= n || eu[e] == ev[e])
      fail(EAMG_ERR_INVALID_ARG, "edge ends must be distinct nodes in [0, n)");
    ++ptr[eu[e] + 1];
    ++ptr[ev[e] + 1];
  }
  for (int i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
  std::vector<int> fill(ptr.begin(), ptr.end() - 1);
  for (int64_t e = 0; e < m; ++e) {   // ascending edge order within each node
    inc[fill[eu[e]]++] = int(e);
    inc[fill[ev[e]]++] = int(e);
  }
  for (int64_t q = 0; q < m * kGnnF; ++q)
    if (!std::isfinite(X[q])) fail(EAMG_ERR_INVALID_ARG, "features must be finite");
  g.m = m;
  g.n = n;
  g.X = arena.upload(X, size_t(m) * kGnnF, s);
  g.eu = arena.upload(eu, s);
  g.ev = arena.upload(ev, s);
  g.inc_ptr = arena.upload(ptr, s);
  g.inc = arena.upload(inc, s);
  if (y) {
    g.y = arena.upload(y, size_t(m), s);
    g.w = arena.upload(w, size_t(m), s);
    wsum = 0.0;
    for (int64_t e = 0; e < m; ++e) wsum += w[e];
  }
  wk.a1 = arena.alloc<float>(size_t(m) * kGnnH);
  wk.a2 = arena.alloc<float>(size_t(m) * kGnnH);
  wk.node = arena.alloc<float>(size_t(n) * kGnnH);
  wk.z = arena.alloc<float>(size_t(2 * m));
  if (y) {
    wk.d1 = arena.alloc<float>(size_t(m) * kGnnH);
    wk.d2 = arena.alloc<float>(size_t(m) * kGnnH);
    wk.ds = arena.alloc<float>(size_t(m) * kGnnH);
    wk.dnode = arena.alloc<float>(size_t(n) * kGnnH);
    wk.chunks = gnn_chunks(m);
    wk.part = arena.alloc<float>(size_t(wk.chunks) * kGnnParams);
    wk.lpart = arena.alloc<float>(size_t((m + 255) / 256));
  }
}

void gnn_logits(eamg_gnn *net, DeviceGraph &dg, hipStream_t s, std::vector<float> &z) {
  hip_check(launch_gnn_round(net->master, net->used, s), "gnn_round");
  hip_check(launch_gnn_forward(net->used, dg.g, dg.wk, s), "gnn_forward");
  z.resize(size_t(dg.m));
  if (dg.m)
    hip_check(hipMemcpyAsync(z.data(), dg.wk.z, sizeof(float) * size_t(dg.m), hipMemcpyDeviceToHost, s),
              "download");
  hip_check(hipStreamSynchronize(s), "sync");
}

}  // namespace eamg

using namespace eamg;

namespace {

void check_graph_args(int64_t m, int32_t n, const float *X, const int32_t *edges) {
  if (m < 1 || n < 2) fail(EAMG_ERR_INVALID_ARG, "need m >= 1 edges over n >= 2 nodes");
  if (!X || !edges) fail(EAMG_ERR_INVALID_ARG, "NULL features or edges");
}

}  // namespace

extern "C" {

eamg_status eamg_gnn_create(const float *params, uint64_t seed, eamg_gnn **out) {
  return guarded([&] {
    if (!out) fail(EAMG_ERR_INVALID_ARG, "NULL out");
    *out = nullptr;
    auto net = std::make_unique<eamg_gnn>();
    std::vector<float> p = params ? std::vector<float>(params, params + kGnnParams) : init_params(seed);
    for (float v : p)
      if (!std::isfinite(v)) fail(EAMG_ERR_INVALID_ARG, "parameters must be finite");
    hipStream_t s = nullptr;
    net->master = net->arena.upload(p, s);
    net->used = net->arena.alloc<float>(kGnnParams);
    std::vector<float> zero(size_t(kGnnParams), 0.0f);
    net->m1 = net->arena.upload(zero, s);
    net->m2 = net->arena.upload(zero, s);
    net->grad = net->arena.alloc<float>(kGnnParams);
    net->loss = net->arena.alloc<float>(1);
    *out = net.release();
  });
}

eamg_status eamg_gnn_params(const eamg_gnn *g, float *params) {
  return guarded([&] {
    if (!g || !params) fail(EAMG_ERR_INVALID_ARG, "NULL argument");
    const auto v = download(g->master, size_t(kGnnParams), nullptr);
    std::copy(v.begin(), v.end(), params);
  });
}

eamg_status eamg_gnn_forward(eamg_gnn *g, int64_t m, int32_t n, const float *X, const int32_t *edges,
                             float *logits) {
  return guarded([&] {
    if (!g || !logits) fail(EAMG_ERR_INVALID_ARG, "NULL argument");
    check_graph_args(m, n, X, edges);
    hipStream_t s = nullptr;
    DeviceGraph dg(m, n, X, edges, nullptr, nullptr, s);
    std::vector<float> z;
    gnn_logits(g, dg, s, z);
    std::copy(z.begin(), z.end(), logits);
  });
}

eamg_status eamg_gnn_loss_grad(eamg_gnn *g, int64_t m, int32_t n, const float *X,
                               const int32_t *edges, const float *y, const float *w, double *loss,
                               float *grad) {
  return guarded([&] {
    if (!g || !y || !w) fail(EAMG_ERR_INVALID_ARG, "NULL argument");
    check_graph_args(m, n, X, edges);
    hipStream_t s = nullptr;
    DeviceGraph dg(m, n, X, edges, y, w, s);
    if (!(dg.wsum > 0.0)) fail(EAMG_ERR_INVALID_ARG, "sample weights must sum to > 0");
    hip_check(launch_gnn_round(g->master, g->used, s), "gnn_round");
    hip_check(launch_gnn_forward(g->used, dg.g, dg.wk, s), "gnn_forward");
    hip_check(launch_gnn_backward(g->used, dg.g, dg.wk, float(dg.wsum), g->grad, g->loss, s), "gnn_backward");
    if (grad) {
      const auto v = download(g->grad, size_t(kGnnParams), s);
      std::copy(v.begin(), v.end(), grad);
    }
    if (loss) *loss = double(download(g->loss, 1, s)[0]);
  });
}

eamg_status eamg_gnn_train(eamg_gnn *g, int32_t ngraphs, const int64_t *m, const int32_t *n,
                           const float *const *X, const int32_t *const *edges,
                           const float *const *y, const float *const *w, int32_t epochs, float lr,
                           float *loss_history) {
  return guarded([&] {
    if (!g || ngraphs < 1 || !m || !n || !X || !edges || !y || !w)
      fail(EAMG_ERR_INVALID_ARG, "NULL argument or ngraphs < 1");
    if (epochs < 1 || !(lr > 0.0f)) fail(EAMG_ERR_INVALID_ARG, "need epochs >= 1 and lr > 0");
    hipStream_t s = nullptr;
    std::vector<std::unique_ptr<DeviceGraph>> gs;
    for (int k = 0; k < ngraphs; ++k) {
      check_graph_args(m[k], n[k], X[k], edges[k]);
      if (!y[k] || !w[k]) fail(EAMG_ERR_INVALID_ARG, "NULL labels or weights");
      gs.emplace_back(std::make_unique<DeviceGraph>(m[k], n[k], X[k], edges[k], y[k], w[k], s));
      if (!(gs.back()->wsum > 0.0)) fail(EAMG_ERR_INVALID_ARG, "sample weights must sum to > 0");
    }
    for (int ep = 0; ep < epochs; ++ep) {
      double lsum = 0.0;
      for (auto &dg : gs) {
        hip_check(launch_gnn_round(g->master, g->used, s), "gnn_round");
        hip_check(launch_gnn_forward(g->used, dg->g, dg->wk, s), "gnn_forward");
        hip_check(launch_gnn_backward(g->used, dg->g, dg->wk, float(dg->wsum), g->grad, g->loss, s),
                  "gnn_backward");
        hip_check(launch_gnn_adam(g->master, g->m1, g->m2, g->grad, lr, ++g->steps, s), "gnn_adam");
        if (loss_history) lsum += double(download(g->loss, 1, s)[0]);
      }
      if (loss_history) loss_history[ep] = float(lsum / ngraphs);
    }
    hip_check(hipStreamSynchronize(s), "sync");
  });
}

void eamg_gnn_destroy(eamg_gnn *g) { delete g; }

}  // extern "C"
