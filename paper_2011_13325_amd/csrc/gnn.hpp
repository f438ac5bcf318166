// Edge-scoring network for learned pairwise aggregation: device kernels (gnn.hip).
//
// Network (F inputs, H = 64 hidden):
//   a1 = W1 x_e + b1, h1 = relu(a1)                       edge layer
//   m_i = mean over candidate edges e at node i of h1_e     one round of message passing
//   a2 = W2a h1_e + W2b (m_u + m_v) + b2, h2 = relu(a2)
//   z_e = w3 . h2 + b3                                     logit of "the exact criterion accepts"
// W1, W2a, W2b, w3 are used rounded to bfloat16 (round to nearest even); biases, activations
// and every sum are FP32.  Loss: weighted mean binary cross-entropy on the logits.  All
// reductions run in a fixed order (node sums over an incidence list in ascending edge order,
// weight gradients over fixed edge chunks then over chunks in order), so results are bitwise
// reproducible.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eamg {

constexpr int kGnnF = 12;
constexpr int kGnnH = 64;
// packed parameter layout: W1 (H x F), b1 (H), W2a (H x H), W2b (H x H), b2 (H), w3 (H), b3 (1)
constexpr int kGnnOffW1 = 0;
constexpr int kGnnOffB1 = kGnnOffW1 + kGnnH * kGnnF;
constexpr int kGnnOffW2a = kGnnOffB1 + kGnnH;
constexpr int kGnnOffW2b = kGnnOffW2a + kGnnH * kGnnH;
constexpr int kGnnOffB2 = kGnnOffW2b + kGnnH * kGnnH;
constexpr int kGnnOffW3 = kGnnOffB2 + kGnnH;
constexpr int kGnnOffB3 = kGnnOffW3 + kGnnH;
constexpr int kGnnParams = kGnnOffB3 + 1;

// Device buffers of one graph: m candidate edges over n nodes.
struct GnnGraph {
  int64_t m = 0;
  int n = 0;
  const float *X = nullptr;        // m x F
  const int *eu = nullptr, *ev = nullptr;   // edge ends
  const int *inc_ptr = nullptr;    // n + 1: incidence lists (edges at each node, ascending)
  const int *inc = nullptr;        // 2m
  const float *y = nullptr;        // labels (training)
  const float *w = nullptr;        // sample weights (training; 0 = unlabelled)
};

// Activations kept for the backward pass (m x H each, n x H for node means).
struct GnnWork {
  float *a1 = nullptr, *a2 = nullptr, *node = nullptr, *z = nullptr;
  float *d1 = nullptr, *d2 = nullptr, *dnode = nullptr, *ds = nullptr;
  float *part = nullptr;           // weight-gradient partials: chunks x kGnnParams
  float *lpart = nullptr;          // loss partials
  int chunks = 0;
};

int gnn_chunks(int64_t m);
// used = master with W1, W2a, W2b, w3 rounded to bfloat16
hipError_t launch_gnn_round(const float *master, float *used, hipStream_t s);
// forward: a1, node means, a2, z
hipError_t launch_gnn_forward(const float *used, const GnnGraph &g, GnnWork &wk, hipStream_t s);
// backward of the weighted mean BCE (wsum = sum of w), gradient into grad (kGnnParams), loss into
// *loss_dev
hipError_t launch_gnn_backward(const float *used, const GnnGraph &g, GnnWork &wk, float wsum,
                               float *grad, float *loss_dev, hipStream_t s);
// Adam step t (1-based) on the masters
hipError_t launch_gnn_adam(float *master, float *mom1, float *mom2, const float *grad, float lr,
                           int t, hipStream_t s);

}  // namespace eamg
