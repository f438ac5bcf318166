// Host side of the edge-scoring network shared by the C ABI (gnn_api.cpp) and the learned
// matching walk (api.cpp): a graph uploaded to the device with its incidence lists, and the
// logits of its edges.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "gnn.hpp"
#include "hierarchy.hpp"

struct eamg_gnn;

namespace eamg {

// m candidate edges over n nodes: features X (m x kGnnF), ends edges (m x 2); labels y and
// weights w (both m, or both NULL for inference).  Owns its device buffers.
struct DeviceGraph {
  DevArena arena;
  GnnGraph g;
  GnnWork wk;
  int64_t m = 0;
  int n = 0;
  double wsum = 0.0;
  DeviceGraph(int64_t m, int n, const float *X, const int32_t *edges, const float *y,
              const float *w, hipStream_t s);
};

// Logits of every edge of dg with the network's current parameters.
void gnn_logits(eamg_gnn *net, DeviceGraph &dg, hipStream_t s, std::vector<float> &z);

}  // namespace eamg
