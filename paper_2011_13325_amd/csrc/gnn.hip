// Edge-scoring network kernels for gfx950 (layout and network in gnn.hpp).
#include <hip/hip_runtime.h>

#include <cmath>

#include "gnn.hpp"

namespace eamg {
namespace {

constexpr int kT = 256;          // threads per workgroup
constexpr int kEdgesPW = kT / kGnnH;   // edges per workgroup step (one wavefront per edge)
constexpr int kChunk = 2048;     // edges per weight-gradient partial
constexpr int kTile = 32;        // edges staged in LDS by the weight-gradient kernel

inline unsigned grid_of(int64_t items, int per) { return unsigned((items + per - 1) / per); }

__device__ inline float bf16_round(float x) {
  if (isnan(x)) return x;
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

__device__ inline bool is_bf16_param(int j) {
  return (j >= kGnnOffW1 && j < kGnnOffB1) || (j >= kGnnOffW2a && j < kGnnOffB2) ||
         (j >= kGnnOffW3 && j < kGnnOffB3);
}

__global__ void k_gnn_round(const float *master, float *used) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < kGnnParams) used[j] = is_bf16_param(j) ? bf16_round(master[j]) : master[j];
}

__device__ inline float relu(float v) { return v > 0.0f ? v : 0.0f; }

// a1[e, h] = b1[h] + W1[h, :] . x_e
__global__ __launch_bounds__(kT) void k_gnn_l1(int64_t m, const float *__restrict__ P,
                                               const float *__restrict__ X, float *__restrict__ a1) {
  const int h = threadIdx.x & (kGnnH - 1);
  const int64_t e = int64_t(blockIdx.x) * kEdgesPW + threadIdx.x / kGnnH;
  if (e >= m) return;
  float acc = P[kGnnOffB1 + h];
#pragma unroll
  for (int f = 0; f < kGnnF; ++f) acc = fmaf(P[kGnnOffW1 + h * kGnnF + f], X[e * kGnnF + f], acc);
  a1[e * kGnnH + h] = acc;
}

// node[i, h] = mean over incident edges of relu(a1[e, h]) (ascending edge order)
__global__ __launch_bounds__(kT) void k_gnn_agg(int n, const int *__restrict__ ptr,
                                                const int *__restrict__ inc,
                                                const float *__restrict__ a1, float *__restrict__ node) {
  const int h = threadIdx.x & (kGnnH - 1);
  const int i = blockIdx.x * kEdgesPW + threadIdx.x / kGnnH;
  if (i >= n) return;
  const int p0 = ptr[i], p1 = ptr[i + 1];
  float s = 0.0f;
  for (int p = p0; p < p1; ++p) s += relu(a1[int64_t(inc[p]) * kGnnH + h]);
  node[int64_t(i) * kGnnH + h] = p1 > p0 ? s / float(p1 - p0) : 0.0f;
}

// Butterfly sum over the 64 lanes of a wavefront (fixed order); every lane gets the total.
__device__ inline float wave_sum(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// a2 = W2a h1 + W2b (m_u + m_v) + b2 ; z = w3 . relu(a2) + b3.  W2a^T, W2b^T staged in LDS.
__global__ __launch_bounds__(kT) void k_gnn_l2(int64_t m, const float *__restrict__ P,
                                               const int *__restrict__ eu, const int *__restrict__ ev,
                                               const float *__restrict__ a1,
                                               const float *__restrict__ node, float *__restrict__ a2,
                                               float *__restrict__ z) {
  __shared__ float Wa[kGnnH * kGnnH], Wb[kGnnH * kGnnH];
  __shared__ float vin[kEdgesPW][2 * kGnnH];
  for (int j = threadIdx.x; j < kGnnH * kGnnH; j += kT) {
    const int h = j / kGnnH, k = j % kGnnH;   // element (h, k) of W2a / W2b
    Wa[k * kGnnH + h] = P[kGnnOffW2a + j];
    Wb[k * kGnnH + h] = P[kGnnOffW2b + j];
  }
  __syncthreads();
  const int h = threadIdx.x & (kGnnH - 1);
  const int wv = threadIdx.x / kGnnH;
  const float b2 = P[kGnnOffB2 + h], w3 = P[kGnnOffW3 + h], b3 = P[kGnnOffB3];
  for (int64_t base = int64_t(blockIdx.x) * kEdgesPW; base < m; base += int64_t(gridDim.x) * kEdgesPW) {
    const int64_t e = base + wv;
    const bool valid = e < m;   // uniform per wavefront
    if (valid) {
      vin[wv][h] = relu(a1[e * kGnnH + h]);
      vin[wv][kGnnH + h] = node[int64_t(eu[e]) * kGnnH + h] + node[int64_t(ev[e]) * kGnnH + h];
    }
    __syncthreads();
    if (valid) {
      float acc = b2;
#pragma unroll 8
      for (int k = 0; k < kGnnH; ++k) acc = fmaf(Wa[k * kGnnH + h], vin[wv][k], acc);
#pragma unroll 8
      for (int k = 0; k < kGnnH; ++k) acc = fmaf(Wb[k * kGnnH + h], vin[wv][kGnnH + k], acc);
      a2[e * kGnnH + h] = acc;
      const float t = wave_sum(w3 * relu(acc));
      if (h == 0) z[e] = t + b3;
    }
    __syncthreads();
  }
}

// dz = w (sigmoid(z) - y) / wsum, loss partials per workgroup
__global__ __launch_bounds__(kT) void k_gnn_dz(int64_t m, const float *__restrict__ z,
                                               const float *__restrict__ y, const float *__restrict__ w,
                                               float inv_wsum, float *__restrict__ dz,
                                               float *__restrict__ lpart) {
  __shared__ float sh[kT];
  const int64_t e = int64_t(blockIdx.x) * kT + threadIdx.x;
  float l = 0.0f;
  if (e < m) {
    const float zz = z[e], yy = y[e], ww = w[e] * inv_wsum;
    const float sp = log1pf(expf(-fabsf(zz))) + relu(zz);   // softplus(z)
    l = ww * (sp - yy * zz);
    dz[e] = ww * (1.0f / (1.0f + expf(-zz)) - yy);
  }
  sh[threadIdx.x] = l;
  __syncthreads();
  for (int st = kT / 2; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = sh[0];
}

// da2 = dz w3 [a2 > 0] (stored over a2's slot in d2); d1 = W2a^T da2 (direct part of dh1);
// ds = W2b^T da2
__global__ __launch_bounds__(kT) void k_gnn_b2(int64_t m, const float *__restrict__ P,
                                               const float *__restrict__ a2, const float *__restrict__ dz,
                                               float *__restrict__ d2, float *__restrict__ d1,
                                               float *__restrict__ ds) {
  __shared__ float Wa[kGnnH * kGnnH], Wb[kGnnH * kGnnH];
  __shared__ float g[kEdgesPW][kGnnH];
  for (int j = threadIdx.x; j < kGnnH * kGnnH; j += kT) {
    Wa[j] = P[kGnnOffW2a + j];   // (h, k) at h * H + k: lane k reads a row-contiguous column
    Wb[j] = P[kGnnOffW2b + j];
  }
  __syncthreads();
  const int k = threadIdx.x & (kGnnH - 1);
  const int wv = threadIdx.x / kGnnH;
  const float w3k = P[kGnnOffW3 + k];
  for (int64_t base = int64_t(blockIdx.x) * kEdgesPW; base < m; base += int64_t(gridDim.x) * kEdgesPW) {
    const int64_t e = base + wv;
    const bool valid = e < m;
    if (valid) {
      const float v = a2[e * kGnnH + k] > 0.0f ? dz[e] * w3k : 0.0f;   // lane k holds da2[k]
      g[wv][k] = v;
      d2[e * kGnnH + k] = v;
    }
    __syncthreads();
    if (valid) {
      float s1 = 0.0f, s2 = 0.0f;
#pragma unroll 8
      for (int hh = 0; hh < kGnnH; ++hh) {
        s1 = fmaf(Wa[hh * kGnnH + k], g[wv][hh], s1);
        s2 = fmaf(Wb[hh * kGnnH + k], g[wv][hh], s2);
      }
      d1[e * kGnnH + k] = s1;
      ds[e * kGnnH + k] = s2;
    }
    __syncthreads();
  }
}

// dnode[i, k] = (sum over incident edges of ds[e, k]) / deg_i
__global__ __launch_bounds__(kT) void k_gnn_bagg(int n, const int *__restrict__ ptr,
                                                 const int *__restrict__ inc,
                                                 const float *__restrict__ ds, float *__restrict__ dnode) {
  const int k = threadIdx.x & (kGnnH - 1);
  const int i = blockIdx.x * kEdgesPW + threadIdx.x / kGnnH;
  if (i >= n) return;
  const int p0 = ptr[i], p1 = ptr[i + 1];
  float s = 0.0f;
  for (int p = p0; p < p1; ++p) s += ds[int64_t(inc[p]) * kGnnH + k];
  dnode[int64_t(i) * kGnnH + k] = p1 > p0 ? s / float(p1 - p0) : 0.0f;
}

// da1 = (d1 + dnode[u] + dnode[v]) [a1 > 0], in place over d1
__global__ __launch_bounds__(kT) void k_gnn_b1(int64_t m, const int *__restrict__ eu,
                                               const int *__restrict__ ev, const float *__restrict__ a1,
                                               const float *__restrict__ dnode, float *__restrict__ d1) {
  const int k = threadIdx.x & (kGnnH - 1);
  const int64_t e = int64_t(blockIdx.x) * kEdgesPW + threadIdx.x / kGnnH;
  if (e >= m) return;
  const int64_t q = e * kGnnH + k;
  const float t = d1[q] + dnode[int64_t(eu[e]) * kGnnH + k] + dnode[int64_t(ev[e]) * kGnnH + k];
  d1[q] = a1[q] > 0.0f ? t : 0.0f;
}

// Weight-gradient partials of one chunk of edges: tiles of kTile edges staged in LDS, each
// thread summing its parameters over the tile in edge order.
__global__ __launch_bounds__(kT) void k_gnn_wgrad(int64_t m, const float *__restrict__ X,
                                                  const int *__restrict__ eu, const int *__restrict__ ev,
                                                  const float *__restrict__ a1, const float *__restrict__ a2,
                                                  const float *__restrict__ node,
                                                  const float *__restrict__ da1,
                                                  const float *__restrict__ da2,
                                                  const float *__restrict__ dz, float *__restrict__ part) {
  __shared__ float sx[kTile][kGnnF], sh1[kTile][kGnnH], ss[kTile][kGnnH], sh2[kTile][kGnnH];
  __shared__ float sd1[kTile][kGnnH], sd2[kTile][kGnnH], sdz[kTile];
  constexpr int kPer = (kGnnParams + kT - 1) / kT;
  float acc[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) acc[q] = 0.0f;
  const int64_t c0 = int64_t(blockIdx.x) * kChunk;
  const int64_t c1 = c0 + kChunk < m ? c0 + kChunk : m;
  for (int64_t t0 = c0; t0 < c1; t0 += kTile) {
    const int nt = int(c1 - t0 < kTile ? c1 - t0 : kTile);
    for (int j = threadIdx.x; j < kTile * kGnnH; j += kT) {
      const int r = j / kGnnH, k = j % kGnnH;
      if (r < nt) {
        const int64_t e = t0 + r, q = e * kGnnH + k;
        sh1[r][k] = relu(a1[q]);
        sh2[r][k] = relu(a2[q]);
        ss[r][k] = node[int64_t(eu[e]) * kGnnH + k] + node[int64_t(ev[e]) * kGnnH + k];
        sd1[r][k] = da1[q];
        sd2[r][k] = da2[q];
      }
    }
    for (int j = threadIdx.x; j < kTile * kGnnF; j += kT) {
      const int r = j / kGnnF, f = j % kGnnF;
      if (r < nt) sx[r][f] = X[(t0 + r) * kGnnF + f];
    }
    if (int(threadIdx.x) < kTile && int(threadIdx.x) < nt) sdz[threadIdx.x] = dz[t0 + threadIdx.x];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int j = int(threadIdx.x) + q * kT;
      if (j >= kGnnParams) break;
      float s = acc[q];
      if (j < kGnnOffB1) {
        const int h = (j - kGnnOffW1) / kGnnF, f = (j - kGnnOffW1) % kGnnF;
        for (int r = 0; r < nt; ++r) s = fmaf(sd1[r][h], sx[r][f], s);
      } else if (j < kGnnOffW2a) {
        const int h = j - kGnnOffB1;
        for (int r = 0; r < nt; ++r) s += sd1[r][h];
      } else if (j < kGnnOffW2b) {
        const int h = (j - kGnnOffW2a) / kGnnH, k = (j - kGnnOffW2a) % kGnnH;
        for (int r = 0; r < nt; ++r) s = fmaf(sd2[r][h], sh1[r][k], s);
      } else if (j < kGnnOffB2) {
        const int h = (j - kGnnOffW2b) / kGnnH, k = (j - kGnnOffW2b) % kGnnH;
        for (int r = 0; r < nt; ++r) s = fmaf(sd2[r][h], ss[r][k], s);
      } else if (j < kGnnOffW3) {
        const int h = j - kGnnOffB2;
        for (int r = 0; r < nt; ++r) s += sd2[r][h];
      } else if (j < kGnnOffB3) {
        const int h = j - kGnnOffW3;
        for (int r = 0; r < nt; ++r) s = fmaf(sdz[r], sh2[r][h], s);
      } else {
        for (int r = 0; r < nt; ++r) s += sdz[r];
      }
      acc[q] = s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int j = int(threadIdx.x) + q * kT;
    if (j < kGnnParams) part[int64_t(blockIdx.x) * kGnnParams + j] = acc[q];
  }
}

__global__ void k_gnn_wreduce(int chunks, const float *__restrict__ part, float *__restrict__ grad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kGnnParams) return;
  float s = 0.0f;
  for (int c = 0; c < chunks; ++c) s += part[int64_t(c) * kGnnParams + j];
  grad[j] = s;
}

__global__ void k_gnn_lreduce(int n, const float *__restrict__ lpart, float *__restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float s = 0.0f;
  for (int i = 0; i < n; ++i) s += lpart[i];
  *loss = s;
}

__global__ void k_gnn_adam(float *master, float *m1, float *m2, const float *grad, float lr,
                           float c1, float c2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kGnnParams) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float g = grad[j];
  const float u = b1 * m1[j] + (1.0f - b1) * g;
  const float v = b2 * m2[j] + (1.0f - b2) * g * g;
  m1[j] = u;
  m2[j] = v;
  master[j] -= lr * (u / c1) / (sqrtf(v / c2) + eps);
}

}  // namespace

int gnn_chunks(int64_t m) { return int((m + kChunk - 1) / kChunk); }

hipError_t launch_gnn_round(const float *master, float *used, hipStream_t s) {
  hipLaunchKernelGGL(k_gnn_round, dim3(grid_of(kGnnParams, kT)), dim3(kT), 0, s, master, used);
  return hipGetLastError();
}

hipError_t launch_gnn_forward(const float *used, const GnnGraph &g, GnnWork &wk, hipStream_t s) {
  if (g.m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gnn_l1, dim3(grid_of(g.m, kEdgesPW)), dim3(kT), 0, s, g.m, used, g.X, wk.a1);
  hipLaunchKernelGGL(k_gnn_agg, dim3(grid_of(g.n, kEdgesPW)), dim3(kT), 0, s, g.n, g.inc_ptr, g.inc,
                     wk.a1, wk.node);
  const unsigned gl2 = grid_of(g.m, kEdgesPW) < 4096u ? grid_of(g.m, kEdgesPW) : 4096u;
  hipLaunchKernelGGL(k_gnn_l2, dim3(gl2), dim3(kT), 0, s, g.m, used, g.eu, g.ev, wk.a1, wk.node,
                     wk.a2, wk.z);
  return hipGetLastError();
}

hipError_t launch_gnn_backward(const float *used, const GnnGraph &g, GnnWork &wk, float wsum,
                               float *grad, float *loss_dev, hipStream_t s) {
  if (g.m == 0 || !(wsum > 0.0f)) return hipErrorInvalidValue;
  float *dz = wk.z + g.m;   // z buffer holds 2m floats: logits, then dz
  const unsigned gdz = grid_of(g.m, kT);
  hipLaunchKernelGGL(k_gnn_dz, dim3(gdz), dim3(kT), 0, s, g.m, wk.z, g.y, g.w, 1.0f / wsum, dz, wk.lpart);
  const unsigned gb = grid_of(g.m, kEdgesPW) < 4096u ? grid_of(g.m, kEdgesPW) : 4096u;
  hipLaunchKernelGGL(k_gnn_b2, dim3(gb), dim3(kT), 0, s, g.m, used, wk.a2, dz, wk.d2, wk.d1, wk.ds);
  hipLaunchKernelGGL(k_gnn_bagg, dim3(grid_of(g.n, kEdgesPW)), dim3(kT), 0, s, g.n, g.inc_ptr, g.inc,
                     wk.ds, wk.dnode);
  hipLaunchKernelGGL(k_gnn_b1, dim3(grid_of(g.m, kEdgesPW)), dim3(kT), 0, s, g.m, g.eu, g.ev, wk.a1,
                     wk.dnode, wk.d1);
  const int nc = gnn_chunks(g.m);
  hipLaunchKernelGGL(k_gnn_wgrad, dim3(nc), dim3(kT), 0, s, g.m, g.X, g.eu, g.ev, wk.a1, wk.a2, wk.node,
                     wk.d1, wk.d2, dz, wk.part);
  hipLaunchKernelGGL(k_gnn_wreduce, dim3(grid_of(kGnnParams, kT)), dim3(kT), 0, s, nc, wk.part, grad);
  hipLaunchKernelGGL(k_gnn_lreduce, dim3(1), dim3(64), 0, s, int(gdz), wk.lpart, loss_dev);
  return hipGetLastError();
}

hipError_t launch_gnn_adam(float *master, float *mom1, float *mom2, const float *grad, float lr,
                           int t, hipStream_t s) {
  const float c1 = 1.0f - std::pow(0.9f, float(t)), c2 = 1.0f - std::pow(0.999f, float(t));
  hipLaunchKernelGGL(k_gnn_adam, dim3(grid_of(kGnnParams, kT)), dim3(kT), 0, s, master, mom1, mom2,
                     grad, lr, c1, c2);
  return hipGetLastError();
}

}  // namespace eamg
