// C ABI of libeamg (include/eamg.h): input validation, the setup driver (host coarsening and
// sparse structure, device numerics), the PCG / V-cycle drivers, statistics and export.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <future>
#include <memory>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/eamg.h"
#include "coarsen.hpp"
#include "criteria.hpp"
#include "dense.hpp"
#include "gnn_host.hpp"
#include "hierarchy.hpp"
#include "kernels.hpp"
#include "structure.hpp"

namespace eamg {

thread_local std::string g_last_error;

namespace {

eamg_setup_params defaults() {
  eamg_setup_params p;
  p.sigma = 20.0;
  p.delta = 1;
  p.R = 1;
  p.rounds = 2;
  p.coarsest_max_dofs = 500;
  p.max_levels = 25;
  p.omega = 2.0 / 3.0;
  p.cap_aux = 4;
  p.cap_std_l0 = 8;
  p.cap_std = 6;
  p.pinv_rtol = 1e-10;
  p.tie_rtol = 1e-12;
  p.vcycle_fp32 = 0;
  p.gnn = nullptr;
  p.gnn_skip = 0.0;
  p.gnn_record = 0;
  p.mu_s_only = 0;
  p.gpu_criteria = 1;
  p.dense_tail_dofs = 0;
  p.dense_tail_fp32 = 0;
  return p;
}

void validate_params(const eamg_setup_params &p) {
  if (!(p.sigma > 0.0) || !std::isfinite(p.sigma)) fail(EAMG_ERR_INVALID_ARG, "sigma must be positive");
  if (p.delta != 1) fail(EAMG_ERR_INVALID_ARG, "only delta = 1 is supported");
  if (p.R != 1) fail(EAMG_ERR_INVALID_ARG, "only R = 1 (mu_s candidate choice) is supported");
  if (p.rounds < 1 || p.rounds > 4) fail(EAMG_ERR_INVALID_ARG, "rounds must be in 1..4");
  if (p.coarsest_max_dofs < 1 || p.coarsest_max_dofs > kMaxCoarsestDofs)
    fail(EAMG_ERR_INVALID_ARG, "coarsest_max_dofs must be in 1.." + std::to_string(kMaxCoarsestDofs));
  if (p.max_levels < 1 || p.max_levels > 64) fail(EAMG_ERR_INVALID_ARG, "max_levels must be in 1..64");
  if (!std::isfinite(p.omega)) fail(EAMG_ERR_INVALID_ARG, "omega must be finite");
  if (p.cap_aux < 1 || p.cap_aux > 16 || p.cap_std_l0 < 1 || p.cap_std_l0 > 16 || p.cap_std < 1 ||
      p.cap_std > 16)
    fail(EAMG_ERR_INVALID_ARG, "row caps must be in 1..16");
  if (!(p.pinv_rtol > 0.0 && p.pinv_rtol <= 1e-2)) fail(EAMG_ERR_INVALID_ARG, "pinv_rtol must be in (0, 1e-2]");
  if (!(p.tie_rtol >= 0.0 && p.tie_rtol <= 1e-6)) fail(EAMG_ERR_INVALID_ARG, "tie_rtol must be in [0, 1e-6]");
  if (p.vcycle_fp32 != 0 && p.vcycle_fp32 != 1) fail(EAMG_ERR_INVALID_ARG, "vcycle_fp32 must be 0 or 1");
  if (!(p.gnn_skip >= 0.0 && p.gnn_skip < 1.0)) fail(EAMG_ERR_INVALID_ARG, "gnn_skip must be in [0, 1)");
  if (p.gnn_record != 0 && p.gnn_record != 1) fail(EAMG_ERR_INVALID_ARG, "gnn_record must be 0 or 1");
  if (p.mu_s_only != 0 && p.mu_s_only != 1) fail(EAMG_ERR_INVALID_ARG, "mu_s_only must be 0 or 1");
  if (p.gpu_criteria < 0 || p.gpu_criteria > 2)
    fail(EAMG_ERR_INVALID_ARG, "gpu_criteria must be 0, 1 or 2");
  if (p.dense_tail_dofs < 0 || p.dense_tail_dofs > kMaxCoarsestDofs)
    fail(EAMG_ERR_INVALID_ARG, "dense_tail_dofs must be in [0, 16384]");
  if (p.dense_tail_fp32 != 0 && p.dense_tail_fp32 != 1)
    fail(EAMG_ERR_INVALID_ARG, "dense_tail_fp32 must be 0 or 1");
  if (p.dense_tail_fp32 && !p.vcycle_fp32) fail(EAMG_ERR_INVALID_ARG, "dense_tail_fp32 needs vcycle_fp32 = 1");
}

void validate_problem(const eamg_problem *pb) {
  if (!pb) fail(EAMG_ERR_INVALID_ARG, "problem is NULL");
  if (pb->dim != 1 && pb->dim != 3) fail(EAMG_ERR_UNSUPPORTED_KERNEL, "dim must be 1 or 3");
  if (pb->k_kernel != (pb->dim == 3 ? 6 : 1))
    fail(EAMG_ERR_UNSUPPORTED_KERNEL, "k_kernel must be 6 (dim 3) or 1 (dim 1)");
  if (pb->n_vertices < 1) fail(EAMG_ERR_INVALID_ARG, "n_vertices must be positive");
  if (!pb->coords || !pb->row_ptr || !pb->col_idx || !pb->vals)
    fail(EAMG_ERR_INVALID_ARG, "coords, row_ptr, col_idx and vals are required");
  const int n = pb->n_vertices;
  if (pb->row_ptr[0] != 0) fail(EAMG_ERR_INVALID_ARG, "row_ptr[0] must be 0");
  for (int i = 0; i < n; ++i)
    if (pb->row_ptr[i + 1] < pb->row_ptr[i]) fail(EAMG_ERR_INVALID_ARG, "row_ptr must be non-decreasing");
  const int64_t nnz = pb->row_ptr[n];
  for (int i = 0; i < n; ++i) {
    bool has_diag = false;
    for (int32_t p = pb->row_ptr[i]; p < pb->row_ptr[i + 1]; ++p) {
      const int j = pb->col_idx[p];
      if (j < 0 || j >= n) fail(EAMG_ERR_INVALID_ARG, "column index out of range in row " + std::to_string(i));
      if (p > pb->row_ptr[i] && pb->col_idx[p - 1] >= j)
        fail(EAMG_ERR_INVALID_ARG, "column indices must be strictly ascending (row " + std::to_string(i) + ")");
      if (j == i) has_diag = true;
    }
    if (!has_diag) fail(EAMG_ERR_INVALID_ARG, "missing diagonal block in row " + std::to_string(i));
  }
  for (int i = 0; i < n; ++i)
    for (int32_t p = pb->row_ptr[i]; p < pb->row_ptr[i + 1]; ++p) {
      const int j = pb->col_idx[p];
      const int32_t *b = pb->col_idx + pb->row_ptr[j], *e = pb->col_idx + pb->row_ptr[j + 1];
      if (!std::binary_search(b, e, i)) fail(EAMG_ERR_INVALID_ARG, "block pattern is not symmetric");
    }
  const int64_t nv = nnz * pb->dim * pb->dim;
  for (int64_t q = 0; q < nv; ++q)
    if (!std::isfinite(pb->vals[q])) fail(EAMG_ERR_INVALID_ARG, "non-finite matrix entry");
  for (int64_t q = 0; q < int64_t(3) * n; ++q)
    if (!std::isfinite(pb->coords[q])) fail(EAMG_ERR_INVALID_ARG, "non-finite coordinate");
  if (pb->edges && pb->n_edges < 0) fail(EAMG_ERR_INVALID_ARG, "n_edges must be >= 0");
  if (pb->kernel) {
    // the given kernel vectors must span the rigid body modes (or the constants)
    const int dim = pb->dim, k = pb->k_kernel;
    const int64_t N = int64_t(n) * dim;
    std::vector<std::vector<double>> Q;   // orthonormalized given vectors
    for (int c = 0; c < k; ++c) {
      std::vector<double> v(pb->kernel + c * N, pb->kernel + (c + 1) * N);
      double nv0 = 0.0;
      for (double a : v) nv0 += a * a;
      for (const auto &u : Q) {
        double d = 0.0;
        for (int64_t t = 0; t < N; ++t) d += u[t] * v[t];
        for (int64_t t = 0; t < N; ++t) v[t] -= d * u[t];
      }
      double nv1 = 0.0;
      for (double a : v) nv1 += a * a;
      if (!(nv1 > 1e-20 * nv0) || !std::isfinite(nv1))
        fail(EAMG_ERR_UNSUPPORTED_KERNEL, "kernel vectors are linearly dependent");
      for (double &a : v) a /= std::sqrt(nv1);
      Q.push_back(std::move(v));
    }
    for (int c = 0; c < k; ++c) {
      std::vector<double> m(size_t(N), 0.0);
      for (int i = 0; i < n; ++i) {
        const double *x = pb->coords + 3 * int64_t(i);
        if (dim == 1) {
          m[i] = 1.0;
        } else if (c < 3) {
          m[3 * int64_t(i) + c] = 1.0;
        } else {
          double e[3] = {0, 0, 0};
          e[c - 3] = 1.0;   // x cross e_m
          m[3 * int64_t(i) + 0] = x[1] * e[2] - x[2] * e[1];
          m[3 * int64_t(i) + 1] = x[2] * e[0] - x[0] * e[2];
          m[3 * int64_t(i) + 2] = x[0] * e[1] - x[1] * e[0];
        }
      }
      double n0 = 0.0;
      for (double a : m) n0 += a * a;
      for (const auto &u : Q) {
        double d = 0.0;
        for (int64_t t = 0; t < N; ++t) d += u[t] * m[t];
        for (int64_t t = 0; t < N; ++t) m[t] -= d * u[t];
      }
      double n1 = 0.0;
      for (double a : m) n1 += a * a;
      if (n1 > 1e-20 * n0)
        fail(EAMG_ERR_UNSUPPORTED_KERNEL, "kernel vectors do not span the rigid body modes / constants");
    }
  }
}

Pattern pattern_from_input(const eamg_problem *pb) {
  Pattern P;
  P.n_rows = P.n_cols = pb->n_vertices;
  P.rp.assign(pb->row_ptr, pb->row_ptr + pb->n_vertices + 1);
  P.col.assign(pb->col_idx, pb->col_idx + pb->row_ptr[pb->n_vertices]);
  return P;
}

std::vector<int> crow_of(const Pattern &C) {
  std::vector<int> r(size_t(C.nnz()));
  for (int i = 0; i < C.n_rows; ++i)
    for (int64_t q = C.rp[i]; q < C.rp[i + 1]; ++q) r[q] = i;
  return r;
}

std::vector<int> to_i32(const std::vector<int64_t> &v) {
  std::vector<int> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) {
    if (v[i] > int64_t(2147483647)) fail(EAMG_ERR_INVALID_ARG, "a level exceeds 2^31 blocks");
    o[i] = int(v[i]);
  }
  return o;
}

}  // namespace

SolveMat make_solve_mat(DevArena &ar, const Pattern &Pp, const std::vector<int64_t> &src, int br, int bc,
                        const double *aos, hipStream_t s, std::vector<int> *diag_out,
                        bool transpose_blocks, bool fp32) {
  SolveMat M;
  M.n_rows = Pp.n_rows;
  M.n_cols = Pp.n_cols;
  M.br = br;
  M.bc = bc;
  M.nnz = Pp.nnz();
  M.group = pick_group(M.nnz, M.n_rows);
  // long rows of a square level matrix: one row per workgroup, so that a row is one round of
  // loads (at most one block per lane) instead of a loop over its blocks
  if (diag_out && M.n_rows > 0 && double(M.nnz) / M.n_rows > kWideRowBlocks) M.group = kBlock;
  M.rp = ar.upload(to_i32(Pp.rp), s);
  M.col = ar.upload(Pp.col, s);
  int64_t *src_d = ar.upload(src, s);
  double *v = ar.alloc<double>(size_t(M.nnz) * br * bc);
  float *v32 = fp32 ? ar.alloc<float>(size_t(M.nnz) * br * bc) : nullptr;
  if (transpose_blocks) {
    // input blocks are bc x br: gathered and transposed in one pass
    hip_check(launch_transpose_blocks(M.nnz, bc, br, src_d, aos, v, s), "transpose");
    if (fp32) hip_check(launch_convert<double, float>(M.nnz * br * bc, v, v32, s), "convert");
    hip_check(hipStreamSynchronize(s), "sync");
  } else {
    hip_check(launch_gather_blocks(M.nnz, br * bc, src_d, aos, v, s), "gather_blocks");
    if (fp32) hip_check(launch_gather_blocks_f32(M.nnz, br * bc, src_d, aos, v32, s), "gather_blocks_f32");
    hip_check(hipStreamSynchronize(s), "sync");
  }
  ar.release(src_d);
  M.val = v;
  M.val32 = v32;
  if (diag_out) {
    std::vector<int> dg(size_t(M.n_rows), -1);
    for (int i = 0; i < M.n_rows; ++i)
      for (int64_t q = Pp.rp[i]; q < Pp.rp[i + 1]; ++q)
        if (Pp.col[q] == i) dg[i] = int(q);
    *diag_out = dg;
    M.diag = ar.upload(dg, s);
  }
  return M;
}



// Bytes of a row range [r0, r1) of a colour-major square level: blocks [lo(row), hi(row)) read,
// plus `per_row` bytes per row and every distinct column of those blocks gathered once.
// Blocks, rows and distinct columns of rows [r0, r1) of the colour-major pattern; part 0: lower
// blocks and the diagonal, 1: whole rows, 2: blocks right of the diagonal.
LaunchShape range_shape(const Pattern &Ap, const std::vector<int> &dg, int r0, int r1, int part,
                        std::vector<int> &mark, int stamp) {
  LaunchShape sh;
  sh.rows = r1 - r0;
  for (int i = r0; i < r1; ++i) {
    const int64_t lo = part == 2 ? dg[i] + 1 : Ap.rp[i];
    const int64_t hi = part == 0 ? dg[i] + 1 : Ap.rp[i + 1];
    sh.blocks += double(hi - lo);
    for (int64_t q = lo; q < hi; ++q)
      if (mark[Ap.col[q]] != stamp) {
        mark[Ap.col[q]] = stamp;
        sh.uniq += 1.0;
      }
  }
  return sh;
}

LaunchShape matrix_shape(const Pattern &M) {
  LaunchShape sh;
  sh.rows = M.n_rows;
  sh.blocks = double(M.nnz());
  std::vector<char> seen(size_t(M.n_cols), 0);
  for (int c : M.col)
    if (!seen[c]) {
      seen[c] = 1;
      sh.uniq += 1.0;
    }
  return sh;
}

void attach_split_parts(DevArena &ar, const Pattern &Ap, const std::vector<int64_t> &src,
                        const std::vector<int> &dg, int bs, const double *vals, hipStream_t s,
                        bool f32, SolveMat &Am) {
  const int n = Ap.n_rows;
  Pattern Plo, Pup, Pd;
  std::vector<int64_t> slo, sup, sd;
  for (Pattern *P : {&Plo, &Pup, &Pd}) {
    P->n_rows = P->n_cols = n;
    P->rp.assign(size_t(n) + 1, 0);
  }
  for (int i = 0; i < n; ++i) {
    for (int64_t q = Ap.rp[i]; q < dg[i]; ++q) {
      Plo.col.push_back(Ap.col[q]);
      slo.push_back(src[q]);
    }
    for (int64_t q = dg[i] + 1; q < Ap.rp[i + 1]; ++q) {
      Pup.col.push_back(Ap.col[q]);
      sup.push_back(src[q]);
    }
    Pd.col.push_back(i);
    sd.push_back(src[size_t(dg[i])]);
    Plo.rp[i + 1] = int64_t(Plo.col.size());
    Pup.rp[i + 1] = int64_t(Pup.col.size());
    Pd.rp[i + 1] = i + 1;
  }
  const SolveMat lo = make_solve_mat(ar, Plo, slo, bs, bs, vals, s, nullptr, false, f32);
  const SolveMat up = make_solve_mat(ar, Pup, sup, bs, bs, vals, s, nullptr, false, f32);
  const SolveMat dm = make_solve_mat(ar, Pd, sd, bs, bs, vals, s, nullptr, false, f32);
  Am.lo_rp = lo.rp;
  Am.lo_col = lo.col;
  Am.lo_val = lo.val;
  Am.lo_val32 = lo.val32;
  Am.lo_nnz = lo.nnz;
  Am.up_rp = up.rp;
  Am.up_col = up.col;
  Am.up_val = up.val;
  Am.up_val32 = up.val32;
  Am.up_nnz = up.nnz;
  Am.dg_val = dm.val;
  Am.dg_val32 = dm.val32;
}

void level_shapes(Level &L, const Pattern &Ap, const std::vector<int> &dg) {
  L.nnz_lower = 0;
  for (int i = 0; i < L.n; ++i) L.nnz_lower += dg[i] - Ap.rp[i];
  L.sh_spmv = matrix_shape(Ap);
  // one task per colour and sweep part plus the residual, each with its own marks
  const int nc = L.ncolors;
  L.sh_fwd.assign(size_t(nc), LaunchShape());
  L.sh_bwd.assign(size_t(nc), LaunchShape());
  parallel_for_dynamic(2 * int64_t(nc) + 1, [&](int64_t t) {
    std::vector<int> mark(size_t(L.n), -1);
    if (t == 2 * int64_t(nc)) {
      L.sh_resid = range_shape(Ap, dg, 0, L.smooth_rows(), 2, mark, 0);
      L.upper_blocks.assign(size_t(nc), 0.0);
      for (int c = 0; c < nc; ++c)
        for (int i = L.color_ptr[c]; i < L.color_ptr[c + 1]; ++i)
          L.upper_blocks[size_t(c)] += double(Ap.rp[i + 1] - dg[i] - 1);
      return;
    }
    const int c = int(t / 2), part = int(t % 2);
    (part == 0 ? L.sh_fwd : L.sh_bwd)[size_t(c)] =
        range_shape(Ap, dg, L.color_ptr[c], L.color_ptr[c + 1], part, mark, 0);
  }, 1);
}

namespace {

static_assert(std::is_nothrow_move_constructible<Level>::value,
              "levels must move without copying their patterns");

void build_level_layout(eamg_hierarchy *h, size_t l, hipStream_t s) {
  Level &L = h->lv[l];
  DevArena &ar = h->arena;
  const bool coarsest = (l + 1 == h->lv.size());
  const int bs = L.bs;
  // colour-major numbering (identity on the coarsest level, which has no smoother)
  L.perm.resize(size_t(L.n));
  L.inv.resize(size_t(L.n));
  if (coarsest) {
    for (int i = 0; i < L.n; ++i) L.perm[i] = L.inv[i] = i;
    L.ncolors = 0;
    L.color.assign(size_t(L.n), -1);
    L.color_ptr = {0, L.n};
  } else {
    if (L.color.size() != size_t(L.n)) {
      PhaseTimer tc;
      L.color = greedy_coloring(L.A, L.ncolors);
      tc.mark("layout: colouring");
    }
    L.color_ptr.assign(size_t(L.ncolors) + 1, 0);
    for (int c : L.color) L.color_ptr[c + 1]++;
    for (int c = 0; c < L.ncolors; ++c) L.color_ptr[c + 1] += L.color_ptr[c];
    std::vector<int> fill(L.color_ptr.begin(), L.color_ptr.end() - 1);
    for (int i = 0; i < L.n; ++i) L.perm[fill[L.color[i]]++] = i;
    for (int r = 0; r < L.n; ++r) L.inv[L.perm[r]] = r;
  }
  PhaseTimer tl;
  L.perm_d = ar.upload(L.perm, s);
  std::vector<int64_t> src;
  const Pattern Ap = permute_pattern(L.A, L.perm, L.inv, src);
  tl.mark("layout: permute");
  std::vector<int> dg;
  const bool f32 = h->prm.vcycle_fp32 != 0;
  L.Am = make_solve_mat(ar, Ap, src, bs, bs, L.A_val, s, &dg, false, f32);
  // the blocks left of the diagonal, right of it, and the diagonal blocks, each stored on its
  // own for the forward sweep and the residual update (SolveMat)
  if (!coarsest) attach_split_parts(ar, Ap, src, dg, bs, L.A_val, s, f32, L.Am);
  tl.mark("layout: A blocks");
  if (coarsest) {
    L.nnz_lower = 0;
    for (int i = 0; i < L.n; ++i) L.nnz_lower += dg[i] - Ap.rp[i];
    L.sh_spmv = matrix_shape(Ap);
  } else {
    level_shapes(L, Ap, dg);
  }
  tl.mark("layout: launch shapes");
  if (coarsest) {
    L.b = ar.alloc<double>(size_t(L.n) * bs);
    L.x = ar.alloc<double>(size_t(L.n) * bs);
    if (f32) {
      L.b32 = ar.alloc<float>(size_t(L.n) * bs);
      L.x32 = ar.alloc<float>(size_t(L.n) * bs);
    }
    return;
  }
  // smoother diagonals (natural), then rows gathered into colour-major order
  double *Dn = ar.alloc<double>(size_t(L.n) * bs * bs);
  hip_check(launch_diag_pinv(L.n, bs, L.A_rp, L.A_col, L.A_val, Dn, h->prm.pinv_rtol, s), "diag_pinv");
  L.Dinv = ar.alloc<double>(size_t(L.n) * bs * bs);
  hip_check(launch_gather_rows(L.n, bs * bs, L.perm_d, Dn, L.Dinv, s), "gather_rows");
  if (f32) {
    L.Dinv32 = ar.alloc<float>(size_t(L.n) * bs * bs);
    hip_check(launch_convert(int64_t(L.n) * bs * bs, L.Dinv, L.Dinv32, s), "convert");
  }
  hip_check(hipStreamSynchronize(s), "sync");
  ar.release(Dn);
  // transfers: fine rows colour-major, coarse columns in the coarse level's colour-major order
  const Level &C = h->lv[l + 1];
  std::vector<int64_t> srcP;
  const Pattern Pp = permute_rect(L.P, L.perm, C.inv, srcP);
  L.Pm = make_solve_mat(ar, Pp, srcP, bs, L.kc, L.P_val, s, nullptr, false, f32);
  std::vector<int64_t> srcT;
  const Pattern Rp = transpose_pattern(Pp, srcT);
  std::vector<int64_t> srcR(srcT.size());
  for (size_t q = 0; q < srcT.size(); ++q) srcR[q] = srcP[size_t(srcT[q])];
  L.Rm = make_solve_mat(ar, Rp, srcR, L.kc, bs, L.P_val, s, nullptr, true, f32);
  L.sh_R = matrix_shape(Rp);
  L.sh_P = matrix_shape(Pp);
  tl.mark("layout: D+ and transfers");
  L.r = ar.alloc<double>(size_t(L.n) * bs);
  if (l > 0) {
    L.b = ar.alloc<double>(size_t(L.n) * bs);
    L.x = ar.alloc<double>(size_t(L.n) * bs);
  }
  if (f32) {
    L.r32 = ar.alloc<float>(size_t(L.n) * bs);
    L.b32 = ar.alloc<float>(size_t(L.n) * bs);
    L.x32 = ar.alloc<float>(size_t(L.n) * bs);
  }
}

void coarsest_factor(eamg_hierarchy *h, hipStream_t s) {
  Level &L = h->lv.back();
  const int bs = L.bs;
  const int N = L.n * bs;
  if (N > kMaxCoarsestDofs)
    fail(EAMG_ERR_INVALID_ARG, "coarsening stalled: coarsest level has " + std::to_string(N) +
                                   " dofs (the direct solve takes at most " +
                                   std::to_string(kMaxCoarsestDofs) + ")");
  // regularization: the projector onto the kernel of every diagonal block
  const std::vector<double> vals = download(L.A_val, size_t(L.A.nnz()) * bs * bs, s);
  std::vector<double> reg(size_t(L.n) * bs * bs, 0.0);
  for (int i = 0; i < L.n; ++i) {
    int64_t qd = -1;
    for (int64_t q = L.A.rp[i]; q < L.A.rp[i + 1]; ++q)
      if (L.A.col[q] == i) qd = q;
    Mat blk(bs, bs);
    if (qd >= 0)
      for (int a = 0; a < bs; ++a)
        for (int c = 0; c < bs; ++c) blk(a, c) = vals[size_t(qd) * bs * bs + a * bs + c];
    const Mat U0 = kernel_basis(blk, h->prm.pinv_rtol);
    for (int a = 0; a < bs; ++a)
      for (int c = 0; c < bs; ++c) {
        double v = 0.0;
        for (int t = 0; t < U0.c; ++t) v += U0(a, t) * U0(c, t);
        reg[size_t(i) * bs * bs + a * bs + c] = v;
      }
  }
  // dense assembly and in-place inversion on the device
  const int ld = dense_ld(N);
  h->nL = N;
  h->ldL = ld;
  h->Ainv = h->arena.alloc<double>(size_t(ld) * ld);
  double *reg_d = h->arena.upload(reg, s);
  double *work = h->arena.alloc<double>(gj_work_doubles(ld));
  int *flag = h->arena.alloc<int>(1);
  hip_check(hipMemsetAsync(flag, 0, sizeof(int), s), "memset");
  hip_check(launch_dense_assemble(L.n, bs, L.A_rp, L.A_col, L.A_val, reg_d, ld, h->Ainv, s), "dense_assemble");
  hip_check(launch_gj_invert(ld, h->Ainv, work, flag, s), "gj_invert");
  const int bad = download(flag, 1, s)[0];
  h->arena.release(flag);
  h->arena.release(work);
  h->arena.release(reg_d);
  if (bad) fail(EAMG_ERR_NOT_SPD, "coarsest level matrix is not positive definite");
}

// r -= (blocks right of the diagonal) x on every row of level L: one launch, or one per colour
// range of L.resid_cut, each with its own lanes per row.
template <class T>
hipError_t resid_update(const Level &L, const T *x, T *r, hipStream_t s) {
  const SolveMat M = L.resid_mat();
  if (L.resid_cut.empty()) return launch_resid_upper<T>(M, 0, L.smooth_rows(), x, r, s);
  for (size_t k = 0; k + 1 < L.resid_cut.size(); ++k) {
    SolveMat m = M;
    if (k < L.g_resid.size() && L.g_resid[k]) m.group = L.g_resid[k];
    const hipError_t e = launch_resid_upper<T>(m, L.color_ptr[size_t(L.resid_cut[k])],
                                               L.color_ptr[size_t(L.resid_cut[k + 1])], x, r, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Algorithmic bytes of one dense-tail apply: the packed upper tiles (FP32 or FP64), both passes
// over the partial sums, and x and y.
double tail_apply_bytes(const eamg_hierarchy *h, bool fp32_matrix, size_t vec_bytes) {
  return double(sym_entries(h->nT)) * (fp32_matrix ? 4.0 : 8.0) + 2.0 * 8.0 * double(sym_work_doubles(h->nT)) +
         2.0 * h->nT * double(vec_bytes);
}

// The dense operators of a fused hierarchy's level: x = D b on each of their systems' rows.
template <class T>
void dense_sets(eamg_hierarchy *h, size_t l, const T *b, T *x, hipStream_t s);
template <>
void dense_sets<double>(eamg_hierarchy *h, size_t l, const double *b, double *x, hipStream_t s) {
  const DenseSet &d = h->lv[l].dense[0];
  if (!d.count) return;
  timed(h, "dense parts", lvname(h, l, "k_dense_symv_multi<double, double>"), d.bytes, s, [&] {
    return launch_dense_symv_multi<double, double>(d.count, d.parts, d.tiles, d.rows, d.active, b, x, d.W, s);
  });
}
template <>
void dense_sets<float>(eamg_hierarchy *h, size_t l, const float *b, float *x, hipStream_t s) {
  const DenseSet &d32 = h->lv[l].dense[1], &d64 = h->lv[l].dense[2];
  if (d32.count)
    timed(h, "dense parts", lvname(h, l, "k_dense_symv_multi<float, float>"), d32.bytes, s, [&] {
      return launch_dense_symv_multi<float, float>(d32.count, d32.parts, d32.tiles, d32.rows, d32.active, b, x,
                                                   d32.W, s);
    });
  if (d64.count)
    timed(h, "dense parts", lvname(h, l, "k_dense_symv_multi<double, float>"), d64.bytes, s, [&] {
      return launch_dense_symv_multi<double, float>(d64.count, d64.parts, d64.tiles, d64.rows, d64.active, b, x,
                                                    d64.W, s);
    });
}

template <class T>
void vcycle_t(eamg_hierarchy *h, size_t l, const T *b, T *x, hipStream_t s) {
  Level &L = h->lv[l];
  const bool f32 = sizeof(T) == 4;
  const std::string ty = type_name<T>();
  if (h->fused) {
    // systems whose V-cycle ends here are applied as dense operators; the others are smoothed
    dense_sets<T>(h, l, b, x, s);
    if (L.smooth_rows() == 0) return;
  }
  if (int(l) == h->tail_level) {
    // the V-cycle of this level and every level below it, as one dense matrix (FP64 unless the
    // FP32 V-cycle was set up with an FP32 copy), its upper tiles packed
    const bool m32 = f32 && h->tailS32;
    const double by = tail_apply_bytes(h, m32, sizeof(T));
    if (m32)
      timed(h, "dense tail", lvname(h, l, "k_dense_symv<float, float>"), by, s, [&] {
        return launch_dense_symv<float, float>(h->nT, h->tailS32, reinterpret_cast<const float *>(b),
                                               reinterpret_cast<float *>(x), h->tailW, s);
      });
    else
      timed(h, "dense tail", lvname(h, l, "k_dense_symv<double, " + ty + ">"), by, s,
            [&] { return launch_dense_symv<double, T>(h->nT, h->tailS, b, x, h->tailW, s); });
    return;
  }
  if (l + 1 == h->lv.size()) {
    const double by = double(h->nL) * h->nL * 8.0 + 2.0 * h->nL * double(sizeof(T));
    timed(h, "coarsest", lvname(h, l, "k_dense_gemv<" + ty + ">"), by, s,
          [&] { return launch_dense_gemv<T>(h->nL, h->ldL, h->Ainv, b, x, s); });
    return;
  }
  const LevelBufs<T> B = bufs<T>(L);
  const int bs = L.bs;
  const double vs = sizeof(T);
  double fwd_bytes = 0.0, bwd_bytes = 0.0;
  for (int c = 0; c < L.ncolors; ++c) {
    fwd_bytes += launch_bytes(L.sh_fwd[c], LK_GS_FWD, bs, bs, vs, 1);
    bwd_bytes += launch_bytes(L.sh_bwd[c], LK_GS_BWD, bs, bs, vs, 1);
  }
  const std::string gs = "k_gs_color<" + ty + ", " + std::to_string(bs);
  // the colours of a sweep are back-to-back launches of one kernel: one profiler record (events
  // per launch would add their own dispatch to every launch)
  if (h->prof_colours) {
    for (int c = 0; c < L.ncolors; ++c)
      timed(h, "gs_fwd", lvname(h, l, "c" + std::to_string(c) + " " + gs + ", true>"),
            launch_bytes(L.sh_fwd[c], LK_GS_FWD, bs, bs, vs, 1), s, [&] {
              return launch_gs_fwd<T>(L.fwd_mat(c), B.Dinv, L.color_ptr[c], L.color_ptr[c + 1], b, x, B.r, s);
            });
  } else {
    timed_n(h, "gs_fwd", lvname(h, l, gs + ", true>"), fwd_bytes, L.ncolors, s, [&] {
      for (int c = 0; c < L.ncolors; ++c) {
        const hipError_t e = launch_gs_fwd<T>(L.fwd_mat(c), B.Dinv, L.color_ptr[c], L.color_ptr[c + 1], b, x, B.r, s);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    });
  }
  const int nres = L.resid_cut.empty() ? 1 : int(L.resid_cut.size()) - 1;
  timed_n(h, "resid_upper", lvname(h, l, "k_resid_upper<" + ty + ", " + std::to_string(bs) + ">"),
          launch_bytes(L.sh_resid, LK_RESID, bs, bs, vs, 1), nres, s, [&] {
            return resid_update<T>(L, x, B.r, s);
          });
  Level &C = h->lv[l + 1];
  const LevelBufs<T> CB = bufs<T>(C);
  timed(h, "restrict", lvname(h, l, "k_rect<" + ty + ", " + std::to_string(L.kc) + ", " + std::to_string(bs) + ">"),
        launch_bytes(L.sh_R, LK_RECT, L.kc, bs, vs, 1), s, [&] { return launch_rect<T>(L.Rm, B.r, CB.b, false, s); });
  vcycle_t<T>(h, l + 1, CB.b, CB.x, s);
  timed(h, "prolong", lvname(h, l, "k_rect<" + ty + ", " + std::to_string(bs) + ", " + std::to_string(L.kc) + ">"),
        launch_bytes(L.sh_P, LK_RECT_ACC, bs, L.kc, vs, 1), s, [&] { return launch_rect<T>(L.Pm, CB.x, x, true, s); });
  if (h->prof_colours) {
    for (int c = L.ncolors - 1; c >= 0; --c)
      timed(h, "gs_bwd", lvname(h, l, "c" + std::to_string(c) + " " + gs + ", false>"),
            launch_bytes(L.sh_bwd[c], LK_GS_BWD, bs, bs, vs, 1), s, [&] {
              return launch_gs_bwd<T>(L.bwd_mat(c), B.Dinv, L.color_ptr[c], L.color_ptr[c + 1], b, x, s);
            });
    return;
  }
  timed_n(h, "gs_bwd", lvname(h, l, gs + ", false>"), bwd_bytes, L.ncolors, s, [&] {
    for (int c = L.ncolors - 1; c >= 0; --c) {
      const hipError_t e = launch_gs_bwd<T>(L.bwd_mat(c), B.Dinv, L.color_ptr[c], L.color_ptr[c + 1], b, x, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  });
}

// z = V(r) on colour-major level-0 vectors: FP64, or FP32 with conversions at the boundary.
void vcycle(eamg_hierarchy *h, const double *r, double *z, bool f32, hipStream_t s) {
  if (f32) {
    Level &L0 = h->lv[0];
    const int64_t N = int64_t(L0.n) * L0.bs;
    timed(h, "convert", "k_convert<double, float>", 12.0 * N, s,
          [&] { return launch_convert<double, float>(N, r, L0.b32, s); });
    vcycle_t<float>(h, 0, L0.b32, L0.x32, s);
    timed(h, "convert", "k_convert<float, double>", 12.0 * N, s,
          [&] { return launch_convert<float, double>(N, L0.x32, z, s); });
  } else {
    vcycle_t<double>(h, 0, r, z, s);
  }
}

// One PCG iteration after the stopping test: z = V(r), beta, p = z + beta p, q = A p, alpha,
// x += alpha p, r -= alpha q, r.r, and the scalars copied to pinned host memory.
void enqueue_iteration(eamg_hierarchy *h, bool f32, hipStream_t s) {
  const Level &L0 = h->lv[0];
  const SolveMat &A = L0.Am;
  const int64_t N = int64_t(L0.n) * L0.bs;
  const int nd = dot_blocks(N);
  const int ns = spmv_blocks(A);
  if (nd > h->part_cap || ns > h->part_cap) fail(EAMG_ERR_INVALID_ARG, "partial-sum buffer too small");
  if (f32) {
    // the FP32 V-cycle reads r's FP32 copy (written with r by the previous update) and its output
    // z is read in FP32 by the dot product and the p update
    vcycle_t<float>(h, 0, L0.b32, L0.x32, s);
    hip_check(launch_dot(N, h->r, L0.x32, h->part, s), "dot");
    hip_check(launch_reduce(nd, h->part, h->scal, SC_RZ, RED_BETA, s), "reduce");
    hip_check(launch_update_p(N, h->scal, L0.x32, h->p, s), "update_p");
  } else {
    vcycle(h, h->r, h->z, false, s);
    hip_check(launch_dot(N, h->r, h->z, h->part, s), "dot");
    hip_check(launch_reduce(nd, h->part, h->scal, SC_RZ, RED_BETA, s), "reduce");
    hip_check(launch_update_p(N, h->scal, h->z, h->p, s), "update_p");
  }
  hip_check(launch_spmv(A, h->p, h->q, h->part, s), "spmv");
  hip_check(launch_reduce(ns, h->part, h->scal, SC_PQ, RED_ALPHA, s), "reduce");
  hip_check(launch_update_xr(N, h->scal, h->x, h->r, h->p, h->q, h->part, s, f32 ? L0.b32 : nullptr),
            "update_xr");
  hip_check(launch_reduce(nd, h->part, h->scal, SC_RR, RED_STORE, s), "reduce");
  hip_check(hipMemcpyAsync(h->scal_h, h->scal, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost, s),
            "copy");
}

// Capture enqueue_iteration once; on any failure fall back to eager launches.
void try_build_graph(eamg_hierarchy *h, bool f32) {
  h->graph_tried[f32] = true;
  if (const char *e = std::getenv("EAMG_GRAPH"))
    if (std::atoi(e) == 0) return;
  if (!h->cap_stream && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    h->cap_stream = nullptr;
    return;
  }
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) return;
  bool ok = true;
  try {
    enqueue_iteration(h, f32, h->cap_stream);
  } catch (const Failure &) {
    ok = false;
  }
  if (hipStreamEndCapture(h->cap_stream, &g) != hipSuccess || !ok) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return;
  }
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) h->g_iter[f32] = ex;
  (void)hipGraphDestroy(g);
  (void)hipGetLastError();
}


double bytes_bcsr(int64_t nnzb, int r, int c, int rows) {
  return double(nnzb) * (r * c * 8.0 + 4.0) + 4.0 * (rows + 1);
}

// One PCG solve on one hierarchy, in phases, so that several solves can be interleaved
// (eamg_solve_multi): init, start (b in, x0, z = V(r), p = z, first iteration), next (the
// stopping test; true while an iteration is due), the iteration itself (graph replay,
// enqueue_iteration or eager_iteration), finish (true residual, x out) and report.
struct SolveRun {
  eamg_hierarchy *h = nullptr;
  eamg_solve_params sp{};
  bool f32 = false;
  hipStream_t s = nullptr;
  int64_t N = 0;
  int nd = 0, ns = 0;
  double vecb = 0.0, bnorm = 0.0;
  int iters = 0;
  double rel = 0.0, rel_true = 0.0, ms = 0.0;
  bool converged = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~SolveRun() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }

  void init(eamg_hierarchy *hh, const eamg_solve_params *params, hipStream_t st) {
    h = hh;
    s = st;
    eamg_default_solve_params(&sp);
    if (params) sp = *params;
    if (sp.max_it < 1) fail(EAMG_ERR_INVALID_ARG, "max_it must be >= 1");
    if (!(sp.rtol >= 0.0)) fail(EAMG_ERR_INVALID_ARG, "rtol must be >= 0");
    if (sp.precond < EAMG_PRECOND_NONE || sp.precond > EAMG_PRECOND_VCYCLE_FP32)
      fail(EAMG_ERR_INVALID_ARG, "precond must be 0, 1 or 2");
    if (sp.precond == EAMG_PRECOND_VCYCLE_FP32 && !h->prm.vcycle_fp32)
      fail(EAMG_ERR_INVALID_ARG, "FP32 V-cycle needs setup with vcycle_fp32 = 1");
    f32 = sp.precond == EAMG_PRECOND_VCYCLE_FP32;
    const Level &L0 = h->lv[0];
    N = int64_t(L0.n) * L0.bs;
    nd = dot_blocks(N);
    ns = spmv_blocks(L0.Am);
    if (nd > h->part_cap || ns > h->part_cap) fail(EAMG_ERR_INVALID_ARG, "partial-sum buffer too small");
    vecb = double(N) * 8.0;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
  }

  // z = V(r): with the FP32 V-cycle z is the level-0 FP32 vector x32 (read as it is by the dot
  // product and the p update) and the V-cycle reads r's FP32 copy b32, which the start and every
  // r update write along with r
  void precondition() {
    const Level &L0 = h->lv[0];
    if (f32)
      vcycle_t<float>(h, 0, L0.b32, L0.x32, s);
    else if (sp.precond)
      vcycle(h, h->r, h->z, false, s);
    else
      hip_check(launch_copy(N, h->r, h->z, s), "copy");
  }
  float *r32() const { return f32 ? h->lv[0].b32 : nullptr; }
  // r.z (partials into part) and p = z + beta p, z in FP64 or the FP32 V-cycle's output
  void dot_rz() {
    if (f32)
      timed(h, "dot", "k_dot<float>", vecb + 4.0 * N + 8.0 * nd, s,
            [&] { return launch_dot(N, h->r, h->lv[0].x32, h->part, s); });
    else
      timed(h, "dot", "k_dot", 2.0 * vecb + 8.0 * nd, s,
            [&] { return launch_dot(N, h->r, h->z, h->part, s); });
  }
  void update_p() {
    if (f32)
      timed(h, "update_p", "k_update_p<float>", 2.0 * vecb + 4.0 * N, s,
            [&] { return launch_update_p(N, h->scal, h->lv[0].x32, h->p, s); });
    else
      timed(h, "update_p", "k_update_p", 3.0 * vecb, s,
            [&] { return launch_update_p(N, h->scal, h->z, h->p, s); });
  }
  void update_xr() {
    timed(h, "update_xr", "k_update_xr", 6.0 * vecb + (f32 ? 4.0 * N : 0.0) + 8.0 * nd, s,
          [&] { return launch_update_xr(N, h->scal, h->x, h->r, h->p, h->q, h->part, s, r32()); });
  }

  double spmv_bytes() const {
    const Level &L0 = h->lv[0];
    return launch_bytes(L0.sh_spmv, LK_SPMV, L0.bs, L0.bs, 8.0, 1) + 8.0 * ns;
  }

  void copy_scalars() {
    hip_check(hipMemcpyAsync(h->scal_h, h->scal, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost, s),
              "copy");
  }
  void wait() { hip_check(hipStreamSynchronize(s), "sync"); }

  // start() in phases: each enqueue_* ends with the scalars copied to the host, each complete_*
  // (after the stream has been synchronised) reads them.  Interleaving the phases of several
  // systems lets their start-up launches overlap.
  bool active_start = true;   // false once start() has settled the solve

  void enqueue_start_a(const double *b_dev, const double *x_dev) {
    const Level &L0 = h->lv[0];
    const SolveMat &A = L0.Am;
    h->cg_alpha.clear();
    h->cg_beta.clear();
    hip_check(hipEventRecord(e0, s), "event");
    hip_check(launch_fill(SC_COUNT, 0.0, h->scal, s), "fill");
    hip_check(launch_perm_in(L0.n, L0.bs, L0.perm_d, h->dir, b_dev, h->bp, s), "perm_in");
    hip_check(launch_finite_check(N, h->bp, h->scal, SC_NONFINITE, s), "finite");
    hip_check(launch_dot(N, h->bp, h->bp, h->part, s), "dot");
    hip_check(launch_reduce(nd, h->part, h->scal, SC_BB, RED_STORE, s), "reduce");
    if (sp.use_x0) {
      hip_check(launch_perm_in(L0.n, L0.bs, L0.perm_d, h->dir, x_dev, h->x, s), "perm_in");
      hip_check(launch_spmv(A, h->x, h->q, nullptr, s), "spmv");
      hip_check(launch_sub(N, h->bp, h->q, h->r, s), "sub");
    } else {
      hip_check(launch_fill(N, 0.0, h->x, s), "fill");
      hip_check(launch_copy(N, h->bp, h->r, s), "copy");
    }
    if (f32) hip_check(launch_convert<double, float>(N, h->r, r32(), s), "convert");
    copy_scalars();
  }
  void complete_start_a() {
    if (h->scal_h[SC_NONFINITE] != 0.0) fail(EAMG_ERR_BREAKDOWN, "right-hand side is not finite");
    bnorm = std::sqrt(h->scal_h[SC_BB]);
    if (bnorm == 0.0) {
      hip_check(launch_fill(N, 0.0, h->x, s), "fill");
      converged = true;
      active_start = false;
    }
  }
  void enqueue_start_b() {
    precondition();
    if (f32)
      hip_check(launch_convert<float, double>(N, h->lv[0].x32, h->p, s), "convert");
    else
      hip_check(launch_copy(N, h->z, h->p, s), "copy");
    dot_rz();
    hip_check(launch_reduce(nd, h->part, h->scal, SC_RHO, RED_STORE, s), "reduce");
    copy_scalars();
  }
  void complete_start_b() {
    const double rho0 = h->scal_h[SC_RHO];
    if (!(rho0 > 0.0) || !std::isfinite(rho0)) {
      // r = b - A x0 may already be zero (exact x0); otherwise the preconditioner is not SPD
      hip_check(launch_dot(N, h->r, h->r, h->part, s), "dot");
      hip_check(launch_reduce(nd, h->part, h->scal, SC_RR, RED_STORE, s), "reduce");
      fetch_scalars(h, s);
      if (h->scal_h[SC_RR] != 0.0) fail(EAMG_ERR_BREAKDOWN, "r.z <= 0 at the start (preconditioner not SPD)");
      converged = true;
      active_start = false;
    }
  }
  // first iteration (p = z already set)
  void enqueue_start_c() {
    const Level &L0 = h->lv[0];
    const SolveMat &A = L0.Am;
    timed(h, "spmv", tname("k_spmv", L0.bs, L0.bs), spmv_bytes(), s,
          [&] { return launch_spmv(A, h->p, h->q, h->part, s); });
    timed(h, "reduce", "k_reduce", 8.0 * ns, s,
          [&] { return launch_reduce(ns, h->part, h->scal, SC_PQ, RED_ALPHA, s); });
    update_xr();
    timed(h, "reduce", "k_reduce", 8.0 * nd, s,
          [&] { return launch_reduce(nd, h->part, h->scal, SC_RR, RED_STORE, s); });
    copy_scalars();
  }

  void start(const double *b_dev, const double *x_dev) {
    enqueue_start_a(b_dev, x_dev);
    wait();
    complete_start_a();
    if (!active_start) return;
    enqueue_start_b();
    wait();
    complete_start_b();
    if (!active_start) return;
    enqueue_start_c();
    wait();
  }

  // The stopping test on the scalars of the last iteration (in h->scal_h); true when another
  // iteration is due.
  bool next() {
    if (converged) return false;
    ++iters;
    h->cg_alpha.push_back(h->scal_h[SC_ALPHA]);
    h->cg_beta.push_back(iters == 1 ? 0.0 : h->scal_h[SC_BETA]);
    if (h->scal_h[SC_BAD] != 0.0) fail(EAMG_ERR_BREAKDOWN, "p.Ap <= 0 or r.z <= 0 (operator or preconditioner not SPD)");
    const double rr = h->scal_h[SC_RR];
    if (!std::isfinite(rr)) fail(EAMG_ERR_BREAKDOWN, "residual is not finite");
    rel = std::sqrt(rr) / bnorm;
    if (std::sqrt(rr) <= sp.rtol * bnorm) {
      converged = true;
      return false;
    }
    return iters < sp.max_it;
  }

  void eager_iteration() {
    const Level &L0 = h->lv[0];
    const SolveMat &A = L0.Am;
    precondition();
    dot_rz();
    timed(h, "reduce", "k_reduce", 8.0 * nd, s,
          [&] { return launch_reduce(nd, h->part, h->scal, SC_RZ, RED_BETA, s); });
    update_p();
    timed(h, "spmv", tname("k_spmv", L0.bs, L0.bs), spmv_bytes(), s,
          [&] { return launch_spmv(A, h->p, h->q, h->part, s); });
    timed(h, "reduce", "k_reduce", 8.0 * ns, s,
          [&] { return launch_reduce(ns, h->part, h->scal, SC_PQ, RED_ALPHA, s); });
    update_xr();
    timed(h, "reduce", "k_reduce", 8.0 * nd, s,
          [&] { return launch_reduce(nd, h->part, h->scal, SC_RR, RED_STORE, s); });
    fetch_scalars(h, s);
  }

  void enqueue_finish(double *x_dev) {
    const Level &L0 = h->lv[0];
    hip_check(launch_spmv(L0.Am, h->x, h->q, nullptr, s), "spmv");
    hip_check(launch_sub(N, h->bp, h->q, h->z, s), "sub");
    hip_check(launch_dot(N, h->z, h->z, h->part, s), "dot");
    hip_check(launch_reduce(nd, h->part, h->scal, SC_RR, RED_STORE, s), "reduce");
    hip_check(launch_perm_out(L0.n, L0.bs, L0.perm_d, h->x, x_dev, s), "perm_out");
    hip_check(hipEventRecord(e1, s), "event");
    copy_scalars();
  }
  void complete_finish() {
    const double bn = std::sqrt(h->scal_h[SC_BB]);
    rel_true = bn > 0.0 ? std::sqrt(h->scal_h[SC_RR]) / bn : 0.0;
    if (bn == 0.0) rel = 0.0;
    float fms = 0.0f;
    hip_check(hipEventElapsedTime(&fms, e0, e1), "event");
    ms = fms;
  }
  void finish(double *x_dev) {
    enqueue_finish(x_dev);
    wait();
    complete_finish();
  }

  eamg_status report(eamg_status st, eamg_solve_info *info) const {
    const eamg_status out = (st == EAMG_OK && !converged) ? EAMG_NOT_CONVERGED : st;
    if (out == EAMG_NOT_CONVERGED) g_last_error = "iteration limit reached";
    if (info) {
      info->iterations = iters;
      info->rel_res = rel;
      info->rel_res_true = rel_true;
      info->ms = ms;
      info->status = out;
    }
    return out;
  }
};

// Streams of eamg_solve_multi: as many as the runtime's default hardware queues per process;
// more streams than queues only adds queue switching (measured slower).
constexpr int kMultiStreams = 4;

// Streams for the systems of eamg_solve_multi: each iteration forks from the solve stream,
// replays every active system's own iteration graph on a stream of its own, and joins.
struct MultiStreams {
  std::vector<hipStream_t> st;
  std::vector<hipEvent_t> ev;
  hipEvent_t fork = nullptr;
  ~MultiStreams() {
    for (hipStream_t x : st) (void)hipStreamDestroy(x);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
  }
  void ensure(size_t n) {
    if (!fork) hip_check(hipEventCreateWithFlags(&fork, hipEventDisableTiming), "event");
    while (st.size() < n) {
      hipStream_t x = nullptr;
      hip_check(hipStreamCreateWithFlags(&x, hipStreamNonBlocking), "stream");
      st.push_back(x);
      hipEvent_t e = nullptr;
      hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
      ev.push_back(e);
    }
  }
};

}  // namespace

void vcycle_apply(eamg_hierarchy *h, const double *r, double *z, bool f32, hipStream_t s) {
  vcycle(h, r, z, f32, s);
}

void vcycle_staged(eamg_hierarchy *h, const double *r_dev, double *z_dev, bool f32, double *rp,
                   double *zp, hipStream_t s) {
  const Level &L0 = h->lv[0];
  hip_check(launch_perm_in(L0.n, L0.bs, L0.perm_d, h->dir, r_dev, rp, s), "perm_in");
  vcycle(h, rp, zp, f32, s);
  hip_check(launch_perm_out(L0.n, L0.bs, L0.perm_d, zp, z_dev, s), "perm_out");
}

}  // namespace eamg

using namespace eamg;

extern "C" {

void eamg_default_setup_params(eamg_setup_params *out) {
  if (out) *out = defaults();
}

void eamg_default_solve_params(eamg_solve_params *out) {
  if (!out) return;
  out->rtol = 1e-8;
  out->max_it = 1000;
  out->use_x0 = 0;
  out->precond = EAMG_PRECOND_VCYCLE;
}

const char *eamg_last_error(void) { return g_last_error.c_str(); }

void eamg_destroy(eamg_hierarchy *h) {
  if (h && h->fused_users > 0) {
    h->destroy_pending = true;   // freed with the last fused hierarchy that reads it
    return;
  }
  delete h;
}

eamg_status eamg_setup(const eamg_problem *pb, const eamg_setup_params *params, void *stream,
                       eamg_hierarchy **out) {
  return guarded([&] {
    if (!out) fail(EAMG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    validate_problem(pb);
    const eamg_setup_params prm = params ? *params : defaults();
    validate_params(prm);
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::unique_ptr<eamg_hierarchy> h(new eamg_hierarchy());
    hip_check(hipGetDevice(&h->device), "hipGetDevice");
    const int n = pb->n_vertices, dim = pb->dim;
    h->dim = dim;
    h->k = pb->k_kernel;
    h->n0 = n;
    h->prm = prm;
    PhaseTimer tm;
    std::vector<std::pair<std::string, double>> phases;
    tm.sink = &phases;
    AuxLevel aux;
    std::string err;
    if (!finest_aux(dim, n, pb->coords, pb->row_ptr, pb->col_idx, pb->vals, pb->edges, pb->n_edges,
                    aux, err))
      fail(EAMG_ERR_INVALID_ARG, err);
    tm.mark("setup: finest weights");
    DevArena &ar = h->arena;
    {
      Level L0;
      L0.n = n;
      L0.bs = dim;
      L0.A = pattern_from_input(pb);
      L0.A_rp = ar.upload(L0.A.rp, s);
      L0.A_col = ar.upload(L0.A.col, s);
      L0.A_val = ar.upload(pb->vals, size_t(L0.A.nnz()) * dim * dim, s);
      hip_check(hipStreamSynchronize(s), "sync");
      tm.mark("setup: level-0 matrix upload");
      std::vector<uint8_t> dir(static_cast<size_t>(n), 0);
      if (pb->dirichlet)
        for (int i = 0; i < n; ++i) dir[i] = pb->dirichlet[i] ? 1 : 0;
      h->dir = ar.upload(dir, s);
      hip_check(launch_dirichlet(n, dim, L0.A_rp, L0.A_col, L0.A_val, h->dir, s), "dirichlet");
      hip_check(hipStreamSynchronize(s), "sync");
      h->lv.push_back(std::move(L0));
    }
    std::vector<char> vd(static_cast<size_t>(n), 0);
    if (pb->dirichlet)
      for (int i = 0; i < n; ++i) vd[i] = pb->dirichlet[i] ? 1 : 0;
    MatchParams mp;
    mp.sigma = prm.sigma;
    mp.rounds = prm.rounds;
    mp.mu_s_only = prm.mu_s_only != 0;
    mp.tie_rtol = prm.tie_rtol;
    mp.tau = prm.pinv_rtol;
    mp.record = prm.gnn_record != 0;
    tm.mark("setup: Dirichlet rows");
    std::unique_ptr<CritBatch> crit_dev;
    if (prm.gpu_criteria) {
      crit_dev = make_device_criteria(s);
      mp.batch = crit_dev.get();
      if (prm.gpu_criteria == 1) {
        mp.batch_min_pairs = kGpuCritMinPairs;
        mp.batch_min_unions = kGpuCritMinUnions;
      }
    }
    if (prm.gnn && prm.gnn_skip > 0.0) {
      eamg_gnn *net = const_cast<eamg_gnn *>(prm.gnn);
      mp.skip = prm.gnn_skip;
      mp.scorer = [net, s](const PassSamples &ps, std::vector<float> &z) {
        DeviceGraph dg(int64_t(ps.edges.size() / 2), ps.n, ps.X.data(), ps.edges.data(), nullptr,
                       nullptr, s);
        gnn_logits(net, dg, s, z);
      };
    }
    // The smoother's colouring of a level depends on its pattern only: it runs on a thread of its
    // own beside the matching of that level and of the levels below.  The thread reads the
    // pattern's buffers, which stay in place while the levels move (nothrow moves).
    struct Colouring {
      std::vector<int> color;
      int ncolors = 0;
    };
    std::vector<std::future<Colouring>> colourings;
    while (true) {
      const size_t l = h->lv.size() - 1;
      {
        const Level &L = h->lv[l];
        if (int64_t(L.bs) * L.n < prm.coarsest_max_dofs || int(h->lv.size()) >= prm.max_levels) break;
        const int nr = L.A.n_rows;
        const int64_t *rp = L.A.rp.data();
        const int *cl = L.A.col.data();
        colourings.push_back(std::async(std::launch::async, [nr, rp, cl] {
          Colouring c;
          c.color = greedy_coloring(nr, rp, cl, c.ncolors);
          return c;
        }));
      }
      tm.mark("setup: level upload");
      MatchResult mr = successive_matching(aux, l == 0 ? vd : std::vector<char>(), mp);
      tm.mark("setup: matching");
      h->crit_evaluated += mr.evaluated;
      h->crit_evaluated_g += mr.evaluated_g;
      h->crit_skipped += mr.skipped;
      for (auto &smp : mr.samples) h->samples.push_back(std::move(smp));
      const int nc = int(mr.aggs.size());
      if (nc == 0 || double(nc) > 0.9 * h->lv[l].n) break;
      Level &L = h->lv[l];
      const int bs = L.bs, kc = aux.k;
      L.agg.assign(size_t(L.n), -1);
      for (int I = 0; I < nc; ++I)
        for (int i : mr.aggs[I]) L.agg[i] = I;
      const ProlongPlan pl = plan_prolongation(L.A, aux, L.agg, mr.dmask,
                                               l == 0 ? prm.cap_std_l0 : prm.cap_std, prm.cap_aux,
                                               prm.tie_rtol);
      L.P = pl.P;
      L.kc = kc;
      tm.mark("setup: P_s plan");
      const int64_t nP = L.P.nnz();
      // auxiliary smoothed prolongation, numeric (device)
      int *type_d = ar.upload(pl.type, s);
      int *agg_d = ar.upload(L.agg, s);
      double *x_d = ar.upload(aux.x, s);
      double *xc_d = ar.upload(mr.ccoords, s);
      int64_t *Prp_d = ar.upload(L.P.rp, s);
      int *Pcol_d = ar.upload(L.P.col, s);
      int64_t *Fptr_d = ar.upload(pl.F_ptr, s);
      int *Fvtx_d = ar.upload(pl.F_vtx, s);
      int *Fedge_d = ar.upload(pl.F_edge, s);
      double *E_d = ar.upload(aux.E, s);
      L.P_val = ar.alloc<double>(size_t(nP) * bs * kc);
      PsArgs a;
      a.n = L.n;
      a.k = kc;
      a.bs = bs;
      a.type = type_d;
      a.agg = agg_d;
      a.x = x_d;
      a.xc = xc_d;
      a.Prp = Prp_d;
      a.Pcol = Pcol_d;
      a.Arp = L.A_rp;
      a.Acol = L.A_col;
      a.Aval = L.A_val;
      a.Fptr = Fptr_d;
      a.Fvtx = Fvtx_d;
      a.Fedge = Fedge_d;
      a.E = E_d;
      a.omega = prm.omega;
      a.tau = prm.pinv_rtol;
      a.Pval = L.P_val;
      hip_check(launch_ps_numeric(a, s), "ps_numeric");
      // Galerkin product A_{l+1} = R (A_l P_s), R = P_s^T (structural patterns on the host)
      const Pattern AP = spgemm_symbolic(L.A, L.P);
      std::vector<int64_t> srcT;
      const Pattern Rt = transpose_pattern(L.P, srcT);
      Pattern Ac = spgemm_symbolic(Rt, AP);
      tm.mark("setup: Galerkin symbolic");
      int *APcrow = ar.upload(crow_of(AP), s);
      int *APcol = ar.upload(AP.col, s);
      int64_t *APrp = ar.upload(AP.rp, s);
      int64_t *Rrp = ar.upload(Rt.rp, s);
      int *Rcol = ar.upload(Rt.col, s);
      int64_t *srcT_d = ar.upload(srcT, s);
      int *Accrow = ar.upload(crow_of(Ac), s);
      double *R_val = ar.alloc<double>(size_t(nP) * kc * bs);
      hip_check(launch_transpose_blocks(nP, bs, kc, srcT_d, L.P_val, R_val, s), "transpose");
      double *AP_val = ar.alloc<double>(size_t(AP.nnz()) * bs * kc);
      hip_check(launch_spgemm_numeric(AP.nnz(), bs, bs, kc, APcrow, APcol, L.A_rp, L.A_col, L.A_val,
                                      Prp_d, Pcol_d, L.P_val, AP_val, s),
                "spgemm AP");
      Level C;
      C.n = nc;
      C.bs = kc;
      C.A = std::move(Ac);
      C.A_rp = ar.upload(C.A.rp, s);
      C.A_col = ar.upload(C.A.col, s);
      C.A_val = ar.alloc<double>(size_t(C.A.nnz()) * kc * kc);
      hip_check(launch_spgemm_numeric(C.A.nnz(), kc, bs, kc, Accrow, C.A_col, Rrp, Rcol, R_val, APrp,
                                      APcol, AP_val, C.A_val, s),
                "spgemm RAP");
      hip_check(hipStreamSynchronize(s), "sync");
      for (void *p : {(void *)type_d, (void *)agg_d, (void *)x_d, (void *)xc_d, (void *)Prp_d,
                      (void *)Pcol_d, (void *)Fptr_d, (void *)Fvtx_d, (void *)Fedge_d, (void *)E_d,
                      (void *)APcrow, (void *)APcol, (void *)APrp, (void *)Rrp, (void *)Rcol,
                      (void *)srcT_d, (void *)Accrow, (void *)R_val, (void *)AP_val})
        ar.release(p);
      tm.mark("setup: P_s / Galerkin numeric");
      aux = std::move(mr.coarse);
      h->lv.push_back(std::move(C));
    }
    coarsest_factor(h.get(), s);
    tm.mark("setup: coarsest factor");
    for (size_t l = 0; l < colourings.size(); ++l) {
      Colouring c = colourings[l].get();
      h->lv[l].color = std::move(c.color);
      h->lv[l].ncolors = c.ncolors;
    }
    tm.mark("setup: colouring (wait)");
    for (size_t l = h->lv.size(); l-- > 0;) build_level_layout(h.get(), l, s);
    tm.mark("setup: solve layout");
    if (prm.dense_tail_dofs > 0) {
      for (size_t l = 1; l + 1 < h->lv.size(); ++l)
        if (int64_t(h->lv[l].n) * h->lv[l].bs <= prm.dense_tail_dofs) {
          build_dense_tail(h.get(), l, s);
          break;
        }
      tm.mark("setup: dense tail");
    }
    const int64_t N0 = int64_t(n) * dim;
    h->x = ar.alloc<double>(size_t(N0));
    h->r = ar.alloc<double>(size_t(N0));
    h->z = ar.alloc<double>(size_t(N0));
    h->p = ar.alloc<double>(size_t(N0));
    h->q = ar.alloc<double>(size_t(N0));
    h->bp = ar.alloc<double>(size_t(N0));
    // partial sums of the dots and of the SpMV's fused p.q: the SpMV launches one workgroup per
    // kBlock / G rows, so size for the widest row team it can be given (G = 64, the most
    // workgroups), whatever the autotuner picks later
    SolveMat widest = h->lv[0].Am;
    widest.group = 64;
    h->part_cap = std::max(dot_blocks(N0), spmv_blocks(widest));
    h->part = ar.alloc<double>(size_t(h->part_cap));
    h->scal = ar.alloc<double>(SC_COUNT);

    hip_check(hipHostMalloc(reinterpret_cast<void **>(&h->scal_h), sizeof(double) * SC_COUNT, 0),
              "hipHostMalloc");
    hip_check(hipStreamSynchronize(s), "sync");
    tm.mark("setup: solve vectors");
    for (const auto &ph : phases) {
      auto it = std::find_if(h->setup_phases.begin(), h->setup_phases.end(),
                             [&](const std::pair<std::string, double> &q) { return q.first == ph.first; });
      if (it == h->setup_phases.end())
        h->setup_phases.push_back(ph);
      else
        it->second += ph.second;
    }
    *out = h.release();
  });
}

eamg_status eamg_coarsening_stats(const eamg_hierarchy *h, int64_t *evaluated, int64_t *evaluated_g,
                                  int64_t *skipped, int32_t *sample_passes) {
  return guarded([&] {
    if (!h) fail(EAMG_ERR_INVALID_ARG, "NULL hierarchy");
    reject_fused(h);
    if (evaluated) *evaluated = h->crit_evaluated;
    if (evaluated_g) *evaluated_g = h->crit_evaluated_g;
    if (skipped) *skipped = h->crit_skipped;
    if (sample_passes) *sample_passes = int32_t(h->samples.size());
  });
}

eamg_status eamg_gnn_samples(const eamg_hierarchy *h, int32_t pass, int64_t *m, int32_t *n, float *X,
                             int32_t *edges, float *y, float *w) {
  return guarded([&] {
    if (!h) fail(EAMG_ERR_INVALID_ARG, "NULL hierarchy");
    reject_fused(h);
    if (pass < 0 || pass >= int(h->samples.size())) fail(EAMG_ERR_INVALID_ARG, "pass out of range");
    const PassSamples &ps = h->samples[size_t(pass)];
    const size_t np = ps.edges.size() / 2;
    if (m) *m = int64_t(np);
    if (n) *n = ps.n;
    if (X) std::copy(ps.X.begin(), ps.X.end(), X);
    if (edges) std::copy(ps.edges.begin(), ps.edges.end(), edges);
    if (y) std::copy(ps.y.begin(), ps.y.end(), y);
    if (w) std::copy(ps.w.begin(), ps.w.end(), w);
  });
}

eamg_status eamg_autotune(eamg_hierarchy *h, int32_t panel_width, void *stream, double *ms_before,
                          double *ms_after) {
  return guarded([&] {
    if (!h) fail(EAMG_ERR_INVALID_ARG, "NULL hierarchy");
    if (panel_width < 0 || panel_width > 64) fail(EAMG_ERR_INVALID_ARG, "panel_width must be in [0, 64]");
    if (h->fused && panel_width > 0) fail(EAMG_ERR_INVALID_ARG, "a fused hierarchy has no panel kernels to tune");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int reps = 5;
    double before = 0.0, after = 0.0;
    auto time_ms = [&](auto &&f) {
      hipEvent_t a, b;
      hip_check(hipEventCreate(&a), "event");
      hip_check(hipEventCreate(&b), "event");
      std::vector<float> t;
      for (int r = 0; r < reps; ++r) {
        hip_check(hipEventRecord(a, s), "event");
        f();
        hip_check(hipEventRecord(b, s), "event");
        hip_check(hipEventSynchronize(b), "sync");
        float ms = 0.0f;
        hip_check(hipEventElapsedTime(&ms, a, b), "event");
        t.push_back(ms);
      }
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      std::sort(t.begin(), t.end());
      return double(t[t.size() / 2]);
    };
    // median time of each of the nparts launches of run_all(mark), which calls mark(k) right
    // after enqueueing part k
    std::vector<hipEvent_t> pev;
    auto part_times = [&](int nparts, auto &&run_all) {
      while (int(pev.size()) < nparts + 1) {
        hipEvent_t e;
        hip_check(hipEventCreate(&e), "event");
        pev.push_back(e);
      }
      std::vector<std::vector<float>> t(static_cast<size_t>(nparts));
      for (int r = 0; r < 3; ++r) {
        hip_check(hipEventRecord(pev[0], s), "event");
        run_all([&](int k) { hip_check(hipEventRecord(pev[size_t(k) + 1], s), "event"); });
        hip_check(hipEventSynchronize(pev[size_t(nparts)]), "sync");
        for (int k = 0; k < nparts; ++k) {
          float ms = 0.0f;
          hip_check(hipEventElapsedTime(&ms, pev[size_t(k)], pev[size_t(k) + 1]), "event");
          t[size_t(k)].push_back(ms);
        }
      }
      std::vector<double> med(static_cast<size_t>(nparts));
      for (int k = 0; k < nparts; ++k) {
        std::sort(t[size_t(k)].begin(), t[size_t(k)].end());
        med[size_t(k)] = t[size_t(k)][1];
      }
      return med;
    };
    struct EventPool {
      std::vector<hipEvent_t> &ev;
      ~EventPool() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
      }
    } pev_guard{pev};
    // single right-hand side: lanes per row of each level's sweeps (FP64 kernels; the FP32 ones
    // share the choice)
    for (size_t l = 0; l + 1 < h->lv.size(); ++l) {
      if (h->tail_level >= 0 && int(l) >= h->tail_level) break;   // applied as the dense tail
      Level &L = h->lv[l];
      const int64_t nv = int64_t(L.n) * L.bs;
      double *b = l == 0 ? h->r : L.b, *x = l == 0 ? h->z : L.x;
      for (double *v : {b, x, L.r}) hip_check(launch_fill(nv, 0.0, v, s), "fill");
      auto fwd_part = [&] {
        for (int c = 0; c < L.ncolors; ++c)
          hip_check(launch_gs_fwd<double>(L.fwd_mat(c), L.Dinv, L.color_ptr[c], L.color_ptr[c + 1], b, x, L.r, s), "gs");
      };
      auto resid_part = [&] { hip_check(resid_update<double>(L, x, L.r, s), "resid"); };
      auto bwd_part = [&] {
        for (int c = L.ncolors - 1; c >= 0; --c)
          hip_check(launch_gs_bwd<double>(L.bwd_mat(c), L.Dinv, L.color_ptr[c], L.color_ptr[c + 1], b, x, s), "gs");
      };
      L.g_fwd.clear();
      L.g_bwd.clear();
      L.resid_cut.clear();
      L.g_resid.clear();
      // EAMG_FORCE_GROUP = 8, 16, 32, 64, 128 or 256 sets every level's lanes per row without
      // timing (tests use it to run each row-team shape)
      if (const char *fg = std::getenv("EAMG_FORCE_GROUP")) {
        const int g = std::atoi(fg);
        if (g != 8 && g != 16 && g != 32 && g != 64 && g != 128 && g != kBlock)
          fail(EAMG_ERR_INVALID_ARG, "EAMG_FORCE_GROUP must be 8, 16, 32, 64, 128 or 256");
        L.Am.group = g;
        L.Am.group_bwd = 0;
        L.group_resid = 0;
        continue;
      }
      // forward sweep, residual update and backward sweep: lanes per row chosen apart
      const int cand[] = {8, 16, 32, 64, 128, kBlock};
      L.Am.group_bwd = 0;
      L.group_resid = 0;
      const int orig = L.Am.group;
      const double f0 = time_ms(fwd_part), r0 = time_ms(resid_part), b0 = time_ms(bwd_part);
      double bf = f0, br = r0, bb = b0;
      int gf = orig, gr = orig, gb = orig;
      for (int g : cand) {
        if (g == orig) continue;
        L.Am.group = g;
        L.Am.group_bwd = g;
        L.group_resid = g;
        const double tf = time_ms(fwd_part), tr = time_ms(resid_part), tb = time_ms(bwd_part);
        if (tf < bf) {
          bf = tf;
          gf = g;
        }
        if (tr < br) {
          br = tr;
          gr = g;
        }
        if (tb < bb) {
          bb = tb;
          gb = g;
        }
      }
      L.Am.group = gf;
      L.Am.group_bwd = gb == gf ? 0 : gb;
      L.group_resid = gr == gf ? 0 : gr;
      // then per colour (the sweeps) and per range of colours (the residual update): each part
      // is timed inside whole sweeps, so its matrix streams from memory as in a V-cycle; a
      // refinement is kept only if the whole part gets faster
      const int nc = L.ncolors;
      auto refine = [&](std::vector<int> &choice, int nparts, auto &&run_all, double level_best) {
        std::vector<std::vector<double>> t(static_cast<size_t>(nparts));
        for (int g : cand) {
          choice.assign(size_t(nparts), g);
          const std::vector<double> tg = part_times(nparts, run_all);
          for (int k = 0; k < nparts; ++k) t[size_t(k)].push_back(tg[size_t(k)]);
        }
        for (int k = 0; k < nparts; ++k) {
          const auto &tk = t[size_t(k)];
          choice[size_t(k)] = cand[std::min_element(tk.begin(), tk.end()) - tk.begin()];
        }
        const double tsum = time_ms([&] { run_all([](int) {}); });
        if (tsum >= level_best) choice.clear();
        return choice.empty() ? level_best : tsum;
      };
      bf = refine(L.g_fwd, nc, [&](auto &&mark) {
        for (int c = 0; c < nc; ++c) {
          hip_check(launch_gs_fwd<double>(L.fwd_mat(c), L.Dinv, L.color_ptr[c], L.color_ptr[c + 1], b, x, L.r, s), "gs");
          mark(c);
        }
      }, bf);
      bb = refine(L.g_bwd, nc, [&](auto &&mark) {
        for (int c = nc - 1; c >= 0; --c) {
          hip_check(launch_gs_bwd<double>(L.bwd_mat(c), L.Dinv, L.color_ptr[c], L.color_ptr[c + 1], b, x, s), "gs");
          mark(nc - 1 - c);
        }
      }, bb);
      // residual update in up to four launches over colour ranges of about equal upper blocks
      {
        std::vector<int> cut{0};
        double tot = 0.0, acc = 0.0;
        for (double u : L.upper_blocks) tot += u;
        for (int c = 0; c < nc; ++c) {
          acc += L.upper_blocks[size_t(c)];
          if (c + 1 < nc && acc >= tot * double(cut.size()) / 4.0) cut.push_back(c + 1);
        }
        cut.push_back(nc);
        if (cut.size() > 2) {
          L.resid_cut = cut;
          const int nr = int(cut.size()) - 1;
          br = refine(L.g_resid, nr, [&](auto &&mark) {
            for (int k = 0; k < nr; ++k) {
              SolveMat m = L.resid_mat();
              if (size_t(k) < L.g_resid.size() && L.g_resid[size_t(k)]) m.group = L.g_resid[size_t(k)];
              hip_check(launch_resid_upper<double>(m, L.color_ptr[size_t(cut[size_t(k)])],
                                                   L.color_ptr[size_t(cut[size_t(k) + 1])], x, L.r, s),
                        "resid");
              mark(k);
            }
          }, br);
          if (L.g_resid.empty()) L.resid_cut.clear();
        }
      }
      before += f0 + r0 + b0;
      after += bf + br + bb;
    }
    for (int p = 0; p < 2; ++p) {
      if (h->g_iter[p]) (void)hipGraphExecDestroy(h->g_iter[p]);
      h->g_iter[p] = nullptr;
      h->graph_tried[p] = false;
    }
    invalidate_fused_graphs(h);
    if (panel_width > 0) {
      int K = 1;
      while (K < panel_width) K <<= 1;
      const auto pa = tune_panels(h, K, s);
      before += pa.first;
      after += pa.second;
    }
    hip_check(hipStreamSynchronize(s), "sync");
    if (ms_before) *ms_before = before;
    if (ms_after) *ms_after = after;
  });
}

eamg_status eamg_solve_multi(int32_t nsys, eamg_hierarchy *const *hs, const double *const *b_dev,
                             double *const *x_dev, const eamg_solve_params *params, void *stream,
                             eamg_solve_info *infos) {
  bool all = true;
  const eamg_status st = guarded([&] {
    if (nsys < 1 || !hs || !b_dev || !x_dev) fail(EAMG_ERR_INVALID_ARG, "NULL argument or nsys < 1");
    for (int m = 0; m < nsys; ++m) {
      if (!hs[m] || !b_dev[m] || !x_dev[m]) fail(EAMG_ERR_INVALID_ARG, "NULL hierarchy or vector");
      reject_fused(hs[m]);
      if (b_dev[m] == x_dev[m]) fail(EAMG_ERR_INVALID_ARG, "b and x may not alias");
      for (int l = 0; l < m; ++l)
        if (hs[l] == hs[m]) fail(EAMG_ERR_INVALID_ARG, "a hierarchy may appear only once");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<std::unique_ptr<SolveRun>> runs;
    for (int m = 0; m < nsys; ++m) {
      runs.emplace_back(std::make_unique<SolveRun>());
      runs[m]->init(hs[m], params, s);
    }
    // a system that breaks down stops with its status; the others go on
    std::vector<eamg_status> sst(size_t(nsys), EAMG_OK);
    std::vector<char> live(size_t(nsys), 1);
    auto guard_sys = [&](int m, auto &&f) {
      try {
        f();
      } catch (const Failure &e) {
        if (e.code != EAMG_ERR_BREAKDOWN) throw;
        sst[m] = e.code;
        live[m] = 0;
      }
    };
    // start-up and finish of all systems in interleaved phases on the streams
    MultiStreams ms;
    ms.ensure(size_t(std::min(nsys, kMultiStreams)));
    for (int m = 0; m < nsys; ++m) runs[m]->s = ms.st[size_t(m) % ms.st.size()];
    // the caller's work on `s` (b and x0 written asynchronously, say) comes before anything the
    // systems' streams do
    hip_check(hipEventRecord(ms.fork, s), "event");
    for (hipStream_t x : ms.st) hip_check(hipStreamWaitEvent(x, ms.fork, 0), "wait");
    auto phase = [&](auto &&enq, auto &&done) {
      for (int m = 0; m < nsys; ++m)
        if (live[m]) guard_sys(m, [&] { enq(m); });
      for (hipStream_t x : ms.st) hip_check(hipStreamSynchronize(x), "sync");
      for (int m = 0; m < nsys; ++m)
        if (live[m]) guard_sys(m, [&] {
            done(m);
            if (!runs[m]->active_start) live[m] = 2;   // settled: no iterations, but finish
          });
    };
    phase([&](int m) { runs[m]->enqueue_start_a(b_dev[m], x_dev[m]); },
          [&](int m) { runs[m]->complete_start_a(); });
    for (int m = 0; m < nsys; ++m) live[m] = live[m] == 1;
    phase([&](int m) { runs[m]->enqueue_start_b(); }, [&](int m) { runs[m]->complete_start_b(); });
    for (int m = 0; m < nsys; ++m) live[m] = live[m] == 1;
    phase([&](int m) { runs[m]->enqueue_start_c(); }, [](int) {});
    for (int m = 0; m < nsys; ++m) runs[m]->s = s;
    bool graphs = runs[0]->sp.precond != EAMG_PRECOND_NONE;
    for (int m = 0; m < nsys; ++m) graphs = graphs && !hs[m]->prof_on;
    if (const char *e = std::getenv("EAMG_GRAPH"))
      if (std::atoi(e) == 0) graphs = false;
    const bool f32 = runs[0]->f32;
    for (int m = 0; m < nsys && graphs; ++m) {
      if (!hs[m]->graph_tried[f32]) try_build_graph(hs[m], f32);
      graphs = hs[m]->g_iter[f32] != nullptr;
    }
    // estimated time of one iteration of each system: its launches (the colour sweeps dominate
    // the small systems) plus its bytes at a fraction of the HBM rate
    std::vector<double> cost(size_t(nsys), 0.0);
    for (int m = 0; m < nsys; ++m) {
      double launches = 8.0, bytes = 0.0;
      for (const Level &L : hs[m]->lv) {
        launches += 2.0 * L.ncolors + 4.0;
        bytes += double(L.A.nnz()) * L.bs * L.bs * (f32 ? 4.0 : 8.0) * 2.0;
      }
      cost[m] = launches * 6e-6 + bytes / 2e12;
    }
    std::vector<int> active;
    for (;;) {
      active.clear();
      for (int m = 0; m < nsys; ++m) {
        if (!live[m]) continue;
        bool more = false;
        guard_sys(m, [&] { more = runs[m]->next(); });
        if (more)
          active.push_back(m);
        else
          live[m] = 0;
      }
      if (active.empty()) break;
      if (graphs) {
        // largest first onto the least loaded of the streams
        std::vector<int> ord = active;
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        const size_t nst = std::min(ord.size(), ms.st.size());
        std::vector<double> load(nst, 0.0);
        hip_check(hipEventRecord(ms.fork, s), "event");
        for (size_t i = 0; i < nst; ++i) hip_check(hipStreamWaitEvent(ms.st[i], ms.fork, 0), "wait");
        for (int m : ord) {
          const size_t i = size_t(std::min_element(load.begin(), load.end()) - load.begin());
          load[i] += cost[m];
          hip_check(hipGraphLaunch(hs[m]->g_iter[f32], ms.st[i]), "graph launch");
        }
        for (size_t i = 0; i < nst; ++i) {
          hip_check(hipEventRecord(ms.ev[i], ms.st[i]), "event");
          hip_check(hipStreamWaitEvent(s, ms.ev[i], 0), "wait");
        }
        hip_check(hipStreamSynchronize(s), "sync");
      } else {
        for (int m : active) runs[m]->eager_iteration();
      }
    }
    for (int m = 0; m < nsys; ++m) {
      runs[m]->s = ms.st[size_t(m) % ms.st.size()];
      if (sst[m] == EAMG_OK) runs[m]->enqueue_finish(x_dev[m]);
    }
    // and the caller's later work on `s` comes after every x is written
    for (size_t i = 0; i < ms.st.size(); ++i) {
      hip_check(hipEventRecord(ms.ev[i], ms.st[i]), "event");
      hip_check(hipStreamWaitEvent(s, ms.ev[i], 0), "wait");
    }
    for (hipStream_t x : ms.st) hip_check(hipStreamSynchronize(x), "sync");
    for (int m = 0; m < nsys; ++m) {
      if (sst[m] == EAMG_OK) runs[m]->complete_finish();
      const eamg_status o = runs[m]->report(sst[m], infos ? infos + m : nullptr);
      all = all && o == EAMG_OK;
    }
  });
  if (st == EAMG_OK && !all) {
    g_last_error = "some systems did not converge";
    return EAMG_NOT_CONVERGED;
  }
  return st;
}

eamg_status eamg_vcycle(eamg_hierarchy *h, const double *r_dev, double *z_dev, int32_t precision,
                        void *stream) {
  return guarded([&] {
    if (!h || !r_dev || !z_dev) fail(EAMG_ERR_INVALID_ARG, "NULL argument");
    reject_fused(h);
    if (precision != EAMG_PRECOND_VCYCLE && precision != EAMG_PRECOND_VCYCLE_FP32)
      fail(EAMG_ERR_INVALID_ARG, "precision must be EAMG_PRECOND_VCYCLE or EAMG_PRECOND_VCYCLE_FP32");
    if (precision == EAMG_PRECOND_VCYCLE_FP32 && !h->prm.vcycle_fp32)
      fail(EAMG_ERR_INVALID_ARG, "FP32 V-cycle needs setup with vcycle_fp32 = 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Level &L0 = h->lv[0];
    hip_check(launch_perm_in(L0.n, L0.bs, L0.perm_d, h->dir, r_dev, h->bp, s), "perm_in");
    vcycle(h, h->bp, h->z, precision == EAMG_PRECOND_VCYCLE_FP32, s);
    hip_check(launch_perm_out(L0.n, L0.bs, L0.perm_d, h->z, z_dev, s), "perm_out");
    hip_check(hipStreamSynchronize(s), "sync");
  });
}

eamg_status eamg_solve(eamg_hierarchy *h, const double *b_dev, double *x_dev,
                       const eamg_solve_params *params, void *stream, eamg_solve_info *info) {
  SolveRun run;
  const eamg_status st = guarded([&] {
    if (!h || !b_dev || !x_dev) fail(EAMG_ERR_INVALID_ARG, "NULL argument");
    reject_fused(h);
    run.init(h, params, static_cast<hipStream_t>(stream));
    run.start(b_dev, x_dev);
    if (!run.converged) {
      const bool graphs = run.sp.precond && !h->prof_on;
      if (graphs && !h->graph_tried[run.f32]) try_build_graph(h, run.f32);
      while (run.next()) {
        if (graphs && h->g_iter[run.f32]) {
          hip_check(hipGraphLaunch(h->g_iter[run.f32], run.s), "graph launch");
          hip_check(hipStreamSynchronize(run.s), "sync");
        } else {
          run.eager_iteration();
        }
      }
    }
    run.finish(x_dev);
  });
  return run.report(st, info);
}

eamg_status eamg_stats(const eamg_hierarchy *h, int32_t *n_levels, int64_t *per_level_n,
                       int64_t *per_level_nnzb, double *vc, double *oc) {
  return guarded([&] {
    if (!h) fail(EAMG_ERR_INVALID_ARG, "NULL hierarchy");
    reject_fused(h);
    if (n_levels) *n_levels = int32_t(h->lv.size());
    double sn = 0.0, snz = 0.0;
    for (size_t l = 0; l < h->lv.size(); ++l) {
      const Level &L = h->lv[l];
      if (per_level_n) per_level_n[l] = L.n;
      if (per_level_nnzb) per_level_nnzb[l] = L.A.nnz();
      sn += L.n;
      snz += double(L.A.nnz()) * L.bs * L.bs;
    }
    const Level &L0 = h->lv[0];
    if (vc) *vc = sn / L0.n;
    if (oc) *oc = snz / (double(L0.A.nnz()) * L0.bs * L0.bs);
  });
}

eamg_status eamg_level_info_get(const eamg_hierarchy *h, int32_t level, eamg_level_info *out) {
  return guarded([&] {
    if (!h || !out) fail(EAMG_ERR_INVALID_ARG, "NULL argument");
    reject_fused(h);
    if (level < 0 || level >= int(h->lv.size())) fail(EAMG_ERR_INVALID_ARG, "level out of range");
    const Level &L = h->lv[level];
    const bool last = level + 1 == int(h->lv.size());
    out->n = L.n;
    out->bs = L.bs;
    out->nnzb_A = L.A.nnz();
    out->n_coarse = last ? 0 : h->lv[level + 1].n;
    out->k_coarse = last ? 0 : L.kc;
    out->nnzb_P = last ? 0 : L.P.nnz();
    out->n_colors = last ? 0 : L.ncolors;
  });
}

eamg_status eamg_export_level(const eamg_hierarchy *h, int32_t level, int32_t *agg,
                              int32_t *P_rowptr, int32_t *P_col, double *P_val, int32_t *A_rowptr,
                              int32_t *A_col, double *A_val, int32_t *color) {
  return guarded([&] {
    if (!h) fail(EAMG_ERR_INVALID_ARG, "NULL hierarchy");
    reject_fused(h);
    if (level < 0 || level >= int(h->lv.size())) fail(EAMG_ERR_INVALID_ARG, "level out of range");
    const Level &L = h->lv[level];
    const bool last = level + 1 == int(h->lv.size());
    hipStream_t s = nullptr;
    if (agg)
      for (int i = 0; i < L.n; ++i) agg[i] = last ? -1 : L.agg[i];
    if (color)
      for (int i = 0; i < L.n; ++i) color[i] = last ? -1 : L.color[i];
    if (!last) {
      if (P_rowptr)
        for (int i = 0; i <= L.n; ++i) P_rowptr[i] = int32_t(L.P.rp[i]);
      if (P_col) std::copy(L.P.col.begin(), L.P.col.end(), P_col);
      if (P_val) {
        const auto v = download(L.P_val, size_t(L.P.nnz()) * L.bs * L.kc, s);
        std::copy(v.begin(), v.end(), P_val);
      }
    }
    if (A_rowptr)
      for (int i = 0; i <= L.n; ++i) A_rowptr[i] = int32_t(L.A.rp[i]);
    if (A_col) std::copy(L.A.col.begin(), L.A.col.end(), A_col);
    if (A_val) {
      const auto v = download(L.A_val, size_t(L.A.nnz()) * L.bs * L.bs, s);
      std::copy(v.begin(), v.end(), A_val);
    }
  });
}

eamg_status eamg_traffic_model(const eamg_hierarchy *h, int32_t precision, double *vcycle_bytes,
                               double *iteration_bytes) {
  return guarded([&] {
    if (!h) fail(EAMG_ERR_INVALID_ARG, "NULL hierarchy");
    reject_fused(h);
    if (precision != EAMG_PRECOND_VCYCLE && precision != EAMG_PRECOND_VCYCLE_FP32)
      fail(EAMG_ERR_INVALID_ARG, "precision must be EAMG_PRECOND_VCYCLE or EAMG_PRECOND_VCYCLE_FP32");
    if (precision == EAMG_PRECOND_VCYCLE_FP32 && !h->prm.vcycle_fp32)
      fail(EAMG_ERR_INVALID_ARG, "FP32 V-cycle needs setup with vcycle_fp32 = 1");
    const bool f32 = precision == EAMG_PRECOND_VCYCLE_FP32;
    // the V-cycle as the PCG iteration runs it (FP32: on r's FP32 copy, z left in FP32)
    double v = 0.0;
    for (size_t l = 0; l < h->lv.size(); ++l) {
      const Level &L = h->lv[l];
      if (int(l) == h->tail_level) {
        v += tail_apply_bytes(h, f32 && h->tailS32, f32 ? 4 : 8);
        break;
      }
      if (l + 1 == h->lv.size()) {
        v += double(h->nL) * h->nL * 8.0 + 2.0 * h->nL * (f32 ? 4.0 : 8.0);
        break;
      }
      const double vs = f32 ? 4.0 : 8.0;
      const int bs = L.bs;
      for (const LaunchShape &sh : L.sh_fwd) v += launch_bytes(sh, LK_GS_FWD, bs, bs, vs, 1);
      for (const LaunchShape &sh : L.sh_bwd) v += launch_bytes(sh, LK_GS_BWD, bs, bs, vs, 1);
      v += launch_bytes(L.sh_resid, LK_RESID, bs, bs, vs, 1) +
           launch_bytes(L.sh_R, LK_RECT, L.kc, bs, vs, 1) +
           launch_bytes(L.sh_P, LK_RECT_ACC, bs, L.kc, vs, 1);
    }
    const Level &L0 = h->lv[0];
    const double vec0 = double(L0.n) * L0.bs * 8.0;
    // PCG: SpMV with p.q, x / r update (x rw, r rw, p, q; FP32: r's FP32 copy written), r.z,
    // p update (z, p rw); z in FP32 with the FP32 V-cycle
    const double it = launch_bytes(L0.sh_spmv, LK_SPMV, L0.bs, L0.bs, 8.0, 1) +
                      (f32 ? 6.5 * vec0 + 1.5 * vec0 + 2.5 * vec0 : 6.0 * vec0 + 2.0 * vec0 + 3.0 * vec0);
    if (vcycle_bytes) *vcycle_bytes = v;
    if (iteration_bytes) *iteration_bytes = it + v;
  });
}

eamg_status eamg_solve_coefficients(const eamg_hierarchy *h, int32_t max_entries, double *alpha,
                                    double *beta, int32_t *n_out) {
  return guarded([&] {
    if (!h) fail(EAMG_ERR_INVALID_ARG, "NULL hierarchy");
    reject_fused(h);
    if (max_entries < 0) fail(EAMG_ERR_INVALID_ARG, "max_entries < 0");
    const int n = int(h->cg_alpha.size());
    const int m = std::min(n, max_entries);
    for (int k = 0; k < m; ++k) {
      if (alpha) alpha[k] = h->cg_alpha[size_t(k)];
      if (beta) beta[k] = h->cg_beta[size_t(k)];
    }
    if (n_out) *n_out = n;
  });
}

eamg_status eamg_setup_phases(const eamg_hierarchy *h, int32_t max_entries, eamg_setup_phase *out,
                              int32_t *n_out) {
  return guarded([&] {
    if (!h) fail(EAMG_ERR_INVALID_ARG, "NULL hierarchy");
    reject_fused(h);
    if (max_entries < 0) fail(EAMG_ERR_INVALID_ARG, "max_entries < 0");
    // where each phase runs: 0 host, 1 device, 2 host-to-device copies
    auto where = [](const std::string &name) {
      if (name.find("upload") != std::string::npos) return 2;
      for (const char *d : {"Dirichlet", "numeric", "coarsest factor", "dense tail", "solve vectors"})
        if (name.find(d) != std::string::npos) return 1;
      return 0;
    };
    const int n = int(h->setup_phases.size());
    for (int k = 0; k < std::min(n, max_entries); ++k) {
      const auto &ph = h->setup_phases[size_t(k)];
      std::string nm = ph.first.rfind("setup: ", 0) == 0 ? ph.first.substr(7) : ph.first;
      std::snprintf(out[k].name, sizeof(out[k].name), "%s", nm.c_str());
      out[k].seconds = ph.second;
      out[k].where = where(nm);
    }
    if (n_out) *n_out = n;
  });
}

eamg_status eamg_dense_tail(const eamg_hierarchy *h, int32_t *level, int32_t *dofs) {
  return guarded([&] {
    if (!h) fail(EAMG_ERR_INVALID_ARG, "NULL hierarchy");
    reject_fused(h);
    if (level) *level = h->tail_level;
    if (dofs) *dofs = h->tail_level >= 0 ? h->nT : 0;
  });
}

eamg_status eamg_profile_enable(eamg_hierarchy *h, int32_t on) {
  return guarded([&] {
    if (!h) fail(EAMG_ERR_INVALID_ARG, "NULL hierarchy");
    h->prof_on = on != 0;
    h->prof_levels = on >= 2;
    h->prof_colours = on == 3;
    h->prof.clear();
    h->ev_used = 0;
  });
}

eamg_status eamg_profile_read(eamg_hierarchy *h, int32_t max_entries, eamg_kernel_stat *out,
                              int32_t *n_out) {
  return guarded([&] {
    if (!h || !n_out || (max_entries > 0 && !out)) fail(EAMG_ERR_INVALID_ARG, "NULL argument");
    hip_check(hipDeviceSynchronize(), "sync");
    std::vector<eamg_kernel_stat> agg;
    for (const ProfRec &r : h->prof) {
      float ms = 0.0f;
      hip_check(hipEventElapsedTime(&ms, r.a, r.b), "event");
      auto it = std::find_if(agg.begin(), agg.end(),
                             [&](const eamg_kernel_stat &k) { return r.name == k.name; });
      if (it == agg.end()) {
        eamg_kernel_stat k{};
        std::snprintf(k.name, sizeof(k.name), "%s", r.name.c_str());
        agg.push_back(k);
        it = agg.end() - 1;
      }
      it->launches += r.launches;
      it->total_ms += ms;
      it->bytes += r.bytes;
    }
    std::sort(agg.begin(), agg.end(),
              [](const eamg_kernel_stat &x, const eamg_kernel_stat &y) { return x.total_ms > y.total_ms; });
    *n_out = int32_t(agg.size());
    for (int i = 0; i < std::min<int>(max_entries, int(agg.size())); ++i) out[i] = agg[i];
    h->prof.clear();
    h->ev_used = 0;
  });
}

}  // extern "C"

namespace {

// An auxiliary level from host arrays (eamg_host_match / eamg_criteria_eval arguments).
AuxLevel host_level(int32_t k, int32_t n, const double *coords, int64_t n_edges,
                    const int32_t *edges, const double *E, const double *M) {
  if (k != 1 && k != 6) fail(EAMG_ERR_UNSUPPORTED_KERNEL, "k must be 1 or 6");
  if (n < 0 || n_edges < 0 || !coords || !M || (n_edges && (!edges || !E)))
    fail(EAMG_ERR_INVALID_ARG, "bad arguments");
  AuxLevel lev;
  lev.n = n;
  lev.k = k;
  lev.x.assign(coords, coords + size_t(3) * n);
  lev.e0.resize(size_t(n_edges));
  lev.e1.resize(size_t(n_edges));
  for (int64_t e = 0; e < n_edges; ++e) {
    lev.e0[e] = edges[2 * e];
    lev.e1[e] = edges[2 * e + 1];
    if (lev.e0[e] < 0 || lev.e1[e] >= n || lev.e0[e] >= lev.e1[e])
      fail(EAMG_ERR_INVALID_ARG, "edges must satisfy 0 <= i < j < n");
    if (e && (lev.e0[e - 1] > lev.e0[e] || (lev.e0[e - 1] == lev.e0[e] && lev.e1[e - 1] >= lev.e1[e])))
      fail(EAMG_ERR_INVALID_ARG, "edges must be strictly ascending");
  }
  lev.E.assign(E, E + size_t(n_edges) * k * k);
  lev.M.assign(M, M + size_t(n) * k * k);
  lev.build_adjacency();
  return lev;
}

}  // namespace

extern "C" {

eamg_status eamg_criteria_eval(int32_t k, int32_t n, const double *coords, int64_t n_edges,
                               const int32_t *edges, const double *E, const double *M,
                               int64_t n_pairs, const int32_t *pairs, int64_t n_unions,
                               const int32_t *unions, double tau, int32_t use_device,
                               void *stream, double *out_mub, double *out_mug) {
  return guarded([&] {
    if (n_pairs < 0 || n_unions < 0 || (n_pairs && (!pairs || !out_mub)) ||
        (n_unions && (!unions || !out_mug)) || !(tau >= 0.0) || (use_device != 0 && use_device != 1))
      fail(EAMG_ERR_INVALID_ARG, "bad arguments");
    if (n_pairs > INT32_MAX / 2 || n_unions > INT32_MAX / crit::kMaxUnion)
      fail(EAMG_ERR_INVALID_ARG, "too many pairs or unions");
    const AuxLevel lev = host_level(k, n, coords, n_edges, edges, E, M);
    for (int64_t u = 0; u < n_pairs; ++u) {
      const int i = pairs[2 * u], j = pairs[2 * u + 1];
      if (i < 0 || i >= n || j < 0 || j >= n || lev.edge_id(i, j) < 0)
        fail(EAMG_ERR_INVALID_ARG, "every pair must be an edge of the level");
    }
    for (int64_t u = 0; u < n_unions; ++u) {
      const int32_t *m = unions + crit::kMaxUnion * u;
      if (m[0] < 0 || m[0] >= n) fail(EAMG_ERR_INVALID_ARG, "malformed union");
      for (int a = 1; a < crit::kMaxUnion; ++a)
        if (m[a] >= n || (m[a] >= 0 && !(m[a - 1] >= 0 && m[a - 1] < m[a])))
          fail(EAMG_ERR_INVALID_ARG, "union members must be distinct, ascending, -1 padded");
    }
    std::vector<Sq> D;
    dhat_all(lev, D);
    std::vector<int32_t> pv(pairs, pairs + 2 * n_pairs), uv(unions, unions + crit::kMaxUnion * n_unions);
    std::vector<double> mub(static_cast<size_t>(n_pairs)), mug(static_cast<size_t>(n_unions));
    auto host_g = [&](int64_t u) {
      std::vector<int> C;
      for (int a = 0; a < crit::kMaxUnion; ++a)
        if (uv[crit::kMaxUnion * u + a] >= 0) C.push_back(uv[crit::kMaxUnion * u + a]);
      mug[u] = mu_g(lev, C, D, tau);
    };
    if (use_device) {
      std::unique_ptr<CritBatch> cb = make_device_criteria(static_cast<hipStream_t>(stream));
      cb->level(lev, D);
      cb->work(lev, D);
      cb->mu_b(pv, tau, mub);
      cb->mu_g(uv, tau, mug);
      for (int64_t u = 0; u < n_unions; ++u)
        if (std::isnan(mug[u])) host_g(u);
    } else {
      parallel_for_dynamic(n_pairs, [&](int64_t u) { mub[u] = mu_b(lev, pv[2 * u], pv[2 * u + 1], D, tau); }, 16);
      parallel_for_dynamic(n_unions, host_g, 4);
    }
    if (n_pairs) std::copy(mub.begin(), mub.end(), out_mub);
    if (n_unions) std::copy(mug.begin(), mug.end(), out_mug);
  });
}

eamg_status eamg_host_match(int32_t k, int32_t n, const double *coords, int64_t n_edges,
                            const int32_t *edges, const double *E, const double *M,
                            const uint8_t *vd, const eamg_setup_params *params, int32_t *out_agg,
                            int32_t *out_nc, double *out_ccoords, double *out_margin) {
  return guarded([&] {
    if (!out_agg || !out_nc) fail(EAMG_ERR_INVALID_ARG, "bad arguments");
    const eamg_setup_params prm = params ? *params : defaults();
    validate_params(prm);
    const AuxLevel lev = host_level(k, n, coords, n_edges, edges, E, M);
    std::vector<char> vdm(static_cast<size_t>(n), 0);
    if (vd)
      for (int i = 0; i < n; ++i) vdm[i] = vd[i] ? 1 : 0;
    MatchParams mp;
    mp.sigma = prm.sigma;
    mp.rounds = prm.rounds;
    mp.mu_s_only = prm.mu_s_only != 0;
    mp.tie_rtol = prm.tie_rtol;
    mp.tau = prm.pinv_rtol;
    const MatchResult mr = successive_matching(lev, vdm, mp);
    for (int i = 0; i < n; ++i) out_agg[i] = -1;
    for (size_t I = 0; I < mr.aggs.size(); ++I)
      for (int i : mr.aggs[I]) out_agg[i] = int32_t(I);
    *out_nc = int32_t(mr.aggs.size());
    if (out_ccoords) std::copy(mr.ccoords.begin(), mr.ccoords.end(), out_ccoords);
    if (out_margin) *out_margin = mr.min_margin;
  });
}

}  // extern "C"
