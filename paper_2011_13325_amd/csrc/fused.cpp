// Fused multi-system solve (eamg_fuse, eamg_solve_fused): several independent systems, each
// with its own hierarchy, merged into one block-diagonal hierarchy so that every colour launch,
// transfer and CG vector operation covers all systems at once.
//
// Level l of the fused hierarchy holds level l of every system whose V-cycle reaches it.  Rows
// are numbered colour by colour, and inside a colour system by system (each system's rows of
// that colour in its own order), so a fused colour is again one contiguous row range and an
// independent set: the systems share no couplings.  Systems whose V-cycle ends on level l (at
// their dense tail, or at the coarsest inverse) put all their level-l rows after the colour
// ranges and are applied there as dense operators, all in one launch.  Each system's V-cycle is
// therefore its own V-cycle (the same rows, blocks, colours and dense operators), applied
// together with the others'.  The PCG keeps one set of scalars per system (segmented dot
// products and updates, section "res" per system) and stops each system on its own test;
// converged systems keep their x while the others go on.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <memory>
#include <string>
#include <vector>

#include "../../include/eamg.h"
#include "hierarchy.hpp"
#include "panel.hpp"
#include "structure.hpp"

namespace eamg {

struct FusedInfo {
  std::vector<eamg_hierarchy *> sys;   // not owned
  std::vector<int> depth;              // level whose dense operator ends each system's V-cycle
  std::vector<DenseTail> own;          // tails built for the fused hierarchy (T null: none)
  std::vector<int> n0;                 // level-0 vertices of each system
  std::vector<int *> map0;             // device: natural vertex -> fused level-0 row
  int bs0 = 0;
  SegTable seg;
  std::vector<int> bptr;               // host copy of seg.bptr
  hipStream_t cap = nullptr;
  hipGraphExec_t g[3] = {nullptr, nullptr, nullptr};   // per precond
  bool tried[3] = {false, false, false};
  ~FusedInfo() {
    for (hipGraphExec_t e : g)
      if (e) (void)hipGraphExecDestroy(e);
    if (cap) (void)hipStreamDestroy(cap);
    for (eamg_hierarchy *h : sys)
      if (--h->fused_users == 0 && h->destroy_pending) delete h;
  }
};

void destroy_fused(FusedInfo *f) { delete f; }

namespace {

// Rows of the fused level l: u[m][j] = fused row of row j (the system's solve numbering) of
// system m, for the systems that reach level l.
struct FusedOrder {
  std::vector<std::vector<int>> u;
  std::vector<int> color_ptr;
  std::vector<int> dense_off;   // first fused row of each system applied densely here, or -1
  int n = 0, n_smooth = 0, ncolors = 0, bs = 0;
};

FusedOrder fused_order(const std::vector<eamg_hierarchy *> &hs, const std::vector<int> &depth, int l) {
  const int nsys = int(hs.size());
  FusedOrder o;
  o.u.resize(size_t(nsys));
  o.dense_off.assign(size_t(nsys), -1);
  o.bs = -1;
  for (int m = 0; m < nsys; ++m) {
    if (depth[m] < l) continue;
    const Level &L = hs[m]->lv[size_t(l)];
    if (o.bs < 0) o.bs = L.bs;
    if (L.bs != o.bs) fail(EAMG_ERR_INVALID_ARG, "the systems' levels " + std::to_string(l) + " have different block sizes");
    o.u[m].assign(size_t(L.n), -1);
    if (depth[m] > l) o.ncolors = std::max(o.ncolors, L.ncolors);
  }
  int64_t u = 0;
  o.color_ptr.assign(size_t(o.ncolors) + 1, 0);
  for (int c = 0; c < o.ncolors; ++c) {
    o.color_ptr[size_t(c)] = int(u);
    for (int m = 0; m < nsys; ++m) {
      if (depth[m] <= l) continue;
      const Level &L = hs[m]->lv[size_t(l)];
      if (c >= L.ncolors) continue;
      for (int j = L.color_ptr[size_t(c)]; j < L.color_ptr[size_t(c) + 1]; ++j) o.u[m][size_t(j)] = int(u++);
    }
  }
  o.color_ptr[size_t(o.ncolors)] = int(u);
  o.n_smooth = int(u);
  for (int m = 0; m < nsys; ++m) {
    if (depth[m] != l) continue;
    const Level &L = hs[m]->lv[size_t(l)];
    o.dense_off[m] = int(u);
    for (int j = 0; j < L.n; ++j) o.u[m][size_t(j)] = int(u++);
  }
  if (u > int64_t(2147483647) / 8) fail(EAMG_ERR_INVALID_ARG, "fused level too large");
  o.n = int(u);
  return o;
}

// Device copy of several device arrays back to back; returns the start of each.
double *concat_device(DevArena &ar, const std::vector<std::pair<const double *, size_t>> &parts,
                      std::vector<size_t> &start, hipStream_t s) {
  size_t total = 0;
  start.clear();
  for (const auto &p : parts) {
    start.push_back(total);
    total += p.second;
  }
  double *d = ar.alloc<double>(total);
  for (size_t k = 0; k < parts.size(); ++k)
    if (parts[k].second)
      hip_check(hipMemcpyAsync(d + start[k], parts[k].first, parts[k].second * sizeof(double),
                               hipMemcpyDeviceToDevice, s),
                "copy");
  return d;
}

void build_fused_level(eamg_hierarchy *F, const std::vector<eamg_hierarchy *> &hs,
                       const std::vector<int> &depth, const std::vector<FusedOrder> &ord, int l,
                       hipStream_t s) {
  const int nsys = int(hs.size());
  const FusedOrder &o = ord[size_t(l)];
  const bool last = size_t(l) + 1 == ord.size();
  const bool f32 = F->prm.vcycle_fp32 != 0;
  DevArena &ar = F->arena;
  Level &L = F->lv[size_t(l)];
  L.n = o.n;
  L.bs = o.bs;
  L.n_smooth = o.n_smooth;
  L.ncolors = o.ncolors;
  L.color_ptr = o.color_ptr;
  const int bs = o.bs;
  // the level matrices of every system that reaches level l, concatenated in the natural
  // numbering, then permuted into the fused order
  Pattern Acat;
  std::vector<std::pair<const double *, size_t>> vparts;
  std::vector<int> perm(size_t(o.n), -1);
  {
    int64_t nb = 0;
    Acat.rp.push_back(0);
    for (int m = 0; m < nsys; ++m) {
      if (depth[m] < l) continue;
      const Level &S = hs[m]->lv[size_t(l)];
      const int64_t qb = Acat.rp.back();
      for (int i = 0; i < S.n; ++i) Acat.rp.push_back(qb + S.A.rp[size_t(i) + 1]);
      for (int c : S.A.col) Acat.col.push_back(int(nb + c));
      vparts.emplace_back(S.A_val, size_t(S.A.nnz()) * bs * bs);
      for (int j = 0; j < S.n; ++j) perm[size_t(o.u[m][size_t(j)])] = int(nb + S.perm[size_t(j)]);
      nb += S.n;
    }
    Acat.n_rows = Acat.n_cols = int(nb);
    if (nb != o.n) fail(EAMG_ERR_INVALID_ARG, "fused level rows do not add up");
  }
  std::vector<int> inv(size_t(o.n));
  for (int r = 0; r < o.n; ++r) inv[size_t(perm[size_t(r)])] = r;
  std::vector<size_t> vstart;
  double *vcat = concat_device(ar, vparts, vstart, s);
  std::vector<int64_t> src;
  const Pattern Ap = permute_pattern(Acat, perm, inv, src);
  std::vector<int> dg;
  L.Am = make_solve_mat(ar, Ap, src, bs, bs, vcat, s, &dg, false, f32);
  if (o.n_smooth > 0) {
    attach_split_parts(ar, Ap, src, dg, bs, vcat, s, f32, L.Am);
    level_shapes(L, Ap, dg);
  } else {
    L.sh_spmv = matrix_shape(Ap);
  }
  hip_check(hipStreamSynchronize(s), "sync");
  ar.release(vcat);
  if (o.n_smooth > 0) {
    // smoother diagonals of the smoothed rows, gathered from the systems' own (solve order)
    std::vector<std::pair<const double *, size_t>> dparts;
    std::vector<int> sysidx;
    for (int m = 0; m < nsys; ++m)
      if (depth[m] > l) {
        dparts.emplace_back(hs[m]->lv[size_t(l)].Dinv, size_t(hs[m]->lv[size_t(l)].n) * bs * bs);
        sysidx.push_back(m);
      }
    std::vector<size_t> dstart;
    double *dcat = concat_device(ar, dparts, dstart, s);
    std::vector<int> gmap(size_t(o.n_smooth), -1);
    for (size_t k = 0; k < sysidx.size(); ++k) {
      const int m = sysidx[k];
      const int base = int(dstart[k] / size_t(bs * bs));
      for (int j = 0; j < hs[m]->lv[size_t(l)].n; ++j) gmap[size_t(o.u[m][size_t(j)])] = base + j;
    }
    int *gmap_d = ar.upload(gmap, s);
    L.Dinv = ar.alloc<double>(size_t(o.n_smooth) * bs * bs);
    hip_check(launch_gather_rows(o.n_smooth, bs * bs, gmap_d, dcat, L.Dinv, s), "gather_rows");
    if (f32) {
      L.Dinv32 = ar.alloc<float>(size_t(o.n_smooth) * bs * bs);
      hip_check(launch_convert(int64_t(o.n_smooth) * bs * bs, L.Dinv, L.Dinv32, s), "convert");
    }
    // transfers: P of the smoothed systems, rows in the fused order of level l, columns in the
    // fused order of level l + 1
    const FusedOrder &oc = ord[size_t(l) + 1];
    int kc = -1;
    Pattern Pcat;
    std::vector<std::pair<const double *, size_t>> pparts;
    std::vector<int> prow(size_t(o.n_smooth), -1);
    std::vector<int> icol;
    {
      int64_t rb = 0, cb = 0;
      Pcat.rp.push_back(0);
      for (int m : sysidx) {
        const Level &S = hs[m]->lv[size_t(l)];
        const Level &Sc = hs[m]->lv[size_t(l) + 1];
        if (kc < 0) kc = S.kc;
        if (S.kc != kc || Sc.bs != kc) fail(EAMG_ERR_INVALID_ARG, "the systems' coarse block sizes differ");
        const int64_t qb = Pcat.rp.back();
        for (int i = 0; i < S.n; ++i) Pcat.rp.push_back(qb + S.P.rp[size_t(i) + 1]);
        for (int c : S.P.col) Pcat.col.push_back(int(cb + c));
        pparts.emplace_back(S.P_val, size_t(S.P.nnz()) * bs * kc);
        for (int j = 0; j < S.n; ++j) prow[size_t(o.u[m][size_t(j)])] = int(rb + S.perm[size_t(j)]);
        for (int w = 0; w < Sc.n; ++w) icol.push_back(oc.u[m][size_t(Sc.inv[size_t(w)])]);
        rb += S.n;
        cb += Sc.n;
      }
      Pcat.n_rows = int(rb);
      Pcat.n_cols = int(cb);
      if (rb != o.n_smooth || cb != oc.n) fail(EAMG_ERR_INVALID_ARG, "fused transfer sizes do not add up");
    }
    std::vector<size_t> pstart;
    double *pcat = concat_device(ar, pparts, pstart, s);
    std::vector<int64_t> srcP;
    const Pattern Pp = permute_rect(Pcat, prow, icol, srcP);
    L.kc = kc;
    L.Pm = make_solve_mat(ar, Pp, srcP, bs, kc, pcat, s, nullptr, false, f32);
    std::vector<int64_t> srcT;
    const Pattern Rp = transpose_pattern(Pp, srcT);
    std::vector<int64_t> srcR(srcT.size());
    for (size_t q = 0; q < srcT.size(); ++q) srcR[q] = srcP[size_t(srcT[q])];
    L.Rm = make_solve_mat(ar, Rp, srcR, kc, bs, pcat, s, nullptr, true, f32);
    L.sh_R = matrix_shape(Rp);
    L.sh_P = matrix_shape(Pp);
    hip_check(hipStreamSynchronize(s), "sync");
    ar.release(pcat);
    ar.release(dcat);
    ar.release(gmap_d);
  } else if (!last) {
    fail(EAMG_ERR_INVALID_ARG, "fused level without smoothed systems above the last level");
  }
  // dense operators of the systems whose V-cycle ends here, as packed upper tiles (each is a
  // symmetric V-cycle operator or coarsest inverse): [0] the FP64 V-cycle, [1] the FP32 V-cycle
  // with FP32 tails (every system set up with dense_tail_fp32), [2] the FP32 V-cycle with FP64
  // matrices (coarsest inverses, and the tails otherwise)
  struct Part {
    const void *S;
    int64_t off;
    int n, sys;
  };
  std::vector<Part> d64, d32f, d32d;
  for (int m = 0; m < nsys; ++m) {
    if (depth[m] != l) continue;
    const eamg_hierarchy *H = hs[m];
    const int n = H->lv[size_t(l)].n * bs;
    const int64_t off = int64_t(o.dense_off[m]) * bs;
    const DenseTail &own = F->fused->own[size_t(m)];
    const double *S = nullptr;
    const float *S32 = nullptr;
    bool tail = true;
    if (own.T) {
      // built for the fused hierarchy
      if (own.n != n) fail(EAMG_ERR_INVALID_ARG, "dense tail size mismatch");
      double *P = ar.alloc<double>(sym_entries(n));
      hip_check(launch_pack_sym<double>(n, own.ld, own.T, P, s), "pack tail");
      S = P;
      if (f32 && F->prm.dense_tail_fp32) {
        float *P32 = ar.alloc<float>(sym_entries(n));
        hip_check(launch_pack_sym<float>(n, own.ld, own.T, P32, s), "pack tail f32");
        S32 = P32;
      }
    } else if (H->tail_level == l && H->tailS) {
      // the system's own tail
      if (H->nT != n) fail(EAMG_ERR_INVALID_ARG, "dense tail size mismatch");
      S = H->tailS;
      S32 = F->prm.dense_tail_fp32 ? H->tailS32 : nullptr;
    } else {
      if (H->nL != n || !H->Ainv) fail(EAMG_ERR_INVALID_ARG, "coarsest inverse size mismatch");
      double *P = ar.alloc<double>(sym_entries(n));
      hip_check(launch_pack_sym<double>(n, H->ldL, H->Ainv, P, s), "pack coarsest inverse");
      S = P;
      tail = false;
    }
    d64.push_back({S, off, n, m});
    if (f32 && tail && S32)
      d32f.push_back({S32, off, n, m});
    else if (f32)
      d32d.push_back({S, off, n, m});   // FP64 matrix, as the coarsest inverse is read
  }
  auto set_of = [&](const std::vector<Part> &v, size_t tm, size_t tv, DenseSet &d) {
    std::vector<SymPart> sp;
    int rows = 0, tiles = 0;
    int64_t wn = 0;
    double by = 0.0;
    for (const Part &q : v) {
      SymPart x{};
      x.S = q.S;
      x.off = q.off;
      x.woff = wn;
      x.n = q.n;
      x.nb = sym_blocks(q.n);
      x.row0 = rows;
      x.t0 = tiles;
      x.sys = q.sys;
      sp.push_back(x);
      rows += q.n;
      tiles += int(sym_tiles(x.nb));
      wn += int64_t(sym_work_doubles(q.n));
      by += double(sym_entries(q.n)) * tm + 2.0 * 8.0 * double(sym_work_doubles(q.n)) + 2.0 * q.n * double(tv);
    }
    d.count = int(sp.size());
    d.rows = rows;
    d.tiles = tiles;
    d.bytes = by;
    d.parts = sp.empty() ? nullptr : ar.upload(sp, s);
    d.W = sp.empty() ? nullptr : ar.alloc<double>(size_t(wn));
  };
  set_of(d64, 8, 8, L.dense[0]);
  set_of(d32f, 4, 4, L.dense[1]);
  set_of(d32d, 8, 4, L.dense[2]);
  // level vectors (level 0 in FP64 uses the CG vectors r and z)
  const size_t nv = size_t(o.n) * bs;
  if (o.n_smooth > 0) L.r = ar.alloc<double>(nv);
  if (l > 0) {
    L.b = ar.alloc<double>(nv);
    L.x = ar.alloc<double>(nv);
  }
  if (f32) {
    if (o.n_smooth > 0) L.r32 = ar.alloc<float>(nv);
    L.b32 = ar.alloc<float>(nv);
    L.x32 = ar.alloc<float>(nv);
  }
}

void check_params(const eamg_hierarchy *F, const eamg_solve_params &sp) {
  if (sp.max_it < 1) fail(EAMG_ERR_INVALID_ARG, "max_it must be >= 1");
  if (!(sp.rtol >= 0.0)) fail(EAMG_ERR_INVALID_ARG, "rtol must be >= 0");
  if (sp.precond < EAMG_PRECOND_NONE || sp.precond > EAMG_PRECOND_VCYCLE_FP32)
    fail(EAMG_ERR_INVALID_ARG, "precond must be 0, 1 or 2");
  if (sp.precond == EAMG_PRECOND_VCYCLE_FP32 && !F->prm.vcycle_fp32)
    fail(EAMG_ERR_INVALID_ARG, "FP32 V-cycle needs every fused hierarchy set up with vcycle_fp32 = 1");
}

void fused_precondition(eamg_hierarchy *F, int precond, hipStream_t s) {
  const int64_t N = int64_t(F->lv[0].n) * F->lv[0].bs;
  if (precond == EAMG_PRECOND_NONE)
    hip_check(launch_copy(N, F->r, F->z, s), "copy");
  else
    vcycle_apply(F, F->r, F->z, precond == EAMG_PRECOND_VCYCLE_FP32, s);
}

// One PCG iteration of every system after its stopping test (inactive systems keep x, r, p).
void fused_iteration(eamg_hierarchy *F, int precond, hipStream_t s) {
  const SegTable &T = F->fused->seg;
  const SolveMat &A = F->lv[0].Am;
  fused_precondition(F, precond, s);
  hip_check(launch_sdot(T, F->r, F->z, F->part, s), "sdot");
  hip_check(launch_sreduce(T, F->part, F->scal, PS_RZ, PRED_BETA, s), "sreduce");
  hip_check(launch_supdate_p(T, F->scal, F->z, F->p, s), "supdate_p");
  hip_check(launch_spmv(A, F->p, F->q, nullptr, s), "spmv");
  hip_check(launch_sdot(T, F->p, F->q, F->part, s), "sdot");
  hip_check(launch_sreduce(T, F->part, F->scal, PS_PQ, PRED_ALPHA, s), "sreduce");
  hip_check(launch_supdate_xr(T, F->scal, F->x, F->r, F->p, F->q, F->part, s), "supdate_xr");
  hip_check(launch_sreduce(T, F->part, F->scal, PS_RR, PRED_RR, s), "sreduce");
}

// Iterations per round: the host reads the systems' active flags once a round (a system that
// stops inside a round keeps its x, r and p through the rest of it).
constexpr int kRound = 4;

// Capture one round of kRound iterations as one graph.
void fused_graph(eamg_hierarchy *F, int precond) {
  FusedInfo &I = *F->fused;
  I.tried[precond] = true;
  if (const char *e = std::getenv("EAMG_GRAPH"))
    if (std::atoi(e) == 0) return;
  if (!I.cap && hipStreamCreateWithFlags(&I.cap, hipStreamNonBlocking) != hipSuccess) {
    I.cap = nullptr;
    return;
  }
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(I.cap, hipStreamCaptureModeRelaxed) != hipSuccess) return;
  bool ok = true;
  try {
    for (int k = 0; k < kRound; ++k) fused_iteration(F, precond, I.cap);
  } catch (const Failure &) {
    ok = false;
  }
  if (hipStreamEndCapture(I.cap, &g) != hipSuccess || !ok) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return;
  }
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) I.g[precond] = ex;
  (void)hipGraphDestroy(g);
  (void)hipGetLastError();
}

}  // namespace

void invalidate_fused_graphs(eamg_hierarchy *h) {
  if (!h->fused) return;
  for (int p = 0; p < 3; ++p) {
    if (h->fused->g[p]) (void)hipGraphExecDestroy(h->fused->g[p]);
    h->fused->g[p] = nullptr;
    h->fused->tried[p] = false;
  }
}

}  // namespace eamg

using namespace eamg;

extern "C" {

eamg_status eamg_fuse(int32_t nsys, eamg_hierarchy *const *hs, int32_t dense_tail_dofs,
                      void *stream, eamg_hierarchy **out) {
  return guarded([&] {
    if (!out) fail(EAMG_ERR_INVALID_ARG, "NULL output");
    *out = nullptr;
    if (nsys < 1 || !hs) fail(EAMG_ERR_INVALID_ARG, "NULL argument or nsys < 1");
    if (dense_tail_dofs < -1 || dense_tail_dofs > kMaxCoarsestDofs)
      fail(EAMG_ERR_INVALID_ARG, "dense_tail_dofs must be -1 or in [0, 16384]");
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    std::vector<eamg_hierarchy *> sys(hs, hs + nsys);
    for (int m = 0; m < nsys; ++m) {
      if (!sys[m]) fail(EAMG_ERR_INVALID_ARG, "NULL hierarchy");
      if (sys[m]->fused) fail(EAMG_ERR_INVALID_ARG, "a fused hierarchy cannot be fused again");
      if (sys[m]->device != dev) fail(EAMG_ERR_INVALID_ARG, "every hierarchy must live on the current device");
      if (sys[m]->dim != sys[0]->dim || sys[m]->lv[0].bs != sys[0]->lv[0].bs)
        fail(EAMG_ERR_INVALID_ARG, "the systems differ in dimension or block size");
      for (int k = 0; k < m; ++k)
        if (sys[k] == sys[m]) fail(EAMG_ERR_INVALID_ARG, "a hierarchy may appear only once");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto F = std::make_unique<eamg_hierarchy>();
    F->dim = sys[0]->dim;
    F->k = sys[0]->k;
    F->device = dev;
    F->prm = sys[0]->prm;
    F->prm.vcycle_fp32 = 1;
    F->prm.dense_tail_fp32 = 1;
    for (eamg_hierarchy *H : sys) {
      F->prm.vcycle_fp32 = F->prm.vcycle_fp32 && H->prm.vcycle_fp32;
      // FP32 dense tails only if every system asked for them
      F->prm.dense_tail_fp32 = F->prm.dense_tail_fp32 && H->prm.dense_tail_fp32;
    }
    F->tail_level = -1;
    auto info = std::make_unique<FusedInfo>();
    info->sys = sys;
    for (eamg_hierarchy *H : sys) ++H->fused_users;
    int U = 0;
    info->own.resize(size_t(nsys));
    for (int m = 0; m < nsys; ++m) {
      eamg_hierarchy *H = sys[size_t(m)];
      const int nl = int(H->lv.size());
      int d = nl - 1;
      if (dense_tail_dofs < 0 && H->tail_level >= 0) d = H->tail_level;
      if (dense_tail_dofs > 0)
        for (int l = 1; l + 1 < nl; ++l)
          if (int64_t(H->lv[size_t(l)].n) * H->lv[size_t(l)].bs <= dense_tail_dofs) {
            d = l;
            break;
          }
      info->depth.push_back(d);
      U = std::max(U, d + 1);
    }
    std::vector<FusedOrder> ord;
    for (int l = 0; l < U; ++l) ord.push_back(fused_order(sys, info->depth, l));
    F->lv.resize(size_t(U));
    F->fused = info.release();
    // dense tails of the fused hierarchy's own size (the systems' own tails are read in place)
    if (dense_tail_dofs > 0)
      for (int m = 0; m < nsys; ++m) {
        eamg_hierarchy *H = sys[size_t(m)];
        const int d = F->fused->depth[size_t(m)];
        if (d + 1 < int(H->lv.size()) && H->tail_level != d)
          F->fused->own[size_t(m)] =
              make_dense_tail(H, size_t(d), F->arena, s);
      }
    for (int l = 0; l < U; ++l) build_fused_level(F.get(), sys, F->fused->depth, ord, l, s);
    // level 0: natural -> fused maps, segments of the CG vectors, CG workspace
    FusedInfo &I = *F->fused;
    const FusedOrder &o0 = ord[0];
    I.bs0 = o0.bs;
    std::vector<int> bsys;
    std::vector<int64_t> bd0, bd1;
    I.bptr.assign(size_t(nsys) + 1, 0);
    for (int m = 0; m < nsys; ++m) {
      const Level &S = sys[m]->lv[0];
      std::vector<int> mp(size_t(S.n));
      for (int v = 0; v < S.n; ++v) mp[size_t(v)] = o0.u[m][size_t(S.inv[size_t(v)])];
      I.n0.push_back(S.n);
      I.map0.push_back(F->arena.upload(mp, s));
      // runs of consecutive fused rows of system m, in increasing order
      std::vector<int> rows = o0.u[m];
      std::sort(rows.begin(), rows.end());
      size_t a = 0;
      while (a < rows.size()) {
        size_t b = a + 1;
        while (b < rows.size() && rows[b] == rows[b - 1] + 1) ++b;
        const int64_t r0 = int64_t(rows[a]) * I.bs0, r1 = int64_t(rows[b - 1] + 1) * I.bs0;
        for (int64_t c = r0; c < r1; c += kSegChunk) {
          bsys.push_back(m);
          bd0.push_back(c);
          bd1.push_back(std::min(r1, c + kSegChunk));
        }
        a = b;
      }
      I.bptr[size_t(m) + 1] = int(bsys.size());
    }
    I.seg.nsys = nsys;
    I.seg.nblk = int(bsys.size());
    I.seg.sys = F->arena.upload(bsys, s);
    I.seg.d0 = F->arena.upload(bd0, s);
    I.seg.d1 = F->arena.upload(bd1, s);
    I.seg.bptr = F->arena.upload(I.bptr, s);
    const int64_t N = int64_t(o0.n) * I.bs0;
    F->n0 = o0.n;
    for (double **v : {&F->x, &F->r, &F->z, &F->p, &F->q, &F->bp}) *v = F->arena.alloc<double>(size_t(N));
    F->part_cap = std::max(1, I.seg.nblk);
    F->part = F->arena.alloc<double>(size_t(F->part_cap));
    F->scal = F->arena.alloc<double>(size_t(PS_COUNT) * nsys);
    // a system whose CG has stopped skips its dense operator
    for (Level &L : F->lv)
      for (DenseSet &d : L.dense) d.active = F->scal + size_t(PS_ACTIVE) * nsys;
    hip_check(hipHostMalloc(reinterpret_cast<void **>(&F->scal_h), sizeof(double) * PS_COUNT * nsys,
                            hipHostMallocDefault),
              "hipHostMalloc");
    hip_check(hipStreamSynchronize(s), "sync");
    *out = F.release();
  });
}

eamg_status eamg_solve_fused(eamg_hierarchy *F, const double *const *b_dev, double *const *x_dev,
                             const eamg_solve_params *params, void *stream, eamg_solve_info *infos) {
  bool all = true;
  const eamg_status st = guarded([&] {
    if (!F || !F->fused) fail(EAMG_ERR_INVALID_ARG, "not a fused hierarchy (eamg_fuse)");
    if (!b_dev || !x_dev) fail(EAMG_ERR_INVALID_ARG, "NULL argument");
    FusedInfo &I = *F->fused;
    const int nsys = int(I.sys.size());
    for (int m = 0; m < nsys; ++m) {
      if (!b_dev[m] || !x_dev[m]) fail(EAMG_ERR_INVALID_ARG, "NULL vector");
      if (b_dev[m] == x_dev[m]) fail(EAMG_ERR_INVALID_ARG, "b and x may not alias");
    }
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev != F->device) fail(EAMG_ERR_INVALID_ARG, "the current device is not the fused hierarchy's");
    eamg_solve_params sp;
    eamg_default_solve_params(&sp);
    if (params) sp = *params;
    check_params(F, sp);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const SegTable &T = I.seg;
    const Level &L0 = F->lv[0];
    const SolveMat &A = L0.Am;
    const int64_t N = int64_t(L0.n) * L0.bs;
    const int pc = sp.precond;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hip_check(hipEventCreate(&e0), "event");
    struct Ev {
      hipEvent_t &a, &b;
      ~Ev() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
      }
    } ev_guard{e0, e1};
    hip_check(hipEventCreate(&e1), "event");
    hip_check(hipEventRecord(e0, s), "event");
    // start: b in, x0, r, z = V(r), p = z and the first iteration, all systems together
    hip_check(launch_sinit(nsys, sp.rtol, sp.max_it, F->scal, s), "sinit");
    for (int m = 0; m < nsys; ++m)
      hip_check(launch_scatter_in(I.n0[m], I.bs0, I.map0[m], I.sys[m]->dir, b_dev[m], F->bp, s), "scatter");
    hip_check(launch_sfinite(T, F->bp, F->scal, s), "sfinite");
    hip_check(launch_sdot(T, F->bp, F->bp, F->part, s), "sdot");
    hip_check(launch_sreduce(T, F->part, F->scal, PS_BB, PRED_INIT, s), "sreduce");
    if (sp.use_x0) {
      for (int m = 0; m < nsys; ++m)
        hip_check(launch_scatter_in(I.n0[m], I.bs0, I.map0[m], I.sys[m]->dir, x_dev[m], F->x, s), "scatter");
      hip_check(launch_spmv(A, F->x, F->q, nullptr, s), "spmv");
      hip_check(launch_sub(N, F->bp, F->q, F->r, s), "sub");
    } else {
      hip_check(launch_fill(N, 0.0, F->x, s), "fill");
      hip_check(launch_copy(N, F->bp, F->r, s), "copy");
    }
    hip_check(launch_sdot(T, F->r, F->r, F->part, s), "sdot");
    hip_check(launch_sreduce(T, F->part, F->scal, PS_RR0, PRED_STORE, s), "sreduce");
    fused_precondition(F, pc, s);
    hip_check(launch_copy(N, F->z, F->p, s), "copy");
    hip_check(launch_sdot(T, F->r, F->z, F->part, s), "sdot");
    hip_check(launch_sreduce(T, F->part, F->scal, PS_RHO, PRED_RHO0, s), "sreduce");
    hip_check(launch_spmv(A, F->p, F->q, nullptr, s), "spmv");
    hip_check(launch_sdot(T, F->p, F->q, F->part, s), "sdot");
    hip_check(launch_sreduce(T, F->part, F->scal, PS_PQ, PRED_ALPHA, s), "sreduce");
    hip_check(launch_supdate_xr(T, F->scal, F->x, F->r, F->p, F->q, F->part, s), "supdate_xr");
    hip_check(launch_sreduce(T, F->part, F->scal, PS_RR, PRED_RR, s), "sreduce");
    const bool graphs = !F->prof_on;
    if (graphs && !I.tried[pc]) fused_graph(F, pc);
    // rounds of kRound iterations, one graph launch each
    for (;;) {
      hip_check(hipMemcpyAsync(F->scal_h, F->scal + size_t(PS_ACTIVE) * nsys, sizeof(double) * nsys,
                               hipMemcpyDeviceToHost, s),
                "copy");
      hip_check(hipStreamSynchronize(s), "sync");
      bool any = false;
      for (int m = 0; m < nsys; ++m) any = any || F->scal_h[m] != 0.0;
      if (!any) break;
      if (graphs && I.g[pc])
        hip_check(hipGraphLaunch(I.g[pc], s), "graph launch");
      else
        for (int k = 0; k < kRound; ++k) fused_iteration(F, pc, s);
    }
    // true residuals (slot RZ), then x out
    hip_check(launch_spmv(A, F->x, F->q, nullptr, s), "spmv");
    hip_check(launch_sub(N, F->bp, F->q, F->z, s), "sub");
    hip_check(launch_sdot(T, F->z, F->z, F->part, s), "sdot");
    hip_check(launch_sreduce(T, F->part, F->scal, PS_RZ, PRED_STORE, s), "sreduce");
    hip_check(hipMemcpyAsync(F->scal_h, F->scal, sizeof(double) * PS_COUNT * nsys,
                             hipMemcpyDeviceToHost, s),
              "copy");
    hip_check(hipStreamSynchronize(s), "sync");
    std::vector<double> S(F->scal_h, F->scal_h + size_t(PS_COUNT) * nsys);
    for (int m = 0; m < nsys; ++m) {
      auto at = [&](int slot) { return S[size_t(slot) * nsys + m]; };
      if (at(PS_BAD) != 0.0) continue;   // breakdown: x is not written
      const int64_t nm = int64_t(I.n0[m]) * I.bs0;
      if (at(PS_BB) == 0.0)
        hip_check(launch_fill(nm, 0.0, x_dev[m], s), "fill");
      else
        hip_check(launch_gather_out(I.n0[m], I.bs0, I.map0[m], F->x, x_dev[m], s), "gather");
    }
    hip_check(hipEventRecord(e1, s), "event");
    hip_check(hipStreamSynchronize(s), "sync");
    float fms = 0.0f;
    hip_check(hipEventElapsedTime(&fms, e0, e1), "event");
    for (int m = 0; m < nsys; ++m) {
      auto at = [&](int slot) { return S[size_t(slot) * nsys + m]; };
      const double bn = std::sqrt(at(PS_BB));
      const bool bad = at(PS_BAD) != 0.0, conv = at(PS_CONV) != 0.0;
      all = all && conv && !bad;
      if (infos) {
        eamg_solve_info &inf = infos[m];
        inf.iterations = int32_t(at(PS_ITS));
        const bool ok = bn > 0.0 && std::isfinite(bn);
        inf.rel_res = ok ? std::sqrt(at(PS_RR)) / bn : 0.0;
        inf.rel_res_true = ok ? std::sqrt(at(PS_RZ)) / bn : 0.0;
        if (bad && at(PS_ITS) == 0.0) inf.rel_res = inf.rel_res_true = 0.0;
        inf.ms = fms;
        inf.status = bad ? EAMG_ERR_BREAKDOWN : conv ? EAMG_OK : EAMG_NOT_CONVERGED;
      }
    }
  });
  if (st == EAMG_OK && !all) {
    g_last_error = "some systems did not converge";
    return EAMG_NOT_CONVERGED;
  }
  return st;
}

}  // extern "C"
