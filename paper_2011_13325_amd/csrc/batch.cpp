// Batched block-panel PCG (eamg_solve_batch): K right-hand sides share every matrix stream of
// the V-cycle and of the CG operator, each column keeping its own CG recurrence.  The
// preconditioner is the same V-cycle as the single-vector path (same colours, same transfers,
// same coarsest inverse), applied to K columns per launch.
#include <algorithm>
#include <cmath>
#include <functional>
#include <cstdlib>
#include <memory>
#include <string>

#include "hierarchy.hpp"
#include "panel.hpp"

namespace eamg {

struct BatchWork {
  int K = 0;
  DevArena arena;
  // level-0 CG panels (FP64, colour-major, interleaved)
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *bp = nullptr;
  double *part = nullptr, *scal = nullptr;
  double *scal_h = nullptr;   // pinned
  double *dense = nullptr;    // slices of the coarsest panel product
  // V-cycle panels per precision ([0] FP64, [1] FP32) and level: x, b, r
  bool have[2] = {false, false};
  std::vector<void *> vx[2], vb[2], vr[2];
  hipStream_t cap = nullptr;
  hipGraphExec_t g[2] = {nullptr, nullptr};
  bool tried[2] = {false, false};
  ~BatchWork() {
    for (hipGraphExec_t e : g)
      if (e) (void)hipGraphExecDestroy(e);
    if (cap) (void)hipStreamDestroy(cap);
    if (scal_h) (void)hipHostFree(scal_h);
  }
};

void destroy_batch(BatchWork *w) { delete w; }

namespace {

int panel_width(int m) {
  int K = 1;
  while (K < m) K <<= 1;
  return K;
}

int64_t level_dofs(const Level &L) { return int64_t(L.n) * L.bs; }

BatchWork *ensure_work(eamg_hierarchy *h, int K, bool f32) {
  if (h->batch && h->batch->K != K) {
    hip_check(hipDeviceSynchronize(), "sync");
    destroy_batch(h->batch);
    h->batch = nullptr;
  }
  if (!h->batch) {
    auto w = std::make_unique<BatchWork>();
    w->K = K;
    const Level &L0 = h->lv[0];
    const int64_t N = level_dofs(L0) * K;
    w->x = w->arena.alloc<double>(N);
    w->r = w->arena.alloc<double>(N);
    w->z = w->arena.alloc<double>(N);
    w->p = w->arena.alloc<double>(N);
    w->q = w->arena.alloc<double>(N);
    w->bp = w->arena.alloc<double>(N);
    const int nparts = std::max(pdot_blocks(N), pspmv_blocks(L0.Am, K));
    w->part = w->arena.alloc<double>(size_t(nparts) * K);
    w->scal = w->arena.alloc<double>(size_t(PS_COUNT) * K);
    w->dense = w->arena.alloc<double>(std::max<size_t>(
        1, std::max(dense_panel_work_doubles(h->nL, K), dense_panel_work_doubles(h->nT, K))));
    hip_check(hipHostMalloc(reinterpret_cast<void **>(&w->scal_h), sizeof(double) * PS_COUNT * K,
                            hipHostMallocDefault),
              "hipHostMalloc");
    h->batch = w.release();
  }
  BatchWork *w = h->batch;
  const int p = f32 ? 1 : 0;
  if (!w->have[p]) {
    const size_t vsz = f32 ? sizeof(float) : sizeof(double);
    const size_t nl = h->lv.size();
    w->vx[p].assign(nl, nullptr);
    w->vb[p].assign(nl, nullptr);
    w->vr[p].assign(nl, nullptr);
    for (size_t l = 0; l < nl; ++l) {
      const size_t n = size_t(level_dofs(h->lv[l])) * K * vsz;
      const bool coarsest = l + 1 == nl;
      // FP64 level 0 uses the CG panels r (right-hand side) and z (result) directly
      if (l > 0 || f32) {
        w->vx[p][l] = w->arena.alloc<char>(n);
        w->vb[p][l] = w->arena.alloc<char>(n);
      }
      if (!coarsest) w->vr[p][l] = w->arena.alloc<char>(n);
    }
    w->have[p] = true;
  }
  return w;
}

template <class T>
T *vp(void *v) {
  return static_cast<T *>(v);
}

template <class T>
void pvcycle_t(eamg_hierarchy *h, BatchWork *w, size_t l, const T *b, T *x, hipStream_t s) {
  const int K = w->K;
  const int pi = sizeof(T) == 4 ? 1 : 0;
  const std::string ty = type_name<T>();
  const double vs = sizeof(T);
  Level &L = h->lv[l];
  if (int(l) == h->tail_level) {
    const double by = double(h->nT) * h->nT * 8.0 + 2.0 * h->nT * K * vs;
    timed(h, "dense tail", lvname(h, l, "k_dense_panel_mfma<" + ty + ">"), by, s,
          [&] { return launch_dense_panel<T>(h->nT, h->ldT, K, h->tail, b, x, w->dense, s); });
    return;
  }
  if (l + 1 == h->lv.size()) {
    const double by = double(h->nL) * h->nL * 8.0 + 2.0 * h->nL * K * vs;
    timed(h, "coarsest", lvname(h, l, "k_dense_panel_mfma<" + ty + ">"), by, s,
          [&] { return launch_dense_panel<T>(h->nL, h->ldL, K, h->Ainv, b, x, w->dense, s); });
    return;
  }
  const int bs = L.bs;
  const T *Dinv = bufs<T>(L).Dinv;
  T *R = vp<T>(w->vr[pi][l]);
  double fwd_bytes = 0.0, bwd_bytes = 0.0;
  for (int c = 0; c < L.ncolors; ++c) {
    fwd_bytes += launch_bytes(L.sh_fwd[c], LK_GS_FWD, bs, bs, vs, K);
    bwd_bytes += launch_bytes(L.sh_bwd[c], LK_GS_BWD, bs, bs, vs, K);
  }
  const std::string gs = "k_pgs_color<" + ty + ", " + std::to_string(bs);
  timed_n(h, "pgs_fwd", lvname(h, l, gs + ", true>"), fwd_bytes, L.ncolors, s, [&] {
    for (int c = 0; c < L.ncolors; ++c) {
      const hipError_t e = launch_pgs_fwd<T>(L.Am, Dinv, L.color_ptr[c], L.color_ptr[c + 1], K, b, x, R, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  });
  timed(h, "presid_upper", lvname(h, l, "k_presid_upper<" + ty + ", " + std::to_string(bs) + ">"),
        launch_bytes(L.sh_resid, LK_RESID, bs, bs, vs, K), s,
        [&] { return launch_presid_upper<T>(L.panel_mat(L.pw_resid), K, x, R, s); });
  T *Cb = vp<T>(w->vb[pi][l + 1]);
  T *Cx = vp<T>(w->vx[pi][l + 1]);
  timed(h, "prestrict", lvname(h, l, "k_prect<" + ty + ", " + std::to_string(L.kc) + ", " + std::to_string(bs) + ">"),
        launch_bytes(L.sh_R, LK_RECT, L.kc, bs, vs, K), s,
        [&] { return launch_prect<T>(L.Rm, K, R, Cb, false, s); });
  pvcycle_t<T>(h, w, l + 1, Cb, Cx, s);
  timed(h, "pprolong", lvname(h, l, "k_prect<" + ty + ", " + std::to_string(bs) + ", " + std::to_string(L.kc) + ">"),
        launch_bytes(L.sh_P, LK_RECT_ACC, bs, L.kc, vs, K), s,
        [&] { return launch_prect<T>(L.Pm, K, Cx, x, true, s); });
  const SolveMat Mb = L.panel_mat(L.pw_bwd);
  timed_n(h, "pgs_bwd", lvname(h, l, gs + ", false>"), bwd_bytes, L.ncolors, s, [&] {
    for (int c = L.ncolors - 1; c >= 0; --c) {
      const hipError_t e = launch_pgs_bwd<T>(Mb, Dinv, L.color_ptr[c], L.color_ptr[c + 1], K, b, x, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  });
}

// Z = V(R) for the K columns of the level-0 CG panels.
void pvcycle(eamg_hierarchy *h, BatchWork *w, bool f32, hipStream_t s) {
  if (f32) {
    const int64_t N = level_dofs(h->lv[0]) * w->K;
    float *b32 = vp<float>(w->vb[1][0]), *x32 = vp<float>(w->vx[1][0]);
    timed(h, "convert", "k_convert<double, float>", 12.0 * N, s,
          [&] { return launch_convert<double, float>(N, w->r, b32, s); });
    pvcycle_t<float>(h, w, 0, b32, x32, s);
    timed(h, "convert", "k_convert<float, double>", 12.0 * N, s,
          [&] { return launch_convert<float, double>(N, x32, w->z, s); });
  } else {
    pvcycle_t<double>(h, w, 0, w->r, w->z, s);
  }
}

// One batched PCG iteration after the stopping test (the columns that are still active).
void penqueue_iteration(eamg_hierarchy *h, BatchWork *w, bool precond, bool f32, hipStream_t s) {
  const Level &L0 = h->lv[0];
  const int K = w->K;
  const int64_t N = level_dofs(L0) * K;
  const int nd = pdot_blocks(N), ns = pspmv_blocks(L0.Am, K);
  const double vecb = 8.0 * N;
  if (precond)
    pvcycle(h, w, f32, s);
  else
    hip_check(launch_copy(N, w->r, w->z, s), "copy");
  timed(h, "pdot", "k_pdot", 2.0 * vecb + 8.0 * nd * K, s,
        [&] { return launch_pdot(N, K, w->r, w->z, w->part, s); });
  timed(h, "preduce", "k_preduce", 8.0 * nd * K, s,
        [&] { return launch_preduce(nd, K, w->part, w->scal, PS_RZ, PRED_BETA, s); });
  timed(h, "pupdate_p", "k_pupdate_p", 3.0 * vecb, s,
        [&] { return launch_pupdate_p(N, K, w->scal, w->z, w->p, s); });
  timed(h, "pspmv", tname("k_pspmv", L0.bs), launch_bytes(L0.sh_spmv, LK_SPMV, L0.bs, L0.bs, 8.0, K) + 8.0 * ns * K, s,
        [&] { return launch_pspmv(L0.Am, K, w->p, w->q, w->part, s); });
  timed(h, "preduce", "k_preduce", 8.0 * ns * K, s,
        [&] { return launch_preduce(ns, K, w->part, w->scal, PS_PQ, PRED_ALPHA, s); });
  timed(h, "pupdate_xr", "k_pupdate_xr", 6.0 * vecb + 8.0 * nd * K, s,
        [&] { return launch_pupdate_xr(N, K, w->scal, w->x, w->r, w->p, w->q, w->part, s); });
  timed(h, "preduce", "k_preduce", 8.0 * nd * K, s,
        [&] { return launch_preduce(nd, K, w->part, w->scal, PS_RR, PRED_RR, s); });
  hip_check(hipMemcpyAsync(w->scal_h, w->scal, sizeof(double) * PS_COUNT * K, hipMemcpyDeviceToHost, s),
            "copy");
}

void ptry_graph(eamg_hierarchy *h, BatchWork *w, bool f32) {
  w->tried[f32] = true;
  if (const char *e = std::getenv("EAMG_GRAPH"))
    if (std::atoi(e) == 0) return;
  if (!w->cap && hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking) != hipSuccess) {
    w->cap = nullptr;
    return;
  }
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(w->cap, hipStreamCaptureModeRelaxed) != hipSuccess) return;
  bool ok = true;
  try {
    penqueue_iteration(h, w, true, f32, w->cap);
  } catch (const Failure &) {
    ok = false;
  }
  if (hipStreamEndCapture(w->cap, &g) != hipSuccess || !ok) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return;
  }
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) w->g[f32] = ex;
  (void)hipGraphDestroy(g);
  (void)hipGetLastError();
}

void pfetch(BatchWork *w, hipStream_t s) {
  hip_check(hipMemcpyAsync(w->scal_h, w->scal, sizeof(double) * PS_COUNT * w->K, hipMemcpyDeviceToHost, s),
            "copy");
  hip_check(hipStreamSynchronize(s), "sync");
}

bool any_active(const BatchWork *w) {
  for (int k = 0; k < w->K; ++k)
    if (w->scal_h[PS_ACTIVE * w->K + k] != 0.0) return true;
  return false;
}

// Solve the m <= 64 columns of one panel; returns whether all of them converged.
bool solve_panel(eamg_hierarchy *h, int m, const double *B, int64_t ld, double *X,
                 const eamg_solve_params &sp, hipStream_t s, eamg_solve_info *infos) {
  const int K = panel_width(m);
  const bool precond = sp.precond != EAMG_PRECOND_NONE;
  const bool f32 = sp.precond == EAMG_PRECOND_VCYCLE_FP32;
  BatchWork *w = ensure_work(h, K, f32);
  const Level &L0 = h->lv[0];
  const SolveMat &A = L0.Am;
  const int64_t N = level_dofs(L0) * K;
  const int nd = pdot_blocks(N), ns = pspmv_blocks(A, K);
  struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  hip_check(hipEventCreate(&ev.a), "event");
  hip_check(hipEventCreate(&ev.b), "event");
  hipEvent_t e0 = ev.a, e1 = ev.b;
  hip_check(hipEventRecord(e0, s), "event");
  hip_check(launch_pinit_scal(K, sp.rtol, sp.max_it, w->scal, s), "pinit");
  hip_check(launch_ppack(L0.n, L0.bs, K, m, L0.perm_d, h->dir, B, ld, w->bp, s), "ppack");
  hip_check(launch_pfinite(N, K, w->bp, w->scal, s), "pfinite");
  hip_check(launch_pdot(N, K, w->bp, w->bp, w->part, s), "pdot");
  hip_check(launch_preduce(nd, K, w->part, w->scal, PS_BB, PRED_INIT, s), "preduce");
  if (sp.use_x0) {
    hip_check(launch_ppack(L0.n, L0.bs, K, m, L0.perm_d, h->dir, X, ld, w->x, s), "ppack");
    hip_check(launch_pspmv(A, K, w->x, w->q, nullptr, s), "pspmv");
    hip_check(launch_sub(N, w->bp, w->q, w->r, s), "sub");
  } else {
    hip_check(launch_fill(N, 0.0, w->x, s), "fill");
    hip_check(launch_copy(N, w->bp, w->r, s), "copy");
  }
  hip_check(launch_pdot(N, K, w->r, w->r, w->part, s), "pdot");
  hip_check(launch_preduce(nd, K, w->part, w->scal, PS_RR0, PRED_STORE, s), "preduce");
  if (precond)
    pvcycle(h, w, f32, s);
  else
    hip_check(launch_copy(N, w->r, w->z, s), "copy");
  hip_check(launch_copy(N, w->z, w->p, s), "copy");
  hip_check(launch_pdot(N, K, w->r, w->z, w->part, s), "pdot");
  hip_check(launch_preduce(nd, K, w->part, w->scal, PS_RHO, PRED_RHO0, s), "preduce");
  // first iteration (p = z), then one graph replay per further iteration
  hip_check(launch_pspmv(A, K, w->p, w->q, w->part, s), "pspmv");
  hip_check(launch_preduce(ns, K, w->part, w->scal, PS_PQ, PRED_ALPHA, s), "preduce");
  hip_check(launch_pupdate_xr(N, K, w->scal, w->x, w->r, w->p, w->q, w->part, s), "pupdate_xr");
  hip_check(launch_preduce(nd, K, w->part, w->scal, PS_RR, PRED_RR, s), "preduce");
  pfetch(w, s);
  const bool graphs = precond && !h->prof_on;
  if (graphs && !w->tried[f32]) ptry_graph(h, w, f32);
  // every active column stops by MAXIT; the bound only guards the host loop
  for (int it = 1; any_active(w) && it <= sp.max_it; ++it) {
    if (graphs && w->g[f32]) {
      hip_check(hipGraphLaunch(w->g[f32], s), "graph launch");
      hip_check(hipStreamSynchronize(s), "sync");
    } else {
      penqueue_iteration(h, w, precond, f32, s);
      hip_check(hipStreamSynchronize(s), "sync");
    }
  }
  // true residuals, x of columns that never started, unpack
  hip_check(launch_pspmv(A, K, w->x, w->q, nullptr, s), "pspmv");
  hip_check(launch_sub(N, w->bp, w->q, w->z, s), "sub");
  hip_check(launch_pdot(N, K, w->z, w->z, w->part, s), "pdot");
  hip_check(launch_preduce(nd, K, w->part, w->scal, PS_RZ, PRED_STORE, s), "preduce");
  hip_check(launch_pzero_unstarted(N, K, w->scal, w->x, s), "pzero");
  hip_check(launch_punpack(L0.n, L0.bs, K, m, L0.perm_d, w->x, X, ld, s), "punpack");
  hip_check(hipEventRecord(e1, s), "event");
  pfetch(w, s);
  float fms = 0.0f;
  hip_check(hipEventElapsedTime(&fms, e0, e1), "event");
  bool all = true;
  for (int k = 0; k < m; ++k) {
    const double *S = w->scal_h;
    auto at = [&](int slot) { return S[slot * K + k]; };
    const double bn = std::sqrt(at(PS_BB));
    const bool conv = at(PS_CONV) != 0.0;
    const bool bad = at(PS_BAD) != 0.0;
    all = all && conv && !bad;
    if (infos) {
      eamg_solve_info &inf = infos[k];
      inf.iterations = int32_t(at(PS_ITS));
      inf.rel_res = (bn > 0.0 && std::isfinite(bn)) ? std::sqrt(at(PS_RR)) / bn : 0.0;
      inf.rel_res_true = (bn > 0.0 && std::isfinite(bn)) ? std::sqrt(at(PS_RZ)) / bn : 0.0;
      if (bad && at(PS_ITS) == 0.0) inf.rel_res = inf.rel_res_true = 0.0;
      inf.ms = fms;
      inf.status = bad ? EAMG_ERR_BREAKDOWN : conv ? EAMG_OK : EAMG_NOT_CONVERGED;
    }
  }
  return all;
}

// Time one launch sequence on the stream (events), median of reps.
template <class F>
double time_ms(hipStream_t s, int reps, F &&f) {
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
  return t[t.size() / 2];
}

}  // namespace

// Panel launch shapes measured on the hierarchy's own matrices for K columns (FP64 V-cycle
// kernels): per level, the sweep + upper-residual sequence and each transfer with one or four
// wavefronts per row; the faster is kept in SolveMat::panel_waves.  Returns the summed time of the
// tuned kernels before / after (ms).
DenseTail make_dense_tail(eamg_hierarchy *h, size_t t, DevArena &out, hipStream_t s) {
  if (t == 0 || t + 1 >= h->lv.size()) fail(EAMG_ERR_INVALID_ARG, "dense tail must start above the coarsest level, below the finest");
  const Level &Lt = h->lv[t];
  const int n = Lt.n * Lt.bs;
  if (n > kMaxCoarsestDofs) fail(EAMG_ERR_INVALID_ARG, "dense tail too large");
  // a workspace of 64-column panels for levels t .. coarsest only (the batched solve's own is
  // sized for level 0)
  constexpr int K = 64;
  BatchWork w;
  w.K = K;
  w.dense = w.arena.alloc<double>(std::max<size_t>(1, dense_panel_work_doubles(h->nL, K)));
  const size_t nl = h->lv.size();
  w.vx[0].assign(nl, nullptr);
  w.vb[0].assign(nl, nullptr);
  w.vr[0].assign(nl, nullptr);
  for (size_t l = t; l < nl; ++l) {
    const size_t nd = size_t(level_dofs(h->lv[l])) * K;
    w.vx[0][l] = w.arena.alloc<double>(nd);
    w.vb[0][l] = w.arena.alloc<double>(nd);
    if (l + 1 < nl) w.vr[0][l] = w.arena.alloc<double>(nd);
  }
  w.have[0] = true;
  const int ld = dense_ld(n);
  double *T = out.alloc<double>(size_t(ld) * ld);
  hip_check(launch_fill(int64_t(ld) * ld, 0.0, T, s), "fill");
  double *B = vp<double>(w.vb[0][t]), *X = vp<double>(w.vx[0][t]);
  const bool prof = h->prof_on;
  h->prof_on = false;
  for (int j0 = 0; j0 < n; j0 += K) {
    hip_check(launch_identity_panel(n, K, j0, B, s), "identity panel");
    pvcycle_t<double>(h, &w, t, B, X, s);
    hip_check(launch_scatter_panel(n, K, j0, std::min(K, n - j0), X, ld, T, s), "scatter panel");
  }
  h->prof_on = prof;
  DenseTail d;
  d.T = T;
  d.n = n;
  d.ld = ld;
  hip_check(hipStreamSynchronize(s), "sync");
  return d;
}

void build_dense_tail(eamg_hierarchy *h, size_t t, hipStream_t s) {
  const DenseTail d = make_dense_tail(h, t, h->arena, s);
  h->tail = d.T;
  h->nT = d.n;
  h->ldT = d.ld;
  h->tailS = h->arena.alloc<double>(sym_entries(d.n));
  hip_check(launch_pack_sym<double>(d.n, d.ld, d.T, h->tailS, s), "pack tail");
  if (h->prm.vcycle_fp32 && h->prm.dense_tail_fp32) {
    h->tailS32 = h->arena.alloc<float>(sym_entries(d.n));
    hip_check(launch_pack_sym<float>(d.n, d.ld, d.T, h->tailS32, s), "pack tail f32");
  }
  h->tailW = h->arena.alloc<double>(sym_work_doubles(d.n));
  hip_check(hipStreamSynchronize(s), "sync");
  h->tail_level = int(t);
}

std::pair<double, double> tune_panels(eamg_hierarchy *h, int K, hipStream_t s) {
  BatchWork *w = ensure_work(h, K, false);
  const int reps = 5;
  double before = 0.0, after = 0.0;
  for (size_t l = 0; l + 1 < h->lv.size(); ++l) {
    if (h->tail_level >= 0 && int(l) >= h->tail_level) break;   // applied as the dense tail
    Level &L = h->lv[l];
    double *b = l == 0 ? w->r : vp<double>(w->vb[0][l]);
    double *x = l == 0 ? w->z : vp<double>(w->vx[0][l]);
    double *r = vp<double>(w->vr[0][l]);
    double *cb = vp<double>(w->vb[0][l + 1]);
    double *cx = vp<double>(w->vx[0][l + 1]);
    const int64_t nv = level_dofs(L) * K, nc = level_dofs(h->lv[l + 1]) * K;
    for (double *v : {b, x, r}) hip_check(launch_fill(nv, 0.0, v, s), "fill");
    for (double *v : {cb, cx}) hip_check(launch_fill(nc, 0.0, v, s), "fill");
    // forward sweep, residual update and backward sweep tuned apart (each reads a different part
    // of the rows), then the transfers
    auto fwd = [&] {
      for (int c = 0; c < L.ncolors; ++c)
        hip_check(launch_pgs_fwd<double>(L.Am, L.Dinv, L.color_ptr[c], L.color_ptr[c + 1], K, b, x, r, s), "pgs");
    };
    auto resid = [&] {
      hip_check(launch_presid_upper<double>(L.panel_mat(L.pw_resid), K, x, r, s), "presid");
    };
    auto bwd = [&] {
      const SolveMat Mb = L.panel_mat(L.pw_bwd);
      for (int c = L.ncolors - 1; c >= 0; --c)
        hip_check(launch_pgs_bwd<double>(Mb, L.Dinv, L.color_ptr[c], L.color_ptr[c + 1], K, b, x, s), "pgs");
    };
    auto restrict_ = [&] { hip_check(launch_prect<double>(L.Rm, K, r, cb, false, s), "prect"); };
    auto prolong = [&] { hip_check(launch_prect<double>(L.Pm, K, cx, x, true, s), "prect"); };
    L.pw_resid = L.pw_bwd = 0;
    struct Item {
      int *pw;   // the choice: 0 (built-in / the forward sweep's), 1 or 4 wavefronts per row
      std::function<void()> run;
    } items[] = {{&L.Am.panel_waves, fwd}, {&L.pw_resid, resid}, {&L.pw_bwd, bwd},
                 {&L.Rm.panel_waves, restrict_}, {&L.Pm.panel_waves, prolong}};
    for (Item &it : items) {
      const int orig = *it.pw;
      int best_w = orig;
      const double t0 = time_ms(s, reps, it.run);
      before += t0;
      double best = t0;
      for (int wv : {1, 4}) {
        *it.pw = wv;
        const double t = time_ms(s, reps, it.run);
        if (t < best) {
          best = t;
          best_w = wv;
        }
      }
      *it.pw = best_w;
      after += best;
    }
  }
  // captured iteration graphs hold the old launch shapes
  for (int p = 0; p < 2; ++p) {
    if (w->g[p]) (void)hipGraphExecDestroy(w->g[p]);
    w->g[p] = nullptr;
    w->tried[p] = false;
  }
  return {before, after};
}

}  // namespace eamg

using namespace eamg;

extern "C" eamg_status eamg_solve_batch(eamg_hierarchy *h, int32_t nrhs, const double *B_dev,
                                        int64_t ld, double *X_dev, const eamg_solve_params *params,
                                        void *stream, eamg_solve_info *infos) {
  bool all = true;
  const eamg_status st = guarded([&] {
    if (!h || !B_dev || !X_dev) fail(EAMG_ERR_INVALID_ARG, "NULL argument");
    reject_fused(h);
    if (nrhs < 1) fail(EAMG_ERR_INVALID_ARG, "nrhs must be >= 1");
    const int64_t ndof = level_dofs(h->lv[0]);
    if (ld < ndof) fail(EAMG_ERR_INVALID_ARG, "ld must be >= n*dim");
    {
      const char *b0 = reinterpret_cast<const char *>(B_dev);
      const char *x0 = reinterpret_cast<const char *>(X_dev);
      const int64_t span = (int64_t(nrhs - 1) * ld + ndof) * int64_t(sizeof(double));
      if (b0 < x0 + span && x0 < b0 + span) fail(EAMG_ERR_INVALID_ARG, "B and X may not overlap");
    }
    eamg_solve_params sp;
    eamg_default_solve_params(&sp);
    if (params) sp = *params;
    if (sp.max_it < 1) fail(EAMG_ERR_INVALID_ARG, "max_it must be >= 1");
    if (!(sp.rtol >= 0.0)) fail(EAMG_ERR_INVALID_ARG, "rtol must be >= 0");
    if (sp.precond < EAMG_PRECOND_NONE || sp.precond > EAMG_PRECOND_VCYCLE_FP32)
      fail(EAMG_ERR_INVALID_ARG, "precond must be 0, 1 or 2");
    if (sp.precond == EAMG_PRECOND_VCYCLE_FP32 && !h->prm.vcycle_fp32)
      fail(EAMG_ERR_INVALID_ARG, "FP32 V-cycle needs setup with vcycle_fp32 = 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    constexpr int kMaxPanel = 64;
    for (int c0 = 0; c0 < nrhs; c0 += kMaxPanel) {
      const int m = std::min(kMaxPanel, nrhs - c0);
      all = solve_panel(h, m, B_dev + int64_t(c0) * ld, ld, X_dev + int64_t(c0) * ld, sp, s,
                        infos ? infos + c0 : nullptr) && all;
    }
  });
  if (st == EAMG_OK && !all) {
    g_last_error = "some right-hand sides did not converge";
    return EAMG_NOT_CONVERGED;
  }
  return st;
}
