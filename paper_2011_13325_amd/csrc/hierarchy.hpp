// Device hierarchy of libeamg shared by the setup / PCG driver (api.cpp) and the batched
// block-panel driver (batch.cpp): levels in colour-major solve layout, device arena, the
// per-launch profiler and the error plumbing of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/eamg.h"
#include "coarse.hpp"
#include "fused.hpp"
#include "kernels.hpp"
#include "coarsen.hpp"
#include "staging.hpp"
#include "structure.hpp"

namespace eamg {

extern thread_local std::string g_last_error;

struct Failure {
  eamg_status code;
  std::string msg;
};

[[noreturn]] inline void fail(eamg_status code, const std::string &msg) { throw Failure{code, msg}; }

inline void hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory) fail(EAMG_ERR_OOM, std::string(what) + ": out of device memory");
  fail(EAMG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Device allocations owned by a hierarchy; freed together.
struct DevArena {
  std::vector<void *> ptrs;
  template <class T>
  T *alloc(size_t count) {
    void *p = nullptr;
    if (count == 0) count = 1;
    hip_check(hipMalloc(&p, count * sizeof(T)), "hipMalloc");
    ptrs.push_back(p);
    return static_cast<T *>(p);
  }
  template <class T, class A>
  T *upload(const std::vector<T, A> &v, hipStream_t s) {
    return upload(v.data(), v.size(), s);
  }
  template <class T>
  T *upload(const T *p, size_t count, hipStream_t s) {
    // setup-time upload from pageable memory: wait so the source may be freed on return
    T *d = alloc<T>(count);
    hip_check(copy_h2d_sync(d, p, count * sizeof(T), s), "upload");
    return d;
  }
  void release(void *p) {
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it != ptrs.end()) {
      (void)hipFree(p);
      ptrs.erase(it);
    }
  }
  ~DevArena() {
    for (void *p : ptrs) (void)hipFree(p);
  }
};

template <class T>
std::vector<T> download(const T *d, size_t count, hipStream_t s) {
  std::vector<T> h(count);
  hip_check(copy_d2h_sync(h.data(), d, count * sizeof(T), s), "download");
  return h;
}

inline int pick_group(int64_t nnz, int rows) {
  const double avg = rows ? double(nnz) / rows : 1.0;
  int g = 4;
  while (g < 64 && g < avg) g <<= 1;
  return g;
}

// What one solve-phase launch streams: matrix blocks (each with its column index), block rows,
// and distinct gathered block columns.
struct LaunchShape {
  double blocks = 0, rows = 0, uniq = 0;
};

enum LaunchKind { LK_GS_FWD, LK_GS_BWD, LK_RESID, LK_RECT, LK_RECT_ACC, LK_SPMV };

// Algorithmic HBM bytes of a launch: every matrix block and index read once, every gathered
// vector block once, row data (offsets, D^+ blocks, own vector entries) once; values of vs
// bytes, K right-hand sides per vector entry.  br x bc is the block shape.
//   GS_FWD: lower blocks + diagonal; row offset and diagonal index, D^+; b read, x and r written
//   GS_BWD: whole rows; row offset and diagonal index, D^+; b read, x written
//   RESID : blocks right of the diagonal; row offset and diagonal index; r read and written
//   RECT  : y = M x (RECT_ACC: y += M x, y also read); SPMV: y = A x
inline double launch_bytes(const LaunchShape &sh, LaunchKind kind, int br, int bc, double vs, int K) {
  const double mat = sh.blocks * (br * bc * vs + 4.0);
  const double gat = sh.uniq * bc * K * vs;
  const double vec = br * K * vs;   // one row's vector entries
  switch (kind) {
    case LK_GS_FWD: return mat + gat + sh.rows * (8.0 + br * br * vs + 3.0 * vec);
    case LK_GS_BWD: return mat + gat + sh.rows * (8.0 + br * br * vs + 2.0 * vec);
    case LK_RESID: return mat + gat + sh.rows * (8.0 + 2.0 * vec);
    case LK_RECT: return mat + gat + 4.0 * (sh.rows + 1) + sh.rows * vec;
    case LK_RECT_ACC: return mat + gat + 4.0 * (sh.rows + 1) + 2.0 * sh.rows * vec;
    case LK_SPMV: return mat + gat + 4.0 * (sh.rows + 1) + sh.rows * vec;
  }
  return 0.0;
}

// Dense operators applied on one level of a fused hierarchy, one part per system (device array
// of `count` SymPart entries: packed upper tiles, `tiles` and `rows` in total, partial sums in
// W), and their algorithmic bytes per application.
struct DenseSet {
  const SymPart *parts = nullptr;
  int count = 0, rows = 0, tiles = 0;
  double *W = nullptr;
  double bytes = 0.0;
  const double *active = nullptr;   // per-system CG activity flags: stopped systems are skipped
};

struct Level {
  int n = 0, bs = 0;
  // rows the smoother covers (the colour ranges), -1 for all n rows; a fused hierarchy's level
  // puts the rows of systems whose V-cycle ends on it after them
  int n_smooth = -1;
  int smooth_rows() const { return n_smooth < 0 ? n : n_smooth; }
  // fused hierarchies: dense operators of the systems whose V-cycle ends on this level;
  // [0] FP64 V-cycle (double matrices), [1] FP32 V-cycle with float matrices, [2] FP32 V-cycle
  // with double matrices
  DenseSet dense[3];
  Pattern A;                 // natural pattern
  int64_t *A_rp = nullptr;   // natural pattern on the device
  int *A_col = nullptr;
  double *A_val = nullptr;   // natural AoS values (n_blocks * bs * bs)
  // coarsening products (levels above the coarsest)
  std::vector<int> agg;
  Pattern P;
  int kc = 0;
  double *P_val = nullptr;   // natural AoS values (nnz * bs * kc)
  std::vector<int> color;    // natural
  int ncolors = 0;
  // colour-major solve layout
  std::vector<int> perm, inv, color_ptr;
  int *perm_d = nullptr;
  SolveMat Am, Pm, Rm;
  // lanes per row of the residual update (upper halves of all rows, one launch), or 0 for Am.group
  int group_resid = 0;
  SolveMat resid_mat() const {
    SolveMat m = Am;
    if (group_resid) m.group = group_resid;
    return m;
  }
  // per colour: lanes per row of the forward / backward sweep, 0 (or empty) for the level's
  // choice; the first row of a colour's lower blocks grows from none (colour 0) to a whole row
  // (the last colour), so one choice per level fits neither end
  std::vector<int> g_fwd, g_bwd;
  SolveMat fwd_mat(int c) const {
    SolveMat m = Am;
    if (size_t(c) < g_fwd.size() && g_fwd[size_t(c)]) m.group = g_fwd[size_t(c)];
    return m;
  }
  SolveMat bwd_mat(int c) const {
    SolveMat m = Am;
    if (size_t(c) < g_bwd.size() && g_bwd[size_t(c)]) m.group_bwd = g_bwd[size_t(c)];
    return m;
  }
  // the residual update as launches over consecutive colour ranges [resid_cut[k],
  // resid_cut[k+1]) with lanes per row g_resid[k] (0: resid_mat()'s); empty: one launch
  std::vector<int> resid_cut, g_resid;
  // blocks right of the diagonal in each colour's rows (to split the residual update)
  std::vector<double> upper_blocks;
  // panel kernels: wavefronts per row of the residual update and of the backward sweep, or 0 for
  // Am.panel_waves (the forward sweep's)
  int pw_resid = 0, pw_bwd = 0;
  SolveMat panel_mat(int pw) const {
    SolveMat m = Am;
    if (pw) m.panel_waves = pw;
    return m;
  }
  double *Dinv = nullptr;
  int64_t nnz_lower = 0;     // blocks strictly below the diagonal (colour-major)
  double *x = nullptr, *b = nullptr, *r = nullptr;
  // what every launch streams (for the traffic model and the profiler)
  std::vector<LaunchShape> sh_fwd, sh_bwd;   // per colour
  LaunchShape sh_resid, sh_R, sh_P, sh_spmv;
  // FP32 V-cycle: values in SolveMat::val32, D^+ and level vectors in float
  float *Dinv32 = nullptr, *x32 = nullptr, *b32 = nullptr, *r32 = nullptr;
};

// Per-precision view of a level's V-cycle buffers.
template <class T>
struct LevelBufs {
  const T *Dinv;
  T *x, *b, *r;
};
template <class T>
LevelBufs<T> bufs(Level &L);
template <>
inline LevelBufs<double> bufs<double>(Level &L) {
  return {L.Dinv, L.x, L.b, L.r};
}
template <>
inline LevelBufs<float> bufs<float>(Level &L) {
  return {L.Dinv32, L.x32, L.b32, L.r32};
}
template <class T>
const char *type_name();
template <>
inline const char *type_name<double>() {
  return "double";
}
template <>
inline const char *type_name<float>() {
  return "float";
}

struct ProfRec {
  std::string name;
  double bytes;
  int launches;
  hipEvent_t a, b;
};

struct BatchWork;
void destroy_batch(BatchWork *w);
struct FusedInfo;
void destroy_fused(FusedInfo *f);
// Solve-phase matrix from a host pattern in the solve numbering, src[q] = natural position of
// block q in the AoS values aos (br x bc blocks; transpose_blocks: aos holds bc x br blocks);
// diag_out (square matrices) receives each row's diagonal position.
SolveMat make_solve_mat(DevArena &ar, const Pattern &Pp, const std::vector<int64_t> &src, int br,
                        int bc, const double *aos, hipStream_t s, std::vector<int> *diag_out = nullptr,
                        bool transpose_blocks = false, bool fp32 = false);
// The blocks left of the diagonal, right of it and the diagonal blocks of a square solve matrix,
// each in storage of its own (SolveMat::lo_*, up_*, dg_*).
void attach_split_parts(DevArena &ar, const Pattern &Ap, const std::vector<int64_t> &src,
                        const std::vector<int> &dg, int bs, const double *vals, hipStream_t s,
                        bool f32, SolveMat &Am);
LaunchShape range_shape(const Pattern &Ap, const std::vector<int> &dg, int r0, int r1, int part,
                        std::vector<int> &mark, int stamp);
LaunchShape matrix_shape(const Pattern &M);
// Launch shapes of a smoothed level (colours, residual update over smooth_rows(), SpMV).
void level_shapes(Level &L, const Pattern &Ap, const std::vector<int> &dg);
// z = V(r) on level-0 vectors in the hierarchy's solve numbering (FP64, or the FP32 V-cycle
// with conversions at the boundary).
void vcycle_apply(eamg_hierarchy *h, const double *r, double *z, bool f32, hipStream_t s);
// Panel launch shapes tuned on the hierarchy for K columns; (time before, after) in ms.
std::pair<double, double> tune_panels(eamg_hierarchy *h, int K, hipStream_t s);
// z = V(r) for level-0 vectors in the natural numbering (eamg_vcycle's operation), with the
// colour-major copies of r and z in the caller's device buffers rp and zp (n0 * dim doubles
// each): launches on s only -- no allocation, no synchronization; the profiler must be off.
void vcycle_staged(eamg_hierarchy *h, const double *r_dev, double *z_dev, bool f32, double *rp,
                   double *zp, hipStream_t s);
// The V-cycle on levels t .. coarsest of h as a dense matrix in the colour-major numbering of
// level t, from the batched V-cycle applied to the columns of the identity: FP64, row-major, ld a
// multiple of 128, zero padding, allocated in `out`.
struct DenseTail {
  double *T = nullptr;
  int n = 0, ld = 0;
};
DenseTail make_dense_tail(eamg_hierarchy *h, size_t t, DevArena &out, hipStream_t s);
// make_dense_tail into h's own arena, kept as h->tail with its packed upper tiles (h->tailS, and
// h->tailS32 with dense_tail_fp32); sets h->tail_level = t.
void build_dense_tail(eamg_hierarchy *h, size_t t, hipStream_t s);

}  // namespace eamg

struct eamg_hierarchy {
  int dim = 0, k = 0, n0 = 0;
  int device = 0;             // the HIP device the hierarchy was set up on
  eamg_setup_params prm{};
  std::vector<eamg::Level> lv;
  eamg::DevArena arena;
  double *Ainv = nullptr;
  int nL = 0;                 // coarsest dofs
  int ldL = 0;                // leading dimension of Ainv (nL rounded up to 128)
  // dense V-cycle tail: the V-cycle on levels tail_level .. coarsest as one dense matrix in the
  // colour-major numbering of tail_level (row-major, zero padding), or tail_level = -1
  int tail_level = -1;
  int nT = 0, ldT = 0;
  double *tail = nullptr;
  // the tail's upper tiles, packed (the V-cycle operator is symmetric): FP64 and, with
  // dense_tail_fp32, FP32; the single-vector V-cycle reads these, with tailW as its workspace
  double *tailS = nullptr;
  float *tailS32 = nullptr;
  double *tailW = nullptr;
  uint8_t *dir = nullptr;     // level-0 Dirichlet mask (natural)
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *bp = nullptr;
  double *part = nullptr, *scal = nullptr;
  int part_cap = 0;   // entries of part: the largest partial-sum count any launch shape can need
  double *scal_h = nullptr;   // pinned
  // profiler: events around every launch while enabled
  bool prof_on = false;
  bool prof_levels = false;   // V-cycle records per level
  bool prof_colours = false;  // ... and per colour launch of the single-vector sweeps
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<eamg::ProfRec> prof;
  // PCG iteration captured as a graph (V-cycle .. r.r and the scalar copy), replayed per iteration
  hipStream_t cap_stream = nullptr;
  // one graph per V-cycle precision: [0] FP64, [1] FP32
  hipGraphExec_t g_iter[2] = {nullptr, nullptr};
  bool graph_tried[2] = {false, false};
  // block-panel (multi right-hand side) workspace, allocated by the first batched call
  eamg::BatchWork *batch = nullptr;
  // fused hierarchies (eamg_fuse): the systems, their level-0 maps and the segmented CG state
  eamg::FusedInfo *fused = nullptr;
  // fused hierarchies that read this one's dense operators; eamg_destroy while there are any
  // only marks it, and the last of them frees it
  int fused_users = 0;
  bool destroy_pending = false;
  // wall time of each setup phase (summed over levels), in the order phases first ran
  std::vector<std::pair<std::string, double>> setup_phases;
  // CG coefficients alpha_k, beta_k of the last single-vector solve (beta_1 = 0)
  std::vector<double> cg_alpha, cg_beta;
  // coarsening: criteria evaluations of the matching walks, candidates passed over by the
  // learned walk, and (when asked for) every pass's candidate pairs with features and labels
  int64_t crit_evaluated = 0, crit_evaluated_g = 0, crit_skipped = 0;
  std::vector<eamg::PassSamples> samples;
  ~eamg_hierarchy() {
    eamg::destroy_batch(batch);
    eamg::destroy_fused(fused);
    for (hipGraphExec_t g : g_iter)
      if (g) (void)hipGraphExecDestroy(g);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (scal_h) (void)hipHostFree(scal_h);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }
};

namespace eamg {

inline hipEvent_t next_event(eamg_hierarchy *h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "event");
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_used++];
}

// Run `f`, which enqueues `launches` back-to-back launches of one kernel; while profiling,
// bracket them with one pair of events and record their algorithmic bytes.
template <class F>
void timed_n(eamg_hierarchy *h, const char *what, const std::string &name, double bytes,
             int launches, hipStream_t s, F &&f) {
  if (!h->prof_on) {
    hip_check(f(), what);
    return;
  }
  ProfRec r{name, bytes, launches, next_event(h), next_event(h)};
  hip_check(hipEventRecord(r.a, s), "event");
  hip_check(f(), what);
  hip_check(hipEventRecord(r.b, s), "event");
  h->prof.push_back(r);
}

template <class F>
void timed(eamg_hierarchy *h, const char *what, const std::string &name, double bytes,
           hipStream_t s, F &&f) {
  timed_n(h, what, name, bytes, 1, s, std::forward<F>(f));
}

// Profiler name of a V-cycle launch on level l.
inline std::string lvname(const eamg_hierarchy *h, size_t l, const std::string &name) {
  return h->prof_levels ? "L" + std::to_string(l) + " " + name : name;
}

inline std::string tname(const char *base, int a) { return std::string(base) + "<" + std::to_string(a) + ">"; }
inline std::string tname(const char *base, int a, int b) {
  return std::string(base) + "<" + std::to_string(a) + ", " + std::to_string(b) + ">";
}

// Entry points other than eamg_solve_fused, eamg_autotune, the profiler and eamg_destroy need a
// hierarchy of one system.
inline void reject_fused(const eamg_hierarchy *h) {
  if (h && h->fused)
    fail(EAMG_ERR_INVALID_ARG, "a fused hierarchy (eamg_fuse) supports only eamg_solve_fused, "
                               "eamg_autotune, the profiler and eamg_destroy");
}
// Drop a fused hierarchy's captured iteration graphs (their launch shapes changed).
void invalidate_fused_graphs(eamg_hierarchy *h);

inline void fetch_scalars(eamg_hierarchy *h, hipStream_t s) {
  hip_check(hipMemcpyAsync(h->scal_h, h->scal, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost, s), "copy");
  hip_check(hipStreamSynchronize(s), "sync");
}

template <class F>
eamg_status guarded(F &&f) {
  try {
    f();
    g_last_error.clear();
    return EAMG_OK;
  } catch (const Failure &e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return EAMG_ERR_OOM;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return EAMG_ERR_INVALID_ARG;
  }
}

}  // namespace eamg
