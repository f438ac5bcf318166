/*
 * eamg.h -- C ABI of the MI355X edge-matrix AMG-PCG library (libeamg.so).
 *
 * The library solves A u = b for the symmetric positive definite block matrix A of a P1 finite
 * element discretization (paper section "fem": Problem prob:gg, scalar, and Problem prob:epseps,
 * linear elasticity) with conjugate gradients preconditioned by one V-cycle of auxiliary
 * topology ("edge matrix") AMG (section "res"): coarsening by successive matching on edge and
 * vertex weight matrices (Algorithm alg:pwagg; Thms thm:deng_elast and thm:cemats), auxiliary
 * smoothed prolongation (Def. def:aux_sp), Galerkin coarse operators, a symmetric multicolour
 * block Gauss-Seidel smoother with pseudo-inverted diagonal blocks and a regularized coarsest
 * level inverted densely on the GPU (section "sing2").
 *
 * Conventions shared by every entry point:
 *  - Plain C types only.  Integers are int32_t unless stated, reals are IEEE double.
 *  - "Host" pointers are CPU memory, "device" pointers are HIP device memory on the current
 *    device.  All input arrays are borrowed for the duration of the call and never retained.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All device work of
 *    a call is ordered on it.  eamg_setup and eamg_solve return after their work is complete.
 *  - Errors are returned as eamg_status; no exception or abort crosses the ABI.  A message for
 *    the last failure on the calling thread is available from eamg_last_error().
 *  - A hierarchy handle must not be used by two threads at once, and its calls must not run on
 *    the device at the same time (calls on two streams): they share the hierarchy's level
 *    vectors and workspaces.  Separate handles are independent.
 */
#ifndef EAMG_H
#define EAMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eamg_hierarchy eamg_hierarchy; /* opaque, owned by the library */

typedef enum {
  EAMG_OK = 0,
  EAMG_NOT_CONVERGED = 1,          /* warning: max_it reached, x holds the last iterate       */
  EAMG_ERR_INVALID_ARG = -1,       /* malformed input (message says which)                    */
  EAMG_ERR_UNSUPPORTED_KERNEL = -2,/* dim / k_kernel / kernel vectors not supported           */
  EAMG_ERR_NOT_SPD = -3,           /* coarsest inversion met a non-positive pivot             */
  EAMG_ERR_BREAKDOWN = -4,         /* non-finite value, p.Ap <= 0 or r.z <= 0 in PCG          */
  EAMG_ERR_HIP = -5,               /* a HIP runtime call failed                               */
  EAMG_ERR_OOM = -6                /* device or host allocation failed                        */
} eamg_status;

/*
 * The problem (section "fem"; kernel vectors: section "amg", eq. qij_epseps).  HOST pointers.
 *  dim         1 (scalar, kernel = constants, k = 1) or 3 (3D elasticity, kernel = the six rigid
 *              body modes, k = 6).
 *  n_vertices  number of mesh vertices n (block rows of A).
 *  coords      n*3 vertex positions (x, y, z) of every vertex (also for dim = 1); they define the
 *              transport maps Q^{i->j} of eq. qij_epseps.
 *  row_ptr     n+1 block CSR row offsets of the boundary-condition-free matrix A_N.
 *  col_idx     row_ptr[n] block column indices, strictly ascending within a row, diagonal present,
 *              pattern symmetric.
 *  vals        row_ptr[n]*dim*dim values, each block row-major.  A_N itself, without Dirichlet
 *              conditions; the library replaces Dirichlet rows/columns by identity/zero blocks.
 *  dirichlet   n flags, 1 = all dim components of that vertex are clamped (may be NULL = none).
 *  kernel      optional (n*dim) x k_kernel column-major kernel vectors.  NULL = derived from
 *              coords.  If given they must span the rigid body modes (dim 3) / constants (dim 1)
 *              to 1e-10 relative, else EAMG_ERR_UNSUPPORTED_KERNEL.
 *  k_kernel    6 for dim 3, 1 for dim 1.
 *  edges       optional n_edges x 2 (i < j) auxiliary topology; NULL = every off-diagonal block
 *              position of A_N.  Each edge must be an off-diagonal position of the pattern.
 */
typedef struct {
  int32_t dim;
  int32_t n_vertices;
  const double *coords;
  const int32_t *row_ptr;
  const int32_t *col_idx;
  const double *vals;
  const uint8_t *dirichlet;
  const double *kernel;
  int32_t k_kernel;
  const int32_t *edges;
  int64_t n_edges;
} eamg_problem;

/*
 * Setup parameters (Algorithm alg:pwagg inputs sigma, delta, R, N; row caps of the smoothed
 * prolongation of section "res").  Pass NULL for the defaults, or fill from
 * eamg_default_setup_params().
 *  sigma              matching threshold (default 20)
 *  delta              1 (neighbour term in mu_g / mu_b; only 1 is supported)
 *  R                  1 (candidate chosen by mu_s; only 1 is supported)
 *  rounds             matching passes per level N (default 2, 1..4)
 *  coarsest_max_dofs  level l is the coarsest once bs_l * n_l < this (default 500, <= 16384).
 *                     The coarsest matrix, regularized (section on singular coarse levels), is
 *                     inverted on the GPU at setup (dense, FP64, ld^2 doubles with ld = dofs
 *                     rounded up to 128) and applied by one dense product per V-cycle: on one
 *                     GPU a coarsest level of several thousand dofs replaces the many colour
 *                     launches of the small levels below it.
 *  max_levels         maximum number of levels (default 25)
 *  omega              prolongation smoothing damping (default 2/3)
 *  cap_aux            columns per edge-matrix row of P_s (default 4, 1..16)
 *  cap_std_l0, cap_std columns per real-matrix row of P_s, finest / coarser (defaults 8, 6; 1..16)
 *  pinv_rtol          relative eigenvalue threshold of pseudo-inverses (default 1e-10)
 *  tie_rtol           relative band in which mu_s values tie (default 1e-12)
 *  vcycle_fp32        0: FP64 V-cycle only (default).  1: also keep FP32 copies of the V-cycle
 *                     matrices (A_l, P_s, R, D^+) and FP32 level vectors, so that solves and
 *                     V-cycles may ask for EAMG_PRECOND_VCYCLE_FP32 (about +50% V-cycle memory).
 *  gnn, gnn_skip      learned walk (NULL / 0: the exact walk, default).  With a network (see
 *                     eamg_gnn_*) and gnn_skip in (0, 1): in every matching pass the candidate
 *                     pairs are scored once on the GPU; the walk passes over candidates whose
 *                     predicted acceptance is below gnn_skip without evaluating mu_b / mu_g, and
 *                     a vertex whose candidates were all passed over evaluates its best scored
 *                     one.  Every pair formed is accepted by the exact criteria.  The network
 *                     is borrowed for the call only.
 *  gnn_record         1: keep every pass's candidate pairs with features and exact labels
 *                     (eamg_gnn_samples), for training.  Default 0.
 *  mu_s_only          0: the robust criteria, a pair is formed only if mu_b < sigma and (unions
 *                     of more than two vertices) mu_g < sigma (Alg. alg:pwagg; default).  1: the
 *                     candidate of smallest mu_s is paired without evaluating mu_b / mu_g, the
 *                     scalar-only coarsening the paper contrasts with in its coefficient-jump
 *                     example (figures fig:2dc_rob / fig:2dc_norob); for comparisons only.
 *  gpu_criteria       1: the matching walks hand the pairs whose criteria they need to GPU
 *                     kernels in batches (mu_b per pair, mu_g per union of up to four vertices;
 *                     bit-identical to the host code, so the same hierarchy; default); batches
 *                     too small to gain from a launch (under 4096 pairs, 128 unions) stay on host
 *                     threads.  2: every batch on the GPU.  0: host threads only.
 *  dense_tail_dofs    0: every level below the finest runs its own sweeps, residual and
 *                     transfers in the V-cycle (default).  > 0 (at most 16384): the V-cycle on
 *                     the first level l >= 1 with bs_l * n_l <= dense_tail_dofs and on every level
 *                     below it is one fixed linear map of that level's right-hand side (Alg.
 *                     alg:tg applied recursively, starting from x = 0); it is computed at setup
 *                     by running that part of the V-cycle on the columns of the identity
 *                     (the batched V-cycle of eamg_solve_batch, 64 columns per pass) and
 *                     applied as one dense product per V-cycle (an FP64 matrix with FP64
 *                     accumulation, in either V-cycle precision unless dense_tail_fp32).  The
 *                     operator is symmetric, so the product reads only the 128 x 128 tiles of
 *                     its upper block triangle, symmetrized.  The hierarchy, and the V-cycle as
 *                     an operator, are those of the sparse path; only the rounding differs.  No
 *                     tail when that level is the coarsest or no level qualifies.  Memory: about
 *                     1.5 ld^2 doubles (the full matrix, kept for the block panels, and the upper
 *                     tiles; + 0.5 ld^2 floats with dense_tail_fp32), ld = the tail's dofs
 *                     rounded up to 128.
 *  dense_tail_fp32    0: the FP32 V-cycle applies the dense tail, which holds the coarsest
 *                     level's inverse, from its FP64 matrix with FP64 accumulation (FP32 vectors
 *                     in and out), as it applies the coarsest inverse without a tail (default).
 *                     1 (needs vcycle_fp32): the upper tiles are also kept in FP32 and the FP32
 *                     V-cycle reads those instead (FP64 accumulation), half the bytes.
 */
typedef struct eamg_gnn eamg_gnn;
typedef struct {
  double sigma;
  int32_t delta, R, rounds, coarsest_max_dofs, max_levels;
  double omega;
  int32_t cap_aux, cap_std_l0, cap_std;
  double pinv_rtol, tie_rtol;
  int32_t vcycle_fp32;
  const eamg_gnn *gnn;
  double gnn_skip;
  int32_t gnn_record;
  int32_t mu_s_only;
  int32_t gpu_criteria;
  int32_t dense_tail_dofs;
  int32_t dense_tail_fp32;
} eamg_setup_params;

/* Preconditioners of the PCG.  EAMG_PRECOND_VCYCLE_FP32 runs the whole V-cycle (smoothers,
 * residual, transfers, their matrices, D^+ and level vectors) in FP32 with FP32 accumulation,
 * except the coarsest level's inverse and the dense tail that holds it (FP64 matrix, FP64
 * accumulation, FP32 vectors; the tail in FP32 with dense_tail_fp32 = 1); the CG
 * operator, vectors, inner products and the stopping test stay FP64, with one conversion of r
 * to FP32 and of z to FP64 per iteration.  It needs a setup with vcycle_fp32 = 1. */
enum {
  EAMG_PRECOND_NONE = 0,
  EAMG_PRECOND_VCYCLE = 1,      /* one FP64 V-cycle (default) */
  EAMG_PRECOND_VCYCLE_FP32 = 2  /* one FP32 V-cycle           */
};

/* Solve parameters.  rtol: stop when ||r||_2 <= rtol ||b||_2 (recursive residual, x0 = 0 unless
 * use_x0); max_it: iteration limit (>= 1); use_x0: 1 = start from the given x; precond: one of
 * EAMG_PRECOND_* (INVALID_ARG for FP32 without vcycle_fp32 at setup). */
typedef struct {
  double rtol;
  int32_t max_it;
  int32_t use_x0;
  int32_t precond;
} eamg_solve_params;

/* Solve report: iterations done, final recursive and true relative residual, the wall time of
 * the solve in milliseconds measured with events on the stream (for a batch: of the whole
 * batch), and the status of this right-hand side (OK, NOT_CONVERGED or BREAKDOWN). */
typedef struct {
  int32_t iterations;
  double rel_res;
  double rel_res_true;
  double ms;
  int32_t status;
} eamg_solve_info;

/* Per-level sizes, for sizing eamg_export_level buffers. */
typedef struct {
  int32_t n;          /* vertices (block rows) of A_l                                    */
  int32_t bs;         /* real dofs per vertex (block size of A_l)                        */
  int64_t nnzb_A;     /* blocks of A_l                                                   */
  int32_t n_coarse;   /* vertices of level l+1 (0 on the coarsest level)                 */
  int32_t k_coarse;   /* columns per P_s block (dofs per coarse vertex)                  */
  int64_t nnzb_P;     /* blocks of P_s (0 on the coarsest level)                         */
  int32_t n_colors;   /* colours of the smoother (0 on the coarsest level)               */
} eamg_level_info;

/* Default parameters (all fields set). */
void eamg_default_setup_params(eamg_setup_params *out);
void eamg_default_solve_params(eamg_solve_params *out);

/*
 * Build the hierarchy (host coarsening; device P_s assembly, Galerkin products, smoother
 * diagonals and coarsest factor).  Paper: the system of section "fem" (Problems prob:gg /
 * prob:epseps on V_h0) with the auxiliary topology of section "deng" (finest edge and vertex
 * weights); per level the successive matching of Algorithm alg:pwagg with the criteria of
 * section "crs" and the coarse weights of Thm thm:cemats, the auxiliary smoothed prolongation
 * P_s of Def. def:aux_sp, A_{l+1} = P_s^T A_l P_s (section "prol"), and the pseudo-inverted
 * smoother diagonals and regularized coarsest level of section "amg".  On success *out owns
 * all device memory of the hierarchy.
 * Errors: INVALID_ARG (NULL pointers, sizes, unsorted/asymmetric pattern, missing diagonal,
 * parameters out of range), UNSUPPORTED_KERNEL, NOT_SPD (coarsest level), HIP, OOM.
 */
eamg_status eamg_setup(const eamg_problem *problem, const eamg_setup_params *params,
                       void *stream, eamg_hierarchy **out);

/*
 * Solve A x = b by PCG, preconditioned by one V-cycle per iteration: CG with the AMG V-cycle
 * as in section "res", the V-cycle being Alg. alg:tg (smoother M before, M^T after the coarse
 * correction) applied recursively down the levels.  b_dev, x_dev: DEVICE arrays of n*dim
 * doubles, caller-owned, may not alias.  b is ignored at Dirichlet dofs; x is 0 there on return.  Returns OK, NOT_CONVERGED
 * (x = last iterate), BREAKDOWN (non-finite b or residual, or a non-positive curvature /
 * preconditioned inner product), INVALID_ARG or HIP.  info may be NULL.
 */
eamg_status eamg_solve(eamg_hierarchy *h, const double *b_dev, double *x_dev,
                       const eamg_solve_params *params, void *stream, eamg_solve_info *info);

/*
 * Solve A X = B for nrhs right-hand sides at once (block panels of up to 64 columns: every
 * matrix of the V-cycle and the CG operator is streamed once per panel).  Each column runs its
 * own PCG recurrence (own alpha, beta and stopping test, exactly as eamg_solve) and stops on
 * its own; converged columns are frozen while the others continue.
 *   B_dev, X_dev  DEVICE arrays, column-major: column c is the n*dim doubles at offset c*ld;
 *                 ld >= n*dim; caller-owned; may not overlap.
 *   infos         HOST array of nrhs reports (may be NULL); infos[c].status is OK,
 *                 NOT_CONVERGED or BREAKDOWN (non-finite b column, non-positive curvature or
 *                 preconditioned inner product in that column; its x column is the last
 *                 iterate, or 0 when it never started).
 * Returns OK when every column converged, NOT_CONVERGED when at least one did not (iteration
 * limit or breakdown of that column), INVALID_ARG or HIP.  The first call with a given panel
 * width allocates the panel workspace (about 7 * n*dim*K doubles plus the V-cycle levels).
 */
eamg_status eamg_solve_batch(eamg_hierarchy *h, int32_t nrhs, const double *B_dev, int64_t ld,
                             double *X_dev, const eamg_solve_params *params, void *stream,
                             eamg_solve_info *infos);

/* ---- learned coarsening: edge-scoring network ---------------------------------------------
 *
 * A three-layer graph network scores the candidate pairs of a matching pass (Algorithm
 * alg:pwagg) with the logit of "the exact criterion (mu_b, and mu_g for larger unions;
 * Thm thm:mu1, Lemma thm:mu2) accepts this pair".  Per pair it reads EAMG_GNN_FEATURES inputs
 * built from the quantities of the criteria (log mu_s; the spectrum of E^{ij} / tr E^{ij}; the
 * traces of D-hat and M at both ends; the aggregate sizes; the trace-strength ratio):
 *   a1 = W1 x + b1, h1 = relu(a1); m_i = mean of h1 over the candidate pairs at node i;
 *   a2 = W2a h1 + W2b (m_u + m_v) + b2, h2 = relu(a2); z = w3 . h2 + b3.
 * Hidden width 64; W1, W2a, W2b, w3 are used rounded to bfloat16, all sums are FP32.
 * Parameters are EAMG_GNN_PARAMS floats packed as W1 (64 x 12, row-major), b1 (64),
 * W2a (64 x 64), W2b (64 x 64), b2 (64), w3 (64), b3 (1).
 * Graph arguments are HOST arrays: X (m x 12 floats), edges (m x 2 int32 node ids in [0, n),
 * distinct ends), labels y and weights w (m floats; weight 0 = unlabelled).  The network and all
 * its arithmetic run on the GPU; parameters live on the device.
 */
#define EAMG_GNN_FEATURES 12
#define EAMG_GNN_PARAMS 9153

/* New network from params (HOST, EAMG_GNN_PARAMS floats) or, if params is NULL, from a seeded
 * He-uniform initialisation (biases 0).  INVALID_ARG for non-finite parameters. */
eamg_status eamg_gnn_create(const float *params, uint64_t seed, eamg_gnn **out);
/* Copy the current FP32 parameters to params (HOST, EAMG_GNN_PARAMS floats). */
eamg_status eamg_gnn_params(const eamg_gnn *g, float *params);
/* Logits of the m pairs (HOST output, m floats). */
eamg_status eamg_gnn_forward(eamg_gnn *g, int64_t m, int32_t n, const float *X,
                             const int32_t *edges, float *logits);
/* Weighted mean binary cross-entropy of the logits against y and its gradient with respect to
 * the parameters (as used: the gradient of the bfloat16-rounded weights is applied to the FP32
 * masters).  loss, grad (HOST, EAMG_GNN_PARAMS) may be NULL. */
eamg_status eamg_gnn_loss_grad(eamg_gnn *g, int64_t m, int32_t n, const float *X,
                               const int32_t *edges, const float *y, const float *w, double *loss,
                               float *grad);
/* Adam (beta 0.9 / 0.999, eps 1e-8, step lr) over `epochs` passes of the ngraphs graphs, one
 * step per graph.  loss_history (HOST, epochs floats, may be NULL): mean loss per epoch. */
eamg_status eamg_gnn_train(eamg_gnn *g, int32_t ngraphs, const int64_t *m, const int32_t *n,
                           const float *const *X, const int32_t *const *edges,
                           const float *const *y, const float *const *w, int32_t epochs, float lr,
                           float *loss_history);
void eamg_gnn_destroy(eamg_gnn *g);

/* Coarsening statistics of a hierarchy (HOST outputs, any may be NULL): criteria evaluations of
 * the matching walks (mu_b; evaluated_g of them also mu_g), candidates the learned walk passed
 * over, and the number of recorded passes (gnn_record). */
eamg_status eamg_coarsening_stats(const eamg_hierarchy *h, int64_t *evaluated, int64_t *evaluated_g,
                                  int64_t *skipped, int32_t *sample_passes);
/* Recorded pass `pass` (gnn_record = 1): m candidate pairs over n working-level vertices, their
 * features X (m x 12), ends (m x 2), labels y (1: the exact criteria accept) and weights w (1:
 * evaluated by the walk, 0: unlabelled).  HOST arrays sized from a first call with NULLs. */
eamg_status eamg_gnn_samples(const eamg_hierarchy *h, int32_t pass, int64_t *m, int32_t *n, float *X,
                             int32_t *edges, float *y, float *w);

/*
 * Autotuner: measure candidate launch shapes on this hierarchy's own matrices (events on
 * `stream`, median of 5) and keep the fastest.  Single right-hand side: lanes per block row of
 * every level's smoother and residual kernels (8, 16, 32, 64 or a whole workgroup).  If
 * panel_width > 0, also the panel kernels for that many right-hand sides (rounded up to a power
 * of two): one or four wavefronts per row for every level matrix and transfer.  Later solves use
 * the tuned shapes (captured iteration graphs are rebuilt); results then differ from the
 * untuned ones only in summation order.  ms_before / ms_after (may be NULL): summed time of the
 * tuned launch sequences with the previous and the chosen shapes.  Allocates the panel
 * workspace when panel_width > 0.  Returns OK, INVALID_ARG (panel_width outside [0, 64]) or HIP.
 */
eamg_status eamg_autotune(eamg_hierarchy *h, int32_t panel_width, void *stream, double *ms_before,
                          double *ms_after);

/*
 * Solve nsys independent systems (each with its own hierarchy, e.g. meshes of different sizes)
 * together: each PCG iteration replays the captured iteration graph of every system that is
 * still iterating, each on a stream of its own, so the small launches of different systems can
 * overlap; the host then applies every system's stopping test.
 * Each system follows exactly the eamg_solve recurrence (same kernels in the same order, so its
 * result is eamg_solve's bit for bit) and stops on its own test.
 *   hs[nsys]          distinct hierarchies (a hierarchy may appear only once)
 *   b_dev[m], x_dev[m] DEVICE arrays of system m (n_m * dim doubles, natural order)
 *   params            shared by all systems (precond FP32 needs vcycle_fp32 on every hierarchy)
 *   infos             HOST array of nsys reports (may be NULL); infos[m].status is OK,
 *                     NOT_CONVERGED or BREAKDOWN (that system's x is not written on BREAKDOWN)
 * Returns OK when every system converged, NOT_CONVERGED otherwise, INVALID_ARG or HIP.
 */
eamg_status eamg_solve_multi(int32_t nsys, eamg_hierarchy *const *hs, const double *const *b_dev,
                             double *const *x_dev, const eamg_solve_params *params, void *stream,
                             eamg_solve_info *infos);

/*
 * Fuse nsys hierarchies into one block-diagonal hierarchy for eamg_solve_fused.  Level l of the
 * fused hierarchy holds level l of every system whose V-cycle reaches it, numbered colour by
 * colour and, inside a colour, system by system; a colour is then still an independent set
 * (the systems share no couplings), so each colour launch, transfer and CG vector operation of
 * the fused solve covers every system at once.  A system whose V-cycle ends on a level (its
 * dense tail, or the coarsest inverse) has its rows there after the colour ranges and is
 * applied as a dense operator, all such systems in one launch (a system whose CG has stopped
 * skips its dense operator).  Every system keeps exactly its
 * own preconditioner: the V-cycle of Algorithm alg:tg with the multicolour block Gauss-Seidel
 * smoother, its transfers P_s (Def. def:aux_sp) and Galerkin levels (section "prol"); only the
 * order in which sums are formed can differ from eamg_solve.
 *   hs[nsys]  distinct hierarchies on the current device, with equal dimension and block sizes
 *             level by level.  Their level matrices, transfers and smoother diagonals are copied;
 *             their own dense tails and coarsest inverses are read in place, so each stays alive as
 *             long as a fused hierarchy uses it (eamg_destroy on it then only marks it, and the
 *             last such fused hierarchy frees it).
 *   dense_tail_dofs  where each system's V-cycle ends (the operator is the same up to rounding
 *             in every case: a dense tail is the V-cycle of the levels below as a matrix):
 *             -1  at the system's own dense tail (dense_tail_dofs at its setup) if it has one,
 *                 as in eamg_solve, else at its coarsest inverse;
 *              0  at the coarsest inverse (every level smoothed);
 *             >0  at the first level below the finest with at most this many dofs (not the
 *                 coarsest), as a dense tail the fused hierarchy computes and owns (or the
 *                 system's own tail if it starts on that level); at most 16384.
 *             Fused, a small level's launches serve every system at once while the tails'
 *             bytes add up, so tails far smaller than a single system's best pay off.
 *             Anything else: INVALID_ARG.
 *   stream    the setup work is enqueued on it and waited for
 *   out       the fused hierarchy (free with eamg_destroy).  It accepts eamg_solve_fused,
 *             eamg_autotune (panel_width 0: lanes per row of its colour sweeps),
 *             eamg_profile_enable / eamg_profile_read and eamg_destroy; every other entry point
 *             returns EAMG_ERR_INVALID_ARG for it.
 * Returns OK, INVALID_ARG (repeated, fused or mismatched systems, another device), OOM or HIP.
 */
eamg_status eamg_fuse(int32_t nsys, eamg_hierarchy *const *hs, int32_t dense_tail_dofs,
                      void *stream, eamg_hierarchy **out);

/*
 * PCG with one V-cycle per iteration (section "res") on every system of a fused hierarchy at
 * once, each system with its own CG scalars and its own stopping test; a system that stops keeps
 * its x while the others go on.  Iterations run in rounds of 4, each round one captured graph
 * (eager launches while profiling); the host reads the systems' flags once a round.
 *   b_dev[m], x_dev[m]  DEVICE arrays of system m (hs order of eamg_fuse), n_m * dim doubles in
 *                       its natural order; Dirichlet dofs of b are treated as 0
 *   params              shared by all systems (rtol, max_it, use_x0, precond; precond FP32
 *                       needs vcycle_fp32 on every fused hierarchy)
 *   infos               HOST array of nsys reports (may be NULL): iterations, residuals,
 *                       status OK, NOT_CONVERGED or BREAKDOWN (that system's x is not written);
 *                       ms is the whole call
 * Runs on `stream` and waits for it.  Returns OK when every system converged, NOT_CONVERGED
 * otherwise, INVALID_ARG (not a fused hierarchy, NULL or aliased vectors) or HIP.
 */
eamg_status eamg_solve_fused(eamg_hierarchy *fused, const double *const *b_dev,
                             double *const *x_dev, const eamg_solve_params *params, void *stream,
                             eamg_solve_info *infos);

/*
 * Apply one V-cycle z = B^{-1} r (DEVICE arrays, n*dim doubles, level-0 natural order).
 * Dirichlet dofs of r are treated as 0.  precision: EAMG_PRECOND_VCYCLE (FP64) or
 * EAMG_PRECOND_VCYCLE_FP32 (needs vcycle_fp32 = 1 at setup); anything else is INVALID_ARG.
 */
eamg_status eamg_vcycle(eamg_hierarchy *h, const double *r_dev, double *z_dev, int32_t precision,
                        void *stream);

/*
 * eamg_vcycle without allocating or synchronizing, for callers that cannot call hipMalloc or
 * wait on the stream: code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same operation, arguments and errors as eamg_vcycle (z = B^{-1} r, DEVICE
 * arrays of n*dim doubles in level-0 natural order, Dirichlet dofs of r treated as 0), but
 *  - the colour-major copies of r and z are staged in a fixed device array of the library
 *    (32 MiB per device, held until the process ends) instead of the hierarchy's buffers: a
 *    level 0 of more than 2,097,152 dofs gives EAMG_ERR_INVALID_ARG;
 *  - the work is only enqueued on `stream`; the call returns without waiting, so z is valid
 *    once the stream has reached that point;
 *  - the profiler must be off (EAMG_ERR_INVALID_ARG otherwise) and the current device must be
 *    the one the hierarchy was set up on.
 * Every call on one GPU shares that staging array, and every call on one hierarchy its level
 * vectors: calls that overlap in time on one GPU (other streams, other threads) race.
 */
eamg_status eamg_vcycle_noalloc(eamg_hierarchy *h, const double *r_dev, double *z_dev,
                                int32_t precision, void *stream);

/* Hierarchy statistics (HOST outputs, any may be NULL).  per_level_n / per_level_nnzb must hold
 * max_levels entries.  vc and oc are the vertex and operator complexities of the tables of
 * section "res" (Tables tab:ucu, tab:3dbeam, tab:co3d): vc = sum n_l / n_0, oc = sum nnz_l /
 * nnz_0 counting scalar entries. */
eamg_status eamg_stats(const eamg_hierarchy *h, int32_t *n_levels, int64_t *per_level_n,
                       int64_t *per_level_nnzb, double *vc, double *oc);

eamg_status eamg_level_info_get(const eamg_hierarchy *h, int32_t level, eamg_level_info *out);

/*
 * Copy one level to HOST buffers in the level's natural vertex numbering (coarse vertex I is
 * the I-th agglomerate of the matching): the agglomerates of Algorithm alg:pwagg, P_s of
 * Def. def:aux_sp, A_l = P_s^T A_{l-1} P_s (section "prol") and the smoother's colours.  Any pointer may be NULL to skip it.  Sizes from
 * eamg_level_info_get:
 *   agg      n       coarse vertex of each vertex, -1 for the dropped set D (coarsest: all -1)
 *   P_rowptr n+1, P_col nnzb_P, P_val nnzb_P*bs*k_coarse (row-major blocks)
 *   A_rowptr n+1, A_col nnzb_A, A_val nnzb_A*bs*bs
 *   color    n       smoother colour of each vertex (coarsest: all -1)
 */
eamg_status eamg_export_level(const eamg_hierarchy *h, int32_t level, int32_t *agg,
                              int32_t *P_rowptr, int32_t *P_col, double *P_val,
                              int32_t *A_rowptr, int32_t *A_col, double *A_val, int32_t *color);

/* Bytes of one V-cycle's algorithmic HBM traffic and of one PCG iteration (matrix and vector
 * streams counted once per kernel), from the real per-level sizes, for the V-cycle precision
 * EAMG_PRECOND_VCYCLE or EAMG_PRECOND_VCYCLE_FP32. */
eamg_status eamg_traffic_model(const eamg_hierarchy *h, int32_t precision, double *vcycle_bytes,
                               double *iteration_bytes);

/* The CG coefficients of the last eamg_solve (or of its system in eamg_solve_multi) on h, one
 * pair per iteration: alpha_k = rho_{k-1} / (p_k . A p_k) and beta_k = rho_{k-1} / rho_{k-2}
 * (beta_1 = 0), rho = r . z (section "res": CG with the V-cycle as preconditioner).  They give
 * the Lanczos tridiagonal matrix of the preconditioned operator, whose extreme eigenvalues
 * estimate its condition number.  Up to max_entries pairs are copied to the HOST arrays alpha
 * and beta (either may be NULL); *n_out = the number of iterations recorded. */
eamg_status eamg_solve_coefficients(const eamg_hierarchy *h, int32_t max_entries, double *alpha,
                                    double *beta, int32_t *n_out);

/* Wall time of the setup phases of h (each summed over the levels), in the order the phases
 * first ran.  where: 0 host (the weights of the finest level, the matching walks -- whose
 * criteria batches may run on the GPU inside them --, the P_s plan, the symbolic Galerkin
 * products, the colouring and the solve layout), 1 device (Dirichlet rows, the P_s and
 * Galerkin numerics, the coarsest inverse, the dense tail, the solve vectors), 2 host-to-device
 * copies of the input.  Up to max_entries phases are copied to out (HOST); *n_out = the number
 * of phases. */
typedef struct {
  char name[48];
  double seconds;
  int32_t where;
} eamg_setup_phase;

eamg_status eamg_setup_phases(const eamg_hierarchy *h, int32_t max_entries, eamg_setup_phase *out,
                              int32_t *n_out);

/* The dense V-cycle tail of a hierarchy (setup parameter dense_tail_dofs): *level = the first
 * level whose V-cycle is applied as one dense matrix, or -1 when there is none; *dofs = its
 * size (0 when none).  Either pointer may be NULL. */
eamg_status eamg_dense_tail(const eamg_hierarchy *h, int32_t *level, int32_t *dofs);

/*
 * Per-kernel timing, for measuring each kernel against its bandwidth roofline.  While enabled,
 * eamg_solve / eamg_solve_batch / eamg_vcycle launch eagerly (no graph) and every launch -- or
 * run of back-to-back launches of one kernel, such as the colours of one smoother sweep -- is
 * bracketed by events on the solve stream and its algorithmic HBM bytes (matrix blocks and
 * index arrays read once, vectors read or written once, gathered vector entries counted once
 * per launch) are recorded.  eamg_profile_read synchronizes the device, aggregates the records
 * by kernel name (the template instance, e.g. "k_gs_color<double, 6, false>"), sorts them by
 * total time, copies up to max_entries of them into out, stores the number of kernels in
 * *n_out and clears the records.  on: 0 off, 1 per kernel, 2 per kernel and level (V-cycle
 * names prefixed "L<level> "), 3 as 2 with every colour launch of the single-vector sweeps
 * timed on its own (names "L<level> c<colour> ...").  Enabling resets the records.
 */
typedef struct {
  char name[48];
  int64_t launches;
  double total_ms;
  double bytes;
} eamg_kernel_stat;

eamg_status eamg_profile_enable(eamg_hierarchy *h, int32_t on);
eamg_status eamg_profile_read(eamg_hierarchy *h, int32_t max_entries, eamg_kernel_stat *out,
                              int32_t *n_out);

/* Free a hierarchy (NULL-safe).  A hierarchy that a fused hierarchy (eamg_fuse) still reads is
 * only marked, and freed with the last such fused hierarchy. */
void eamg_destroy(eamg_hierarchy *h);

/* Message of the last failure on the calling thread ("" if none). */
const char *eamg_last_error(void);

/*
 * The exact coarsening criteria of given pairs and unions of one auxiliary level, evaluated by the
 * GPU kernels the setup uses (use_device = 1, on `stream`) or by the host code (use_device = 0):
 * for checking the two against each other and against an independent evaluation.  HOST arrays;
 * the level as in eamg_host_match (D-hat blocks computed from it).
 *  n_pairs, pairs     2 per pair: vertices i, j joined by an edge -> out_mub[n_pairs], mu_b of
 *                     Lemma thm:mu2 (delta = 1)
 *  n_unions, unions   4 per union: distinct ascending vertex ids, padded with -1 at the end ->
 *                     out_mug[n_unions], mu_g of Thm thm:mu1 for C = the union (delta = 1); a
 *                     union the device cannot hold (more than 384 edges leaving it) is
 *                     evaluated on the host
 *  tau                relative eigenvalue cut of the pseudo-inverses (pinv_rtol)
 * Pairs that are not edges and malformed unions give EAMG_ERR_INVALID_ARG; nothing is written.
 */
eamg_status eamg_criteria_eval(int32_t k, int32_t n, const double *coords, int64_t n_edges,
                               const int32_t *edges, const double *E, const double *M,
                               int64_t n_pairs, const int32_t *pairs, int64_t n_unions,
                               const int32_t *unions, double tau, int32_t use_device,
                               void *stream, double *out_mub, double *out_mug);

/*
 * Host-only successive matching of one level (Algorithm alg:pwagg), exposed so the coarsening
 * can be checked without a GPU.  HOST pointers; no device work.
 *  k            1 or 6 (dofs of the auxiliary space)
 *  n, coords    vertices and positions (n*3)
 *  n_edges, edges, E   auxiliary edges (i < j, ascending (i, j)) and their k*k weights
 *  M            n*k*k vertex weights
 *  vd           n flags of V_D (may be NULL)
 *  out_agg      n: coarse vertex or -1 (D)
 *  out_nc       number of coarse vertices
 *  out_ccoords  may be NULL, else n*3 capacity: coarse positions
 *  out_margin   may be NULL: min |mu - sigma| / sigma over all threshold decisions
 */
eamg_status eamg_host_match(int32_t k, int32_t n, const double *coords, int64_t n_edges,
                            const int32_t *edges, const double *E, const double *M,
                            const uint8_t *vd, const eamg_setup_params *params,
                            int32_t *out_agg, int32_t *out_nc, double *out_ccoords,
                            double *out_margin);

#ifdef __cplusplus
}
#endif

#endif /* EAMG_H */
