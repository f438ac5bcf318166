// Launchers of the block-panel (multi right-hand side) kernels (panel.hip).
//
// A panel holds K right-hand sides of one level interleaved: entry (dof d, column k) of a panel
// vector lives at v[d * K + k], so the K values of one dof are contiguous.  Every sparse matrix
// kernel gives one block row to a wavefront: 64 / K sub-teams of K lanes share out the row's
// blocks, lane k of a sub-team computing column k, and a shuffle reduction adds the sub-teams'
// sums.  A matrix block is read once per sub-team (its K lanes load the same address) and
// reused for all K columns; the gathered vector entries are K-wide contiguous loads.  K is a
// power of two in [1, 64]; lanes of different columns never combine values, so the columns
// stay independent in every kernel.
//
// Matrices are the SolveMat block storage of the single-vector path (kernels.hpp), with rows
// in the level's colour-major order.  All pointers are device pointers; every launcher
// enqueues on `s` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace eamg {

// Forward colour sweep with X = 0 initially on rows [r0, r1):
//   T_i = B_i - sum_{j < i} A_ij X_j ; X_i = Dinv_i T_i ; R_i = T_i - A_ii X_i
template <class T>
hipError_t launch_pgs_fwd(const SolveMat &A, const T *Dinv, int r0, int r1, int K, const T *b, T *x,
                          T *r, hipStream_t s);
// Backward colour sweep on rows [r0, r1): X_i += Dinv_i (B_i - sum_j A_ij X_j).
template <class T>
hipError_t launch_pgs_bwd(const SolveMat &A, const T *Dinv, int r0, int r1, int K, const T *b, T *x,
                          hipStream_t s);
// R_i -= sum_{j > i} A_ij X_j on all rows.
template <class T>
hipError_t launch_presid_upper(const SolveMat &A, int K, const T *x, T *r, hipStream_t s);
// Y = M X or Y += M X (rectangular transfer).
template <class T>
hipError_t launch_prect(const SolveMat &M, int K, const T *x, T *y, bool accumulate, hipStream_t s);
// FP64 CG operator: Y = A X; if part != nullptr also per-workgroup, per-column partial sums of
// X.Y into part[wg * K + k] (pspmv_blocks(A, K) workgroups).
hipError_t launch_pspmv(const SolveMat &A, int K, const double *x, double *y, double *part,
                        hipStream_t s);
int pspmv_blocks(const SolveMat &A, int K);

// ---- panel CG vectors (FP64, n = dofs * K entries) -------------------------------------------
// Per-column state of the batched PCG, scal[slot * K + k].
enum PanelScalar : int {
  PS_RHO = 0, PS_PQ = 1, PS_RR = 2, PS_ALPHA = 3, PS_BETA = 4, PS_RZ = 5, PS_BB = 6,
  PS_BAD = 7, PS_NONFINITE = 8, PS_ACTIVE = 9, PS_CONV = 10, PS_ITS = 11, PS_RTOL = 12,
  PS_MAXIT = 13, PS_RR0 = 14, PS_COUNT = 16
};
// What a panel reduction derives besides storing the column sums in scal[slot]:
//   PRED_STORE  nothing
//   PRED_INIT   slot BB: ACTIVE = (bb > 0 and b finite), CONV = (bb == 0), BAD = b not finite
//   PRED_RHO0   slot RHO: active columns with rho <= 0 stop: converged if RR0 == 0 (exact
//               initial guess), else BAD
//   PRED_ALPHA  slot PQ: ALPHA = RHO / pq for active columns (pq <= 0 or non-finite: BAD, stop)
//   PRED_BETA   slot RZ: BETA = rz / RHO, RHO = rz for active columns (rz <= 0: BAD, stop)
//   PRED_RR     slot RR: active columns count one more iteration (ITS) and stop when
//               sqrt(rr) <= RTOL sqrt(bb) (CONV) or ITS >= MAXIT; non-finite rr: BAD, stop
enum PanelReduceOp : int {
  PRED_STORE = 0, PRED_INIT = 1, PRED_RHO0 = 2, PRED_ALPHA = 3, PRED_BETA = 4, PRED_RR = 5
};
int pdot_blocks(int64_t n);
// part[wg * K + k] <- per-column partials of a.b over the n entries
hipError_t launch_pdot(int64_t n, int K, const double *a, const double *b, double *part,
                       hipStream_t s);
hipError_t launch_preduce(int nparts, int K, const double *part, double *scal, int slot, int op,
                          hipStream_t s);
// Active columns: X += ALPHA P ; R -= ALPHA Q ; part <- per-column partials of R.R
hipError_t launch_pupdate_xr(int64_t n, int K, const double *scal, double *x, double *r,
                             const double *p, const double *q, double *part, hipStream_t s);
// Active columns: P = Z + BETA P
hipError_t launch_pupdate_p(int64_t n, int K, const double *scal, const double *z, double *p,
                            hipStream_t s);
// Per-column solve state: RTOL, MAXIT, zero everything else.
hipError_t launch_pinit_scal(int K, double rtol, int max_it, double *scal, hipStream_t s);
// NONFINITE[k] = 1 if column k of a holds a non-finite entry (NONFINITE pre-zeroed)
hipError_t launch_pfinite(int64_t n, int K, const double *a, double *scal, hipStream_t s);
// Columns that did not start (b = 0 or not finite) get x = 0.
hipError_t launch_pzero_unstarted(int64_t n, int K, const double *scal, double *x, hipStream_t s);
// natural column-major user panel (nrhs columns of n*bs) -> interleaved colour-major, Dirichlet
// rows zeroed, columns nrhs..K-1 zero
hipError_t launch_ppack(int n, int bs, int K, int nrhs, const int *perm, const uint8_t *mask,
                        const double *in, int64_t ld, double *out, hipStream_t s);
// interleaved colour-major -> natural column-major (columns < nrhs)
hipError_t launch_punpack(int n, int bs, int K, int nrhs, const int *perm, const double *in,
                          double *out, int64_t ld, hipStream_t s);

}  // namespace eamg
