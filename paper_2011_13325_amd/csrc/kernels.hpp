// Launchers of the gfx950 kernels (kernels.hip).  All pointers are device pointers; every
// launcher enqueues on `s` and returns the launch status.
//
// Solve-phase matrices (SolveMat) are block CSR with row-major blocks stored one after another:
// value (r, c) of block q lives at val[q * BR * BC + r * BC + c], so a lane that owns a block
// reads it as a few wide loads of consecutive bytes (measured on a level-1-shaped 6 x 6 FP32
// matrix: 11 % more bandwidth than element planes, where value (r, c) of every block forms one
// array).  Rows of every level are numbered colour-major, so a colour is a contiguous row range
// and, within a row, the columns below the row index are exactly the neighbours of lower colour.
// diag[i] is the position of the diagonal block of row i.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eamg {

// ---- setup -------------------------------------------------------------------------------
// Dirichlet rows / columns of A_N -> identity / zero blocks (AoS row-major blocks).
hipError_t launch_dirichlet(int n, int bs, const int64_t *rp, const int *col, double *val,
                            const uint8_t *dir, hipStream_t s);

// Dinv[i] = pinv_tau(A_ii) for every row (AoS blocks, natural numbering).
hipError_t launch_diag_pinv(int n, int bs, const int64_t *rp, const int *col, const double *val,
                            double *Dinv, double tau, hipStream_t s);

struct PsArgs {
  int n, k, bs;
  const int *type;        // ROW_S / ROW_A / ROW_D
  const int *agg;         // coarse vertex or -1
  const double *x;        // fine positions n*3
  const double *xc;       // coarse positions nc*3
  const int64_t *Prp;     // P_s pattern
  const int *Pcol;
  const int64_t *Arp;     // A_l (AoS bs x bs)
  const int *Acol;
  const double *Aval;
  const int64_t *Fptr;    // filtered neighbours of edge-matrix rows
  const int *Fvtx, *Fedge;
  const double *E;        // edge weights m*k*k
  double omega, tau;
  double *Pval;           // out: nnz(P) * bs * k (AoS)
};
hipError_t launch_ps_numeric(const PsArgs &a, hipStream_t s);

// C = A * B on a given pattern (AoS blocks: A ra x ca, B ca x cb, C ra x cb).
// crow[q] = block row of entry q of C.
hipError_t launch_spgemm_numeric(int64_t nnzC, int ra, int ca, int cb, const int *crow,
                                 const int *Ccol, const int64_t *Arp, const int *Acol,
                                 const double *Aval, const int64_t *Brp, const int *Bcol,
                                 const double *Bval, double *Cval, hipStream_t s);

// out[q] = transpose(in[src[q]]) for r x c input blocks (AoS).
hipError_t launch_transpose_blocks(int64_t nnz, int r, int c, const int64_t *src, const double *in,
                                   double *out, hipStream_t s);

// Block gather: out[q * bsz + e] = in[src[q] * bsz + e].
hipError_t launch_gather_blocks(int64_t nnz, int bsz, const int64_t *src, const double *in, double *out,
                                hipStream_t s);

// AoS -> AoS row gather: out[r * bsz + e] = in[perm[r] * bsz + e].
hipError_t launch_gather_rows(int n, int bsz, const int *perm, const double *in, double *out,
                              hipStream_t s);

// ---- solve -------------------------------------------------------------------------------
constexpr int kBlock = 256;          // threads per workgroup of the solve kernels
constexpr double kWideRowBlocks = 96; // square matrices with longer average rows: group = kBlock

struct SolveMat {
  // group: lanes per row (a power of two <= 64), or 128 / kBlock for two wavefronts / a whole
  // workgroup per row (square matrices with diag only)
  int n_rows = 0, n_cols = 0, br = 0, bc = 0, group = 16;
  // lanes per row of the backward sweep (whole rows), or 0 for `group` (forward sweep and the
  // residual update read about half of each row)
  int group_bwd = 0;
  // panel kernels: wavefronts per row (1 or 4), or 0 for the built-in choice
  int panel_waves = 0;
  int64_t nnz = 0;
  const int *rp = nullptr;   // int32 row offsets (nnz < 2^31 for one level)
  const int *col = nullptr;
  const double *val = nullptr;
  const float *val32 = nullptr;  // FP32 copy of val (FP32 V-cycle), or nullptr
  const int *diag = nullptr; // square matrices only
  // Square colour-major level matrices also hold the blocks left of the diagonal, the blocks
  // right of it and the diagonal blocks each in storage of their own (row offsets, columns,
  // blocks; the diagonal block of row i is block i of dg_val), so that the forward sweep and
  // the residual update, which read one side of every row, stream contiguous memory instead of
  // touching partly used cache lines at both ends of every row segment.
  const int *lo_rp = nullptr, *lo_col = nullptr;
  const double *lo_val = nullptr;
  const float *lo_val32 = nullptr;
  int64_t lo_nnz = 0;
  const int *up_rp = nullptr, *up_col = nullptr;
  const double *up_val = nullptr;
  const float *up_val32 = nullptr;
  int64_t up_nnz = 0;
  const double *dg_val = nullptr;   // nnz = n_rows
  const float *dg_val32 = nullptr;
};

// y = A x ; if part != nullptr also writes per-workgroup partial sums of x.y (spmv_blocks(A)
// entries)
hipError_t launch_spmv(const SolveMat &A, const double *x, double *y, double *part, hipStream_t s);
int spmv_blocks(const SolveMat &A);
// The V-cycle kernels are instantiated for T = double (values SolveMat::val) and T = float
// (values SolveMat::val32); they accumulate in T.
// Forward colour sweep with x = 0 initially on rows [r0, r1):
//   t = b_i - sum_{j < i} A_ij x_j ; x_i = Dinv_i t ; r_i = t - A_ii x_i
template <class T>
hipError_t launch_gs_fwd(const SolveMat &A, const T *Dinv, int r0, int r1, const T *b, T *x, T *r,
                         hipStream_t s);
// r_i -= sum_{j > i} A_ij x_j on rows [r0, r1) (completes r = b - A x after the forward sweep).
template <class T>
hipError_t launch_resid_upper(const SolveMat &A, int r0, int r1, const T *x, T *r, hipStream_t s);
// Backward colour sweep on rows [r0, r1): x_i += Dinv_i (b_i - sum_j A_ij x_j).
template <class T>
hipError_t launch_gs_bwd(const SolveMat &A, const T *Dinv, int r0, int r1, const T *b, T *x,
                         hipStream_t s);
// y = M x (rectangular, overwrite) or y += M x (accumulate = true).
template <class T>
hipError_t launch_rect(const SolveMat &M, const T *x, T *y, bool accumulate, hipStream_t s);
// out[i] = D(in[i])
template <class S, class D>
hipError_t launch_convert(int64_t n, const S *in, D *out, hipStream_t s);
// Block gather to FP32: out[q * bsz + e] = float(in[src[q] * bsz + e]).
hipError_t launch_gather_blocks_f32(int64_t nnz, int bsz, const int64_t *src, const double *in,
                                    float *out, hipStream_t s);

// Vector operations with deterministic reductions; grid size fixed by the length.
int dot_blocks(int64_t n);
// part <- partials of a.b (b in double, or in float: the FP32 V-cycle's output, each value
// converted exactly)
hipError_t launch_dot(int64_t n, const double *a, const double *b, double *part, hipStream_t s);
hipError_t launch_dot(int64_t n, const double *a, const float *b, double *part, hipStream_t s);
// Reduce partials into scal[slot]; op selects what else is derived (see kernels.hip).
enum ReduceOp : int { RED_STORE = 0, RED_ALPHA = 1, RED_BETA = 2 };
hipError_t launch_reduce(int nparts, const double *part, double *scal, int slot, int op,
                         hipStream_t s);
// x += alpha p ; r -= alpha q ; part <- partials of r.r   (alpha = scal[SC_ALPHA]); with r32,
// also r32 = float(r) (the next FP32 V-cycle's right-hand side)
hipError_t launch_update_xr(int64_t n, const double *scal, double *x, double *r, const double *p,
                            const double *q, double *part, hipStream_t s, float *r32 = nullptr);
// p = z + beta p (beta = scal[SC_BETA]); z in double or float
hipError_t launch_update_p(int64_t n, const double *scal, const double *z, double *p, hipStream_t s);
hipError_t launch_update_p(int64_t n, const double *scal, const float *z, double *p, hipStream_t s);
// y = a - b
hipError_t launch_sub(int64_t n, const double *a, const double *b, double *y, hipStream_t s);
hipError_t launch_copy(int64_t n, const double *a, double *y, hipStream_t s);
// out[r*bs+c] = mask[perm[r]] ? 0 : in[perm[r]*bs+c]   (natural -> colour-major, Dirichlet zeroed)
hipError_t launch_perm_in(int n, int bs, const int *perm, const uint8_t *mask, const double *in,
                          double *out, hipStream_t s);
// out[perm[r]*bs+c] = in[r*bs+c]   (colour-major -> natural)
hipError_t launch_perm_out(int n, int bs, const int *perm, const double *in, double *out,
                           hipStream_t s);
// flag non-finite entries: scal[slot] = 1 if any a[i] is not finite (scal[slot] pre-zeroed)
hipError_t launch_finite_check(int64_t n, const double *a, double *scal, int slot, hipStream_t s);
hipError_t launch_fill(int64_t n, double v, double *a, hipStream_t s);

// Scalar slots on the device.
enum Scalar : int {
  SC_RHO = 0, SC_PQ = 1, SC_RR = 2, SC_ALPHA = 3, SC_BETA = 4, SC_RZ = 5, SC_BB = 6,
  SC_BAD = 7, SC_NONFINITE = 8, SC_COUNT = 16
};

}  // namespace eamg
