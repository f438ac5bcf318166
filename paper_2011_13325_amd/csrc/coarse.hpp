// Coarsest-level direct solve on the device (coarse.hip).
//
// The regularized coarsest matrix A_L + sum_i Pi_ker(A_L,ii) (section on singular coarse
// levels: SPD by construction) is inverted once at setup, in place, by blocked Gauss-Jordan
// elimination without pivoting; every V-cycle then applies the inverse as one dense
// matrix-vector (or matrix-panel) product, a stream of n^2 doubles at HBM bandwidth.  On one
// GPU this makes a coarsest level of thousands of dofs cheaper than the many colour launches of
// the small levels it replaces.
//
// Storage: row-major with a leading dimension ld = n rounded up to a multiple of 128; before the
// inversion the padding rows and columns hold the identity, so the padded matrix is diag(A, I)
// and its inverse diag(A^{-1}, I): every kernel works on whole 64 x 64 tiles, and the columns
// n..ld-1 of the first n rows of the inverse are exactly zero.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace eamg {

constexpr int kDenseTile = 64;            // Gauss-Jordan block size
constexpr int kMaxCoarsestDofs = 16384;   // inverse <= 2 GiB of FP64

inline int dense_ld(int n) { return (n + 127) / 128 * 128; }

// Scratch of launch_gj_invert: the inverted pivot block, the row panel and the saved column
// panel of one block step.
inline size_t gj_work_doubles(int ld) {
  return size_t(kDenseTile) * kDenseTile + 2 * size_t(ld) * kDenseTile;
}

// D (ld x ld) := the n x n block CSR matrix (rp, col on the device; AoS bs x bs blocks in val)
// with reg (n blocks of bs x bs, device) added to its diagonal blocks, zero elsewhere, and the
// identity on the padding rows n * bs .. ld - 1.
hipError_t launch_dense_assemble(int n, int bs, const int64_t *rp, const int *col,
                                 const double *val, const double *reg, int ld, double *D,
                                 hipStream_t s);

// A (ld x ld, ld a multiple of 128, SPD) := A^{-1}, then symmetrized as (A + A^T) / 2.  *flag
// (device int, zeroed by the caller) becomes 1 if a pivot is not positive and finite, i.e. A is
// not positive definite (the result is then meaningless).  Deterministic.
hipError_t launch_gj_invert(int ld, double *A, double *work, int *flag, hipStream_t s);

// y = D x for the first n rows of D (leading dimension ld); x, y of length n; FP64 accumulation.
template <class T>
hipError_t launch_dense_gemv(int n, int ld, const double *D, const T *x, T *y, hipStream_t s);

// Packed symmetric storage: the tiles (i, j), i <= j, of kSymTile x kSymTile entries of the upper
// block triangle of an n x n symmetric matrix (nb = ceil(n / kSymTile) block rows), tile (i, j)
// at index i * nb - i * (i - 1) / 2 + j - i, row-major inside, zero past n: about half the bytes
// of the full matrix.
constexpr int kSymTile = 128;
inline int sym_blocks(int n) { return (n + kSymTile - 1) / kSymTile; }
inline int64_t sym_tiles(int nb) { return int64_t(nb) * (nb + 1) / 2; }
inline size_t sym_entries(int n) { return size_t(sym_tiles(sym_blocks(n))) * kSymTile * kSymTile; }
// Workspace of launch_dense_symv: nb * nb partial blocks of kSymTile doubles.
inline size_t sym_work_doubles(int n) { return size_t(sym_blocks(n)) * sym_blocks(n) * kSymTile; }

// S (packed, sym_entries(n) values of TM) := the upper tiles of (D + D^T) / 2, D n x n with
// leading dimension ld (a multiple of kSymTile).
template <class TM>
hipError_t launch_pack_sym(int n, int ld, const double *D, TM *S, hipStream_t s);

// y = S x for the packed symmetric S (TM values; FP64 accumulation; x, y of length n; TV double
// with TM double, float with either).  Two launches: one workgroup per stored tile writes its
// row sums and (off the diagonal) its column sums into W (sym_work_doubles(n)); a second sums
// the parts of every output in a fixed order, so the result is reproducible.  Calls that share W
// must not overlap.
template <class TM, class TV>
hipError_t launch_dense_symv(int n, const TM *S, const TV *x, TV *y, double *W, hipStream_t s);

// One matrix of a multi-part symmetric product: packed upper tiles S (TM values) of an n x n
// matrix (nb = sym_blocks(n)) applied to x[off .. off + n) into y[off .. off + n).  Among all
// parts of a launch it has tiles t0 .. t0 + sym_tiles(nb) - 1 and rows row0 .. row0 + n - 1, and
// its partial sums start at W[woff]; sys indexes its activity flag.
struct SymPart {
  const void *S;
  int64_t off, woff;
  int n, nb, row0, t0, sys;
};
// y = S_p x for every part p (nparts entries, device array, t0 and row0 increasing from 0; tiles
// and rows in total; W holds every part's sym_work_doubles(n)): one workgroup per stored tile,
// then one thread per row, as launch_dense_symv.  With active (device, indexed by sys), parts
// whose flag is 0 are skipped and leave y as it is.
template <class TM, class TV>
hipError_t launch_dense_symv_multi(int nparts, const SymPart *parts, int tiles, int rows,
                                   const double *active, const TV *x, TV *y, double *W, hipStream_t s);

// B (n x K panel, entry (dof, k) at dof * K + k) := columns j0 .. j0 + K - 1 of the identity.
hipError_t launch_identity_panel(int n, int K, int j0, double *B, hipStream_t s);

// Columns j0 .. j0 + ncols - 1 (ncols <= K) of the row-major D (leading dimension ld) := the
// first ncols columns of the n x K panel X.
hipError_t launch_scatter_panel(int n, int K, int j0, int ncols, const double *X, int ld, double *D,
                                hipStream_t s);

// Y = D X for a panel of K columns (K a power of two in [1, 64]; entry (dof, k) at dof * K + k),
// on the matrix cores in FP64, summed over dense_panel_splits(n) slices of the inner dimension
// through `work` (device, dense_panel_work_doubles(n, K) doubles); deterministic.
int dense_panel_splits(int n);
size_t dense_panel_work_doubles(int n, int K);
template <class T>
hipError_t launch_dense_panel(int n, int ld, int K, const double *D, const T *X, T *Y,
                              double *work, hipStream_t s);

}  // namespace eamg
