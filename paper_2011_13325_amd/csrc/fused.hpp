// Launchers of the fused multi-system kernels (fused.hip).
//
// A fused hierarchy holds several independent systems as one block-diagonal hierarchy: level l
// is the union of the systems' levels l, one row range per system and colour.  The CG of each
// system keeps its own scalars, so its vector operations run on *segments*: block k of a
// segmented launch covers the dofs [d0[k], d1[k]) of the concatenated level-0 vector, all of
// one system sys[k]; the blocks of system m are [bptr[m], bptr[m+1]), in increasing order of
// their dofs, so a system's sums always add the same partials in the same order.
//
// Per-system scalars use the slots of the block-panel CG (PanelScalar, panel.hpp) with the system
// in place of the column: scal[slot * nsys + m].  All pointers are device pointers; every
// launcher enqueues on `s` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eamg {

struct SegTable {
  int nsys = 0, nblk = 0;
  const int *sys = nullptr;      // nblk
  const int64_t *d0 = nullptr;   // nblk
  const int64_t *d1 = nullptr;   // nblk
  const int *bptr = nullptr;     // nsys + 1
};

// dofs of one block of a segmented launch (a segment is split into blocks of at most this many)
constexpr int kSegChunk = 2048;

// part[k] <- sum over block k of a.b
hipError_t launch_sdot(const SegTable &T, const double *a, const double *b, double *part,
                       hipStream_t s);
// scal[slot * nsys + m] <- sum of part over system m's blocks, in block order, then the
// per-system bookkeeping of `op` (PanelReduceOp, panel.hpp)
hipError_t launch_sreduce(const SegTable &T, const double *part, double *scal, int slot, int op,
                          hipStream_t s);
// active systems: x += ALPHA p ; r -= ALPHA q ; part[k] <- r.r over block k (every system)
hipError_t launch_supdate_xr(const SegTable &T, const double *scal, double *x, double *r,
                             const double *p, const double *q, double *part, hipStream_t s);
// active systems: p = z + BETA p
hipError_t launch_supdate_p(const SegTable &T, const double *scal, const double *z, double *p,
                            hipStream_t s);
// NONFINITE of system m = 1 if its segment of a holds a non-finite entry (NONFINITE pre-zeroed)
hipError_t launch_sfinite(const SegTable &T, const double *a, double *scal, hipStream_t s);
// every slot zero, then RTOL and MAXIT of every system
hipError_t launch_sinit(int nsys, double rtol, int max_it, double *scal, hipStream_t s);
// out[map[v] * bs + c] = mask[v] ? 0 : in[v * bs + c]  for v < n (natural -> fused order)
hipError_t launch_scatter_in(int n, int bs, const int *map, const uint8_t *mask, const double *in,
                             double *out, hipStream_t s);
// out[v * bs + c] = in[map[v] * bs + c]  for v < n (fused -> natural order)
hipError_t launch_gather_out(int n, int bs, const int *map, const double *in, double *out,
                             hipStream_t s);

}  // namespace eamg
