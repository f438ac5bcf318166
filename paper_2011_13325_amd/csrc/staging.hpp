// Host <-> device copies of setup data through pinned staging buffers.
//
// The setup hands the device large arrays that live in pageable host memory (the input matrix,
// level weights, patterns) and reads large results back (coarse edge weights).  Pageable copies
// run at a few GB/s; these copies go through two pinned chunks instead, the host copy of one
// chunk overlapping the DMA of the other.  Both calls return when the data has arrived.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace eamg {

// `bytes` from host `src` (pageable) to device `dst`, on stream `s`; waits for the copy.
hipError_t copy_h2d_sync(void *dst, const void *src, size_t bytes, hipStream_t s);
// `bytes` from device `src` to host `dst` (pageable), on stream `s`; waits for the copy.
hipError_t copy_d2h_sync(void *dst, const void *src, size_t bytes, hipStream_t s);

}  // namespace eamg
