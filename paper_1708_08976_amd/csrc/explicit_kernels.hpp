// The straightforward MTTKRP that the paper takes as its baseline
// (Section 2.3): the mode-n matricization X_(n) is formed explicitly by
// reordering the tensor's entries, the full Khatri-Rao product is formed
// explicitly, and the MTTKRP is one matrix multiplication of the two.  The
// external modes need no reordering: X_(0) is the tensor's memory read as a
// column-major I_0 x (I / I_0) matrix and X_(N-1) as a row-major one.  This
// file holds the reordering kernel; the Khatri-Rao rows come from
// k_krp_rows and the multiplication from hipBLASLt.
#pragma once

#include "device_common.hpp"

namespace cpm {

// Y[r][l][i] = X[r][i][l]: the 3-index view of mode n (l over the IL left
// entries, i over I_n, r over the IR right entries) with i made the fastest
// index, so that Y is X_(n) stored column-major (I_n x IL*IR, column index
// l + IL * r, the natural order of the other modes).  64 x 64 tiles go
// through LDS (one padding word per row); tile t of the grid stride covers
// (l tile, i tile, r).  E is the element's bit pattern type.
template <typename E>
__global__ __launch_bounds__(kThreads) void k_unfold(const E *__restrict__ X, int64_t IL, int64_t In, int64_t IR,
                                                     E *__restrict__ Y) {
    __shared__ E tile[64][65];
    const int64_t tl = (IL + 63) / 64, ti = (In + 63) / 64;
    const int64_t ntiles = tl * ti * IR;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4 threads
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t bl = t % tl, bi = (t / tl) % ti, r = t / (tl * ti);
        const int64_t l0 = bl * 64, i0 = bi * 64;
        const E *src = X + r * In * IL;
        E *dst = Y + r * In * IL;
        __syncthreads();
        for (int k = ty; k < 64; k += 4) {  // read rows i of the tile, l contiguous
            const int64_t i = i0 + k, l = l0 + tx;
            if (i < In && l < IL) tile[k][tx] = src[i * IL + l];
        }
        __syncthreads();
        for (int k = ty; k < 64; k += 4) {  // write rows l, i contiguous
            const int64_t l = l0 + k, i = i0 + tx;
            if (i < In && l < IL) dst[l * In + i] = tile[tx][k];
        }
    }
}

}  // namespace cpm
