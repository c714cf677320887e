// Symmetric-pair packed storage (the linearised triangle of a symmetric
// pair of modes that Section 5.3.3 uses for its fMRI tensor).
//
// A tensor with I_0 = I_1 = n and X(i, j, rest) = X(j, i, rest) is held as
// its triangle i <= j: pair index p = j (j + 1) / 2 + i (i fastest, then j),
// then modes 2..N-1 in natural order, P = n (n + 1) / 2 pairs.  The packed
// tensor is itself a natural-layout tensor with modes (P, I_2, ..., I_{N-1}),
// so its MTTKRPs run on the ordinary kernels:
//   * a mode k >= 2 is the view's mode k - 1 with the pair factor
//     W(p, c) = U_0(i, c) U_1(j, c) + U_0(j, c) U_1(i, c) for i < j and
//     U_0(i, c) U_1(i, c) on the diagonal (k_sympair_rows): every packed
//     entry stands for (i, j, .) and (j, i, .);
//   * the pair modes 0 and 1 share one pass: the view's mode-0 MTTKRP
//     T(p, c) = sum_rest Xp(p, rest) K_rest(rest, c), then
//     M_0(a, c) = sum_j T(pair(a, j), c) U_1(j, c) and
//     M_1(b, c) = sum_i T(pair(i, b), c) U_0(i, c) (k_sympair_leaf).
#pragma once

#include "device_common.hpp"

namespace cpm {

// Pair (i, j), i <= j, of packed index p.
__device__ inline void sympair_of(int64_t p, int64_t &i, int64_t &j) {
    int64_t jj = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while (jj * (jj + 1) / 2 > p) --jj;
    while ((jj + 1) * (jj + 2) / 2 <= p) ++jj;
    j = jj;
    i = p - jj * (jj + 1) / 2;
}
__device__ inline int64_t sympair_index(int64_t a, int64_t b) {
    const int64_t i = a < b ? a : b, j = a < b ? b : a;
    return j * (j + 1) / 2 + i;
}

// W (P x R, row-major): the pair factor, each entry formed in float64 and
// rounded once.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_sympair_rows(const T *__restrict__ U0, const T *__restrict__ U1,
                                                           int64_t P, int R, T *__restrict__ W) {
    const int64_t total = P * R;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total; e += (int64_t)gridDim.x * kThreads) {
        const int64_t p = e / R;
        const int c = (int)(e - p * R);
        int64_t i, j;
        sympair_of(p, i, j);
        double v = (double)U0[i * R + c] * (double)U1[j * R + c];
        if (i != j) v += (double)U0[j * R + c] * (double)U1[i * R + c];
        W[e] = (T)v;
    }
}

// out(a, c) = sum_{j < n} T(pair(a, j), c) * Uo(j, c), for the pair modes.
// grid.x = output row a, grid.y = block of 64 rank columns (one per lane);
// the four waves take quarters of the j range and their float64 sums are
// added in wave order.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_sympair_leaf(const T *__restrict__ Tm, const T *__restrict__ Uo,
                                                           int64_t n, int R, T *__restrict__ out) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t a = blockIdx.x;
    const int c = (int)blockIdx.y * 64 + lane;
    const int64_t q = (n + 3) / 4;
    const int64_t j0 = wave * q, j1 = min(n, j0 + q);
    double s = 0.0;
    if (c < R)
        for (int64_t j = j0; j < j1; ++j) s += (double)Tm[sympair_index(a, j) * R + c] * (double)Uo[j * R + c];
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && c < R) out[a * R + c] = (T)(((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]);
}

// Xp(p, r) = X(i_p, j_p, r) for the packed triangle; E is the element's bit
// pattern type (2, 4 or 8 bytes).  grid.x covers the pairs (one per
// thread, decoded once), grid.y strides over r; grid.z = plane (the hi and
// lo planes of a split-bf16 tensor).  Pure data movement.
template <typename E>
__global__ __launch_bounds__(kThreads) void k_pack_sympair(const E *__restrict__ X, int64_t n, int64_t rest,
                                                           E *__restrict__ Xp) {
    const int64_t P = n * (n + 1) / 2;
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= P) return;
    int64_t i, j;
    sympair_of(p, i, j);
    const int64_t full = n * n * rest;
    const E *src = X + blockIdx.z * full + i + n * j;
    E *dst = Xp + blockIdx.z * P * rest + p;
    for (int64_t r = blockIdx.y; r < rest; r += gridDim.y) dst[r * P] = src[r * n * n];
}

}  // namespace cpm
