// Last step of the all-mode MTTKRP with cross-mode reuse (the reuse of
// partial results across the MTTKRPs of different modes that the paper's
// Conclusion names as the next step, after Phan et al., Section III.C).
//
// The modes are split into two groups, [0, s) and [s, N).  One pass over X
// contracts the right group (an external-mode MTTKRP of X viewed as
// (I_0 ... I_{s-1} flattened, I_s, ..., I_{N-1})), leaving
//   T_L(l, c) = sum_r X(l, r) K_R(r, c)      l over the left group's entries,
// and one pass contracts the left group the same way, leaving T_R(r, c).
// Every mode's MTTKRP then follows from the intermediate of its own group:
//   M_n(i, c) = sum over l with l_n = i of T(l, c) * prod_{k in group, k != n} U_k(l_k, c),
// which is the MTTKRP definition with the other group's sum already done.
// This file holds that last step; the two passes are ordinary MTTKRP
// launches.
#pragma once

#include "device_common.hpp"

namespace cpm {

// Product of factors 1..Z-1 of a Khatri-Rao descriptor at row g (all but
// the fastest), digits decoded with 32-bit division when the operands allow.
template <typename T>
__device__ inline T krp_slow_value(const Krp<T> &k, int R, int64_t g, int c) {
    T v = T(1);
    for (int z = 1; z < k.Z; ++z) v *= k.U[z][mod64(div64(g, k.stride[z]), k.J[z]) * R + c];
    return v;
}

// One group mode's MTTKRP from the group intermediate T (rows of R values;
// the row index is the group's multi-index, first mode fastest).  Writing a
// row as l = b + Ll * (i + It * a) (b over the group modes before this one,
// a over those after), and q = b + Ll * a for the pair, M(i, c) = sum_q
// T(l, c) K(q, c), with K the Khatri-Rao product of the group's other
// modes in order (descriptor kk).
//
// grid.x strides over the It output rows, grid.y splits the pairs into
// ranges of per_split, grid.z takes blocks of 2^rc_shift rank columns.
// Within a wave, 64 >> rc_shift sub-rows run side by side; each of the
// block's 4 * (64 >> rc_shift) sub-rows walks a contiguous run of pairs as
// Algorithm 1 walks Khatri-Rao rows: the product of the slower factors is
// held and refreshed only when the fastest index wraps, and the T row
// advances by one (by Ll * (It - 1) more when b wraps).  The block's sum is
// formed in a fixed order in float64: a butterfly over each wave's
// sub-rows, then the four waves in order through LDS.  With
// grid.y == 1 the result goes to M directly, otherwise to slice blockIdx.y
// of the partial buffer [grid.y][It][R], summed afterwards in slice order.
constexpr int kLeafBatch = 8;
template <typename T>
__global__ __launch_bounds__(kThreads) void k_tree_leaf(const T *__restrict__ Tm, int64_t Ll, int64_t It,
                                                        int64_t pairs, int64_t per_split, Krp<T> kk, int R,
                                                        int rc_shift, T *__restrict__ out) {
    __shared__ double red[kThreads];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int RC = 1 << rc_shift;
    const int subs = 64 >> rc_shift;
    const int sub = lane >> rc_shift;
    const int c = (int)blockIdx.z * RC + (lane & (RC - 1));
    const bool col_ok = c < R;
    const int cc = col_ok ? c : 0;
    const int64_t p0 = (int64_t)blockIdx.y * per_split;
    const int64_t p1 = p0 + per_split < pairs ? p0 + per_split : pairs;
    const int workers = 4 * subs;
    const int64_t run = (p1 - p0 + workers - 1) / workers;
    const int64_t wk = wave * subs + sub;
    const int64_t q0 = p0 + wk * run < p1 ? p0 + wk * run : p1;
    const int64_t q1 = q0 + run < p1 ? q0 + run : p1;
    const int64_t J0 = kk.Z > 0 ? kk.J[0] : 1;
    const T *U0 = kk.Z > 0 ? kk.U[0] : nullptr;
    for (int64_t i = blockIdx.x; i < It; i += gridDim.x) {
        double acc = 0.0;
        if (q0 < q1) {
            const int64_t a = div64(q0, Ll);
            int64_t b = q0 - a * Ll;
            int64_t row = b + Ll * (i + It * a);
            int64_t d0 = kk.Z > 0 ? mod64(q0, J0) : 0;
            T slow = krp_slow_value(kk, R, q0, cc);
            // kLeafBatch pairs per step: rows and weights first, then the
            // loads of all of them in flight together, then the adds in
            // pair order
            for (int64_t q = q0; q < q1; q += kLeafBatch) {
                int64_t rows[kLeafBatch];
                T ws[kLeafBatch];
#pragma unroll
                for (int u = 0; u < kLeafBatch; ++u) {
                    const bool ok = q + u < q1;
                    rows[u] = ok ? row : -1;
                    ws[u] = ok ? (kk.Z > 0 ? slow * U0[d0 * R + cc] : T(1)) : T(0);
                    if (ok) {
                        ++row;
                        if (++b == Ll) {
                            b = 0;
                            row += Ll * (It - 1);
                        }
                        if (++d0 == J0) {
                            d0 = 0;
                            if (q + u + 1 < q1) slow = krp_slow_value(kk, R, q + u + 1, cc);
                        }
                    }
                }
                double v[kLeafBatch];
#pragma unroll
                for (int u = 0; u < kLeafBatch; ++u)
                    v[u] = (col_ok && rows[u] >= 0) ? (double)Tm[rows[u] * R + c] : 0.0;
#pragma unroll
                for (int u = 0; u < kLeafBatch; ++u) acc += v[u] * (double)ws[u];
            }
        }
        // the wave's sub-rows first (a butterfly over the lanes that hold the
        // same columns: a fixed pattern, so the sum is reproducible), then
        // the four waves in order
        for (int off = RC; off < 64; off <<= 1) acc += __shfl_xor(acc, off);
        if (lane < RC) red[wave * 64 + lane] = acc;
        __syncthreads();
        if (tid < RC) {
            const double s = ((red[tid] + red[64 + tid]) + red[128 + tid]) + red[192 + tid];
            const int oc = (int)blockIdx.z * RC + tid;
            if (oc < R) out[((int64_t)blockIdx.y * It + i) * R + oc] = (T)s;
        }
        __syncthreads();
    }
}

// Float32 form of k_tree_leaf for R a multiple of 4 with 16-byte aligned
// factors: each lane takes 4 consecutive rank columns (16-byte loads of T
// rows and factor rows), 2^rc_shift lanes cover a row's column block of
// 4 * 2^rc_shift columns, and 64 >> rc_shift sub-rows run side by side.
// Same walk, batching and fixed-order float64 sums as k_tree_leaf.
__device__ inline f32x4 krp_slow_value4(const Krp<float> &k, int R, int64_t g, int c4) {
    f32x4 v = {1.f, 1.f, 1.f, 1.f};
    for (int z = 1; z < k.Z; ++z)
        v *= *reinterpret_cast<const f32x4 *>(k.U[z] + mod64(div64(g, k.stride[z]), k.J[z]) * R + c4);
    return v;
}

__global__ __launch_bounds__(kThreads) void k_tree_leaf4(const float *__restrict__ Tm, int64_t Ll, int64_t It,
                                                         int64_t pairs, int64_t per_split, Krp<float> kk, int R,
                                                         int rc_shift, float *__restrict__ out) {
    __shared__ double red[4][kThreads];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int RC = 1 << rc_shift;
    const int subs = 64 >> rc_shift;
    const int sub = lane >> rc_shift;
    const int c4 = ((int)blockIdx.z * RC + (lane & (RC - 1))) * 4;
    const bool col_ok = c4 < R;
    const int cc = col_ok ? c4 : 0;
    const int64_t p0 = (int64_t)blockIdx.y * per_split;
    const int64_t p1 = p0 + per_split < pairs ? p0 + per_split : pairs;
    const int workers = 4 * subs;
    const int64_t run = (p1 - p0 + workers - 1) / workers;
    const int64_t wk = wave * subs + sub;
    const int64_t q0 = p0 + wk * run < p1 ? p0 + wk * run : p1;
    const int64_t q1 = q0 + run < p1 ? q0 + run : p1;
    const int64_t J0 = kk.Z > 0 ? kk.J[0] : 1;
    const float *U0 = kk.Z > 0 ? kk.U[0] : nullptr;
    const f32x4 ones = {1.f, 1.f, 1.f, 1.f}, zeros = {0.f, 0.f, 0.f, 0.f};
    for (int64_t i = blockIdx.x; i < It; i += gridDim.x) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (q0 < q1) {
            const int64_t a = div64(q0, Ll);
            int64_t b = q0 - a * Ll;
            int64_t row = b + Ll * (i + It * a);
            int64_t d0 = kk.Z > 0 ? mod64(q0, J0) : 0;
            f32x4 slow = krp_slow_value4(kk, R, q0, cc);
            for (int64_t q = q0; q < q1; q += kLeafBatch) {
                int64_t rows[kLeafBatch];
                f32x4 ws[kLeafBatch];
#pragma unroll
                for (int u = 0; u < kLeafBatch; ++u) {
                    const bool ok = q + u < q1;
                    rows[u] = ok ? row : -1;
                    ws[u] = ok ? (kk.Z > 0 ? slow * *reinterpret_cast<const f32x4 *>(U0 + d0 * R + cc) : ones)
                               : zeros;
                    if (ok) {
                        ++row;
                        if (++b == Ll) {
                            b = 0;
                            row += Ll * (It - 1);
                        }
                        if (++d0 == J0) {
                            d0 = 0;
                            if (q + u + 1 < q1) slow = krp_slow_value4(kk, R, q + u + 1, cc);
                        }
                    }
                }
                f32x4 v[kLeafBatch];
#pragma unroll
                for (int u = 0; u < kLeafBatch; ++u)
                    v[u] = (col_ok && rows[u] >= 0) ? *reinterpret_cast<const f32x4 *>(Tm + rows[u] * R + c4)
                                                    : zeros;
#pragma unroll
                for (int u = 0; u < kLeafBatch; ++u)
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[e] += (double)v[u][e] * (double)ws[u][e];
            }
        }
        // the wave's sub-rows first (a butterfly over the lanes that hold the
        // same columns: a fixed pattern, so the sum is reproducible), then
        // the four waves in order
        for (int off = RC; off < 64; off <<= 1)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] += __shfl_xor(acc[e], off);
        if (lane < RC)
#pragma unroll
            for (int e = 0; e < 4; ++e) red[e][wave * 64 + lane] = acc[e];
        __syncthreads();
        if (tid < RC) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double s = ((red[e][tid] + red[e][64 + tid]) + red[e][128 + tid]) + red[e][192 + tid];
                const int oc = c4 + e;
                if (oc < R) out[((int64_t)blockIdx.y * It + i) * R + oc] = (float)s;
            }
        }
        __syncthreads();
    }
}

// Both MTTKRPs of a two-mode group from one pass over its intermediate.
// The rows of T are l = b + B * a (b the group's first mode, a its second):
//   M_b(b, c) = sum_a T(l, c) U_a(a, c),   M_a(a, c) = sum_b T(l, c) U_b(b, c).
// A wave covers 4 * RC rank columns with RC = 64 / WPW lanes of 4 columns
// each, so WPW workers share it.  A work-group takes kPairTB values of b
// and 4 * TA values of a (TA per wave); worker w of a wave takes
// b = b0 + w + WPW * j for j < kPairTB / WPW, so one load instruction reads
// WPW consecutive rows of T.  TA (a multiple of WPW, at most kPairTA) is
// the number of a values per wave: the host takes fewer when the grid would
// otherwise be too small to fill the chip.  (A compile-time TA matters: with
// the loop bound at run time the 512^2 x 32 pair took 15 us instead of 10.)  The loads of WPW values of a
// are issued together, then:
//   M_a: each worker adds its b products in j order; the wave's workers
//     then reduce-scatter the WPW rows (a butterfly that halves the rows
//     each lane keeps at every step: worker w ends with the sum of row w),
//     written to slice blockIdx.x of PA [gridDim.x][A][R];
//   M_b: each worker adds over its wave's a values in order; the four
//     waves are added in order through LDS and written to slice blockIdx.y
//     of PB [gridDim.y][B][R].
// All sums in float64 in a fixed order; k_sum_jobs adds the slices.  A
// grid dimension of 1 makes the slice the result itself.  Needs R a
// multiple of 4, R <= 4 * RC, 16-byte aligned T, factors and PA, and
// (A * B + kPairTB) * R * 4 below 2^32 (buffer offsets).
constexpr int kPairTA = 8;
constexpr int kPairTB = 16;
template <int WPW, int TA>
__global__ __launch_bounds__(kThreads) void k_pair_leaf(const float *__restrict__ Tm, int64_t A, int64_t B,
                                                        const float *__restrict__ Ua,
                                                        const float *__restrict__ Ub, int R,
                                                        float *__restrict__ PA, float *__restrict__ PB) {
    static_assert(TA % WPW == 0 && TA <= kPairTA, "a values per wave: whole chunks of WPW");
    constexpr int RC = 64 / WPW;
    constexpr int KB = kPairTB / WPW;
    __shared__ double red[4][kPairTB][4 * RC];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int w = lane / RC;
    const int c4 = 4 * (lane % RC);
    const bool col_ok = c4 < R;
    const int cc = col_ok ? c4 : 0;
    const int64_t b0 = (int64_t)blockIdx.x * kPairTB;
    const int64_t a0 = (int64_t)blockIdx.y * (4 * TA) + wave * TA;
    const f32x4 zeros = {0.f, 0.f, 0.f, 0.f};
    // T and U_a through buffer resources: a lane offset plus a wave-uniform
    // row offset.  T is read once, with the non-temporal hint (15 -> 10 us
    // for the 512^2 x 32 intermediate of the 512^3 tensor).  The host keeps every offset of T below 2^32; lanes past B
    // or R read a neighbouring row (or zeros past the end) and are masked.
    const rsrc_t rt = make_rsrc(Tm, (uint32_t)(A * B * R * 4));
    const rsrc_t ru = make_rsrc(Ua, (uint32_t)(A * R * 4));
    const uint32_t lane_off = (uint32_t)((w * R + c4) * 4);
    f32x4 ub[KB];
    bool bok[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        const int64_t b = b0 + w + WPW * j;
        bok[j] = col_ok && b < B;
        ub[j] = bok[j] ? *reinterpret_cast<const f32x4 *>(Ub + b * R + cc) : zeros;
    }
    double accb[KB][4];
#pragma unroll
    for (int j = 0; j < KB; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) accb[j][e] = 0.0;
    // one chunk of loads in flight per wave: the resident waves overlap them
#pragma unroll 1
    for (int ac = 0; ac < TA; ac += WPW) {
        f32x4 v[WPW][KB];
#pragma unroll
        for (int u = 0; u < WPW; ++u) {
            const int64_t a = a0 + ac + u;
#pragma unroll
            for (int j = 0; j < KB; ++j) {
                const uint32_t row_off = (uint32_t)(((a * B) + b0 + WPW * j) * R * 4);
                const f32x4 x = __builtin_bit_cast(
                    f32x4, __builtin_amdgcn_raw_buffer_load_b128(rt, lane_off, (int)row_off, kStream));
                v[u][j] = (a < A && bok[j]) ? x : zeros;
            }
        }
        double pa[WPW][4];
#pragma unroll
        for (int u = 0; u < WPW; ++u) {
            const int64_t a = a0 + ac + u;
            const f32x4 x = __builtin_bit_cast(
                f32x4, __builtin_amdgcn_raw_buffer_load_b128(ru, (uint32_t)(c4 * 4), (int)(uint32_t)(a * R * 4), 0));
            const f32x4 ua = (a < A && col_ok) ? x : zeros;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < KB; ++j) {
                    s += (double)v[u][j][e] * (double)ub[j][e];
                    accb[j][e] += (double)v[u][j][e] * (double)ua[e];
                }
                pa[u][e] = s;
            }
        }
        // reduce-scatter over the wave's workers: at the step of bit m a
        // lane keeps the half of its rows selected by bit m of w and adds
        // the partner's copy of that half
#pragma unroll
        for (int m = WPW / 2; m >= 1; m >>= 1) {
            const bool hi = (w & m) != 0;
#pragma unroll
            for (int i = 0; i < m; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double keep = hi ? pa[i + m][e] : pa[i][e];
                    const double send = hi ? pa[i][e] : pa[i + m][e];
                    pa[i][e] = keep + __shfl_xor(send, m * RC);
                }
        }
        const int64_t a = a0 + ac + w;
        if (a < A && col_ok) {
            const f32x4 o = {(float)pa[0][0], (float)pa[0][1], (float)pa[0][2], (float)pa[0][3]};
            *reinterpret_cast<f32x4 *>(PA + ((int64_t)blockIdx.x * A + a) * R + c4) = o;
        }
    }
#pragma unroll
    for (int j = 0; j < KB; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) red[wave][w + WPW * j][c4 + e] = accb[j][e];
    __syncthreads();
    for (int q = tid; q < kPairTB * R; q += kThreads) {
        const int bl = q / R, c = q % R;
        const int64_t b = b0 + bl;
        if (b < B)
            PB[((int64_t)blockIdx.y * B + b) * R + c] =
                (float)(((red[0][bl][c] + red[1][bl][c]) + red[2][bl][c]) + red[3][bl][c]);
    }
}

// Sums of partial slices for up to kSumJobs outputs in one launch (the
// slices of k_pair_leaf, and a pass's split-K partials when the pass writes
// a result): job j takes blocks [first[j], first[j + 1]), each 64
// consecutive entries e of M_j = sum over q < S_j of P_j[q * n_j + e].  The
// four waves of a block take interleaved slices and are added in wave
// order, in float64: the order of k_reduce's plain sums.
constexpr int kSumJobs = 4;
struct SumJobs {
    const float *P[kSumJobs];
    float *M[kSumJobs];
    int64_t S[kSumJobs], n[kSumJobs];
    int64_t first[kSumJobs + 1];
    int count;
};
__global__ __launch_bounds__(kThreads) void k_sum_jobs(SumJobs J) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int j = 0;
    while (j + 1 < J.count && (int64_t)blockIdx.x >= J.first[j + 1]) ++j;
    const float *P = J.P[j];
    const int64_t S = J.S[j], total = J.n[j];
    const int64_t e = ((int64_t)blockIdx.x - J.first[j]) * 64 + lane;
    double s = 0.0;
    if (e < total) {
#pragma unroll 4
        for (int64_t q = wave; q < S; q += 4) s += (double)P[q * total + e];
    }
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && e < total) J.M[j][e] = (float)(((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]);
}

}  // namespace cpm
