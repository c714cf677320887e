// Device-side building blocks shared by the cpmttkrp kernels: the Khatri-Rao
// row descriptor, the on-the-fly row builder, MFMA wrappers and bf16 helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cpmttkrp.h"

namespace cpm {

constexpr int kMaxModes = CPM_MAX_MODES;
constexpr int kThreads = 256;  // every tiled kernel runs 4 waves of 64

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef f32x4 type; };
template <> struct Vec4<double> { typedef f64x4 type; };

// ---------------------------------------------------------------------------
// Khatri-Rao product of Z factor matrices, described fastest-index first:
// row g has multi-index (g_0, ..., g_{Z-1}) with g = sum_z g_z * stride[z],
// stride[0] = 1, and value K(g, c) = prod_z U[z][g_z * R + c].
//
// With the factors of the modes left of n listed as U_0, U_1, ..., U_{n-1}
// this is K_L = U_{n-1} kr ... kr U_0 (mode 0 fastest, as the row-wise
// definition of Section 2.1 puts the last operand's index fastest); with
// U_{n+1}, ..., U_{N-1} it is K_R = U_{N-1} kr ... kr U_{n+1}.  Z = 0 is the
// empty product: a row of ones.
// ---------------------------------------------------------------------------
template <typename T> struct Krp {
    int Z;
    int64_t rows;                 // prod_z J[z] (1 when Z == 0)
    int64_t J[kMaxModes];
    int64_t stride[kMaxModes];
    const T *U[kMaxModes];
};

// K(g, c) from scratch: one Hadamard product over all Z factors.
template <typename T>
__device__ inline T krp_value(const Krp<T> &k, int R, int64_t g, int c) {
    T v = T(1);
    for (int z = 0; z < k.Z; ++z) {
        int64_t gz = (g / k.stride[z]) % k.J[z];
        v *= k.U[z][gz * R + c];
    }
    return v;
}

// Product of all factors except the fastest one (the partial Hadamard
// product that Algorithm 1 keeps while the fastest index runs).
template <typename T>
__device__ inline T krp_slow_part(const Krp<T> &k, int R, int64_t g, int c) {
    T v = T(1);
    for (int z = 1; z < k.Z; ++z) {
        int64_t gz = (g / k.stride[z]) % k.J[z];
        v *= k.U[z][gz * R + c];
    }
    return v;
}

// Rows [row0, row0 + nrows) of K, columns [coff, coff + RP), written through
// store(q, c, value) with q the row offset in the tile and c relative to
// coff.  R is the factors' row stride; rows at or past row_limit and
// columns at or past R are written as zero.
//
// Work split: thread t owns column c = t % RP and a contiguous run of rows,
// and walks it like Algorithm 1 (Section 4.1): the product of the slower
// factors is held in a register and refreshed only when the fastest index
// wraps, so each row costs one multiply by a row of the fastest factor.
// Each thread starts its run by decoding its own first row, as in the
// parallel variant of that algorithm.
template <typename T, typename Store>
__device__ inline void build_krp_rows(const Krp<T> &k, int R, int coff, int RP, int64_t row0,
                                      int nrows, int64_t row_limit, Store store) {
    const int t = threadIdx.x;
    if (RP > kThreads) return;  // host never launches this
    const int groups = kThreads / RP;
    const int cl = t % RP;
    const int c = coff + cl;
    const int g = t / RP;
    if (g >= groups) return;
    const int run = (nrows + groups - 1) / groups;
    const int q0 = g * run;
    const int q1 = min(nrows, q0 + run);
    if (q0 >= q1) return;
    const int64_t lim = min(row_limit, k.rows);
    const bool col_ok = c < R;
    if (k.Z == 0) {
        for (int q = q0; q < q1; ++q)
            store(q, cl, (col_ok && row0 + q < lim) ? T(1) : T(0));
        return;
    }
    const T *__restrict__ U0 = k.U[0];
    const int64_t J0 = k.J[0];
    int64_t grow = row0 + q0;
    int64_t i0 = grow % J0;
    T slow = (col_ok && grow < lim) ? krp_slow_part(k, R, grow, c) : T(0);
    for (int q = q0; q < q1; ++q, ++grow) {
        T v = T(0);
        if (col_ok && grow < lim) v = slow * U0[i0 * R + c];
        store(q, cl, v);
        if (++i0 == J0) {
            i0 = 0;
            if (col_ok && grow + 1 < lim) slow = krp_slow_part(k, R, grow + 1, c);
        }
    }
}

// ---------------------------------------------------------------------------
// MFMA wrappers.  16x16x4 (f32, f64): lane l holds A[l%16][l/16] and
// B[l/16][l%16].  Accumulator element j (0..3) of lane l holds
// D[acc_row<T>(l, j)][l%16]: row 4*(l/16)+j for f32 but 4*j+l/16 for f64
// (measured on gfx950).  16x16x32 bf16: lane l holds A[l%16][8*(l/16)+e]
// and B[8*(l/16)+e][l%16] for e = 0..7, accumulator as for f32.
// ---------------------------------------------------------------------------
template <typename T> __device__ inline int acc_row(int lane, int j);
template <> __device__ inline int acc_row<float>(int lane, int j) { return 4 * (lane >> 4) + j; }
template <> __device__ inline int acc_row<double>(int lane, int j) { return 4 * j + (lane >> 4); }

__device__ inline f32x4 mfma4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f64x4 mfma4(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Round-to-nearest-even float -> bfloat16 bit pattern (finite inputs; NaN is
// kept a quiet NaN).
__device__ inline uint16_t bf16_rne_bits(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_bits_to_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

}  // namespace cpm
