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
// Buffer loads.  A buffer resource holds a base address and a byte range; a
// load whose byte offset falls outside the range returns zero instead of
// touching memory.  The kernels give a lane with nothing to load the offset
// kNoLoad, so every load is issued unconditionally (no branch around it) and
// inactive lanes read zeros.  Offsets are unsigned 32-bit: callers keep
// every live offset below kRsrcRange.
// ---------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr uint32_t kRsrcRange = 0xFFFFFF00u;
constexpr uint32_t kNoLoad = 0xFFFFFFF0u;
// dword 3 of the resource: 32-bit data format, raw (untyped) access
constexpr int kRsrcWord3 = 0x00020000;

// Cache policy of a buffer load: bit 1 of the policy operand is the
// non-temporal hint.  On MI355X a plain 512 MiB read in 16-byte loads ran at
// about 6.0 TB/s without it and 6.9 TB/s with it.  It is set where it
// measured faster: the 16- and 8-byte tensor loads of the float32
// right-first kernel (the 512^3 passes 7-14% faster) and the fused
// residual's tensor loads (141 -> 131 us at 512^3).  The left-first kernels
// (128-byte row segments in 16-byte loads), the 4-byte loads of rows that
// are not 16-byte aligned and the split-bf16 planes were as fast or slower
// with it (down to half the rate on 225 x 59 x 200 x 200).
constexpr int kStream = 2;

__device__ inline rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kRsrcWord3);
}
template <int AUX = 0>
__device__ inline float buf_load1(rsrc_t r, uint32_t off, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX));
}
template <int AUX = 0>
__device__ inline double buf_load1(rsrc_t r, uint32_t off, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX));
}
template <int AUX = 0>
__device__ inline f32x4 buf_load4(rsrc_t r, uint32_t off, float) {
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX));
}
template <int AUX = 0>
__device__ inline f64x4 buf_load4(rsrc_t r, uint32_t off, double) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 lo = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX));
    const d2 hi = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, off == kNoLoad ? kNoLoad : off + 16, 0, AUX));
    return f64x4{lo[0], lo[1], hi[0], hi[1]};
}

// a / b and a % b for non-negative 64-bit values, in 32-bit arithmetic when
// both fit (the common case, and far cheaper on the GPU).
__device__ inline int64_t div64(int64_t a, int64_t b) {
    if (((a | b) >> 31) == 0) return (int64_t)((uint32_t)a / (uint32_t)b);
    return a / b;
}
__device__ inline int64_t mod64(int64_t a, int64_t b) {
    if (((a | b) >> 31) == 0) return (int64_t)((uint32_t)a % (uint32_t)b);
    return a % b;
}

// One-time tile build for the streaming kernels: rows [row0, row0 + nrows)
// of K, columns [coff, coff + RP), written through store(q, c, v) (zero past
// row_limit and past column R).  Thread t owns column t % RP and consecutive
// runs of PR rows; for each run it decodes the first row once, steps the
// multi-index with carries (the row order of Algorithm 1), and issues all of
// the run's factor loads before multiplying, so a run costs about one memory
// latency rather than one per row.  Products of more than kCursorZ factors
// decode every row instead.
template <typename T, int RP, int PR, typename Store>
__device__ inline void build_tile_batched(const Krp<T> &k, int R, int coff, int64_t row0, int nrows,
                                          int64_t row_limit, Store store) {
    constexpr int ZM = 4;
    const int t = threadIdx.x;
    const int cl = t % RP;
    const int c = coff + cl;
    const int groups = kThreads / RP;
    const int64_t lim = min(row_limit, k.rows);
    const bool col_ok = c < R;
    for (int base = (t / RP) * PR; base < nrows; base += groups * PR) {
        T v[PR];
        if (k.Z == 0) {
#pragma unroll
            for (int i = 0; i < PR; ++i) v[i] = (col_ok && row0 + base + i < lim) ? T(1) : T(0);
        } else if (k.Z <= ZM) {
            int64_t d[ZM];
            const int64_t g0 = row0 + base;
#pragma unroll
            for (int z = 0; z < ZM; ++z) d[z] = (z < k.Z) ? mod64(div64(g0, k.stride[z]), k.J[z]) : 0;
            T f[PR][ZM];
#pragma unroll
            for (int i = 0; i < PR; ++i) {
                const bool ok = col_ok && base + i < nrows && g0 + i < lim;
#pragma unroll
                for (int z = 0; z < ZM; ++z) {
                    f[i][z] = T(1);
                    if (z < k.Z) {
                        const rsrc_t rz = make_rsrc(k.U[z], (uint32_t)(k.J[z] * R * (int64_t)sizeof(T)));
                        const uint32_t off = ok ? (uint32_t)((d[z] * R + c) * (int64_t)sizeof(T)) : kNoLoad;
                        f[i][z] = buf_load1(rz, off, T(0));
                    }
                }
                // next row: carry through the digits
                bool carry = true;
#pragma unroll
                for (int z = 0; z < ZM; ++z) {
                    if (carry && z < k.Z) {
                        if (++d[z] < k.J[z]) carry = false;
                        else d[z] = 0;
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < PR; ++i) {
                T p = f[i][0];
#pragma unroll
                for (int z = 1; z < ZM; ++z)
                    if (z < k.Z) p *= f[i][z];
                v[i] = p;
            }
        } else {
#pragma unroll
            for (int i = 0; i < PR; ++i) {
                const int64_t g = row0 + base + i;
                v[i] = (col_ok && base + i < nrows && g < lim) ? krp_value(k, R, g, c) : T(0);
            }
        }
#pragma unroll
        for (int i = 0; i < PR; ++i)
            if (base + i < nrows) store(base + i, cl, v[i]);
    }
}

// Multi-index of one row of a Khatri-Rao product, advanced one row at a time
// with carries (no division after the first decode).  Digit z is the row of
// factor z (fastest first).  Only the first kCursorZ factors are tracked
// incrementally; products of more factors fall back to decoding.
constexpr int kCursorZ = 4;
template <typename T>
struct KrpCursor {
    int64_t g;                 // row of the product
    int64_t d[kCursorZ];       // digits of the first kCursorZ factors

    __device__ inline void set(const Krp<T> &k, int64_t row) {
        g = row;
#pragma unroll
        for (int z = 0; z < kCursorZ; ++z) d[z] = (z < k.Z) ? mod64(div64(row, k.stride[z]), k.J[z]) : 0;
    }
    __device__ inline void next(const Krp<T> &k) {
        ++g;
#pragma unroll
        for (int z = 0; z < kCursorZ; ++z) {
            if (z >= k.Z) break;
            if (++d[z] < k.J[z]) return;
            d[z] = 0;
        }
    }
};

// Raw factor values of one row of a Khatri-Rao product for NB lane columns
// (cbase, cbase + CS, ...), fetched ahead of use (first ZS factors) and
// multiplied when needed.  The row index is the same in every lane, so the
// index arithmetic is scalar; the loads are unconditional buffer loads (a
// column past R reads zero).
template <typename T, int NB, int CS = 16>
struct KrpRowVals {
    static constexpr int ZS = kCursorZ;
    T f[NB][ZS];
    int64_t g;

    __device__ inline void fetch(const Krp<T> &k, int R, int cbase, const KrpCursor<T> &cur) {
        g = cur.g;
#pragma unroll
        for (int z = 0; z < ZS; ++z) {
            const int zz = z < k.Z ? z : 0;  // k.Z >= 1 whenever this is used
            const rsrc_t rs = make_rsrc(k.U[zz], (uint32_t)(k.J[zz] * R * (int64_t)sizeof(T)));
            const int64_t rowz = (z < k.Z) ? cur.d[z] : 0;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int c = cbase + CS * nb;
                const uint32_t off = (c < R) ? (uint32_t)((rowz * R + c) * (int64_t)sizeof(T)) : kNoLoad;
                f[nb][z] = buf_load1(rs, off, T(0));  // not touched until value(): no wait here
            }
        }
    }
    __device__ inline T value(const Krp<T> &k, int R, int cbase, int nb) const {
        const int c = cbase + CS * nb;
        if (c >= R) return T(0);
        T v = f[nb][0];
#pragma unroll
        for (int z = 1; z < ZS; ++z)
            if (z < k.Z) v *= f[nb][z];
        for (int z = ZS; z < k.Z; ++z) v *= k.U[z][mod64(div64(g, k.stride[z]), k.J[z]) * R + c];
        return v;
    }
};

// Outer scales S(o, c) of up to scale_blocks<RP>() consecutive blocks, for
// the work-group's RP rank columns, held in LDS ([block][RP], 6 KB).  The
// stream runs in chunks of that many blocks; the table is refilled between
// chunks (a barrier and one round of factor loads), outside the unrolled
// step loop.  Reading a scale in the stream is an LDS access, so it never
// waits on the in-order completion counter of the X loads in flight.  The
// chunk length is a multiple of the register rings of the streaming kernels
// (3 and 6), so every chunk starts on ring slot 0.
constexpr int kScaleTableBytes = 6144;
template <int RP>
__host__ __device__ constexpr int scale_blocks() {
    return kScaleTableBytes / 4 / RP;
}
static_assert(scale_blocks<128>() % 6 == 0 && scale_blocks<16>() % 6 == 0, "chunk must align with the rings");
template <int RP>
__device__ inline void fill_scales(const Krp<float> &kout, int R, int c0, int64_t ob, int64_t o_end, float *stab) {
    constexpr int NBLK = scale_blocks<RP>();
    if (kout.Z == 0) {
        for (int e = threadIdx.x; e < NBLK * RP; e += kThreads) stab[e] = 1.f;
        return;
    }
    build_tile_batched<float, RP, (NBLK * RP >= 8 * kThreads ? 8 : 4)>(
        kout, R, c0, ob, NBLK, o_end, [&](int q, int c, float v) { stab[q * RP + c] = v; });
}

// ---------------------------------------------------------------------------
// MFMA wrappers.  16x16x4 (f32, f64): lane l holds A[l%16][l/16] and
// B[l/16][l%16].  Accumulator element j (0..3) of lane l holds
// D[acc_row<T>(l, j)][l%16]: row 4*(l/16)+j for f32 but 4*j+l/16 for f64
// (measured on gfx950).  16x16x32 bf16: lane l holds A[l%16][8*(l/16)+e]
// and B[8*(l/16)+e][l%16] for e = 0..7, accumulator as for f32.
// ---------------------------------------------------------------------------
// 32x32x2 f32: lane l holds A[l%32][l/32] and B[l/32][l%32]; accumulator
// element j (0..15) of lane l holds D[acc32_row(l, j)][l%32].
typedef float f32x16 __attribute__((ext_vector_type(16)));
__device__ inline f32x16 mfma32(float a, float b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ inline int acc32_row(int lane, int j) { return 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3); }

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
