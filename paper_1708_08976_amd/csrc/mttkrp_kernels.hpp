// MTTKRP contraction kernels over the 3-index view of the tensor.
//
// For mode n let IL = prod_{k<n} I_k, In = I_n, IR = prod_{k>n} I_k.  The
// natural linearisation (Section 2.1) makes the tensor, without any
// movement, a stack of IR contiguous slabs X3[r], each an In x IL row-major
// matrix: entry (r, i, l) sits at offset l + i*IL + r*IL*In.  (These slabs
// are the row-major column blocks of X_(n) of Section 4.2.)  Then
//
//     M(i, c) = sum_r K_R(r, c) * sum_l X3[r][i][l] * K_L(l, c)
//
// with K_L = U_{n-1} kr ... kr U_0 and K_R = U_{N-1} kr ... kr U_{n+1}.
//
// Two tilings realise this sum; both read X exactly once, in its own layout:
//   * left-first (k_contract_left): for each slab, the partial MTTKRP
//     X3[r] * K_L on MFMA, then the multi-TTV with the right Khatri-Rao
//     product applied as a per-slab scaling of the output tile by K_R(r,:)
//     (the left-first 2-step scheme of Section 4.3, fused so the
//     intermediate never leaves registers).  Covers the last mode (IR = 1)
//     and internal modes.
//   * right-first (k_contract_right): X viewed as IR rows of length
//     J = In*IL, T = X * K_R on MFMA with the long dimension r contracted.
//     For mode 0 (IL = 1) T is M; for an internal mode with short IL the
//     multi-TTV against K_L runs in the reduction (the right-first 2-step
//     scheme of Section 4.3).
// Each work-group owns a contiguous share of the contracted index and writes
// a private partial result; k_reduce sums the partials in a fixed order (the
// private-buffer reduction of Algorithm 3), so results are reproducible.
#pragma once

#include "device_common.hpp"

namespace cpm {

// ---------------------------------------------------------------------------
// Left-first contraction.
//   grid.x = row tile, grid.y = split s (contiguous range of work units; a
//            unit is one l-chunk of one slab, units ordered slab-major),
//   grid.z = column block (16*NB columns starting at c0 = z*16*NB).
//   The 4 waves are arranged WI (row groups of 16*MB rows) x WL (waves that
//   share rows and interleave the 16-wide l-steps of each chunk).
// partial: [gridDim.y][In][R].
// ---------------------------------------------------------------------------
template <typename T, int NB, int MB, bool V4>
__global__ __launch_bounds__(kThreads) void k_contract_left(
    const T *__restrict__ X, int64_t IL, int64_t In, int64_t IR, Krp<T> kl, Krp<T> kr, int R,
    int LC, int WI, int64_t nlc, int64_t units_per_split, int64_t total_units,
    T *__restrict__ partial) {
    typedef typename Vec4<T>::type acc_t;
    constexpr int RP = NB * 16;
    constexpr int PITCH = RP + 4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kg = lane >> 4;
    const int WL = 4 / WI;
    const int wi = wave % WI, wl = wave / WI;
    const int c0 = blockIdx.z * RP;
    const int64_t TI = (int64_t)WI * 16 * MB;
    const int64_t row_base = (int64_t)blockIdx.x * TI + (int64_t)wi * 16 * MB;
    const int64_t u_begin = (int64_t)blockIdx.y * units_per_split;
    const int64_t u_end = min(total_units, u_begin + units_per_split);
    const bool single_chunk = (nlc == 1);
    const int tile_elems = LC * PITCH;

    acc_t acc[MB][NB], tot[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            acc[mb][nb] = acc_t{0, 0, 0, 0};
            tot[mb][nb] = acc_t{0, 0, 0, 0};
        }

    auto build = [&](int64_t u, int buf) {
        const int64_t l0 = (u % nlc) * (int64_t)LC;
        T *dst = tile + buf * tile_elems;
        build_krp_rows<T>(kl, R, c0, RP, l0, LC, IL, [&](int q, int c, T v) {
            dst[q * PITCH + c] = v;
        });
    };

    if (u_begin < u_end) build(u_begin, 0);
    __syncthreads();
    int buf = 0;
    for (int64_t u = u_begin; u < u_end; ++u) {
        const int64_t r = u / nlc, lc = u % nlc;
        if (!single_chunk && u + 1 < u_end) build(u + 1, buf ^ 1);
        const T *K = tile + buf * tile_elems;
        const int64_t l0 = lc * (int64_t)LC;
        const int64_t lend = min(IL, l0 + (int64_t)LC);
        const int nsteps = (int)((lend - l0 + 15) / 16);
        const T *xr[MB];
        bool rok[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int64_t row = row_base + 16 * mb + m;
            rok[mb] = row < In;
            xr[mb] = X + ((r * In + (rok[mb] ? row : 0)) * IL);
        }
        for (int st = wl; st < nsteps; st += WL) {
            const int64_t lb = l0 + (int64_t)st * 16 + 4 * kg;
            T a[MB][4];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                if (V4) {
                    if (rok[mb] && lb < lend) {
                        const acc_t v = *reinterpret_cast<const acc_t *>(xr[mb] + lb);
                        a[mb][0] = v[0]; a[mb][1] = v[1]; a[mb][2] = v[2]; a[mb][3] = v[3];
                    } else {
                        a[mb][0] = a[mb][1] = a[mb][2] = a[mb][3] = T(0);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        a[mb][e] = (rok[mb] && lb + e < lend) ? xr[mb][lb + e] : T(0);
                }
            }
            const int qb = st * 16 + 4 * kg;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                T b[NB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) b[nb] = K[(qb + t) * PITCH + 16 * nb + m];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[mb][nb] = mfma4(a[mb][t], b[nb], acc[mb][nb]);
            }
        }
        const bool slab_end = (lc == nlc - 1) || (u + 1 == u_end);
        // (a right product exists whenever mode n is not the last mode, even
        // if every mode to the right has size 1)
        if (kr.Z > 0 && slab_end) {
            // multi-TTV with the right Khatri-Rao product: scale this slab's
            // partial MTTKRP by K_R(r, c) for the lane's columns.
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int c = c0 + 16 * nb + m;
                const T kv = (c < R) ? krp_value(kr, R, r, c) : T(0);
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    tot[mb][nb] += acc[mb][nb] * kv;
                    acc[mb][nb] = acc_t{0, 0, 0, 0};
                }
            }
        }
        if (!single_chunk) {
            __syncthreads();
            buf ^= 1;
        }
    }
    if (kr.Z == 0) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) tot[mb][nb] = acc[mb][nb];
    }

    // Sum the WL waves that share rows, in wave order, and store the partial.
    __syncthreads();
    T *red = tile;  // [wave][mb][nb][j][lane]
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                red[(((wave * MB + mb) * NB + nb) * 4 + j) * 64 + lane] = tot[mb][nb][j];
    __syncthreads();
    const int per_wi = MB * NB * 4 * 64;
    for (int e = tid; e < WI * per_wi; e += kThreads) {
        const int wi2 = e / per_wi, rem = e % per_wi;
        const int ln = rem & 63, j = (rem >> 6) & 3, blk = rem >> 8;
        const int nb = blk % NB, mb = blk / NB;
        T s = T(0);
        for (int w2 = 0; w2 < WL; ++w2) {
            const int wave2 = w2 * WI + wi2;
            s += red[(((wave2 * MB + mb) * NB + nb) * 4 + j) * 64 + ln];
        }
        const int64_t row = (int64_t)blockIdx.x * TI + (int64_t)wi2 * 16 * MB + 16 * mb + acc_row<T>(ln, j);
        const int c = c0 + 16 * nb + (ln & 15);
        if (row < In && c < R) partial[((int64_t)blockIdx.y * In + row) * R + c] = s;
    }
}

// ---------------------------------------------------------------------------
// Right-first contraction over the slow index r of X viewed as [IR][J].
//   grid.x = tile of 64*MJ entries of J, grid.y = split s (rows
//   [s*rows_per_split, ...)), grid.z = rank-column block.  The 4 waves interleave
//   the 4-row k-steps of each chunk of RC rows of K_R.
// Lane (m, kg) loads 4 consecutive j at 4m + 64g; component e feeds m-block
// 4g + e, so output row j = jt0 + 64g + 4*m' + e for accumulator row m'.
// partial: [gridDim.y][J][R].
// ---------------------------------------------------------------------------
template <typename T, int NB, int MJ, bool V4>
__global__ __launch_bounds__(kThreads) void k_contract_right(
    const T *__restrict__ X, int64_t J, int64_t IR, Krp<T> kr, int R, int RC,
    int64_t rows_per_split, T *__restrict__ partial) {
    typedef typename Vec4<T>::type acc_t;
    constexpr int RP = NB * 16;
    constexpr int PITCH = RP + 16;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kg = lane >> 4;
    const int c0 = blockIdx.z * RP;
    const int64_t jt0 = (int64_t)blockIdx.x * 64 * MJ;
    const int64_t r_begin = (int64_t)blockIdx.y * rows_per_split;
    const int64_t r_end = min(IR, r_begin + rows_per_split);
    const int tile_elems = RC * PITCH;

    acc_t acc[MJ][4][NB];
#pragma unroll
    for (int g = 0; g < MJ; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[g][e][nb] = acc_t{0, 0, 0, 0};

    auto build = [&](int64_t rc0, int buf) {
        T *dst = tile + buf * tile_elems;
        build_krp_rows<T>(kr, R, c0, RP, rc0, RC, r_end, [&](int q, int c, T v) {
            dst[q * PITCH + c] = v;
        });
    };

    bool jok[MJ];
    const T *xc[MJ];
#pragma unroll
    for (int g = 0; g < MJ; ++g) {
        const int64_t j = jt0 + 64 * g + 4 * m;
        jok[g] = j < J;
        xc[g] = X + (jok[g] ? j : 0);
    }

    if (r_begin < r_end) build(r_begin, 0);
    __syncthreads();
    int buf = 0;
    for (int64_t rc0 = r_begin; rc0 < r_end; rc0 += RC) {
        if (rc0 + RC < r_end) build(rc0 + RC, buf ^ 1);
        const T *K = tile + buf * tile_elems;
        const int nsteps = (int)((min((int64_t)RC, r_end - rc0) + 3) / 4);
        for (int st = wave; st < nsteps; st += 4) {
            const int64_t rk = rc0 + (int64_t)st * 4 + kg;
            const bool rrow = rk < r_end;
            T a[MJ][4];
#pragma unroll
            for (int g = 0; g < MJ; ++g) {
                const T *p = xc[g] + rk * J;
                if (V4) {
                    if (rrow && jok[g]) {
                        const acc_t v = *reinterpret_cast<const acc_t *>(p);
                        a[g][0] = v[0]; a[g][1] = v[1]; a[g][2] = v[2]; a[g][3] = v[3];
                    } else {
                        a[g][0] = a[g][1] = a[g][2] = a[g][3] = T(0);
                    }
                } else {
                    const int64_t j = jt0 + 64 * g + 4 * m;
#pragma unroll
                    for (int e = 0; e < 4; ++e) a[g][e] = (rrow && j + e < J) ? p[e] : T(0);
                }
            }
            T b[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) b[nb] = K[(st * 4 + kg) * PITCH + 16 * nb + m];
#pragma unroll
            for (int g = 0; g < MJ; ++g)
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) acc[g][e][nb] = mfma4(a[g][e], b[nb], acc[g][e][nb]);
        }
        __syncthreads();
        buf ^= 1;
    }

    // Sum the 4 waves in order and store the partial.
    T *red = tile;  // [wave][g][e][nb][jj][lane]
    const int per_wave = MJ * 4 * NB * 4 * 64;
#pragma unroll
    for (int g = 0; g < MJ; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    red[wave * per_wave + (((g * 4 + e) * NB + nb) * 4 + jj) * 64 + lane] = acc[g][e][nb][jj];
    __syncthreads();
    for (int q = tid; q < per_wave; q += kThreads) {
        const int ln = q & 63, jj = (q >> 6) & 3, blk = q >> 8;
        const int nb = blk % NB, ge = blk / NB, e = ge % 4, g = ge / 4;
        T s = red[q] + red[per_wave + q] + red[2 * per_wave + q] + red[3 * per_wave + q];
        const int64_t j = jt0 + 64 * g + 4 * acc_row<T>(ln, jj) + e;
        const int c = c0 + 16 * nb + (ln & 15);
        if (j < J && c < R) partial[((int64_t)blockIdx.y * J + j) * R + c] = s;
    }
}

// ---------------------------------------------------------------------------
// Fixed-order reduction of the split partials, accumulated in float64:
//   out(i, c) = sum_s sum_l K_L(l, c) * partial[s][i*IL + l][c]
// With kl.Z == 0 this is the plain split-K sum (IL must then be 1); with
// kl.Z > 0 it also applies the multi-TTV of the right-first scheme (IL may
// be 1 when every mode to the left has size 1: K_L is then one factor row).
// Each block owns 64 consecutive outputs; its 4 waves take interleaved
// terms and are summed in wave order.
// ---------------------------------------------------------------------------
template <typename T, typename TOut>
__global__ __launch_bounds__(kThreads) void k_reduce(const T *__restrict__ partial, int64_t S,
                                                     int64_t rows_per_slice, int64_t In, int64_t IL,
                                                     Krp<T> kl, int R, TOut *__restrict__ out) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t e = (int64_t)blockIdx.x * 64 + lane;
    const int64_t total = In * R;
    double s = 0.0;
    if (e < total) {
        const int64_t i = e / R;
        const int c = (int)(e % R);
        if (kl.Z == 0) {
            const T *p = partial + i * R + c;
            const int64_t step = rows_per_slice * R;
#pragma unroll 8
            for (int64_t q = wave; q < S; q += 4) s += (double)p[q * step];
        } else {
            const int64_t terms = S * IL;
            for (int64_t q = wave; q < terms; q += 4) {
                const int64_t sl = q / IL, l = q % IL;
                const double v = (double)partial[(sl * rows_per_slice + i * IL + l) * R + c];
                s += v * (double)krp_value(kl, R, l, c);
            }
        }
    }
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && e < total) out[e] = (TOut)(((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]);
}

}  // namespace cpm
