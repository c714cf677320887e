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
// Shared structure of both contraction kernels.
//
// The contracted Khatri-Rao product of each kernel is split into an inner
// part over the fastest modes of that side and an outer part over the rest:
// K(g_in + G_in * o, c) = K_in(g_in, c) * S(o, c).  (For K_L this is
// Algorithm 1's observation that the partial Hadamard product of the slow
// factors stays fixed while the fast indices run.)  A work-group keeps one
// tile of K_in -- a fixed chunk of its rows, for a fixed block of rank
// columns -- in LDS for its whole life, and streams X block by block over
// the outer index o: each block is contracted against the tile on MFMA, and
// at the block's end the block result is scaled by S(o, :) and added to the
// running total.  That scaling is the multi-TTV of the 2-step scheme; for
// the left-first kernel it carries both the slow left modes and every right
// mode.  No tile is rebuilt and no barrier is taken inside the stream.
//
// Each wave streams "steps" of 16 contracted indices (4 MFMA k-steps of 4)
// and keeps two steps of X in flight in registers ahead of the one it
// multiplies (a ring of three register sets used in rotation).
// ---------------------------------------------------------------------------

// Per-block scale S(o, c) for the lane's NB columns: the factor values of
// the block after the current one are loaded at the current block's end and
// multiplied only when that block ends, so the loads never stall the stream.
template <typename T, int NB>
struct BlockScale {
    KrpRowVals<T, NB> next;
    KrpCursor<T> cur;  // outer index of the block whose values are in flight
    __device__ inline void start(const Krp<T> &k, int R, int cbase, int64_t o) {
        cur.set(k, o);
        next.fetch(k, R, cbase, cur);
    }
    __device__ inline void advance(const Krp<T> &k, int R, int cbase) {
        cur.next(k);
        next.fetch(k, R, cbase, cur);
    }
    __device__ inline T value(const Krp<T> &k, int R, int cbase, int nb) const {
        return next.value(k, R, cbase, nb);
    }
};

// ---------------------------------------------------------------------------
// Left-first contraction (internal and last modes).
// X is viewed as X[r][i][h][l_in]: l_in over the inner left modes (IL_in
// entries, contiguous), h over the outer left modes, i = i_n, r over the
// right modes; row (i, h, r) starts at l_in = 0 and rows of consecutive i
// are IL = IL_in * IL_out apart.  The outer block o = h + IL_out * r.
//   grid.x = row tile of 16*MB rows of i
//   grid.y = lc + nlc * s: inner chunk lc of LC = 64*SPB entries of l_in,
//            split s = a contiguous range of blocks_per_split outer blocks
//   grid.z = column block (16*NB columns from c0 = z*16*NB)
// A step covers 16*Q entries of every row: lane (m, kg) loads Q groups of 4
// consecutive entries at 16q + 4kg, so one row receives Q*64 contiguous
// bytes per step (whole cache lines for Q >= 2), and MFMA k-step (q, t)
// pairs slot kg with entry 16q + 4kg + t.  Wave w owns entries
// [w*16*Q*SPB, (w+1)*16*Q*SPB) of the chunk (LC = 64*Q*SPB) for all rows.
// partial: [gridDim.y][In][R].
// ---------------------------------------------------------------------------
template <typename T, int NB, int MB, bool V4, int Q = 1, int RING = 3>
__global__ __launch_bounds__(kThreads) void k_contract_left(
    const T *__restrict__ X, int64_t IL_in, int64_t IL_out, int64_t In, int64_t n_outer, Krp<T> kin,
    Krp<T> kout, int R, int SPB, int64_t nlc, int64_t blocks_per_split, T *__restrict__ partial) {
    typedef typename Vec4<T>::type acc_t;
    constexpr int RP = NB * 16;
    constexpr int PITCH = RP + 4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kg = lane >> 4;
    const int c0 = blockIdx.z * RP;
    const int WS = 16 * Q;                            // entries per row per step
    const int LC = 4 * WS * SPB;
    const int64_t lc = blockIdx.y % nlc;
    const int64_t split = blockIdx.y / nlc;
    const int64_t l0 = lc * LC;                       // first inner entry of the chunk
    const int64_t lend = min(IL_in, l0 + LC);         // one past the last
    const int64_t IL = IL_in * IL_out;
    const int64_t row_base = (int64_t)blockIdx.x * 16 * MB;
    const int64_t o_begin = split * blocks_per_split;
    const int64_t o_end = min(n_outer, o_begin + blocks_per_split);
    const bool has_out = kout.Z > 0;


    acc_t acc[MB][NB], tot[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            acc[mb][nb] = acc_t{0, 0, 0, 0};
            tot[mb][nb] = acc_t{0, 0, 0, 0};
        }
    int64_t rowoff[MB];
    bool rok[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const int64_t row = row_base + 16 * mb + m;
        rok[mb] = row < In;
        rowoff[mb] = (rok[mb] ? row : 0) * IL;
    }
    const int64_t lane_l = l0 + wave * WS * SPB + 4 * kg;  // this lane's entries: + WS*s + 16*q + e

    // Block o = h + IL_out * r starts at X + r*In*IL + h*IL_in; the load
    // cursor walks (h, r) with a carry instead of dividing.
    int64_t cur_r = o_begin / IL_out, cur_h = o_begin - (o_begin / IL_out) * IL_out;
    auto block_base = [&]() -> const T * { return X + cur_r * In * IL + cur_h * IL_in; };

    // load cursor
    int64_t lo = o_begin;
    int ls = 0;
    // X loads: one buffer resource per m-block, based at the m-block's first
    // row in the current block, so lane offsets are (m * IL + l) entries;
    // rows past In, entries past the chunk and blocks past the split get
    // kNoLoad and read zeros.  No load sits behind a branch, which lets the
    // compiler wait for exactly the step being multiplied.
    rsrc_t rs[MB];
    auto set_block = [&]() {
        const T *b = block_base();
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) rs[mb] = make_rsrc(b + (row_base + 16 * mb) * IL, kRsrcRange);
    };
    set_block();
    const uint32_t lane_row = (uint32_t)(m * IL);
    auto load_step = [&](T (&a)[MB][Q][4]) {
        const bool live = lo < o_end;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int64_t l = lane_l + WS * ls + 16 * q;
                if (V4) {
                    const bool ok = live && rok[mb] && l < lend;
                    const uint32_t off = ok ? (uint32_t)((lane_row + l) * sizeof(T)) : kNoLoad;
                    const acc_t v = buf_load4(rs[mb], off, T(0));
                    a[mb][q][0] = v[0]; a[mb][q][1] = v[1]; a[mb][q][2] = v[2]; a[mb][q][3] = v[3];
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const bool ok = live && rok[mb] && l + e < lend;
                        const uint32_t off = ok ? (uint32_t)((lane_row + l + e) * sizeof(T)) : kNoLoad;
                        a[mb][q][e] = buf_load1(rs[mb], off, T(0));
                    }
                }
            }
        if (++ls == SPB) {
            ls = 0;
            ++lo;
            if (++cur_h == IL_out) {
                cur_h = 0;
                ++cur_r;
            }
            set_block();
        }
    };

    // Start streaming X, then build this work-group's chunk of K_in once
    // (rows past IL_in and columns past R are zero) while those loads fly.
    T x[RING][MB][Q][4];
#pragma unroll
    for (int k = 0; k < RING - 1; ++k) load_step(x[k]);
    build_tile_batched<T, RP, 16>(kin, R, c0, l0, LC, IL_in, [&](int q, int c, T v) { tile[q * PITCH + c] = v; });

    // compute cursor
    int64_t co = o_begin;
    int cs = 0;
    BlockScale<T, NB> sc;
    if (has_out && o_begin < o_end) sc.start(kout, R, c0 + m, o_begin);
    __syncthreads();  // tile ready
    auto compute_step = [&](const T (&a)[MB][Q][4]) {
        const T *kb = tile + (wave * WS * SPB + WS * cs + 4 * kg) * PITCH + m;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            T b[4][NB];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) b[t][nb] = kb[(16 * q + t) * PITCH + 16 * nb];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mfma4(a[mb][q][t], b[t][nb], acc[mb][nb]);
        }
        if (++cs == SPB) {
            cs = 0;
            if (has_out) {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const T s = sc.value(kout, R, c0 + m, nb);
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb) {
                        tot[mb][nb] += acc[mb][nb] * s;
                        acc[mb][nb] = acc_t{0, 0, 0, 0};
                    }
                }
                if (co + 1 < o_end) sc.advance(kout, R, c0 + m);
            }
            ++co;
        }
    };

    // Ring of RING register sets: RING - 1 steps in flight ahead of the one
    // being multiplied (slot indices are compile-time after unrolling).
    const int64_t nsteps = (o_end > o_begin ? o_end - o_begin : 0) * SPB;
    int64_t st = 0;
    for (; st + RING <= nsteps; st += RING) {
#pragma unroll
        for (int k = 0; k < RING; ++k) {
            load_step(x[(k + RING - 1) % RING]);
            compute_step(x[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < RING - 1; ++k)
        if (st + k < nsteps) compute_step(x[k]);
    if (!has_out) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) tot[mb][nb] = acc[mb][nb];
    }

    // Sum the 4 waves (which share rows) in wave order and store the partial.
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
    constexpr int PER_WAVE = MB * NB * 4 * 64;
    for (int e = tid; e < PER_WAVE; e += kThreads) {
        const int ln = e & 63, j = (e >> 6) & 3, blk = e >> 8;
        const int nb = blk % NB, mb = blk / NB;
        const T sum = ((red[e] + red[PER_WAVE + e]) + red[2 * PER_WAVE + e]) + red[3 * PER_WAVE + e];
        const int64_t row = row_base + 16 * mb + acc_row<T>(ln, j);
        const int c = c0 + 16 * nb + (ln & 15);
        if (row < In && c < R) partial[((int64_t)blockIdx.y * In + row) * R + c] = sum;
    }
}

// ---------------------------------------------------------------------------
// Right-first contraction (mode 0, and internal modes with a short left
// product): X viewed as X[o][r_in][j] with j over J = In*IL contiguous
// entries, r_in over the inner right modes (IR_in), o over the outer right
// modes.  T(j, c) = sum_o S(o, c) sum_{r_in} X[o][r_in][j] K_in(r_in, c).
//   grid.x = j-tile of 64*MJ entries
//   grid.y = lc + nlc * s: inner chunk lc of LC = 64*SPB rows of r_in and
//            split s of the outer blocks
//   grid.z = rank-column block
// Wave w owns rows [w*16*SPB, (w+1)*16*SPB) of the chunk; within a step of
// 16 rows, k-step t uses rows 4*kg + t, so lane (m, kg) loads 4 consecutive
// j at 4m + 64g from each of its 4 rows, and component e feeds m-block
// 4g + e (accumulator row m' of that block is j = jt0 + 64g + 4m' + e).
// partial: [gridDim.y][J][R].
// ---------------------------------------------------------------------------
template <typename T, int NB, int MJ, bool V4, int RING = 3>
__global__ __launch_bounds__(kThreads) void k_contract_right(
    const T *__restrict__ X, int64_t J, int64_t IR_in, int64_t n_outer, Krp<T> kin, Krp<T> kout, int R,
    int SPB, int64_t nlc, int64_t blocks_per_split, T *__restrict__ partial) {
    typedef typename Vec4<T>::type acc_t;
    constexpr int RP = NB * 16;
    constexpr int PITCH = RP + 4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kg = lane >> 4;
    const int c0 = blockIdx.z * RP;
    const int LC = 64 * SPB;
    const int64_t lc = blockIdx.y % nlc;
    const int64_t split = blockIdx.y / nlc;
    const int64_t r0 = lc * LC;
    const int64_t rend = min(IR_in, r0 + LC);
    const int64_t jt0 = (int64_t)blockIdx.x * 64 * MJ;
    const int64_t o_begin = split * blocks_per_split;
    const int64_t o_end = min(n_outer, o_begin + blocks_per_split);
    const bool has_out = kout.Z > 0;


    acc_t acc[MJ][4][NB], tot[MJ][4][NB];
#pragma unroll
    for (int g = 0; g < MJ; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                acc[g][e][nb] = acc_t{0, 0, 0, 0};
                tot[g][e][nb] = acc_t{0, 0, 0, 0};
            }
    int64_t jj[MJ];
    bool jok[MJ];
#pragma unroll
    for (int g = 0; g < MJ; ++g) {
        jj[g] = jt0 + 64 * g + 4 * m;
        jok[g] = jj[g] < J;
    }

    // X loads: one buffer resource per block for this wave's rows, based at
    // (row r0 + w*16*SPB, column jt0), so lane offsets are
    // ((16*ls + 4*kg + t) * J + 64*g + 4*m) entries; rows past the chunk,
    // columns past J and blocks past the split read zeros.
    int64_t lo = o_begin;
    int ls = 0;
    const int64_t wrow = r0 + wave * 16 * SPB;
    auto wave_base = [&](int64_t o) { return X + (o * IR_in + wrow) * J + jt0; };
    rsrc_t rs = make_rsrc(wave_base(o_begin < o_end ? o_begin : 0), kRsrcRange);
    auto load_step = [&](T (&a)[4][MJ][4]) {
        const bool live = lo < o_end;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t rl = 16 * ls + 4 * kg + t;  // row within this wave's rows
            const bool rok = live && wrow + rl < rend;
#pragma unroll
            for (int g = 0; g < MJ; ++g) {
                const int64_t jl = 64 * g + 4 * m;  // column within the tile
                if (V4) {
                    const bool ok = rok && jok[g];
                    const uint32_t off = ok ? (uint32_t)((rl * J + jl) * sizeof(T)) : kNoLoad;
                    const acc_t v = buf_load4(rs, off, T(0));
                    a[t][g][0] = v[0]; a[t][g][1] = v[1]; a[t][g][2] = v[2]; a[t][g][3] = v[3];
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const bool ok = rok && jj[g] + e < J;
                        const uint32_t off = ok ? (uint32_t)((rl * J + jl + e) * sizeof(T)) : kNoLoad;
                        a[t][g][e] = buf_load1(rs, off, T(0));
                    }
                }
            }
        }
        if (++ls == SPB) {
            ls = 0;
            ++lo;
            if (lo < o_end) rs = make_rsrc(wave_base(lo), kRsrcRange);
        }
    };

    T x[RING][4][MJ][4];
#pragma unroll
    for (int k = 0; k < RING - 1; ++k) load_step(x[k]);
    build_tile_batched<T, RP, 16>(kin, R, c0, r0, LC, IR_in, [&](int q, int c, T v) { tile[q * PITCH + c] = v; });

    int64_t co = o_begin;
    int cs = 0;
    BlockScale<T, NB> sc;
    if (has_out && o_begin < o_end) sc.start(kout, R, c0 + m, o_begin);
    __syncthreads();
    auto compute_step = [&](const T (&a)[4][MJ][4]) {
        const T *kb = tile + (wave * 16 * SPB + 16 * cs + 4 * kg) * PITCH + m;
        T b[4][NB];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) b[t][nb] = kb[t * PITCH + 16 * nb];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int g = 0; g < MJ; ++g)
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) acc[g][e][nb] = mfma4(a[t][g][e], b[t][nb], acc[g][e][nb]);
        if (++cs == SPB) {
            cs = 0;
            if (has_out) {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const T s = sc.value(kout, R, c0 + m, nb);
#pragma unroll
                    for (int g = 0; g < MJ; ++g)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            tot[g][e][nb] += acc[g][e][nb] * s;
                            acc[g][e][nb] = acc_t{0, 0, 0, 0};
                        }
                }
                if (co + 1 < o_end) sc.advance(kout, R, c0 + m);
            }
            ++co;
        }
    };

    const int64_t nsteps = (o_end > o_begin ? o_end - o_begin : 0) * SPB;
    int64_t st = 0;
    for (; st + RING <= nsteps; st += RING) {
#pragma unroll
        for (int k = 0; k < RING; ++k) {
            load_step(x[(k + RING - 1) % RING]);
            compute_step(x[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < RING - 1; ++k)
        if (st + k < nsteps) compute_step(x[k]);
    if (!has_out) {
#pragma unroll
        for (int g = 0; g < MJ; ++g)
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) tot[g][e][nb] = acc[g][e][nb];
    }

    // Sum the 4 waves in wave order and store the partial.
    __syncthreads();
    constexpr int PER_WAVE = MJ * 4 * NB * 4 * 64;
    T *red = tile;  // [wave][g][e][nb][jj][lane]
#pragma unroll
    for (int g = 0; g < MJ; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    red[wave * PER_WAVE + (((g * 4 + e) * NB + nb) * 4 + q) * 64 + lane] = tot[g][e][nb][q];
    __syncthreads();
    for (int q = tid; q < PER_WAVE; q += kThreads) {
        const int ln = q & 63, qq = (q >> 6) & 3, blk = q >> 8;
        const int nb = blk % NB, ge = blk / NB, e = ge % 4, g = ge / 4;
        const T sum = ((red[q] + red[PER_WAVE + q]) + red[2 * PER_WAVE + q]) + red[3 * PER_WAVE + q];
        const int64_t j = jt0 + 64 * g + 4 * acc_row<T>(ln, qq) + e;
        const int c = c0 + 16 * nb + (ln & 15);
        if (j < J && c < R) partial[((int64_t)blockIdx.y * J + j) * R + c] = sum;
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
