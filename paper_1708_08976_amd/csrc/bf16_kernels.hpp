// Split-bfloat16 MTTKRP: the tensor is stored as two bfloat16 planes, hi and
// lo, with value hi + lo (about 16 significant bits of the float32 it came
// from).  The Khatri-Rao product values are formed in float32 and split the
// same way inside the kernel.  Each contraction step multiplies
//     Xh*Kh + Xh*Kl + Xl*Kh
// on the 16x16x32 bf16 MFMA with float32 accumulation; the dropped Xl*Kl
// term is below 2^-16 of each product.  This recovers float32-level accuracy
// at a fraction of the float32 MFMA cost, and the tensor still moves only
// 4 bytes per entry.
//
// The work decomposition is that of the float32 kernels in
// mttkrp_kernels.hpp (resident inner Khatri-Rao tile, X streamed block by
// block over the outer index, per-block scaling for the outer factors).
#pragma once

#include "device_common.hpp"

namespace cpm {

__device__ inline bf16x8 as_bf16x8(f32x4 raw) { return __builtin_bit_cast(bf16x8, raw); }

// One 16-byte buffer load of 8 consecutive bf16 values.  The planes are
// read without the non-temporal hint: with it, the left-first kernels on the
// 256 x 256 x 512 x 32 tensor at R = 128 took 7-11% longer.
__device__ inline f32x4 buf_load_raw16(rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

// 8 consecutive bf16 values read one at a time (unaligned rows); lanes past
// the row end read zeros.
__device__ inline f32x4 buf_load_raw16_scalar(rsrc_t r, uint32_t off, int64_t l, int64_t lend) {
    u16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const uint32_t oe = (off != kNoLoad && l + e < lend) ? off + 2 * e : kNoLoad;
        v[e] = (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, oe, 0, 0);
    }
    return __builtin_bit_cast(f32x4, v);
}

// ---------------------------------------------------------------------------
// Left-first split-bf16 contraction (internal and last modes).  Geometry as
// k_contract_left: X viewed as X[r][i][h][l_in], outer block o = h + IL_out*r.
//   grid.x = row tile (16*MB rows), grid.y = lc + nlc*split, grid.z = column
//   block (16*NB columns).
// A step covers 32*Q entries of every row: lane (m, kg) loads Q groups of 8
// consecutive entries at 32q + 8kg from each plane (one 16x16x32 MFMA k-step
// per group), so a row receives Q*64 contiguous bytes per plane.  Wave w owns
// entries [w*32*Q*SPB, (w+1)*32*Q*SPB) of the chunk (LC = 128*Q*SPB).
// The tile holds K_in split into bf16 planes, stored column-major
// (Kt[c][l]) so the B operand of a k-step is one 16-byte LDS read.
// partial: [gridDim.y][In][R] float32.
// ---------------------------------------------------------------------------
template <int NB, int MB, int Q, bool V8, int WM = 1, int RING = 3>
__global__ __launch_bounds__(kThreads) void k_contract_left_bf16(
    const uint16_t *__restrict__ Xp, int64_t I, int64_t IL_in, int64_t IL_out, int64_t In, int64_t n_outer,
    Krp<float> kin, Krp<float> kout, int R, int SPB, int64_t nlc, int64_t blocks_per_split,
    float *__restrict__ partial) {
    constexpr int RP = NB * 16;
    constexpr int WC = 4 / WM;  // waves along the chunk; WM wave groups take separate row tiles
    const int WS = 32 * Q;
    const int LC = WC * WS * SPB;
    const int LCP = LC + 8;  // bf16 row pitch of the transposed tile (16-byte pad)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint16_t *kth = reinterpret_cast<uint16_t *>(smem_raw);
    uint16_t *ktl = kth + RP * LCP;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WC, wc = wave % WC;
    const int m = lane & 15, kg = lane >> 4;
    const int c0 = blockIdx.z * RP;
    const int64_t lc = blockIdx.y % nlc;
    const int64_t split = blockIdx.y / nlc;
    const int64_t l0 = lc * LC;
    const int64_t lend = min(IL_in, l0 + LC);
    const int64_t IL = IL_in * IL_out;
    const int64_t row_base = (int64_t)blockIdx.x * 16 * MB * WM + 16 * MB * wm;  // this wave's rows
    const int64_t o_begin = split * blocks_per_split;
    const int64_t o_end = min(n_outer, o_begin + blocks_per_split);
    const bool has_out = kout.Z > 0;

    f32x4 acc[MB][NB], tot[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            acc[mb][nb] = f32x4{0, 0, 0, 0};
            tot[mb][nb] = f32x4{0, 0, 0, 0};
        }
    // Descriptors over each 16-row block of the current outer block: rows
    // past In lie outside the record count, and everything does once the
    // split's blocks are exhausted; only a ragged last chunk needs a
    // per-lane check.
    int64_t rows_valid[MB];
    uint32_t rec[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        rows_valid[mb] = max((int64_t)0, min((int64_t)16, In - row_base - 16 * mb));
        rec[mb] = rows_valid[mb] == 16 ? kRsrcRange : (uint32_t)(rows_valid[mb] * IL * 2);
    }
    const bool ragged = lend - l0 < LC;
    const uint32_t lane_row = (uint32_t)(m * IL);
    const int64_t lane_l = l0 + wc * WS * SPB + 8 * kg;

    int64_t cur_r = o_begin / IL_out, cur_h = o_begin - (o_begin / IL_out) * IL_out;
    int64_t lo = o_begin;
    rsrc_t rh[MB], rl[MB];
    auto set_block = [&]() {
        const int64_t b = cur_r * In * IL + cur_h * IL_in;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const bool live = lo < o_end && rows_valid[mb] > 0;
            const int64_t e = live ? b + (row_base + 16 * mb) * IL : 0;
            rh[mb] = make_rsrc(Xp + e, live ? rec[mb] : 0u);
            rl[mb] = make_rsrc(Xp + I + e, live ? rec[mb] : 0u);
        }
    };
    set_block();

    int ls = 0;
    // a[mb][q][0] = hi, a[mb][q][1] = lo
    auto load_step = [&](f32x4 (&a)[MB][Q][2]) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int64_t l = lane_l + WS * ls + 32 * q;
                uint32_t off = (uint32_t)((lane_row + l) * 2);
                if (V8) {
                    if (ragged) off = l < lend ? off : kNoLoad;
                    a[mb][q][0] = buf_load_raw16(rh[mb], off);
                    a[mb][q][1] = buf_load_raw16(rl[mb], off);
                } else {
                    if (l >= lend) off = kNoLoad;
                    a[mb][q][0] = buf_load_raw16_scalar(rh[mb], off, l, lend);
                    a[mb][q][1] = buf_load_raw16_scalar(rl[mb], off, l, lend);
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

    f32x4 x[RING][MB][Q][2];
#pragma unroll
    for (int k = 0; k < RING - 1; ++k) load_step(x[k]);
    // Build this work-group's chunk of K_in once: float32 values split into
    // the hi/lo planes of the transposed tile.
    build_tile_batched<float, RP, 16>(kin, R, c0, l0, LC, IL_in, [&](int q, int c, float v) {
        const uint16_t h = bf16_rne_bits(v);
        kth[c * LCP + q] = h;
        ktl[c * LCP + q] = bf16_rne_bits(v - bf16_bits_to_float(h));
    });

    float *stab = reinterpret_cast<float *>(ktl + RP * LCP);  // [scale_blocks<RP>()][RP] outer scales
    if (has_out) fill_scales<RP>(kout, R, c0, o_begin, o_end, stab);
    int64_t co = o_begin, tb0 = o_begin;
    int cs = 0;

    auto compute_step = [&](const f32x4 (&a)[MB][Q][2]) {
        const int kbase = wc * WS * SPB + WS * cs + 8 * kg;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int c = 16 * nb + m;
                const bf16x8 bh = as_bf16x8(*reinterpret_cast<const f32x4 *>(kth + c * LCP + kbase + 32 * q));
                const bf16x8 bl = as_bf16x8(*reinterpret_cast<const f32x4 *>(ktl + c * LCP + kbase + 32 * q));
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    const bf16x8 ah = as_bf16x8(a[mb][q][0]);
                    const bf16x8 al = as_bf16x8(a[mb][q][1]);
                    acc[mb][nb] = mfma_bf16(ah, bh, acc[mb][nb]);
                    acc[mb][nb] = mfma_bf16(ah, bl, acc[mb][nb]);
                    acc[mb][nb] = mfma_bf16(al, bh, acc[mb][nb]);
                }
            }
        }
        if (++cs == SPB) {
            cs = 0;
            if (has_out) {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const float sc = stab[(co - tb0) * RP + 16 * nb + m];
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb) {
                        tot[mb][nb] += acc[mb][nb] * sc;
                        acc[mb][nb] = f32x4{0, 0, 0, 0};
                    }
                }
            }
            ++co;
        }
    };

    // Chunks of scale_blocks<RP>() blocks (a multiple of RING); the scale table is
    // refilled between chunks, outside the unrolled step loop.
    for (; tb0 < o_end; tb0 += scale_blocks<RP>()) {
        if (tb0 != o_begin && has_out) fill_scales<RP>(kout, R, c0, tb0, o_end, stab);
        __syncthreads();
        const int64_t nsteps = (min(o_end, tb0 + scale_blocks<RP>()) - tb0) * SPB;
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
        __syncthreads();
    }
    if (!has_out) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) tot[mb][nb] = acc[mb][nb];
    }

    __syncthreads();
    float *red = reinterpret_cast<float *>(smem_raw);  // [wave][mb][nb][j][lane]
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                red[(((wave * MB + mb) * NB + nb) * 4 + j) * 64 + lane] = tot[mb][nb][j];
    __syncthreads();
    constexpr int PER_WAVE = MB * NB * 4 * 64;
    for (int e = tid; e < WM * PER_WAVE; e += kThreads) {
        const int g = e / PER_WAVE, r = e % PER_WAVE;  // row group, element
        const int ln = r & 63, j = (r >> 6) & 3, blk = r >> 8;
        const int nb = blk % NB, mb = blk / NB;
        const float *src = red + (g * WC) * PER_WAVE + r;
        float sum = src[0];
#pragma unroll
        for (int w = 1; w < WC; ++w) sum += src[w * PER_WAVE];
        const int64_t row = (int64_t)blockIdx.x * 16 * MB * WM + 16 * MB * g + 16 * mb + acc_row<float>(ln, j);
        const int c = c0 + 16 * nb + (ln & 15);
        if (row < In && c < R) partial[((int64_t)blockIdx.y * In + row) * R + c] = sum;
    }
}

// ---------------------------------------------------------------------------
// Right-first split-bf16 contraction (mode 0, and internal modes with a short
// left product).  Geometry as k_contract_right: X viewed as X[o][r_in][j],
// T(j, c) = sum_o S(o, c) sum_{r_in} X[o][r_in][j] K_in(r_in, c).
// The contracted index r_in is the strided one, while the bf16 MFMA packs 8
// consecutive k values per lane, so every step's X tile (32 rows x 64 j, both
// planes) is loaded with 16-byte loads along j and written to LDS transposed
// (Xt[j][r]); lanes then read 8 consecutive r of one j in one 16-byte read.
// The waves split the rank columns (WN ways) and the 4 j-blocks (WM ways),
// so each wave owns distinct output blocks.  X steps are kept DX deep in
// flight in registers; the LDS X tile is double-buffered.
//   grid.x = j tile of 64, grid.y = lc + nlc*split (inner chunk of
//   LC = 32*SPB rows, split of the outer blocks), grid.z = column block.
// partial: [gridDim.y][J][R] float32.
// ---------------------------------------------------------------------------
template <int NB, bool V8, int DX = 6>
__global__ __launch_bounds__(kThreads) void k_contract_right_bf16(
    const uint16_t *__restrict__ Xp, int64_t I, int64_t J, int64_t IR_in, int64_t n_outer, Krp<float> kin,
    Krp<float> kout, int R, int SPB, int64_t nlc, int64_t blocks_per_split, float *__restrict__ partial) {
    constexpr int RP = NB * 16;
    constexpr int WN = NB < 4 ? NB : 4;  // waves along rank blocks
    constexpr int WM = 4 / WN;           // waves along j blocks
    constexpr int NBW = NB / WN;         // rank blocks per wave
    constexpr int MBW = 4 / WM;          // j blocks per wave
    constexpr int JT = 64, RS = 32, XP = RS + 8;
    const int LC = RS * SPB;
    const int LCP = LC + 8;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint16_t *kth = reinterpret_cast<uint16_t *>(smem_raw);
    uint16_t *ktl = kth + RP * LCP;
    uint16_t *xt = ktl + RP * LCP;  // [2 buffers][2 planes][JT][XP]

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform, so the X descriptor stays scalar
    const int m = lane & 15, kg = lane >> 4;
    const int wn = wave % WN, wm = wave / WN;
    const int c0 = blockIdx.z * RP;
    const int64_t jt0 = (int64_t)blockIdx.x * JT;
    const int64_t lc = blockIdx.y % nlc;
    const int64_t split = blockIdx.y / nlc;
    const int64_t r0 = lc * LC;
    const int64_t rend = min(IR_in, r0 + LC);
    const int64_t o_begin = split * blocks_per_split;
    const int64_t o_end = min(n_outer, o_begin + blocks_per_split);
    const bool has_out = kout.Z > 0;

    // X tile loader: thread -> (plane, 8-wide j group, row pair)
    const int plane = wave >> 1, tt = tid & 127, jg = tt & 7, rp = tt >> 3;  // rp in [0, 16)
    const bool jok = V8 ? (jt0 + 8 * jg < J) : true;
    const bool jragged = jt0 + JT > J;
    // Descriptor over the chunk's rows of the current outer block: rows past
    // the chunk end lie outside its record count, and everything does once
    // the split's blocks are exhausted.
    const int64_t rows_valid = rend - r0;
    const uint32_t rec = rows_valid == LC ? kRsrcRange : (uint32_t)(rows_valid * J * 2);
    int64_t lo = o_begin;
    int ls = 0;
    rsrc_t rx;
    auto set_block = [&]() {
        const bool live = lo < o_end;
        rx = make_rsrc(Xp + (live ? (int64_t)plane * I + lo * IR_in * J + r0 * J + jt0 : 0), live ? rec : 0u);
    };
    set_block();
    auto load_step = [&](f32x4 (&a)[2]) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t rl = (int64_t)RS * ls + 2 * rp + h;  // row within the chunk
            uint32_t off = (uint32_t)((rl * J + 8 * jg) * 2);
            if (V8) {
                if (jragged) off = jok ? off : kNoLoad;
                a[h] = buf_load_raw16(rx, off);
            } else {
                a[h] = buf_load_raw16_scalar(rx, off, jt0 + 8 * jg, J);
            }
        }
        if (++ls == SPB) {
            ls = 0;
            ++lo;
            set_block();
        }
    };
    // Transposed write: the two rows of this thread are adjacent in r, so each
    // j gets one 32-bit (2 x bf16) store.  Within a j row the four 8-entry r
    // chunks are XOR-swizzled by (j / 8) % 4: the eight threads that differ
    // only in jg would otherwise store to one bank (8 jg rows of 20 words
    // are a multiple of 32 words apart).  The reads below undo the swizzle;
    // a 16-byte A read stays one contiguous chunk.
    const int rsw = 8 * ((rp >> 2) ^ (jg & 3)) + 2 * (rp & 3);
    auto write_tile = [&](const f32x4 (&a)[2], int buf) {
        const u16x8 v0 = __builtin_bit_cast(u16x8, a[0]);
        const u16x8 v1 = __builtin_bit_cast(u16x8, a[1]);
        uint32_t *dst = reinterpret_cast<uint32_t *>(xt + ((buf * 2 + plane) * JT + 8 * jg) * XP + rsw);
#pragma unroll
        for (int e = 0; e < 8; ++e) dst[e * XP / 2] = (uint32_t)v0[e] | ((uint32_t)v1[e] << 16);
    };

    f32x4 acc[MBW][NBW], tot[MBW][NBW];
#pragma unroll
    for (int a = 0; a < MBW; ++a)
#pragma unroll
        for (int b = 0; b < NBW; ++b) {
            acc[a][b] = f32x4{0, 0, 0, 0};
            tot[a][b] = f32x4{0, 0, 0, 0};
        }

    f32x4 x[DX][2];
#pragma unroll
    for (int k = 0; k < DX; ++k) load_step(x[k]);
    build_tile_batched<float, RP, 16>(kin, R, c0, r0, LC, IR_in, [&](int q, int c, float v) {
        const uint16_t hb = bf16_rne_bits(v);
        kth[c * LCP + q] = hb;
        ktl[c * LCP + q] = bf16_rne_bits(v - bf16_bits_to_float(hb));
    });
    float *stab = reinterpret_cast<float *>(xt + 2 * 2 * JT * XP);  // [scale_blocks<RP>()][RP] outer scales
    if (has_out) fill_scales<RP>(kout, R, c0, o_begin, o_end, stab);
    int64_t co = o_begin, tb0 = o_begin;
    int cs = 0;

    auto compute_step = [&](int buf) {
        const uint16_t *xb = xt + buf * 2 * JT * XP;
#pragma unroll
        for (int a = 0; a < MBW; ++a) {
            const int j = 16 * (wm * MBW + a) + m;
            const int ch = kg ^ ((j >> 3) & 3);  // swizzled position of r chunk kg in row j
            const bf16x8 ah = as_bf16x8(*reinterpret_cast<const f32x4 *>(xb + j * XP + 8 * ch));
            const bf16x8 al = as_bf16x8(*reinterpret_cast<const f32x4 *>(xb + JT * XP + j * XP + 8 * ch));
#pragma unroll
            for (int b = 0; b < NBW; ++b) {
                const int c = 16 * (wn * NBW + b) + m;
                const int koff = c * LCP + RS * cs + 8 * kg;
                const bf16x8 bh = as_bf16x8(*reinterpret_cast<const f32x4 *>(kth + koff));
                const bf16x8 bl = as_bf16x8(*reinterpret_cast<const f32x4 *>(ktl + koff));
                acc[a][b] = mfma_bf16(ah, bh, acc[a][b]);
                acc[a][b] = mfma_bf16(ah, bl, acc[a][b]);
                acc[a][b] = mfma_bf16(al, bh, acc[a][b]);
            }
        }
        if (++cs == SPB) {
            cs = 0;
            if (has_out) {
#pragma unroll
                for (int b = 0; b < NBW; ++b) {
                    const float sval = stab[(co - tb0) * RP + 16 * (wn * NBW + b) + m];
#pragma unroll
                    for (int a = 0; a < MBW; ++a) {
                        tot[a][b] += acc[a][b] * sval;
                        acc[a][b] = f32x4{0, 0, 0, 0};
                    }
                }
            }
            ++co;
        }
    };

    // Global step g is computed from LDS buffer g & 1; its registers were
    // x[g % DX].  Chunks of scale_blocks<RP>() blocks (an even multiple of DX
    // steps) keep both alignments; the scale table is refilled between
    // chunks, behind the per-step barrier.
    const int64_t total = (o_end > o_begin ? o_end - o_begin : 0) * SPB;
    if (total > 0) write_tile(x[0], 0);
    for (int64_t g0 = 0; g0 < total; g0 += (int64_t)scale_blocks<RP>() * SPB) {
        tb0 = o_begin + g0 / SPB;
        if (g0 != 0 && has_out) fill_scales<RP>(kout, R, c0, tb0, o_end, stab);
        __syncthreads();
        const int64_t gend = min(total, g0 + (int64_t)scale_blocks<RP>() * SPB);
        int64_t g = g0;
        for (; g + DX <= gend; g += DX) {
#pragma unroll
            for (int k = 0; k < DX; ++k) {
                compute_step((int)((g + k) & 1));
                if (g + k + 1 < total) write_tile(x[(k + 1) % DX], (int)((g + k + 1) & 1));
                load_step(x[k]);  // step g + k + DX
                __syncthreads();
            }
        }
#pragma unroll
        for (int k = 0; k < DX; ++k) {
            if (g + k < gend) {
                compute_step((int)((g + k) & 1));
                if (g + k + 1 < total) write_tile(x[(k + 1) % DX], (int)((g + k + 1) & 1));
                __syncthreads();
            }
        }
    }
    if (!has_out) {
#pragma unroll
        for (int a = 0; a < MBW; ++a)
#pragma unroll
            for (int b = 0; b < NBW; ++b) tot[a][b] = acc[a][b];
    }
#pragma unroll
    for (int a = 0; a < MBW; ++a)
#pragma unroll
        for (int b = 0; b < NBW; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t j = jt0 + 16 * (wm * MBW + a) + acc_row<float>(lane, q);
                const int c = c0 + 16 * (wn * NBW + b) + m;
                if (j < J && c < R) partial[((int64_t)blockIdx.y * J + j) * R + c] = tot[a][b][q];
            }
}

}  // namespace cpm
