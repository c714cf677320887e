// Float32 MTTKRP contraction kernels on the 32x32x2 f32 MFMA.
//
// Same decomposition as mttkrp_kernels.hpp (3-index view X3[r][i][l], K_in
// tile resident in LDS, X streamed block by block over the outer index o,
// per-block scaling by S(o, :) for the multi-TTV), tuned for the float32
// matrix rate being barely above what HBM delivers at small R:
//   * the 32x32 product moves half the operand bytes per flop of the 16x16
//     one, and one 32-column block covers R = 32 in a single accumulator
//     whose column index is the lane (one scale value per lane);
//   * the K_in tile is stored transposed (Kt[c][row]) with a pitch of
//     4 (mod 32) words, so a lane's B operands for four consecutive
//     k-steps are one conflict-free 16-byte LDS read;
//   * X arrives in 16-byte buffer loads, eight lanes per 128-byte row
//     segment (left-first, staged through LDS into MFMA layout) or 512
//     contiguous bytes per row (right-first), with a ring of RING register
//     sets so RING - 1 steps are in flight; rows need only 4-byte
//     alignment (row lengths need not be multiples of 4: the four entries
//     that straddle a chunk or row end are loaded one by one);
//   * the outer scale S(o, c) of the current block multiplies the B
//     operands as they leave LDS, so the MFMA accumulates full Khatri-Rao
//     values K_in(g, c) * S(o, c) directly: one accumulator set, no
//     per-block epilogue.  The scales of the coming blocks sit in an LDS
//     table (fill_scales), so reading them never waits behind X loads.
#pragma once

#include <type_traits>

#include "device_common.hpp"

namespace cpm {

// ---------------------------------------------------------------------------
// Left-first (internal and last modes).  X viewed as X[r][i][h][l_in]:
// IL_in inner entries contiguous, outer block o = h + IL_out * r.
// A work-group owns 32*WM rows of i (WM row tiles of 32, one per wave group)
// and a chunk of LC inner entries split over WC = 4/WM waves; 32*NC rank
// columns.  Wave (wm, wc) handles rows row_w + (0..31) and entries
// [wc*32*SPB, (wc+1)*32*SPB) of the chunk, 32 entries (128 B of a row) per
// step.
// Loads are row-coalesced: load i of a step gives lane L the 16 bytes at
// chunk ch = L%8 of row 8i + L/8, so eight lanes cover one 128-byte row
// segment.  The wave writes its step into a private LDS slot with the chunk
// position XOR-swizzled by the row (conflict-free in both directions) and
// reads it back in MFMA layout: lane (m, h) of k-step (q, t) takes row m,
// entry 8q + 4h + t.  A slot is private to its wave and LDS operations of a
// wave complete in order, so no barrier is needed.
// Validity is carried by the buffer descriptor: its record count stops at
// the last valid row and is zero once the wave's blocks are exhausted, so
// the loads need no per-lane condition except in a ragged last chunk.
//   grid.x = row tile (32*WM rows), grid.y = lc + nlc*split, grid.z = column
//   block.  partial: [gridDim.y][In][R].
// ---------------------------------------------------------------------------
template <int NC, int WM, int RING = 3>
__global__ __launch_bounds__(kThreads) void k_left32(const float *__restrict__ X, int64_t IL_in, int64_t IL_out,
                                                     int64_t In, int64_t n_outer, Krp<float> kin,
                                                     Krp<float> kout, int R, int SPB, int64_t nlc,
                                                     int64_t blocks_per_split, float *__restrict__ partial) {
    constexpr int RP = 32 * NC;
    constexpr int WC = 4 / WM;  // waves along the chunk
    constexpr int WS = 32;      // entries per row per wave-step
    const int LC = WC * WS * SPB;
    const int PT = LC + 4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *tile = reinterpret_cast<float *>(smem_raw);  // [RP][PT]: K_in transposed

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WC, wc = wave % WC;
    const int m = lane & 31, h = lane >> 5;
    const int c0 = blockIdx.z * RP;
    const int64_t lc = blockIdx.y % nlc;
    const int64_t split = blockIdx.y / nlc;
    const int64_t l0 = lc * LC;
    const int64_t lcount = min(IL_in - l0, (int64_t)LC);  // entries of this chunk
    const bool ragged = lcount < LC;
    const int64_t IL = IL_in * IL_out;
    const int64_t row_w = (int64_t)blockIdx.x * 32 * WM + 32 * wm;  // first row of this wave
    const int64_t o_begin = split * blocks_per_split;
    const int64_t o_end = min(n_outer, o_begin + blocks_per_split);
    const int wl = wc * WS * SPB;  // wave's first entry within the chunk
    float *stg = tile + RP * PT + wave * 32 * WS;  // this wave's staging slot [32 rows][32 entries]

    // Descriptor over the wave's rows of the current block: rows past In are
    // outside its record count, and so is everything once the split ends.
    const int64_t rows_valid = max((int64_t)0, min((int64_t)32, In - row_w));
    const uint32_t rec_rows = rows_valid == 32 ? kRsrcRange : (uint32_t)(rows_valid * IL * 4);
    int64_t cur_r = o_begin / IL_out, cur_h = o_begin - (o_begin / IL_out) * IL_out;
    int64_t lo = o_begin;
    rsrc_t rs;
    auto set_block = [&]() {
        const bool live = lo < o_end && rows_valid > 0;
        rs = make_rsrc(X + (live ? cur_r * In * IL + cur_h * IL_in + row_w * IL + l0 : 0), live ? rec_rows : 0u);
    };
    set_block();
    const int ch = lane & 7;
    uint32_t loff[4];  // byte offset of each load within a step, for the step at entry 0
#pragma unroll
    for (int i = 0; i < 4; ++i) loff[i] = (uint32_t)(((int64_t)(8 * i + (lane >> 3)) * IL + wl + 4 * ch) * 4);
    int ls = 0;
    // One step's loads.  PART (a chunk that ends inside a group of four
    // entries, for inner ranges that are not a multiple of 4) takes single
    // loads of the entries inside the chunk and zeros for the rest, so no
    // load reaches past it.  The two forms are separate copies of the
    // stream below, each with a fixed number of loads per step, so the
    // waits before a step's data is used count only that step's loads and
    // RING - 1 steps stay in flight.
    auto load_step = [&](auto part_c, f32x4 (&a)[4]) {
        constexpr bool PART = decltype(part_c)::value;
        const int e0 = wl + WS * ls + 4 * ch;  // chunk-relative entry of this lane
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t off = loff[i] + (uint32_t)(WS * ls * 4);
            if constexpr (!PART) {
                a[i] = buf_load4(rs, (!ragged || e0 < lcount) ? off : kNoLoad, 0.f);
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) a[i][t] = buf_load1(rs, e0 + t < lcount ? off + 4 * t : kNoLoad, 0.f);
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

    float *stab = stg + (4 - wave) * 32 * WS;  // [scale_blocks<RP>()][RP], after the four staging slots
    int64_t co = o_begin, tb0 = o_begin;
    int cs = 0;
    float scl[NC];
    f32x16 acc[NC];
#pragma unroll
    for (int nc = 0; nc < NC; ++nc) acc[nc] = f32x16{};
    const float *tb = tile + m * PT + wl + 4 * h;
    auto load_scales = [&]() {
#pragma unroll
        for (int nc = 0; nc < NC; ++nc) scl[nc] = stab[(co - tb0) * RP + 32 * nc + m];
    };

    auto compute_step = [&](const f32x4 (&xl)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rho = 8 * i + (lane >> 3);
            *reinterpret_cast<f32x4 *>(stg + rho * WS + ((ch ^ (rho & 7)) * 4)) = xl[i];
        }
        f32x4 a[4], b[NC][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = *reinterpret_cast<const f32x4 *>(stg + m * WS + (((2 * q + h) ^ (m & 7)) * 4));
#pragma unroll
        for (int nc = 0; nc < NC; ++nc)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                b[nc][q] = *reinterpret_cast<const f32x4 *>(tb + 32 * nc * PT + WS * cs + 8 * q) * scl[nc];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int nc = 0; nc < NC; ++nc) acc[nc] = mfma32(a[q][t], b[nc][q][t], acc[nc]);
        if (++cs == SPB) {
            cs = 0;
            if (++co - tb0 < scale_blocks<RP>() && co < o_end) load_scales();
        }
    };

    auto stream = [&](auto part_c) {
        f32x4 x[RING][4];
#pragma unroll
        for (int k = 0; k < RING - 1; ++k) load_step(part_c, x[k]);
        build_tile_batched<float, RP, 16>(kin, R, c0, l0, LC, IL_in,
                                          [&](int q, int c, float v) { tile[c * PT + q] = v; });
        fill_scales<RP>(kout, R, c0, o_begin, o_end, stab);
        // Chunks of scale_blocks<RP>() blocks; within a chunk RING steps per
        // pass with compile-time ring slots.
        for (; tb0 < o_end; tb0 += scale_blocks<RP>()) {
            if (tb0 != o_begin) fill_scales<RP>(kout, R, c0, tb0, o_end, stab);
            __syncthreads();
            co = tb0;
            load_scales();
            const int64_t nsteps = (min(o_end, tb0 + scale_blocks<RP>()) - tb0) * SPB;
            int64_t st = 0;
            for (; st + RING <= nsteps; st += RING) {
#pragma unroll
                for (int k = 0; k < RING; ++k) {
                    load_step(part_c, x[(k + RING - 1) % RING]);
                    compute_step(x[k]);
                }
            }
            // only the last chunk can end off a RING boundary; its remaining
            // steps are already in slots 0 .. RING - 2
#pragma unroll
            for (int k = 0; k < RING - 1; ++k)
                if (st + k < nsteps) compute_step(x[k]);
            __syncthreads();  // every wave is done with this chunk's scales
        }
    };
    if (ragged && (lcount & 3) != 0) stream(std::true_type{});
    else stream(std::false_type{});

    // Sum the WC waves that share rows, in wave order, and store.
    __syncthreads();
    float *red = tile;  // [wave][nc][j][lane]
#pragma unroll
    for (int nc = 0; nc < NC; ++nc)
#pragma unroll
        for (int j = 0; j < 16; ++j) red[((wave * NC + nc) * 16 + j) * 64 + lane] = acc[nc][j];
    __syncthreads();
    constexpr int PER_WAVE = NC * 16 * 64;
    for (int e = tid; e < WM * PER_WAVE; e += kThreads) {
        const int g = e / PER_WAVE, r = e % PER_WAVE;  // row group, element
        const int ln = r & 63, j = (r >> 6) & 15, nc = r >> 10;
        const float *src = red + (g * WC) * PER_WAVE + r;
        float sum = src[0];
#pragma unroll
        for (int w = 1; w < WC; ++w) sum += src[w * PER_WAVE];
        const int64_t row = (int64_t)blockIdx.x * 32 * WM + 32 * g + acc32_row(ln, j);
        const int c = c0 + 32 * nc + (ln & 31);
        if (row < In && c < R) partial[((int64_t)blockIdx.y * In + row) * R + c] = sum;
    }
}

// ---------------------------------------------------------------------------
// Right-first (mode 0, and internal modes with a short left product).  X
// viewed as X[o][r_in][j], J = In*IL contiguous entries per row.
// T(j, c) = sum_o S(o, c) sum_{r_in} X[o][r_in][j] K_in(r_in, c).
// Waves: WJ along j (32*TJ entries each), WR = 4/WJ along the chunk's rows.
// Lane (m, h) of a wave reads TJ consecutive j at TJ*m from rows 4h + s
// (s = 0..3) of each 8-row step; MFMA (s, t) pairs slot h with row 4h + s
// and accumulator t covers j = jw + TJ*row' + t.
//   grid.x = j tile (32*TJ*WJ), grid.y = lc + nlc*split, grid.z = column
//   block.  partial: [gridDim.y][J][R].
// ---------------------------------------------------------------------------
template <int TJ> struct JVec;
template <> struct JVec<1> { typedef float type; };
template <> struct JVec<2> { typedef float __attribute__((ext_vector_type(2))) type; };
template <> struct JVec<4> { typedef f32x4 type; };

template <int TJ>
__device__ inline typename JVec<TJ>::type buf_loadj(rsrc_t r, uint32_t off) {
    if constexpr (TJ == 4) return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kStream));
    else if constexpr (TJ == 2)
        return __builtin_bit_cast(typename JVec<2>::type, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kStream));
    else return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <int TJ>
__device__ inline float jcomp(const typename JVec<TJ>::type &v, int t) {
    if constexpr (TJ == 1) return v;
    else return v[t];
}
template <int TJ>
__device__ inline void jset(typename JVec<TJ>::type &v, int t, float x) {
    if constexpr (TJ == 1) v = x;
    else v[t] = x;
}

template <int NC, int TJ, int WJ, int RING = 3>
__global__ __launch_bounds__(kThreads) void k_right32(const float *__restrict__ X, int64_t J, int64_t IR_in,
                                                      int64_t n_outer, Krp<float> kin, Krp<float> kout, int R,
                                                      int SPB, int64_t nlc, int64_t blocks_per_split,
                                                      float *__restrict__ partial) {
    typedef typename JVec<TJ>::type jv;
    constexpr int RP = 32 * NC;
    constexpr int WR = 4 / WJ;
    constexpr int JW = 32 * TJ;  // j per wave
    const int LC = WR * 8 * SPB;
    const int PT = LC + 4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *tile = reinterpret_cast<float *>(smem_raw);  // [RP][PT]: K_in transposed

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wj = wave % WJ, wr = wave / WJ;
    const int m = lane & 31, h = lane >> 5;
    const int c0 = blockIdx.z * RP;
    const int64_t lc = blockIdx.y % nlc;
    const int64_t split = blockIdx.y / nlc;
    const int64_t r0 = lc * LC;
    const int64_t rend = min(IR_in, r0 + LC);
    const int64_t jw = (int64_t)blockIdx.x * JW * WJ + JW * wj;  // first j of this wave
    const int64_t o_begin = split * blocks_per_split;
    const int64_t o_end = min(n_outer, o_begin + blocks_per_split);
    const int wrow = wr * 8 * SPB;  // wave's first row within the chunk
    const bool jok = jw + TJ * m < J;
    const bool wave_live = jw < J;

    // Descriptor over the wave's rows of the current block: rows past the
    // chunk end are outside its record count, and so is everything once the
    // split ends; lanes past J (a ragged j tile) get an out-of-range offset.
    const int64_t rows_valid = max((int64_t)0, min((int64_t)8 * SPB, rend - r0 - wrow));
    const uint32_t rec_rows = rows_valid == 8 * SPB ? kRsrcRange : (uint32_t)(rows_valid * J * 4);
    int64_t lo = o_begin;
    rsrc_t rs;
    auto set_block = [&]() {
        const bool live = lo < o_end && wave_live && rows_valid > 0;
        rs = make_rsrc(X + (live ? (lo * IR_in + r0 + wrow) * J + jw : 0), live ? rec_rows : 0u);
    };
    set_block();
    const bool jragged = jw + JW > J;
    uint32_t loff[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) loff[s] = (uint32_t)(((int64_t)(4 * h + s) * J + TJ * m) * 4);
    int ls = 0;
    // One step's loads.  PART (the last j tile of rows whose length J is not
    // a multiple of TJ) loads entry by entry, zeros past J, so no lane's
    // loads cross the row end; the two forms are separate copies of the
    // stream below, each with a fixed number of loads per step.
    auto load_step = [&](auto part_c, jv (&a)[4]) {
        constexpr bool PART = decltype(part_c)::value;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const uint32_t off = loff[s] + (uint32_t)(8 * ls * J * 4);
            if constexpr (!PART || TJ == 1) {
                a[s] = buf_loadj<TJ>(rs, (!jragged || jok) ? off : kNoLoad);
            } else {
#pragma unroll
                for (int t = 0; t < TJ; ++t)
                    jset<TJ>(a[s], t, buf_load1(rs, jw + TJ * m + t < J ? off + 4 * t : kNoLoad, 0.f));
            }
        }
        if (++ls == SPB) {
            ls = 0;
            ++lo;
            set_block();
        }
    };

    float *stab = tile + RP * PT;  // [scale_blocks<RP>()][RP]
    int64_t co = o_begin, tb0 = o_begin;
    int cs = 0;
    float scl[NC];
    f32x16 acc[TJ][NC];
#pragma unroll
    for (int t = 0; t < TJ; ++t)
#pragma unroll
        for (int nc = 0; nc < NC; ++nc) acc[t][nc] = f32x16{};
    const float *tb = tile + m * PT + wrow + 4 * h;
    auto load_scales = [&]() {
#pragma unroll
        for (int nc = 0; nc < NC; ++nc) scl[nc] = stab[(co - tb0) * RP + 32 * nc + m];
    };

    auto compute_step = [&](const jv (&a)[4]) {
        f32x4 b[NC];
#pragma unroll
        for (int nc = 0; nc < NC; ++nc)
            b[nc] = *reinterpret_cast<const f32x4 *>(tb + 32 * nc * PT + 8 * cs) * scl[nc];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int t = 0; t < TJ; ++t)
#pragma unroll
                for (int nc = 0; nc < NC; ++nc) acc[t][nc] = mfma32(jcomp<TJ>(a[s], t), b[nc][s], acc[t][nc]);
        if (++cs == SPB) {
            cs = 0;
            if (++co - tb0 < scale_blocks<RP>() && co < o_end) load_scales();
        }
    };

    auto stream = [&](auto part_c) {
        jv x[RING][4];
#pragma unroll
        for (int k = 0; k < RING - 1; ++k) load_step(part_c, x[k]);
        build_tile_batched<float, RP, 16>(kin, R, c0, r0, LC, IR_in,
                                          [&](int q, int c, float v) { tile[c * PT + q] = v; });
        fill_scales<RP>(kout, R, c0, o_begin, o_end, stab);
        for (; tb0 < o_end; tb0 += scale_blocks<RP>()) {
            if (tb0 != o_begin) fill_scales<RP>(kout, R, c0, tb0, o_end, stab);
            __syncthreads();
            co = tb0;
            load_scales();
            const int64_t nsteps = (min(o_end, tb0 + scale_blocks<RP>()) - tb0) * SPB;
            int64_t st = 0;
            for (; st + RING <= nsteps; st += RING) {
#pragma unroll
                for (int k = 0; k < RING; ++k) {
                    load_step(part_c, x[(k + RING - 1) % RING]);
                    compute_step(x[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < RING - 1; ++k)
                if (st + k < nsteps) compute_step(x[k]);
            __syncthreads();
        }
    };
    if (TJ > 1 && jragged && J % TJ != 0) stream(std::true_type{});
    else stream(std::false_type{});

    auto store = [&](int64_t jrow, int c, float v) {
        if (jrow < J && c < R) partial[((int64_t)blockIdx.y * J + jrow) * R + c] = v;
    };
    if (WR == 1) {
#pragma unroll
        for (int t = 0; t < TJ; ++t)
#pragma unroll
            for (int nc = 0; nc < NC; ++nc)
#pragma unroll
                for (int j = 0; j < 16; ++j) store(jw + TJ * acc32_row(lane, j) + t, c0 + 32 * nc + m, acc[t][nc][j]);
        return;
    }
    // Sum the WR waves that share j, in wave order, and store.
    __syncthreads();
    float *red = tile;  // [wave][t][nc][j][lane]
    constexpr int PER_WAVE = TJ * NC * 16 * 64;
#pragma unroll
    for (int t = 0; t < TJ; ++t)
#pragma unroll
        for (int nc = 0; nc < NC; ++nc)
#pragma unroll
            for (int j = 0; j < 16; ++j) red[wave * PER_WAVE + ((t * NC + nc) * 16 + j) * 64 + lane] = acc[t][nc][j];
    __syncthreads();
    for (int e = tid; e < WJ * PER_WAVE; e += kThreads) {
        const int g = e / PER_WAVE, r = e % PER_WAVE;  // j group (wave % WJ), element
        const int ln = r & 63, j = (r >> 6) & 15, tn = r >> 10;
        const int nc = tn % NC, t = tn / NC;
        const float *src = red + g * PER_WAVE + r;
        float sum = src[0];
#pragma unroll
        for (int w = 1; w < WR; ++w) sum += src[w * WJ * PER_WAVE];
        const int64_t j0 = (int64_t)blockIdx.x * JW * WJ + JW * g;
        store(j0 + TJ * acc32_row(ln, j) + t, c0 + 32 * nc + (ln & 31), sum);
    }
}

}  // namespace cpm
