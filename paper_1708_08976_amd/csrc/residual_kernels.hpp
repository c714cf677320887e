// Squared residual ||X - [[U_0..U_{N-1}]]||_F^2 of a CP model, with the model
// entries recomputed on the fly from the factors (the CP model of Section
// 2.2) while X streams past once.  Nothing of the residual is stored.  The
// paper's Conclusion names this computation as the next bottleneck of CP-ALS
// once MTTKRP is fast; here it is one pass over X at MTTKRP cost, and it
// replaces the identity ||X||^2 - 2 <M, U> + sum(Hadamard of Grams), whose
// cancellation costs about log10(||X||^2 / ||X - Y||^2) digits.
//
// X is viewed as Rr rows (the modes s..N-1, slow) of L contiguous entries
// (the modes 0..s-1): Y(r, l) = sum_c K_R(r, c) K_L(l, c), with the same
// inner/outer split of K_L as the MTTKRP kernels, K_L(g + G_in o, c) =
// K_in(g, c) S(o, c).  A 32 x 32 tile of Y is one chain of R/2 MFMAs
// (32x32x2 f32): A = 32 rows of K_R scaled by S(o, :), B = 32 rows of the
// resident K_in tile.  The X entries are loaded straight into the MFMA
// output layout, and the squared differences are formed and summed in
// float64.
#pragma once

#include "als_kernels.hpp"
#include "device_common.hpp"

namespace cpm {

constexpr int kResRows = 128;  // rows of K_R per work-group: 32 per wave

template <int RP>
__host__ __device__ constexpr size_t residual_lds_bytes(int LC) {
    return (size_t)4 * ((size_t)kResRows * (RP + 4) + (size_t)LC * (RP + 4)) + (size_t)kScaleTableBytes;
}

// One work-group per (row tile of kResRows rows r, chunk [LC * ch, LC * (ch +
// 1)) of the inner range G_in, range of bps outer blocks), flattened into
// blockIdx.x = (split * nlc + ch) * ntiles + tile; partial gets one float64
// per work-group at that index.
// BF: X is the split-bf16 pair (hi plane of I entries, then lo plane).
//
// LDS: the K_R tile [kResRows][RP + 4] and the K_in tile [LC][RP + 4], both
// with the rank index permuted to c' = (c & 1) * RP/2 + c / 2, so that a
// lane's operands for four consecutive MFMA steps (c = 2t + lane/32, t..t+3)
// are one 16-byte read; the pitch RP + 4 (4 words mod 32) makes those reads
// conflict-free.  Then the scale table [blocks][RP] (natural order).
template <int RP, bool BF>
__global__ __launch_bounds__(kThreads) void k_residual32(const void *__restrict__ Xv, int64_t I, int64_t Rr,
                                                         int64_t L, int64_t G_in, int64_t n_outer, Krp<float> kr,
                                                         Krp<float> kin, Krp<float> kout, int R, int LC,
                                                         int64_t ntiles, int64_t nlc, int64_t bps,
                                                         double *__restrict__ partial) {
    constexpr int NT = RP / 2;  // MFMA steps (two rank columns each)
    constexpr int PT = RP + 4;
    constexpr int NBLK = scale_blocks<RP>();
    extern __shared__ __attribute__((aligned(16))) float smem[];
    float *krt = smem;
    float *kbt = krt + kResRows * PT;
    float *stab = kbt + LC * PT;
    __shared__ double red[kThreads];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = lane >> 5;
    const int64_t tile = (int64_t)blockIdx.x % ntiles;
    const int64_t rest = (int64_t)blockIdx.x / ntiles;
    const int64_t r0 = tile * kResRows;
    const int64_t g0 = (rest % nlc) * LC;
    const int64_t o_begin = (rest / nlc) * bps;
    const int64_t o_end = o_begin + bps < n_outer ? o_begin + bps : n_outer;
    const int glen = (int)(G_in - g0 < LC ? G_in - g0 : LC);  // valid inner entries of the chunk

    auto perm = [](int c) { return (c & 1) * (RP / 2) + (c >> 1); };
    build_tile_batched<float, RP, 8>(kr, R, 0, r0, kResRows, Rr,
                                     [&](int q, int c, float v) { krt[q * PT + perm(c)] = v; });
    build_tile_batched<float, RP, 8>(kin, R, 0, g0, LC, G_in,
                                     [&](int q, int c, float v) { kbt[q * PT + perm(c)] = v; });

    // This wave's 32 rows r = rbase + acc32_row(lane, j), read through a
    // buffer resource that ends at the last valid row: rows past Rr and
    // columns past the chunk (offset kNoLoad) read zero, with no branch
    // around the loads.  Row offsets stay below 32 L entries (the plan keeps
    // 128 L bytes within the 32-bit offset range).
    const int64_t rbase = r0 + 32 * wave;
    const int64_t vr = Rr - rbase < 32 ? (Rr - rbase > 0 ? Rr - rbase : 0) : 32;
    constexpr int ES = BF ? 2 : 4;
    const char *xb = reinterpret_cast<const char *>(Xv);
    const rsrc_t rx = make_rsrc(xb + rbase * L * ES, (uint32_t)(vr * L * ES));
    const rsrc_t rlo = make_rsrc(xb + (I + rbase * L) * ES, (uint32_t)(vr * L * ES));
    const int tpc = (glen + 31) / 32;  // 32-column tiles per block
    auto load_tile = [&](int64_t o, int jt, float (&x)[16]) {
        const int gl = jt * 32 + (lane & 31);
        const uint32_t col = (uint32_t)(o * G_in + g0 + gl);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const uint32_t off = gl < glen ? ((uint32_t)acc32_row(lane, j) * (uint32_t)L + col) * ES : kNoLoad;
            if (BF) {
                const uint16_t hb = __builtin_amdgcn_raw_buffer_load_b16(rx, off, 0, 0);
                const uint16_t lb = __builtin_amdgcn_raw_buffer_load_b16(rlo, off, 0, 0);
                x[j] = bf16_bits_to_float(hb) + bf16_bits_to_float(lb);
            } else {
                x[j] = buf_load1<kStream>(rx, off, 0.f);
            }
        }
    };
    double sum = 0.0;

    for (int64_t tb0 = o_begin; tb0 < o_end; tb0 += NBLK) {
        const int64_t tb1 = tb0 + NBLK < o_end ? tb0 + NBLK : o_end;
        float xn[16];
        load_tile(tb0, 0, xn);  // the first tile's X is in flight across the refill
        __syncthreads();
        fill_scales<RP>(kout, R, 0, tb0, o_end, stab);
        __syncthreads();
        for (int64_t o = tb0; o < tb1; ++o) {
            // A operands for this block: K_R(r, c) * S(o, c), c = 2t + h
            float a[NT];
            const float *arow = krt + (32 * wave + (lane & 31)) * PT + h * (RP / 2);
            const float *srow = stab + (o - tb0) * RP;
#pragma unroll
            for (int t = 0; t < NT; t += 4) {
                const f32x4 v = *reinterpret_cast<const f32x4 *>(arow + t);
#pragma unroll
                for (int u = 0; u < 4; ++u) a[t + u] = v[u] * srow[2 * (t + u) + h];
            }
            for (int jt = 0; jt < tpc; ++jt) {
                float x[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) x[j] = xn[j];
                // prefetch the next tile of the chunk while this one computes
                const bool more = jt + 1 < tpc || o + 1 < tb1;
                if (more) load_tile(jt + 1 < tpc ? o : o + 1, jt + 1 < tpc ? jt + 1 : 0, xn);
                const int gl = jt * 32 + (lane & 31);
                f32x16 acc = {};
                const float *brow = kbt + gl * PT + h * (RP / 2);
#pragma unroll
                for (int t = 0; t < NT; t += 4) {
                    const f32x4 b = *reinterpret_cast<const f32x4 *>(brow + t);
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc = mfma32(a[t + u], b[u], acc);
                }
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const double d = (double)x[j] - (double)acc[j];
                    sum += d * d;
                }
            }
        }
    }
    sum = block_sum(sum, red);
    if (tid == 0) partial[blockIdx.x] = sum;
}

}  // namespace cpm
