// Kernels around MTTKRP for the CP-ALS update and the CP gradient
// (Section 2.2): float64 Gram matrices and their Hadamard product, a
// one-work-group Cholesky factorisation, row-parallel triangular solves,
// the gradient U_n H_n - M_n, the loss scalars, ||X||^2, the bf16 split of
// a float32 tensor and explicit Khatri-Rao rows.  Every reduction here runs
// in a fixed order, so results are reproducible run to run.
#pragma once

#include "device_common.hpp"

namespace cpm {

// Sets *flag = 0 (a kernel rather than a memset so the sequence can be
// captured into a graph).
__global__ void k_clear_status(int *flag) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *flag = 0;
}

__global__ void k_set_scalar(double *dst, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v;
}

// Partial Gram matrices of row blocks: part[b] = U_b^T U_b (R x R, float64)
// for rows [b*rows_per_block, (b+1)*rows_per_block) (grid.x = b).  Each
// thread owns a 4 x 4 tile of entries (grid.y takes groups of kThreads
// tiles), so a staged row costs 8 LDS reads for 16 multiply-adds.  The
// work-group stages its rows in LDS as float64 (row pitch R rounded up to 4,
// zero padded), and every entry is summed over the rows in row order.
constexpr int kGramStage = 4096;
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gram_partial(const T *__restrict__ U, int64_t I, int R,
                                                           int64_t rows_per_block, double *__restrict__ part) {
    __shared__ __attribute__((aligned(32))) double su[kGramStage];
    const int RP = (R + 3) & ~3;
    const int TR = RP / 4;                  // tiles per row of the Gram matrix
    const int SR = max(1, kGramStage / RP); // rows per stage
    const int64_t i0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t i1 = min(I, i0 + rows_per_block);
    const int t = (int)blockIdx.y * kThreads + threadIdx.x;
    const bool own = t < TR * TR;
    const int a0 = own ? 4 * (t / TR) : 0, c0 = own ? 4 * (t % TR) : 0;
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
    for (int64_t s0 = i0; s0 < i1; s0 += SR) {
        const int nr = (int)min((int64_t)SR, i1 - s0);
        __syncthreads();
        for (int e = threadIdx.x; e < nr * RP; e += kThreads) {
            const int r = e / RP, col = e - r * RP;
            su[e] = col < R ? (double)U[(s0 + r) * R + col] : 0.0;
        }
        __syncthreads();
        if (own) {
            for (int i = 0; i < nr; ++i) {
                double va[4], vc[4];
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    va[x] = su[i * RP + a0 + x];
                    vc[x] = su[i * RP + c0 + x];
                }
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] += va[x] * vc[y];
            }
        }
    }
    if (!own) return;
    double *dst = part + (int64_t)blockIdx.x * R * R;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
            if (a0 + x < R && c0 + y < R) dst[(a0 + x) * R + c0 + y] = acc[x][y];
}

// out[e] = sum_{b < nslices} part[b][e], in slice order.
__global__ __launch_bounds__(kThreads) void k_sum_slices(const double *__restrict__ part, int64_t nslices,
                                                         int64_t count, double *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= count) return;
    double s = 0.0;
    for (int64_t b = 0; b < nslices; ++b) s += part[b * count + e];
    out[e] = s;
}

// H = Hadamard product of grams[k] (R x R each) over k != skip.
__global__ __launch_bounds__(kThreads) void k_hadamard_except(const double *__restrict__ grams, int N, int R,
                                                              int skip, double *__restrict__ H) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= R * R) return;
    double v = 1.0;
    for (int k = 0; k < N; ++k)
        if (k != skip) v *= grams[(int64_t)k * R * R + e];
    H[e] = v;
}

// Cholesky H = L L^T of an R x R float64 matrix held in LDS by one work-group.
// Right-looking on the unscaled trailing matrix: step j subtracts
// A[i][j] A[k][j] / d_j from every (i, k) with k <= i in the trailing block
// (threads tile it 16 x 16), one barrier per step.  The pivot d_j = A[j][j]
// never changes after step j, so L is formed at the end as
// L[i][j] = A[i][j] / sqrt(d_j) (and L[j][j] = sqrt(d_j)).  Writes L
// (row-major, zero above the diagonal) and its transpose Lt.  If a pivot is
// not positive the factorisation stops and *status is set to 1 (it is never
// cleared here, so one failure in a sweep is remembered).
// H itself is formed on the way into LDS: the Hadamard product of grams[k]
// (N matrices of R x R) over k != skip.
__global__ __launch_bounds__(kThreads) void k_cholesky(const double *__restrict__ grams, int N, int skip, int R,
                                                       double *__restrict__ L, double *__restrict__ Lt,
                                                       int *__restrict__ status) {
    extern __shared__ double A[];  // R x R
    const int t = threadIdx.x, ti = t >> 4, tk = t & 15;
    for (int e = t; e < R * R; e += kThreads) {
        double v = 1.0;
        for (int k = 0; k < N; ++k)
            if (k != skip) v *= grams[(int64_t)k * R * R + e];
        A[e] = v;
    }
    __syncthreads();
    for (int j = 0; j < R; ++j) {
        const double d = A[j * R + j];
        if (!(d > 0.0)) {  // d is the same value in every thread: uniform exit
            if (t == 0) *status = 1;
            return;
        }
        const double inv = 1.0 / d;
        for (int i = j + 1 + ti; i < R; i += 16) {
            const double aij = A[i * R + j] * inv;
            for (int k = j + 1 + tk; k <= i; k += 16) A[i * R + k] -= aij * A[k * R + j];
        }
        __syncthreads();
    }
    for (int e = t; e < R * R; e += kThreads) {
        const int i = e / R, k = e % R;
        double v = 0.0;
        if (k == i) v = sqrt(A[e]);
        else if (k < i) v = A[e] / sqrt(A[k * R + k]);
        L[e] = v;
        Lt[k * R + i] = v;
    }
}

// Row-parallel solve x H = m for every row of M (H = L L^T): L y = m^T then
// L^T x^T = y.  One wave per row, rows_per_wave rows in turn; lane k holds
// entries k and k + 64 (R <= 128).  With LDS_L the work-group first copies L
// and L^T into LDS (2 R^2 doubles), so the 2R dependent steps of a row read
// LDS instead of memory.  Skipped entirely when *status is set, leaving out
// untouched.
template <typename T, bool LDS_L>
__global__ __launch_bounds__(kThreads) void k_chol_solve_rows(const double *__restrict__ Lg,
                                                              const double *__restrict__ Ltg,
                                                              const int *__restrict__ status,
                                                              const T *__restrict__ M, int64_t In, int R,
                                                              int rows_per_wave, T *__restrict__ out) {
    if (*status) return;
    extern __shared__ double sl[];
    const double *L = Lg, *Lt = Ltg;
    if (LDS_L) {
        for (int e = threadIdx.x; e < R * R; e += kThreads) {
            sl[e] = Lg[e];
            sl[R * R + e] = Ltg[e];
        }
        __syncthreads();
        L = sl;
        Lt = sl + R * R;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int k0 = lane, k1 = lane + 64;
    // each lane holds the reciprocal pivots of its own entries, so step j
    // takes lane j's value already divided: one multiply and one shuffle on
    // the dependent chain instead of a float64 division and an LDS read
    const double r0 = (k0 < R) ? 1.0 / L[k0 * R + k0] : 0.0;
    const double r1 = (k1 < R) ? 1.0 / L[k1 * R + k1] : 0.0;
    for (int rr = 0; rr < rows_per_wave; ++rr) {
        const int64_t row = ((int64_t)blockIdx.x * 4 + wave) * rows_per_wave + rr;
        if (row >= In) break;
        double v0 = (k0 < R) ? (double)M[row * R + k0] : 0.0;
        double v1 = (k1 < R) ? (double)M[row * R + k1] : 0.0;
        for (int j = 0; j < R; ++j) {  // forward: column j of L is row j of Lt
            const double src = (j < 64) ? v0 * r0 : v1 * r1;
            const double yj = __shfl(src, j & 63);
            if (j < 64) { if (lane == j) v0 = yj; } else { if (lane == j - 64) v1 = yj; }
            const double *col = Lt + (int64_t)j * R;
            if (k0 > j && k0 < R) v0 -= col[k0] * yj;
            if (k1 > j && k1 < R) v1 -= col[k1] * yj;
        }
        for (int j = R - 1; j >= 0; --j) {  // backward: column j of L^T is row j of L
            const double src = (j < 64) ? v0 * r0 : v1 * r1;
            const double xj = __shfl(src, j & 63);
            if (j < 64) { if (lane == j) v0 = xj; } else { if (lane == j - 64) v1 = xj; }
            const double *rowL = L + (int64_t)j * R;
            if (k0 < j) v0 -= rowL[k0] * xj;
            if (k1 < j && k1 < R) v1 -= rowL[k1] * xj;
        }
        if (k0 < R) out[row * R + k0] = (T)v0;
        if (k1 < R) out[row * R + k1] = (T)v1;
    }
}

// grad[i][c] = sum_d U[i][d] H[d][c] - M[i][c], in float64.  A work-group
// owns 64 consecutive outputs (one per lane); its 4 waves take the four
// quarters of the d range and their sums are added in wave order.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_grad(const T *__restrict__ U, const double *__restrict__ H,
                                                   const T *__restrict__ M, int64_t In, int R,
                                                   T *__restrict__ G) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t e = (int64_t)blockIdx.x * 64 + lane;
    const int q = (R + 3) / 4;
    const int d0 = wave * q, d1 = min(R, d0 + q);
    double s = 0.0;
    if (e < In * R) {
        const int64_t i = e / R;
        const int c = (int)(e % R);
        for (int d = d0; d < d1; ++d) s += (double)U[i * R + d] * H[d * R + c];
    }
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && e < In * R)
        G[e] = (T)((((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]) - (double)M[e]);
}

// Fixed-order block sum of 256 per-thread doubles; valid in thread 0.
__device__ inline double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    return sh[0];
}

// part[block] = sum over the block's grid-stride share of a[e] * b[e], in
// float64 (a fixed split; k_sum_vector then adds the parts in order).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dot_partial(const T *__restrict__ a, const T *__restrict__ b,
                                                          int64_t n, double *__restrict__ part) {
    __shared__ double sh[kThreads];
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride)
        s += (double)a[e] * (double)b[e];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// part[block] = sum over the block's grid-stride share of the entries e of
// prod_k G_k[e] (the Hadamard product of all Grams), in float64: a fixed
// split, added in order by k_loss.
__global__ __launch_bounds__(kThreads) void k_hadsum_partial(const double *__restrict__ grams, int N, int R,
                                                             double *__restrict__ part) {
    __shared__ double sh[kThreads];
    const int64_t RR = (int64_t)R * R;
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < RR; e += (int64_t)gridDim.x * kThreads) {
        double v = 1.0;
        for (int k = 0; k < N; ++k) v *= grams[k * RR + e];
        s += v;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// f = 1/2 (||X||^2 - 2 <M_{N-1}, U_{N-1}> + sum_ab prod_k G_k[a][b]), the
// last sum given as nparts partial sums; with want_fit the result is
// 1 - sqrt(max(0, 2 f)) / sqrt(||X||^2) instead.
__global__ void k_loss(const double *__restrict__ xnorm2, const double *__restrict__ inner,
                       const double *__restrict__ hpart, int nparts, int want_fit, double *__restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += hpart[b];
    const double f = 0.5 * (*xnorm2 - 2.0 * *inner + s);
    *out = want_fit ? 1.0 - sqrt(fmax(0.0, 2.0 * f)) / sqrt(*xnorm2) : f;
}

// Per-block partial sums of squares of the tensor entries (bf16 pairs are
// widened to hi + lo, which is exact in float32).  With vec (16-byte aligned
// data, I a multiple of 8) the entries are read 16 bytes at a time: groups of
// 4 floats, or 8 hi and 8 lo values.  A fixed split, summed in float64.
template <int DT>
__global__ __launch_bounds__(kThreads) void k_sumsq_partial(const void *__restrict__ Xv, int64_t I, int vec,
                                                            double *__restrict__ part) {
    __shared__ double sh[kThreads];
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    const int64_t t0 = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (vec && DT == CPM_F32) {
        const f32x4 *x4 = (const f32x4 *)Xv;
        for (int64_t g = t0; g < I / 4; g += stride) {
            const f32x4 v = x4[g];
            s += (double)v[0] * v[0] + (double)v[1] * v[1] + (double)v[2] * v[2] + (double)v[3] * v[3];
        }
    } else if (vec && DT == CPM_BF16X2) {
        const u16x8 *h8 = (const u16x8 *)Xv;
        const u16x8 *l8 = (const u16x8 *)((const uint16_t *)Xv + I);
        for (int64_t g = t0; g < I / 8; g += stride) {
            const u16x8 h = h8[g], l = l8[g];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const double x = (double)(bf16_bits_to_float(h[e]) + bf16_bits_to_float(l[e]));
                s += x * x;
            }
        }
    } else {
        for (int64_t e = t0; e < I; e += stride) {
            double x;
            if (DT == CPM_F32) {
                x = (double)((const float *)Xv)[e];
            } else if (DT == CPM_F64) {
                x = ((const double *)Xv)[e];
            } else {
                const uint16_t *p = (const uint16_t *)Xv;
                x = (double)(bf16_bits_to_float(p[e]) + bf16_bits_to_float(p[I + e]));
            }
            s += x * x;
        }
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_sum_vector(const double *__restrict__ part, int n,
                                                         double *__restrict__ out) {
    __shared__ double sh[kThreads];
    double s = 0.0;
    for (int e = threadIdx.x; e < n; e += kThreads) s += part[e];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) *out = s;
}

// hi = RNE(x), lo = RNE(x - hi): the bf16 pair format.  With vec8 (x 16-byte
// aligned and n a multiple of 8, so both planes are 16-byte aligned too) each
// thread converts groups of 8 values: two 16-byte loads, one 16-byte store
// per plane.
__device__ inline void split_one(float v, uint16_t &h, uint16_t &l) {
    h = bf16_rne_bits(v);
    l = bf16_rne_bits(v - bf16_bits_to_float(h));
}
__global__ __launch_bounds__(kThreads) void k_split_bf16(const float *__restrict__ x, int64_t n, int vec8,
                                                         uint16_t *__restrict__ planes) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    const int64_t t0 = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (vec8) {
        const f32x4 *x4 = reinterpret_cast<const f32x4 *>(x);
        u16x8 *hi8 = reinterpret_cast<u16x8 *>(planes);
        u16x8 *lo8 = reinterpret_cast<u16x8 *>(planes + n);
        auto convert = [&](const f32x4 &a, const f32x4 &b, int64_t g) {
            u16x8 h, l;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                uint16_t hh, ll;
                split_one(a[e], hh, ll);
                h[e] = hh;
                l[e] = ll;
                split_one(b[e], hh, ll);
                h[4 + e] = hh;
                l[4 + e] = ll;
            }
            hi8[g] = h;
            lo8[g] = l;
        };
        const int64_t n8 = n / 8;
        int64_t g = t0;
        // two groups (four 16-byte loads) in flight per thread, then the tail
        for (; g + stride < n8; g += 2 * stride) {
            const f32x4 a0 = x4[2 * g], b0 = x4[2 * g + 1];
            const f32x4 a1 = x4[2 * (g + stride)], b1 = x4[2 * (g + stride) + 1];
            convert(a0, b0, g);
            convert(a1, b1, g + stride);
        }
        for (; g < n8; g += stride) convert(x4[2 * g], x4[2 * g + 1], g);
        return;
    }
    for (int64_t e = t0; e < n; e += stride) {
        uint16_t h, l;
        split_one(x[e], h, l);
        planes[e] = h;
        planes[n + e] = l;
    }
}

// Explicit rows [j0, j0 + nrows) of a Khatri-Rao product, built by the same
// row builder the MTTKRP kernels use; 64 rows per block.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_krp_rows(Krp<T> k, int R, int RP, int64_t j0, int64_t nrows,
                                                       T *__restrict__ out) {
    const int64_t q0 = (int64_t)blockIdx.x * 64;
    const int cnt = (int)min((int64_t)64, nrows - q0);
    build_krp_rows<T>(k, R, 0, RP, j0 + q0, cnt, j0 + nrows, [&](int q, int c, T v) {
        if (c < R) out[(q0 + q) * R + c] = v;
    });
}

}  // namespace cpm
