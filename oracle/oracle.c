/*
 * Reference oracle for dense MTTKRP, CP-ALS and the CP least-squares gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously correct
 * CPU implementation that the GPU library is checked against.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or helper with the HIP library.
 *
 * Everything is computed in IEEE double precision, straight from the
 * definitions of the paper (Hayashi, Ballard, Jiang, Tobia, "Shared-Memory
 * Parallelization of MTTKRP for Dense Tensors", 2018):
 *
 *   - storage order: the natural linearisation of Section 2.1 (Notation),
 *     l = sum_n i_n * prod_{k<n} I_k, so mode 0 is the fastest index;
 *   - MTTKRP: the first bullet of Section 2.2 (CP Decomposition),
 *     M = X_(n) (U_{N-1} kr ... kr U_{n+1} kr U_{n-1} kr ... kr U_0),
 *     evaluated entry by entry as
 *       M(i_n, c) = sum over all entries with mode-n index i_n of
 *                   X(i_0..i_{N-1}) * prod_{k != n} U_k(i_k, c);
 *   - Khatri-Rao product rows: the row-wise definition of Section 2.1,
 *     K(r_B + r_A I_B, :) = A(r_A, :) * B(r_B, :);
 *   - CP-ALS factor update: the three operations of Section 2.2 (MTTKRP,
 *     Hadamard product of Gram matrices, linear solve), with the solve done
 *     by Cholesky factorisation in double precision (the paper writes a
 *     pseudo-inverse; for a positive-definite H the two agree, and a
 *     non-positive-definite H is reported as an error instead);
 *   - CP gradient: Section 2.2 notes that MTTKRP is part of the gradient; for
 *     f = 1/2 ||X - [[U_0..U_{N-1}]]||_F^2 the gradient with respect to U_n is
 *     U_n * H_n - MTTKRP_n with H_n the Hadamard product of the other Grams.
 *
 * Factor matrices are I_k x R, row-major (R contiguous).  MTTKRP outputs and
 * gradients are I_n x R, row-major.  The tensor may be given as float32,
 * float64 or a pair of bfloat16 planes (hi plane followed by lo plane, the
 * value being hi + lo); every entry is widened exactly to double.
 *
 * Parallel loops use OpenMP over fixed contiguous chunks of the storage order
 * with private double accumulators that are summed in chunk order, so the
 * result is deterministic for a fixed thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_F32 = 0, OR_F64 = 1, OR_BF16PAIR = 2 };
enum { OR_OK = 0, OR_EINVAL = 1, OR_ENOTPD = 3, OR_ENOMEM = 6 };

/* Exact widening of one stored tensor entry to double. */
static double load_entry(const void *X, int xtype, int64_t total, int64_t l)
{
    if (xtype == OR_F32) return (double)((const float *)X)[l];
    if (xtype == OR_F64) return ((const double *)X)[l];
    /* bfloat16 pair: a bfloat16 is the upper half of a float32 bit pattern. */
    const uint16_t *p = (const uint16_t *)X;
    uint32_t hb = (uint32_t)p[l] << 16, lb = (uint32_t)p[total + l] << 16;
    float hf, lf;
    memcpy(&hf, &hb, 4);
    memcpy(&lf, &lb, 4);
    return (double)hf + (double)lf;
}

static int num_threads(int req)
{
#ifdef _OPENMP
    return req > 0 ? req : omp_get_max_threads();
#else
    (void)req;
    return 1;
#endif
}

static int check_dims(const int64_t *dims, int N, int R, int64_t *total)
{
    if (N < 1 || N > 64 || R < 1 || !dims) return 0;
    int64_t t = 1;
    for (int k = 0; k < N; ++k) {
        if (dims[k] < 1) return 0;
        if (t > ((int64_t)1 << 62) / dims[k]) return 0;
        t *= dims[k];
    }
    *total = t;
    return 1;
}

/* Multi-index of linear position l in the natural linearisation. */
static void decode(int64_t l, const int64_t *dims, int N, int64_t *idx)
{
    for (int k = 0; k < N; ++k) {
        idx[k] = l % dims[k];
        l /= dims[k];
    }
}

/* Move a multi-index one step forward in storage order (mode 0 fastest). */
static void advance(int64_t *idx, const int64_t *dims, int N)
{
    for (int k = 0; k < N; ++k) {
        if (++idx[k] < dims[k]) return;
        idx[k] = 0;
    }
}

/*
 * Full mode-n MTTKRP from the definition.  out is I_n x R, overwritten.
 */
int oracle_mttkrp(const void *X, int xtype, const int64_t *dims, int N,
                  const double *const *U, int R, int mode, double *out, int nthreads)
{
    int64_t total;
    if (!X || !U || !out || !check_dims(dims, N, R, &total) || mode < 0 || mode >= N)
        return OR_EINVAL;
    int T = num_threads(nthreads);
    int64_t In = dims[mode];
    double *priv = (double *)calloc((size_t)T * (size_t)In * (size_t)R, sizeof(double));
    if (!priv) return OR_ENOMEM;
#pragma omp parallel num_threads(T)
    {
#ifdef _OPENMP
        int t = omp_get_thread_num();
        int nt = omp_get_num_threads();
#else
        int t = 0, nt = 1;
#endif
        int64_t chunk = (total + nt - 1) / nt;
        int64_t lo = (int64_t)t * chunk, hi = lo + chunk < total ? lo + chunk : total;
        double *acc = priv + (size_t)t * (size_t)In * (size_t)R;
        double *w = (double *)malloc(sizeof(double) * (size_t)R);
        int64_t idx[64];
        if (lo < hi) decode(lo, dims, N, idx);
        for (int64_t l = lo; l < hi; ++l) {
            double x = load_entry(X, xtype, total, l);
            for (int c = 0; c < R; ++c) w[c] = x;
            for (int k = 0; k < N; ++k) {
                if (k == mode) continue;
                const double *row = U[k] + idx[k] * R;
                for (int c = 0; c < R; ++c) w[c] *= row[c];
            }
            double *o = acc + idx[mode] * R;
            for (int c = 0; c < R; ++c) o[c] += w[c];
            advance(idx, dims, N);
        }
        free(w);
    }
    for (int64_t e = 0; e < In * R; ++e) {
        double s = 0.0;
        for (int t = 0; t < T; ++t) s += priv[(size_t)t * (size_t)In * (size_t)R + e];
        out[e] = s;
    }
    free(priv);
    return OR_OK;
}

/*
 * Symmetric-pair packed storage.  A tensor whose first two modes have equal
 * size n and X(i, j, rest) = X(j, i, rest) is stored as its triangle i <= j:
 * the pair (i, j) becomes one index p = j (j + 1) / 2 + i (i fastest, then
 * j, the natural linearisation restricted to the triangle), and the packed
 * tensor has modes (p, I_2, ..., I_{N-1}) in natural order, P = n (n + 1) / 2
 * pairs.  Section 5.3.3 stores the region-by-region correlation pair of its
 * fMRI tensor this way (as one linearised triangle of about half the
 * entries); the diagonal is kept here so the packed tensor represents the
 * whole symmetric tensor.
 *
 * Pair (i, j) of packed index p.
 */
static void pair_of(int64_t p, int64_t *i, int64_t *j)
{
    int64_t jj = 0;
    while ((jj + 1) * (jj + 2) / 2 <= p) ++jj;
    *j = jj;
    *i = p - jj * (jj + 1) / 2;
}

/*
 * Mode-n MTTKRP of the full symmetric tensor represented by the packed
 * tensor Xp, from the definition of Section 2.2: every packed entry stands
 * for the full-tensor entries (i, j, rest) and, when i != j, (j, i, rest),
 * each of which adds X * prod_{k != n} U_k(idx_k, :) to row idx_n.
 * dims are the full tensor's (dims[0] == dims[1]); out is I_n x R.
 */
int oracle_mttkrp_sympair(const void *Xp, int xtype, const int64_t *dims, int N,
                          const double *const *U, int R, int mode, double *out, int nthreads)
{
    int64_t total;
    if (!Xp || !U || !out || N < 3 || !check_dims(dims, N, R, &total) || mode < 0 || mode >= N ||
        dims[0] != dims[1])
        return OR_EINVAL;
    const int64_t n = dims[0], P = n * (n + 1) / 2;
    const int64_t rest = total / (n * n), ptotal = P * rest;
    int T = num_threads(nthreads);
    int64_t In = dims[mode];
    double *priv = (double *)calloc((size_t)T * (size_t)In * (size_t)R, sizeof(double));
    if (!priv) return OR_ENOMEM;
#pragma omp parallel num_threads(T)
    {
#ifdef _OPENMP
        int t = omp_get_thread_num();
        int nt = omp_get_num_threads();
#else
        int t = 0, nt = 1;
#endif
        int64_t chunk = (ptotal + nt - 1) / nt;
        int64_t lo = (int64_t)t * chunk, hi = lo + chunk < ptotal ? lo + chunk : ptotal;
        double *acc = priv + (size_t)t * (size_t)In * (size_t)R;
        double *w = (double *)malloc(sizeof(double) * (size_t)R);
        int64_t idx[64];
        for (int64_t l = lo; l < hi; ++l) {
            double x = load_entry(Xp, xtype, ptotal, l);
            int64_t i, j;
            pair_of(l % P, &i, &j);
            decode(l / P, dims + 2, N - 2, idx + 2);
            for (int copy = 0; copy < (i == j ? 1 : 2); ++copy) {
                idx[0] = copy ? j : i;
                idx[1] = copy ? i : j;
                for (int c = 0; c < R; ++c) w[c] = x;
                for (int k = 0; k < N; ++k) {
                    if (k == mode) continue;
                    const double *row = U[k] + idx[k] * R;
                    for (int c = 0; c < R; ++c) w[c] *= row[c];
                }
                double *o = acc + idx[mode] * R;
                for (int c = 0; c < R; ++c) o[c] += w[c];
            }
        }
        free(w);
    }
    for (int64_t e = 0; e < In * R; ++e) {
        double s = 0.0;
        for (int t = 0; t < T; ++t) s += priv[(size_t)t * (size_t)In * (size_t)R + e];
        out[e] = s;
    }
    free(priv);
    return OR_OK;
}

/*
 * Selected rows of the mode-n MTTKRP: out[q][c] = M(rows[q], c).  Each row
 * is a sum over the entries whose mode-n index equals rows[q]; this serves
 * sampled checks on tensors too large for a full oracle pass.
 */
int oracle_mttkrp_rows(const void *X, int xtype, const int64_t *dims, int N,
                       const double *const *U, int R, int mode,
                       const int64_t *rows, int64_t nrows, double *out, int nthreads)
{
    int64_t total;
    if (!X || !U || !out || !rows || !check_dims(dims, N, R, &total) || mode < 0 || mode >= N)
        return OR_EINVAL;
    int64_t In = dims[mode];
    for (int64_t q = 0; q < nrows; ++q)
        if (rows[q] < 0 || rows[q] >= In) return OR_EINVAL;
    int64_t left = 1;
    for (int k = 0; k < mode; ++k) left *= dims[k];
    int64_t rest = total / In; /* entries per row of the unfolding */
    int T = num_threads(nthreads);
    double *priv = (double *)calloc((size_t)T * (size_t)R, sizeof(double));
    if (!priv) return OR_ENOMEM;
    for (int64_t q = 0; q < nrows; ++q) {
        memset(priv, 0, sizeof(double) * (size_t)T * (size_t)R);
#pragma omp parallel num_threads(T)
        {
#ifdef _OPENMP
            int t = omp_get_thread_num();
            int nt = omp_get_num_threads();
#else
            int t = 0, nt = 1;
#endif
            int64_t chunk = (rest + nt - 1) / nt;
            int64_t lo = (int64_t)t * chunk, hi = lo + chunk < rest ? lo + chunk : rest;
            double *acc = priv + (size_t)t * (size_t)R;
            double *w = (double *)malloc(sizeof(double) * (size_t)R);
            int64_t idx[64];
            for (int64_t j = lo; j < hi; ++j) {
                /* column j of X_(n): the remaining modes in natural order */
                int64_t jl = j % left, jr = j / left;
                int64_t l = jl + rows[q] * left + jr * left * In;
                decode(l, dims, N, idx);
                double x = load_entry(X, xtype, total, l);
                for (int c = 0; c < R; ++c) w[c] = x;
                for (int k = 0; k < N; ++k) {
                    if (k == mode) continue;
                    const double *row = U[k] + idx[k] * R;
                    for (int c = 0; c < R; ++c) w[c] *= row[c];
                }
                for (int c = 0; c < R; ++c) acc[c] += w[c];
            }
            free(w);
        }
        for (int c = 0; c < R; ++c) {
            double s = 0.0;
            for (int t = 0; t < T; ++t) s += priv[(size_t)t * (size_t)R + c];
            out[q * R + c] = s;
        }
    }
    free(priv);
    return OR_OK;
}

/*
 * Rows [j0, j0+nrows) of the Khatri-Rao product A_0 kr A_1 kr ... kr A_{Z-1}
 * (A_z is J_z x R, row-major), by the row-wise definition of Section 2.1:
 * the last matrix's row index varies fastest.  out is nrows x R.
 */
int oracle_krp_rows(const double *const *A, const int64_t *J, int Z, int R,
                    int64_t j0, int64_t nrows, double *out)
{
    if (!A || !J || !out || Z < 1 || R < 1 || j0 < 0 || nrows < 0) return OR_EINVAL;
    int64_t rows = 1;
    for (int z = 0; z < Z; ++z) {
        if (J[z] < 1) return OR_EINVAL;
        rows *= J[z];
    }
    if (j0 + nrows > rows) return OR_EINVAL;
    for (int64_t q = 0; q < nrows; ++q) {
        int64_t j = j0 + q;
        for (int c = 0; c < R; ++c) out[q * R + c] = 1.0;
        for (int z = Z - 1; z >= 0; --z) {
            int64_t rz = j % J[z];
            j /= J[z];
            for (int c = 0; c < R; ++c) out[q * R + c] *= A[z][rz * R + c];
        }
    }
    return OR_OK;
}

/* Gram matrix G = U^T U (R x R) of an I x R row-major factor. */
static void gram(const double *U, int64_t I, int R, double *G)
{
    for (int a = 0; a < R; ++a)
        for (int b = 0; b < R; ++b) {
            double s = 0.0;
            for (int64_t i = 0; i < I; ++i) s += U[i * R + a] * U[i * R + b];
            G[a * R + b] = s;
        }
}

/* H = Hadamard product of the Grams of all factors except mode `skip`
 * (skip = -1 keeps all of them). */
static void hadamard_grams(const double *const *U, const int64_t *dims, int N, int R,
                           int skip, double *H, double *G)
{
    for (int e = 0; e < R * R; ++e) H[e] = 1.0;
    for (int k = 0; k < N; ++k) {
        if (k == skip) continue;
        gram(U[k], dims[k], R, G);
        for (int e = 0; e < R * R; ++e) H[e] *= G[e];
    }
}

/* In-place Cholesky H = L L^T (lower triangle kept).  Returns 0 when H is
 * not positive definite. */
static int cholesky(double *H, int R)
{
    for (int j = 0; j < R; ++j) {
        double d = H[j * R + j];
        for (int k = 0; k < j; ++k) d -= H[j * R + k] * H[j * R + k];
        if (!(d > 0.0)) return 0;
        d = sqrt(d);
        H[j * R + j] = d;
        for (int i = j + 1; i < R; ++i) {
            double s = H[i * R + j];
            for (int k = 0; k < j; ++k) s -= H[i * R + k] * H[j * R + k];
            H[i * R + j] = s / d;
        }
    }
    return 1;
}

/* Solve x H = m for every row (H = L L^T): forward then backward substitution. */
static void chol_solve_rows(const double *L, int R, const double *M, int64_t rows, double *out)
{
    double *y = (double *)malloc(sizeof(double) * (size_t)R);
    for (int64_t i = 0; i < rows; ++i) {
        const double *m = M + i * R;
        for (int j = 0; j < R; ++j) {
            double s = m[j];
            for (int k = 0; k < j; ++k) s -= L[j * R + k] * y[k];
            y[j] = s / L[j * R + j];
        }
        double *x = out + i * R;
        for (int j = R - 1; j >= 0; --j) {
            double s = y[j];
            for (int k = j + 1; k < R; ++k) s -= L[k * R + j] * x[k];
            x[j] = s / L[j * R + j];
        }
    }
    free(y);
}

/* ||X||_F^2 in double. */
double oracle_xnorm2(const void *X, int xtype, const int64_t *dims, int N)
{
    int64_t total;
    if (!X || !check_dims(dims, N, 1, &total)) return -1.0;
    double s = 0.0;
    for (int64_t l = 0; l < total; ++l) {
        double x = load_entry(X, xtype, total, l);
        s += x * x;
    }
    return s;
}

/* ||X - [[U_0..U_{N-1}]]||_F^2 computed entry by entry from the CP model of
 * Section 2.2 (each model entry is sum_c prod_k U_k(i_k, c)). */
double oracle_residual2(const void *X, int xtype, const int64_t *dims, int N,
                        const double *const *U, int R, int nthreads)
{
    int64_t total;
    if (!X || !U || !check_dims(dims, N, R, &total)) return -1.0;
    int T = num_threads(nthreads);
    double *part = (double *)calloc((size_t)T, sizeof(double));
#pragma omp parallel num_threads(T)
    {
#ifdef _OPENMP
        int t = omp_get_thread_num();
        int nt = omp_get_num_threads();
#else
        int t = 0, nt = 1;
#endif
        int64_t chunk = (total + nt - 1) / nt;
        int64_t lo = (int64_t)t * chunk, hi = lo + chunk < total ? lo + chunk : total;
        int64_t idx[64];
        double s = 0.0;
        if (lo < hi) decode(lo, dims, N, idx);
        for (int64_t l = lo; l < hi; ++l) {
            double y = 0.0;
            for (int c = 0; c < R; ++c) {
                double p = 1.0;
                for (int k = 0; k < N; ++k) p *= U[k][idx[k] * R + c];
                y += p;
            }
            double d = load_entry(X, xtype, total, l) - y;
            s += d * d;
            advance(idx, dims, N);
        }
        part[t] = s;
    }
    double s = 0.0;
    for (int t = 0; t < T; ++t) s += part[t];
    free(part);
    return s;
}

/*
 * One CP-ALS sweep (Section 2.2), modes updated in order 0..N-1, each with
 * the factors already updated earlier in the sweep.  U is in/out.  On a
 * non-positive-definite H the factors are restored to their input values
 * and OR_ENOTPD is returned.  If fit_out is non-null it receives
 * 1 - ||X - Y|| / ||X|| for the updated model, computed from the residual
 * entry by entry.
 */
int oracle_cp_als_step(const void *X, int xtype, const int64_t *dims, int N,
                       double *const *U, int R, double *fit_out, int nthreads)
{
    int64_t total;
    if (!X || !U || !check_dims(dims, N, R, &total)) return OR_EINVAL;
    int64_t maxI = 0, sumI = 0;
    for (int k = 0; k < N; ++k) {
        if (dims[k] > maxI) maxI = dims[k];
        sumI += dims[k];
    }
    double *save = (double *)malloc(sizeof(double) * (size_t)sumI * (size_t)R);
    double *M = (double *)malloc(sizeof(double) * (size_t)maxI * (size_t)R);
    double *H = (double *)malloc(sizeof(double) * (size_t)R * (size_t)R);
    double *G = (double *)malloc(sizeof(double) * (size_t)R * (size_t)R);
    if (!save || !M || !H || !G) {
        free(save); free(M); free(H); free(G);
        return OR_ENOMEM;
    }
    for (int64_t k = 0, off = 0; k < N; off += dims[k] * R, ++k)
        memcpy(save + off, U[k], sizeof(double) * (size_t)dims[k] * (size_t)R);
    int status = OR_OK;
    for (int n = 0; n < N && status == OR_OK; ++n) {
        status = oracle_mttkrp(X, xtype, dims, N, (const double *const *)U, R, n, M, nthreads);
        if (status != OR_OK) break;
        hadamard_grams((const double *const *)U, dims, N, R, n, H, G);
        if (!cholesky(H, R)) {
            status = OR_ENOTPD;
            break;
        }
        chol_solve_rows(H, R, M, dims[n], U[n]);
    }
    if (status != OR_OK) {
        for (int64_t k = 0, off = 0; k < N; off += dims[k] * R, ++k)
            memcpy(U[k], save + off, sizeof(double) * (size_t)dims[k] * (size_t)R);
    } else if (fit_out) {
        double x2 = oracle_xnorm2(X, xtype, dims, N);
        double r2 = oracle_residual2(X, xtype, dims, N, (const double *const *)U, R, nthreads);
        *fit_out = 1.0 - sqrt(r2) / sqrt(x2);
    }
    free(save); free(M); free(H); free(G);
    return status;
}

/*
 * Gradient of f = 1/2 ||X - [[U]]||_F^2 with respect to every factor:
 * grads[n] = U_n H_n - MTTKRP_n (I_n x R).  loss_direct receives f from the
 * residual entry by entry; loss_identity receives the same quantity from the
 * expansion 1/2 (||X||^2 - 2 <MTTKRP_{N-1}, U_{N-1}> + 1^T (Hadamard of all
 * Grams) 1).  Any output pointer may be null.
 */
int oracle_cp_grad(const void *X, int xtype, const int64_t *dims, int N,
                   const double *const *U, int R, double *const *grads,
                   double *loss_direct, double *loss_identity, int nthreads)
{
    int64_t total;
    if (!X || !U || !check_dims(dims, N, R, &total)) return OR_EINVAL;
    int64_t maxI = 0;
    for (int k = 0; k < N; ++k) if (dims[k] > maxI) maxI = dims[k];
    double *M = (double *)malloc(sizeof(double) * (size_t)maxI * (size_t)R);
    double *H = (double *)malloc(sizeof(double) * (size_t)R * (size_t)R);
    double *G = (double *)malloc(sizeof(double) * (size_t)R * (size_t)R);
    if (!M || !H || !G) {
        free(M); free(H); free(G);
        return OR_ENOMEM;
    }
    int status = OR_OK;
    double inner_last = 0.0;
    for (int n = 0; n < N; ++n) {
        if (!grads && !(loss_identity && n == N - 1)) continue;
        status = oracle_mttkrp(X, xtype, dims, N, U, R, n, M, nthreads);
        if (status != OR_OK) break;
        if (n == N - 1)
            for (int64_t e = 0; e < dims[n] * R; ++e) inner_last += M[e] * U[n][e];
        if (!grads || !grads[n]) continue;
        hadamard_grams(U, dims, N, R, n, H, G);
        for (int64_t i = 0; i < dims[n]; ++i)
            for (int c = 0; c < R; ++c) {
                double s = 0.0;
                for (int d = 0; d < R; ++d) s += U[n][i * R + d] * H[d * R + c];
                grads[n][i * R + c] = s - M[i * R + c];
            }
    }
    if (status == OR_OK && loss_identity) {
        hadamard_grams(U, dims, N, R, -1, H, G);
        double y2 = 0.0;
        for (int e = 0; e < R * R; ++e) y2 += H[e];
        *loss_identity = 0.5 * (oracle_xnorm2(X, xtype, dims, N) - 2.0 * inner_last + y2);
    }
    if (status == OR_OK && loss_direct)
        *loss_direct = 0.5 * oracle_residual2(X, xtype, dims, N, U, R, nthreads);
    free(M); free(H); free(G);
    return status;
}
