// C-ABI of the cpmttkrp library: argument validation, launch planning and
// the entry points declared in include/cpmttkrp.h.
#include <hip/hip_runtime.h>
#include <hipblaslt/hipblaslt.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>

#include "../../include/cpmttkrp.h"
#include "als_kernels.hpp"
#include "bf16_kernels.hpp"
#include "explicit_kernels.hpp"
#include "mttkrp32_kernels.hpp"
#include "mttkrp_kernels.hpp"
#include "residual_kernels.hpp"
#include "sympair_kernels.hpp"
#include "tree_kernels.hpp"

using namespace cpm;

// Split-K partials of mttkrp_scratch: a fixed device array, one copy per
// GPU, alive until the process ends.  In host code this name is only a
// stand-in for the symbol; the device address comes from
// hipGetSymbolAddress (scratch_ptr below) and is the only form of it that
// is ever passed to a kernel.
static __device__ __align__(256) unsigned char scratch[CPM_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

cpm_status fail(cpm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(CPM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

#define LAUNCH_CHECK(what)                                                             \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess) return fail(CPM_EHIP, "launch of %s failed: %s", what,   \
                                          hipGetErrorString(e_));                      \
    } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

size_t dtype_x_bytes(cpm_dtype dt) { return dt == CPM_F64 ? 8 : (dt == CPM_F32 ? 4 : 4); }
size_t dtype_f_bytes(cpm_dtype dt) { return dt == CPM_F64 ? 8 : 4; }

// Shape checks shared by every tensor entry point.  Touches host memory only.
cpm_status check_shape(const int64_t *dims, int N, int R, int64_t *total, int Rmax) {
    if (!dims) return fail(CPM_EINVAL, "dims is null");
    if (N < 2 || N > CPM_MAX_MODES) return fail(CPM_EINVAL, "N=%d outside [2, %d]", N, CPM_MAX_MODES);
    if (R < 1) return fail(CPM_EINVAL, "R=%d < 1", R);
    if (R > Rmax) return fail(CPM_EUNSUPPORTED, "R=%d above the limit %d", R, Rmax);
    int64_t t = 1;
    for (int k = 0; k < N; ++k) {
        if (dims[k] < 1) return fail(CPM_EINVAL, "dims[%d]=%lld < 1", k, (long long)dims[k]);
        if (t > ((int64_t)1 << 62) / dims[k]) return fail(CPM_EUNSUPPORTED, "tensor has 2^62 or more entries");
        t *= dims[k];
    }
    *total = t;
    return CPM_OK;
}

cpm_status check_dtype(cpm_dtype dt) {
    if (dt != CPM_F32 && dt != CPM_F64 && dt != CPM_BF16X2) return fail(CPM_EINVAL, "unknown dtype %d", (int)dt);
    return CPM_OK;
}

constexpr int64_t kMaxBufferOffset = 0xFFFFFF00LL;  // reach of one buffer resource

// Factor rows are read through buffer resources whose range is 32 bits:
// every factor read (all but `skip`, -1 for none) must span less than
// kMaxBufferOffset bytes.
cpm_status check_factor_reach(const int64_t *dims, int N, int R, cpm_dtype dt, int skip) {
    for (int k = 0; k < N; ++k)
        if (k != skip && dims[k] * (int64_t)R * (int64_t)dtype_f_bytes(dt) >= kMaxBufferOffset)
            return fail(CPM_EUNSUPPORTED, "factor %d (%lld x %d) spans 4 GiB or more, beyond one buffer resource",
                        k, (long long)dims[k], R);
    return CPM_OK;
}

// ---------------------------------------------------------------------------
// Launch planning for one mode.
// ---------------------------------------------------------------------------
enum Kind { kLeft = 0, kRight = 1, kBf16Left = 2, kBf16Right = 3, kLeft32 = 4, kRight32 = 5 };

struct Plan {
    Kind kind;
    int64_t IL, In, IR, J;
    int NB, MB, ncb;          // n-blocks per column block, m-blocks (right: MJ), column blocks;
                              // 32x32 kernels: NB = 32-column blocks, MB = row groups (left) or
                              // j-groups of waves (right), Q = j per lane (right)
    int p;                    // left: inner modes [0, p); right: inner modes [mode+1, p)
    int64_t G_in, G_out;      // inner rows of the contracted product; left: outer left extent
    int64_t n_outer;          // outer blocks
    int SPB, LC;              // steps per block per wave, inner chunk
    int Q;                    // left: 16-entry groups per row per step
    int WMg = 1;              // split-bf16 left: wave groups on separate row tiles
    int64_t nlc, bps, S;      // inner chunks, blocks per split, splits
    int64_t ntiles;           // row tiles (left) / j tiles (right)
    bool v4;
    size_t lds;
    bool reduce;              // partials need the reduction kernel
    size_t partial_bytes;
    int64_t max_offset;       // largest byte offset a buffer load uses (must stay below 2^32 - 256)
};

constexpr int kTargetGroups = 512;        // about two resident work-groups per CU
constexpr size_t kTileBytes = 78 * 1024;   // LDS for the resident Khatri-Rao tile

// Splits the outer blocks so the grid holds at most `groups` work-groups
// (one round of resident work-groups): rounding the split count up instead
// put a grid just past a round (516 for 512 slots) in two rounds of the
// same length.  When that round would be less than 85% full (257 tiles for
// 512 slots), the split count with the shortest estimated time is taken
// instead: rounds x (blocks per work-group + 2 for its set-up), with at
// most 1024 partial slices.  Grids of several rounds are left as they are:
// their work-groups do not finish together, so a short last round costs
// less than that estimate says (splitting further measured slower).
void split_outer(Plan &p, int64_t groups) {
    const int64_t T = p.ntiles * p.nlc * p.ncb;
    int64_t S = std::min(std::max<int64_t>(1, groups / T), p.n_outer);
    if (T * S < groups * 85 / 100) {
        const int64_t smax = std::max(S, std::min(p.n_outer, (int64_t)1024 / p.nlc));
        int64_t best = -1;
        for (int64_t s = 1; s <= smax; ++s) {
            const int64_t b = ceil_div(p.n_outer, s), s2 = ceil_div(p.n_outer, b);
            const int64_t cost = ceil_div(T * s2, groups) * (b + 2);
            if (best < 0 || cost < best) {
                best = cost;
                S = s2;
            }
        }
    }
    p.bps = ceil_div(p.n_outer, S);
    p.S = ceil_div(p.n_outer, p.bps);
}

// Chunk length (a multiple of unit, at most lcmax) for an inner range of
// G rows: chunks of equal step counts, the count (up to twice the fewest)
// that pads the fewest steps.  Every block runs a chunk's worth of steps
// whatever the chunk holds, so 256 rows in chunks of 96 ran 288 rows of
// steps, and four chunks of 64 run 256.
int even_chunk(int64_t G, int64_t lcmax, int64_t unit) {
    const int64_t g = ceil_div(G, unit);
    const int64_t c0 = ceil_div(G, lcmax);
    int64_t lc = ceil_div(g, c0) * unit;
    for (int64_t c = c0 + 1; c <= std::min(g, 2 * c0); ++c)
        if (c * ceil_div(g, c) * unit < ceil_div(G, lc) * lc) lc = ceil_div(g, c) * unit;
    return (int)lc;
}

int pow2_at_least(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Split-bf16 tiling.  Left-first once the left product is at least one
// 32-entry k-step long; otherwise right-first (X tiles transposed in LDS).
constexpr size_t kBf16XtBytes = 2 * 2 * 64 * 40 * 2;  // double-buffered hi/lo X tile of the right kernel

void plan_bf16(Plan &p, const int64_t *dims, int N, int R, int mode, const void *X) {
    const int RPtot = (R + 15) / 16 * 16;
    const int nb = RPtot / 16;
    p.NB = nb <= 8 ? pow2_at_least(nb) : 8;
    p.ncb = nb <= 8 ? 1 : (int)ceil_div(nb, 8);
    const int RP = p.NB * 16;
    const int64_t I = p.IL * p.In * p.IR;
    if (p.IL >= 32) {
        p.kind = kBf16Left;
        p.MB = p.NB >= 4 ? 1 : 2;
        while (p.MB > 1 && 16 * p.MB / 2 >= p.In) p.MB /= 2;
        const int64_t lcmax =
            std::max<int64_t>(128, std::min<int64_t>(512, (int64_t)(kTileBytes / (4 * RP) - 8) / 128 * 128));
        // Inner range: the fastest left modes that fit one chunk (a single
        // longer mode is cut into chunks).
        int q = 0;
        p.G_in = 1;
        while (q < mode && p.G_in * dims[q] <= lcmax) p.G_in *= dims[q++];
        if (q == 0) p.G_in = dims[q++];  // one long mode, cut into chunks
        // Rows far apart (8 MB or more): take a longer inner range in chunks,
        // so each row contributes a longer contiguous run per block (fewer
        // pages touched per byte streamed).
        if (p.IL * 2 >= ((int64_t)8 << 20))
            while (q < mode && p.G_in < lcmax) p.G_in *= dims[q++];
        p.p = q;
        p.G_out = p.IL / p.G_in;
        p.n_outer = p.G_out * p.IR;
        // Waves split the chunk (WC ways) and take separate 16*MB-row tiles
        // (WM = 4 / WC ways).  Wide ranks prefer row tiles, so a block spans
        // several steps per wave and its scaling epilogue is amortised; a
        // short inner range needs them, so no step runs past it.
        const int wc_fit = (int)std::max<int64_t>(1, std::min<int64_t>(4, p.G_in / 32));
        int wm = p.NB < 4 ? 1 : (p.In >= 64 ? 4 : (p.In >= 32 ? 2 : 1));
        while (4 / wm > wc_fit) wm *= 2;
        p.WMg = wm;
        // Two k-step groups per step (128 contiguous bytes of a row per plane
        // per step instead of 64) once the chunk is long enough; at NB = 8 it
        // is taken with row-tile wave groups, where it measured 5% (WM = 4)
        // and 14% (WM = 2, I_n = 32) faster on 256 x 256 x 512 x 32 at R = 128.
        bool q2 = p.G_in >= 256;
        q2 = q2 && (p.NB >= 8 ? wm > 1 : wm == 1);
        p.Q = q2 ? 2 : 1;
        const int64_t unit = (4 / p.WMg) * 32 * p.Q;
        p.LC = (int)std::min<int64_t>(std::max<int64_t>(unit, lcmax / unit * unit), ceil_div(p.G_in, unit) * unit);
        p.SPB = p.LC / (int)unit;
        p.nlc = ceil_div(p.G_in, p.LC);
        p.ntiles = ceil_div(p.In, 16 * p.MB * p.WMg);
        const size_t tile = (size_t)4 * RP * (p.LC + 8) + (size_t)kScaleTableBytes;
        const size_t red = (size_t)4 * p.MB * p.NB * 256 * 4;
        p.lds = std::max(tile, red);
        p.v4 = (p.G_in % 8 == 0) && (I % 8 == 0) && ((uintptr_t)X % 16 == 0);
        p.max_offset = (15 * p.IL + p.G_in + 8) * 2;
        p.J = p.In;
    } else {
        p.kind = kBf16Right;
        p.J = p.In * p.IL;
        const int64_t lcmax = std::max<int64_t>(
            32, std::min<int64_t>(512, ((int64_t)((kTileBytes - kBf16XtBytes) / (4 * RP)) - 8) / 32 * 32));
        int q = mode + 1;
        p.G_in = 1;
        while (q < N && p.G_in * dims[q] <= lcmax) p.G_in *= dims[q++];
        if (q == mode + 1 && q < N) p.G_in = dims[q++];
        p.p = q;
        p.n_outer = p.IR / p.G_in;
        p.LC = even_chunk(p.G_in, lcmax, 32);
        p.SPB = p.LC / 32;
        p.nlc = ceil_div(p.G_in, p.LC);
        p.ntiles = ceil_div(p.J, 64);
        p.lds = (size_t)4 * RP * (p.LC + 8) + kBf16XtBytes + (size_t)kScaleTableBytes;
        p.v4 = (p.J % 8 == 0) && (I % 8 == 0) && ((uintptr_t)X % 16 == 0);
        p.max_offset = ((int64_t)p.LC * p.J + 64 + 8) * 2;
    }
    split_outer(p, kTargetGroups);
    p.reduce = p.S * p.nlc > 1 || (p.kind == kBf16Right && mode > 0);
    const int64_t rows = p.kind == kBf16Left ? p.In : p.J;
    p.partial_bytes = p.reduce ? (size_t)p.S * p.nlc * rows * R * 4 : 0;
}

// Float32 tiling on the 32x32 MFMA kernels (mttkrp32_kernels.hpp).
// Left-first once the left product has 32 entries; right-first otherwise.  The inner part of the contracted index
// is grown until it reaches the chunk length (a long inner range is then cut
// into chunks).  Returns false when these kernels do not apply.
constexpr int64_t kF32Chunk = 128;  // inner entries per work-group (tile of 16 KB per 32 columns)
constexpr int kF32GroupsRight = 512;  // wide-output test: j tiles that occupy every CU

// Work-groups of a float32 contraction kernel resident on one CU: each has
// one wave per SIMD, so the waves per SIMD its registers allow (from the
// compiled kernels: k_left32 three at one 32-column block and two at more;
// k_right32 four at one column block and one j per lane, three at two
// columns-times-j, two at four), and what its LDS allows.
int64_t f32_groups(const Plan &p) {
    int regs;
    if (p.kind == kLeft32) regs = p.NB == 1 ? 3 : 2;
    else regs = p.NB * p.Q == 1 ? 4 : (p.NB * p.Q == 2 ? 3 : 2);
    const int64_t lds = std::max<int64_t>(1, (int64_t)(160 * 1024) / (int64_t)p.lds);
    return 256 * std::min<int64_t>(regs, lds);
}

// tight: the inner contracted group grows only while it still fits one
// chunk (at least one mode), so the contracted range is not cut into chunks
// whose partial results are each a whole output; used for wide outputs.
constexpr int64_t kTightChunkMax = 512;
constexpr size_t kTightLds = 80 * 1024;
bool plan_f32(Plan &p, const int64_t *dims, int N, int R, int mode, const void *X, bool tight) {
    const int nct = (R + 31) / 32;
    const bool left = p.IL >= 32;
    const int ncmax = left ? 4 : 2;
    p.NB = nct <= ncmax ? pow2_at_least(nct) : ncmax;
    p.ncb = (int)ceil_div(nct, p.NB);
    const int RP = 32 * p.NB;
    const uintptr_t xa = (uintptr_t)X;
    if (left) {
        p.kind = kLeft32;
        int q = 0;
        p.G_in = 1;
        if (tight) {
            p.G_in = dims[q++];
            while (q < mode && p.G_in * dims[q] <= kF32Chunk) p.G_in *= dims[q++];
        } else {
            // a mode that would make the inner range more than 64 chunks long
            // stays outer once the range holds one k-step group (32)
            while (q < mode && p.G_in < kF32Chunk && !(p.G_in >= 32 && p.G_in * dims[q] > 64 * kF32Chunk))
                p.G_in *= dims[q++];
        }
        if (xa % 4 != 0) return false;  // rows need 4-byte alignment
        p.p = q;
        p.G_out = p.IL / p.G_in;
        p.n_outer = p.G_out * p.IR;
        p.MB = p.G_in >= 128 ? 1 : (p.G_in >= 64 ? 2 : 4);  // wave groups along rows
        while (p.MB > 1 && 32 * p.MB / 2 >= p.In) p.MB /= 2;
        const int64_t unit = (4 / p.MB) * 32;
        p.LC = (int)std::max(unit, std::min(kF32Chunk / unit * unit, ceil_div(p.G_in, unit) * unit));
        p.SPB = p.LC / (int)unit;
        p.nlc = ceil_div(p.G_in, p.LC);
        p.ntiles = ceil_div(p.In, 32 * p.MB);
        p.lds = std::max((size_t)4 * RP * (p.LC + 4) + 16384 + (size_t)kScaleTableBytes, (size_t)16384 * p.NB);
        p.v4 = true;
        p.max_offset = (31 * p.IL + p.LC + 4) * 4;
        p.J = p.In;
    } else {
        p.kind = kRight32;
        p.J = p.In * p.IL;
        if (xa % 4 != 0) return false;
        // Any row length works (a lane whose entries straddle J loads them
        // one by one), but unaligned rows measured slower at TJ = 4 (mode 0
        // of 225 x 59 x 200 x 200: 0.88 ms against 0.65 ms at TJ = 1), so
        // the wide forms are kept for rows of aligned length.
        const bool a4 = p.J % 4 == 0 && xa % 16 == 0, a2 = p.J % 2 == 0 && xa % 8 == 0;
        // Waves split the rows of a narrow j tile: the partial result of a
        // work-group (its j tile x R) stays small next to the X it streams.
        int tj = 1;
        if (p.NB == 1 && a4 && p.J >= 128) tj = 4;
        else if (a2 && p.J >= 32) tj = 2;  // mode 0 of 60^5 (J = 60): 1.09 -> 0.75 ms against TJ = 1
        // A wide output (the cross-mode reuse's pass over a long left
        // product): each wave takes its own j range and streams the whole
        // contracted range, so the work-group needs no cross-wave reduction
        // and writes its 4 x 32 x TJ outputs directly, while there are still
        // enough j tiles to occupy every CU.
        int wj = 1;
        if (tight && ((p.NB == 1 && tj == 4) || (p.NB == 2 && tj == 2)) &&
            ceil_div(p.J, 32 * tj * 4) >= kF32GroupsRight / 2)
            wj = 4;
        p.Q = tj;
        p.MB = wj;
        const int64_t unit = 8 * (4 / wj);
        // tight: the whole inner group in one resident chunk while the tile
        // and scale table stay within kTightLds (up to 512 rows)
        int64_t lcap = kF32Chunk;
        if (tight)
            while (lcap + unit <= kTightChunkMax &&
                   (size_t)4 * RP * (lcap + unit + 4) + (size_t)kScaleTableBytes <= kTightLds)
                lcap += unit;
        int q = mode + 1;
        p.G_in = 1;
        if (tight && q < N) {
            p.G_in = dims[q++];
            while (q < N && p.G_in * dims[q] <= lcap) p.G_in *= dims[q++];
        } else {
            while (q < N && p.G_in < lcap && !(p.G_in >= 32 && p.G_in * dims[q] > 64 * lcap)) p.G_in *= dims[q++];
        }
        p.p = q;
        p.n_outer = p.IR / p.G_in;
        const int64_t lcmax = std::max<int64_t>(unit, lcap / unit * unit);
        p.LC = even_chunk(p.G_in, lcmax, unit);
        p.SPB = p.LC / (int)unit;
        p.nlc = ceil_div(p.G_in, p.LC);
        p.ntiles = ceil_div(p.J, 32 * tj * wj);
        p.lds = std::max((size_t)4 * RP * (p.LC + 4) + (size_t)kScaleTableBytes,
                         wj < 4 ? (size_t)16384 * tj * p.NB : (size_t)0);
        p.v4 = tj > 1;
        p.max_offset = ((int64_t)p.LC * p.J + 32 * tj + 4) * 4;
    }
    split_outer(p, f32_groups(p));
    p.reduce = p.S * p.nlc > 1 || (p.kind == kRight32 && mode > 0);
    p.partial_bytes = p.reduce ? (size_t)p.S * p.nlc * (p.kind == kLeft32 ? p.In : p.J) * R * 4 : 0;
    return true;
}

Plan make_plan(const int64_t *dims, int N, int R, int mode, cpm_dtype dt, const void *X) {
    Plan p{};
    p.IL = 1;
    for (int k = 0; k < mode; ++k) p.IL *= dims[k];
    p.In = dims[mode];
    p.IR = 1;
    for (int k = mode + 1; k < N; ++k) p.IR *= dims[k];
    const size_t sz = dtype_f_bytes(dt);
    const int RPtot = (R + 15) / 16 * 16;
    const bool bf = dt == CPM_BF16X2;
    if (bf) {
        plan_bf16(p, dims, N, R, mode, X);
        return p;
    }
    if (dt == CPM_F32) {
        Plan q = p;
        if (plan_f32(q, dims, N, R, mode, X, false) && q.max_offset < kMaxBufferOffset) {
            // Split-K partials that rival X itself (a wide output, as in a
            // partial contraction over a few modes): prefer the tight inner
            // group when it writes fewer of them.
            if ((int64_t)q.partial_bytes > p.IL * p.In * p.IR / 2) {
                Plan t = p;
                if (plan_f32(t, dims, N, R, mode, X, true) && t.max_offset < kMaxBufferOffset &&
                    t.partial_bytes < q.partial_bytes)
                    return t;
            }
            return q;
        }
    }
    const bool left = p.IL >= 16;
    const bool dbl = dt == CPM_F64;
    // n-blocks (16 rank columns) per work-group; wider ranks take several
    // column blocks.  The right-first kernel keeps four accumulator rows per
    // lane, so it stays at two blocks.
    // (float reaches this tiling only as the fallback of the 32x32 kernels:
    // misaligned rows or offsets beyond one buffer resource)
    const int nbmax = left ? 2 : (dbl ? 1 : 2);
    int nb = RPtot / 16;
    if (nb <= nbmax) {
        p.NB = pow2_at_least(nb);
        p.ncb = 1;
    } else {
        p.NB = nbmax;
        p.ncb = (int)ceil_div(nb, nbmax);
    }
    const int RP = p.NB * 16;
    const int pitch = RP + 4;
    const int64_t lcmax = std::max<int64_t>(64, std::min<int64_t>(512, (int64_t)(kTileBytes / (pitch * sz)) / 64 * 64));
    // Inner part of the contracted product: consecutive modes starting next
    // to the stride-1 end, as many as fit in one tile (at least one mode;
    // a single mode longer than a tile is cut into chunks).
    auto pick_inner = [&](int first, int last, int64_t &G) {
        int q = first;
        G = 1;
        while (q < last && G * dims[q] <= lcmax) G *= dims[q++];
        if (q == first && q < last) G = dims[q++];
        return q;
    };
    if (left) {
        p.kind = kLeft;
        p.MB = (!dbl || p.NB >= 2) ? 1 : 2;
        while (p.MB > 1 && 16 * p.MB / 2 >= p.In) p.MB /= 2;
        p.p = pick_inner(0, mode, p.G_in);
        p.G_out = p.IL / p.G_in;
        p.n_outer = p.G_out * p.IR;
        p.Q = (dbl && p.G_in > 64) ? 2 : 1;  // 128-byte row bursts once rows are long enough
        const int64_t unit = 64 * p.Q;
        p.LC = (int)std::min<int64_t>(lcmax / unit * unit, ceil_div(p.G_in, unit) * unit);
        p.SPB = p.LC / (int)unit;
        p.nlc = ceil_div(p.G_in, p.LC);
        p.ntiles = ceil_div(p.In, 16 * p.MB);
        const size_t red = (size_t)4 * p.MB * p.NB * 256 * sz;
        p.lds = std::max((size_t)p.LC * pitch * sz, red);
        split_outer(p, kTargetGroups);
        p.v4 = (p.G_in % 4 == 0) && ((uintptr_t)X % (4 * sz) == 0);
        p.max_offset = (15 * p.IL + p.G_in + 4) * (int64_t)sz;  // lane offsets within one m-block
        p.J = p.In;
        p.reduce = p.S * p.nlc > 1;
        p.partial_bytes = p.reduce ? (size_t)p.S * p.nlc * p.In * R * sz : 0;
    } else {
        p.kind = kRight;
        p.J = p.In * p.IL;
        p.MB = 1;  // MJ
        p.p = pick_inner(mode + 1, N, p.G_in);
        p.n_outer = p.IR / p.G_in;
        p.LC = (int)std::min<int64_t>(lcmax, ceil_div(p.G_in, 64) * 64);
        p.SPB = p.LC / 64;
        p.nlc = ceil_div(p.G_in, p.LC);
        p.ntiles = ceil_div(p.J, 64 * p.MB);
        const size_t red = (size_t)4 * p.MB * 4 * p.NB * 256 * sz;
        p.lds = std::max((size_t)p.LC * pitch * sz, red);
        split_outer(p, kTargetGroups);
        p.v4 = (p.J % 4 == 0) && ((uintptr_t)X % (4 * sz) == 0);
        p.max_offset = ((16 * (int64_t)p.SPB) * p.J + 64 * p.MB + 4) * (int64_t)sz;  // within one wave's rows
        p.reduce = p.S * p.nlc > 1 || mode > 0;  // mode > 0: the multi-TTV with K_L runs in the reduction
        p.partial_bytes = p.reduce ? (size_t)p.S * p.nlc * p.J * R * sz : 0;
    }
    return p;
}

// ----------------------------- kernel dispatch -----------------------------
template <typename T, int NB, int MB, int Q>
void launch_left_t(const Plan &p, const T *X, const Krp<T> &kin, const Krp<T> &kout, int R, T *partial,
                   hipStream_t st) {
    dim3 grid((unsigned)p.ntiles, (unsigned)(p.S * p.nlc), (unsigned)p.ncb);
    if (p.v4)
        hipLaunchKernelGGL((k_contract_left<T, NB, MB, true, Q>), grid, dim3(kThreads), p.lds, st, X, p.G_in,
                           p.G_out, p.In, p.n_outer, kin, kout, R, p.SPB, p.nlc, p.bps, partial);
    else
        hipLaunchKernelGGL((k_contract_left<T, NB, MB, false, Q>), grid, dim3(kThreads), p.lds, st, X, p.G_in,
                           p.G_out, p.In, p.n_outer, kin, kout, R, p.SPB, p.nlc, p.bps, partial);
}

template <typename T, int NB, int MB>
void launch_left_q(const Plan &p, const T *X, const Krp<T> &kin, const Krp<T> &kout, int R, T *partial,
                   hipStream_t st) {
    if (p.Q == 2) launch_left_t<T, NB, MB, 2>(p, X, kin, kout, R, partial, st);
    else launch_left_t<T, NB, MB, 1>(p, X, kin, kout, R, partial, st);
}

template <typename T, int NB>
void launch_left_m(const Plan &p, const T *X, const Krp<T> &kin, const Krp<T> &kout, int R, T *partial,
                   hipStream_t st) {
    if (p.MB == 2) launch_left_q<T, NB, 2>(p, X, kin, kout, R, partial, st);
    else launch_left_q<T, NB, 1>(p, X, kin, kout, R, partial, st);
}

template <typename T>
void launch_left(const Plan &p, const T *X, const Krp<T> &kin, const Krp<T> &kout, int R, T *partial,
                 hipStream_t st);
template <>
void launch_left<float>(const Plan &p, const float *X, const Krp<float> &kin, const Krp<float> &kout, int R,
                        float *partial, hipStream_t st) {
    if (p.NB == 1) launch_left_t<float, 1, 1, 1>(p, X, kin, kout, R, partial, st);
    else launch_left_t<float, 2, 1, 1>(p, X, kin, kout, R, partial, st);
}
template <>
void launch_left<double>(const Plan &p, const double *X, const Krp<double> &kin, const Krp<double> &kout, int R,
                         double *partial, hipStream_t st) {
    if (p.NB == 1) launch_left_m<double, 1>(p, X, kin, kout, R, partial, st);
    else launch_left_q<double, 2, 1>(p, X, kin, kout, R, partial, st);
}

template <typename T, int NB, int MJ>
void launch_right_t(const Plan &p, const T *X, const Krp<T> &kin, const Krp<T> &kout, int R, T *partial,
                    hipStream_t st) {
    dim3 grid((unsigned)p.ntiles, (unsigned)(p.S * p.nlc), (unsigned)p.ncb);
    if (p.v4)
        hipLaunchKernelGGL((k_contract_right<T, NB, MJ, true>), grid, dim3(kThreads), p.lds, st, X, p.J, p.G_in,
                           p.n_outer, kin, kout, R, p.SPB, p.nlc, p.bps, partial);
    else
        hipLaunchKernelGGL((k_contract_right<T, NB, MJ, false>), grid, dim3(kThreads), p.lds, st, X, p.J, p.G_in,
                           p.n_outer, kin, kout, R, p.SPB, p.nlc, p.bps, partial);
}

template <typename T>
void launch_right(const Plan &p, const T *X, const Krp<T> &kin, const Krp<T> &kout, int R, T *partial,
                  hipStream_t st);
template <>
void launch_right<float>(const Plan &p, const float *X, const Krp<float> &kin, const Krp<float> &kout, int R,
                         float *partial, hipStream_t st) {
    if (p.NB == 1) launch_right_t<float, 1, 1>(p, X, kin, kout, R, partial, st);
    else launch_right_t<float, 2, 1>(p, X, kin, kout, R, partial, st);
}
template <>
void launch_right<double>(const Plan &p, const double *X, const Krp<double> &kin, const Krp<double> &kout, int R,
                          double *partial, hipStream_t st) {
    launch_right_t<double, 1, 1>(p, X, kin, kout, R, partial, st);
    (void)p;
}

template <int NC, int WM>
void launch_left32_t(const Plan &p, const float *X, const Krp<float> &kin, const Krp<float> &kout, int R,
                     float *partial, hipStream_t st) {
    dim3 grid((unsigned)p.ntiles, (unsigned)(p.S * p.nlc), (unsigned)p.ncb);
    hipLaunchKernelGGL((k_left32<NC, WM>), grid, dim3(kThreads), p.lds, st, X, p.G_in, p.G_out, p.In, p.n_outer, kin,
                       kout, R, p.SPB, p.nlc, p.bps, partial);
}

template <int NC>
void launch_left32_m(const Plan &p, const float *X, const Krp<float> &kin, const Krp<float> &kout, int R,
                     float *partial, hipStream_t st) {
    if (p.MB == 4) launch_left32_t<NC, 4>(p, X, kin, kout, R, partial, st);
    else if (p.MB == 2) launch_left32_t<NC, 2>(p, X, kin, kout, R, partial, st);
    else launch_left32_t<NC, 1>(p, X, kin, kout, R, partial, st);
}

void launch_left32(const Plan &p, const float *X, const Krp<float> &kin, const Krp<float> &kout, int R,
                   float *partial, hipStream_t st) {
    if (p.NB == 1) launch_left32_m<1>(p, X, kin, kout, R, partial, st);
    else if (p.NB == 2) launch_left32_m<2>(p, X, kin, kout, R, partial, st);
    else launch_left32_m<4>(p, X, kin, kout, R, partial, st);
}

template <int NC, int TJ, int WJ>
void launch_right32_t(const Plan &p, const float *X, const Krp<float> &kin, const Krp<float> &kout, int R,
                      float *partial, hipStream_t st) {
    dim3 grid((unsigned)p.ntiles, (unsigned)(p.S * p.nlc), (unsigned)p.ncb);
    hipLaunchKernelGGL((k_right32<NC, TJ, WJ>), grid, dim3(kThreads), p.lds, st, X, p.J, p.G_in, p.n_outer, kin,
                       kout, R, p.SPB, p.nlc, p.bps, partial);
}

void launch_right32(const Plan &p, const float *X, const Krp<float> &kin, const Krp<float> &kout, int R,
                    float *partial, hipStream_t st) {
    if (p.MB == 4) {  // one j range per wave (wide outputs)
        if (p.NB == 1) launch_right32_t<1, 4, 4>(p, X, kin, kout, R, partial, st);
        else launch_right32_t<2, 2, 4>(p, X, kin, kout, R, partial, st);
        return;
    }
    if (p.NB == 1) {
        if (p.Q == 4) launch_right32_t<1, 4, 1>(p, X, kin, kout, R, partial, st);
        else if (p.Q == 2) launch_right32_t<1, 2, 1>(p, X, kin, kout, R, partial, st);
        else launch_right32_t<1, 1, 1>(p, X, kin, kout, R, partial, st);
    } else {
        if (p.Q == 2) launch_right32_t<2, 2, 1>(p, X, kin, kout, R, partial, st);
        else launch_right32_t<2, 1, 1>(p, X, kin, kout, R, partial, st);
    }
}

// Enqueue one MTTKRP (arguments already validated).
// Khatri-Rao descriptor over a list of modes, fastest first.
template <typename T>
Krp<T> krp_of(const void *const *factors, const int64_t *dims, const int *modes, int count) {
    Krp<T> k{};
    k.Z = 0;
    k.rows = 1;
    for (int i = 0; i < count; ++i) {
        const int m = modes[i];
        k.J[k.Z] = dims[m];
        k.stride[k.Z] = k.rows;
        k.U[k.Z] = reinterpret_cast<const T *>(factors[m]);
        k.rows *= dims[m];
        ++k.Z;
    }
    return k;
}

// Slice sums queued for one k_sum_jobs launch.  A caller queues only sums
// whose slices stay untouched until the flush, and flushes before anything
// reads their outputs.
struct SumList {
    SumJobs j{};
};

cpm_status sum_flush(SumList &L, hipStream_t st) {
    if (L.j.count == 0) return CPM_OK;
    const int64_t blocks = L.j.first[L.j.count];
    hipLaunchKernelGGL(k_sum_jobs, dim3((unsigned)blocks), dim3(kThreads), 0, st, L.j);
    L.j = SumJobs{};
    LAUNCH_CHECK("k_sum_jobs");
    return CPM_OK;
}

cpm_status sum_add(SumList &L, const float *P, int64_t S, int64_t n, float *M, hipStream_t st) {
    if (L.j.count == kSumJobs) {
        const cpm_status s = sum_flush(L, st);
        if (s) return s;
    }
    const int k = L.j.count++;
    L.j.P[k] = P;
    L.j.M[k] = M;
    L.j.S[k] = S;
    L.j.n[k] = n;
    L.j.first[k + 1] = L.j.first[k] + ceil_div(n, 64);
    return CPM_OK;
}

// Enqueue one MTTKRP (arguments already validated).
template <typename T>
cpm_status run_mttkrp_t(const Plan &p, const void *Xv, const int64_t *dims, int N, const void *const *factors,
                        int R, int mode, void *outv, void *ws, hipStream_t st, SumList *defer = nullptr) {
    int in_modes[CPM_MAX_MODES], out_modes[CPM_MAX_MODES], left_modes[CPM_MAX_MODES];
    int nin = 0, nout = 0, nleft = 0;
    for (int k = 0; k < mode; ++k) left_modes[nleft++] = k;
    const bool lf = p.kind == kLeft || p.kind == kLeft32;
    if (lf) {
        for (int k = 0; k < p.p; ++k) in_modes[nin++] = k;
        for (int k = p.p; k < mode; ++k) out_modes[nout++] = k;
        for (int k = mode + 1; k < N; ++k) out_modes[nout++] = k;
    } else {
        for (int k = mode + 1; k < p.p; ++k) in_modes[nin++] = k;
        for (int k = p.p; k < N; ++k) out_modes[nout++] = k;
    }
    const Krp<T> kin = krp_of<T>(factors, dims, in_modes, nin);
    const Krp<T> kout = krp_of<T>(factors, dims, out_modes, nout);
    const T *X = reinterpret_cast<const T *>(Xv);
    T *out = reinterpret_cast<T *>(outv);
    T *partial = p.reduce ? reinterpret_cast<T *>(ws) : out;
    if constexpr (std::is_same<T, float>::value) {
        if (p.kind == kLeft32) {
            launch_left32(p, X, kin, kout, R, partial, st);
            LAUNCH_CHECK("k_left32");
        } else if (p.kind == kRight32) {
            launch_right32(p, X, kin, kout, R, partial, st);
            LAUNCH_CHECK("k_right32");
        }
    }
    if (p.kind == kLeft) {
        launch_left<T>(p, X, kin, kout, R, partial, st);
        LAUNCH_CHECK("k_contract_left");
    } else if (p.kind == kRight) {
        launch_right<T>(p, X, kin, kout, R, partial, st);
        LAUNCH_CHECK("k_contract_right");
    }
    if constexpr (std::is_same<T, float>::value) {
        // left-first partials are plain slices of the output: the caller
        // may add them in a later k_sum_jobs launch (the same sums)
        if (p.reduce && lf && defer) return sum_add(*defer, partial, p.S * p.nlc, p.In * R, out, st);
    }
    if (p.reduce) {
        const int64_t total = p.In * R;
        const int64_t rows_per_slice = lf ? p.In : p.J;
        // right-first for mode > 0: the multi-TTV with K_L (all left modes)
        Krp<T> kred = krp_of<T>(factors, dims, left_modes, lf ? 0 : nleft);
        const int64_t il = lf ? 1 : p.IL;
        hipLaunchKernelGGL((k_reduce<T, T>), dim3((unsigned)ceil_div(total, 64)), dim3(kThreads), 0, st, partial,
                           p.S * p.nlc, rows_per_slice, p.In, il, kred, R, out);
        LAUNCH_CHECK("k_reduce");
    }
    return CPM_OK;
}

template <int NB, int MB, int Q, int WM = 1>
void launch_left_bf16_t(const Plan &p, const uint16_t *X, int64_t I, const Krp<float> &kin, const Krp<float> &kout,
                        int R, float *partial, hipStream_t st) {
    dim3 grid((unsigned)p.ntiles, (unsigned)(p.S * p.nlc), (unsigned)p.ncb);
    if (p.v4)
        hipLaunchKernelGGL((k_contract_left_bf16<NB, MB, Q, true, WM>), grid, dim3(kThreads), p.lds, st, X, I,
                           p.G_in, p.G_out, p.In, p.n_outer, kin, kout, R, p.SPB, p.nlc, p.bps, partial);
    else
        hipLaunchKernelGGL((k_contract_left_bf16<NB, MB, Q, false, WM>), grid, dim3(kThreads), p.lds, st, X, I,
                           p.G_in, p.G_out, p.In, p.n_outer, kin, kout, R, p.SPB, p.nlc, p.bps, partial);
}

template <int NB, int MB>
void launch_left_bf16_q(const Plan &p, const uint16_t *X, int64_t I, const Krp<float> &kin, const Krp<float> &kout,
                        int R, float *partial, hipStream_t st) {
    if (p.Q == 2) launch_left_bf16_t<NB, MB, 2>(p, X, I, kin, kout, R, partial, st);
    else launch_left_bf16_t<NB, MB, 1>(p, X, I, kin, kout, R, partial, st);
}

template <int NB>
void launch_left_bf16_m(const Plan &p, const uint16_t *X, int64_t I, const Krp<float> &kin, const Krp<float> &kout,
                        int R, float *partial, hipStream_t st) {
    if (p.MB == 2) launch_left_bf16_q<NB, 2>(p, X, I, kin, kout, R, partial, st);
    else launch_left_bf16_q<NB, 1>(p, X, I, kin, kout, R, partial, st);
}

template <int NB>
void launch_right_bf16_t(const Plan &p, const uint16_t *X, int64_t I, const Krp<float> &kin,
                         const Krp<float> &kout, int R, float *partial, hipStream_t st) {
    dim3 grid((unsigned)p.ntiles, (unsigned)(p.S * p.nlc), (unsigned)p.ncb);
    if (p.v4)
        hipLaunchKernelGGL((k_contract_right_bf16<NB, true>), grid, dim3(kThreads), p.lds, st, X, I, p.J, p.G_in,
                           p.n_outer, kin, kout, R, p.SPB, p.nlc, p.bps, partial);
    else
        hipLaunchKernelGGL((k_contract_right_bf16<NB, false>), grid, dim3(kThreads), p.lds, st, X, I, p.J, p.G_in,
                           p.n_outer, kin, kout, R, p.SPB, p.nlc, p.bps, partial);
}

// Narrow ranks with row-tile wave groups (short inner ranges).
template <int NB>
void launch_left_bf16_wm(const Plan &p, const uint16_t *X, int64_t I, const Krp<float> &kin,
                         const Krp<float> &kout, int R, float *partial, hipStream_t st) {
    if (p.MB == 2) {
        if (p.WMg == 4) launch_left_bf16_t<NB, 2, 1, 4>(p, X, I, kin, kout, R, partial, st);
        else launch_left_bf16_t<NB, 2, 1, 2>(p, X, I, kin, kout, R, partial, st);
    } else {
        if (p.WMg == 4) launch_left_bf16_t<NB, 1, 1, 4>(p, X, I, kin, kout, R, partial, st);
        else launch_left_bf16_t<NB, 1, 1, 2>(p, X, I, kin, kout, R, partial, st);
    }
}

cpm_status run_mttkrp_bf16(const Plan &p, const void *Xv, const int64_t *dims, int N, const void *const *factors,
                           int R, int mode, void *outv, void *ws, hipStream_t st) {
    int in_modes[CPM_MAX_MODES], out_modes[CPM_MAX_MODES], left_modes[CPM_MAX_MODES];
    int nin = 0, nout = 0, nleft = 0;
    for (int k = 0; k < mode; ++k) left_modes[nleft++] = k;
    if (p.kind == kBf16Left) {
        for (int k = 0; k < p.p; ++k) in_modes[nin++] = k;
        for (int k = p.p; k < mode; ++k) out_modes[nout++] = k;
        for (int k = mode + 1; k < N; ++k) out_modes[nout++] = k;
    } else {
        for (int k = mode + 1; k < p.p; ++k) in_modes[nin++] = k;
        for (int k = p.p; k < N; ++k) out_modes[nout++] = k;
    }
    const Krp<float> kin = krp_of<float>(factors, dims, in_modes, nin);
    const Krp<float> kout = krp_of<float>(factors, dims, out_modes, nout);
    const uint16_t *X = reinterpret_cast<const uint16_t *>(Xv);
    const int64_t I = p.IL * p.In * p.IR;
    float *out = reinterpret_cast<float *>(outv);
    float *partial = p.reduce ? reinterpret_cast<float *>(ws) : out;
    if (p.kind == kBf16Left) {
        switch (p.NB) {
        case 1:
            if (p.WMg == 1) launch_left_bf16_m<1>(p, X, I, kin, kout, R, partial, st);
            else launch_left_bf16_wm<1>(p, X, I, kin, kout, R, partial, st);
            break;
        case 2:
            if (p.WMg == 1) launch_left_bf16_m<2>(p, X, I, kin, kout, R, partial, st);
            else launch_left_bf16_wm<2>(p, X, I, kin, kout, R, partial, st);
            break;
        case 4:
            if (p.WMg == 4) {
                if (p.Q == 2) launch_left_bf16_t<4, 1, 2, 4>(p, X, I, kin, kout, R, partial, st);
                else launch_left_bf16_t<4, 1, 1, 4>(p, X, I, kin, kout, R, partial, st);
            } else if (p.WMg == 2) {
                if (p.Q == 2) launch_left_bf16_t<4, 1, 2, 2>(p, X, I, kin, kout, R, partial, st);
                else launch_left_bf16_t<4, 1, 1, 2>(p, X, I, kin, kout, R, partial, st);
            } else {
                launch_left_bf16_q<4, 1>(p, X, I, kin, kout, R, partial, st);
            }
            break;
        default:
            if (p.WMg == 4) {
                if (p.Q == 2) launch_left_bf16_t<8, 1, 2, 4>(p, X, I, kin, kout, R, partial, st);
                else launch_left_bf16_t<8, 1, 1, 4>(p, X, I, kin, kout, R, partial, st);
            } else if (p.WMg == 2) {
                if (p.Q == 2) launch_left_bf16_t<8, 1, 2, 2>(p, X, I, kin, kout, R, partial, st);
                else launch_left_bf16_t<8, 1, 1, 2>(p, X, I, kin, kout, R, partial, st);
            } else {
                launch_left_bf16_t<8, 1, 1>(p, X, I, kin, kout, R, partial, st);
            }
            break;
        }
        LAUNCH_CHECK("k_contract_left_bf16");
    } else {
        switch (p.NB) {
        case 1: launch_right_bf16_t<1>(p, X, I, kin, kout, R, partial, st); break;
        case 2: launch_right_bf16_t<2>(p, X, I, kin, kout, R, partial, st); break;
        case 4: launch_right_bf16_t<4>(p, X, I, kin, kout, R, partial, st); break;
        default: launch_right_bf16_t<8>(p, X, I, kin, kout, R, partial, st); break;
        }
        LAUNCH_CHECK("k_contract_right_bf16");
    }
    if (p.reduce) {
        const int64_t rows_per_slice = (p.kind == kBf16Left) ? p.In : p.J;
        const Krp<float> kred = krp_of<float>(factors, dims, left_modes, p.kind == kBf16Left ? 0 : nleft);
        const int64_t il = (p.kind == kBf16Left) ? 1 : p.IL;
        hipLaunchKernelGGL((k_reduce<float, float>), dim3((unsigned)ceil_div(p.In * R, 64)), dim3(kThreads), 0, st,
                           partial, p.S * p.nlc, rows_per_slice, p.In, il, kred, R, out);
        LAUNCH_CHECK("k_reduce");
    }
    return CPM_OK;
}

cpm_status run_mttkrp(const Plan &p, const void *X, const int64_t *dims, int N, const void *const *factors,
                      int R, int mode, void *out, cpm_dtype dt, void *ws, hipStream_t st,
                      SumList *defer = nullptr) {
    if (dt == CPM_F32) return run_mttkrp_t<float>(p, X, dims, N, factors, R, mode, out, ws, st, defer);
    if (dt == CPM_F64) return run_mttkrp_t<double>(p, X, dims, N, factors, R, mode, out, ws, st);
    return run_mttkrp_bf16(p, X, dims, N, factors, R, mode, out, ws, st);
}

cpm_status validate_mttkrp(const void *X, const int64_t *dims, int N, const void *const *factors, int R,
                           int mode, const void *out, cpm_dtype dt, int64_t *total) {
    cpm_status s = check_dtype(dt);
    if (s) return s;
    s = check_shape(dims, N, R, total, CPM_MAX_RANK);
    if (s) return s;
    if (!X) return fail(CPM_EINVAL, "X is null");
    if (!out) return fail(CPM_EINVAL, "out is null");
    if (!factors) return fail(CPM_EINVAL, "factors is null");
    if (mode < 0 || mode >= N) return fail(CPM_EINVAL, "mode=%d outside [0, %d)", mode, N);
    for (int k = 0; k < N; ++k)
        if (k != mode && !factors[k]) return fail(CPM_EINVAL, "factors[%d] is null", k);
    return check_factor_reach(dims, N, R, dt, mode);
}

size_t mttkrp_ws(const int64_t *dims, int N, int R, int mode, cpm_dtype dt) {
    // The tiling may depend on X's alignment (vector width of the loads);
    // size the workspace for every alignment a caller can pass.
    size_t b = 0;
    for (uintptr_t a : {(uintptr_t)4096, (uintptr_t)8, (uintptr_t)4, (uintptr_t)2})
        b = std::max(b, make_plan(dims, N, R, mode, dt, (const void *)a).partial_bytes);
    return align_up(b);
}

// Every mode's tiling must keep its buffer-load offsets within one resource.
cpm_status check_reach(const void *X, const int64_t *dims, int N, int R, cpm_dtype dt) {
    for (int n = 0; n < N; ++n)
        if (make_plan(dims, N, R, n, dt, X).max_offset >= kMaxBufferOffset)
            return fail(CPM_EUNSUPPORTED, "mode %d: rows of the tensor are too far apart for one buffer resource "
                        "(4 GiB reach)", n);
    return CPM_OK;
}

size_t max_mttkrp_ws(const int64_t *dims, int N, int R, cpm_dtype dt) {
    size_t m = 0;
    for (int n = 0; n < N; ++n) m = std::max(m, mttkrp_ws(dims, N, R, n, dt));
    return m;
}

// ------------------- all-mode MTTKRP with cross-mode reuse ------------------
// Modes split into [0, s) and [s, N).  Pass A contracts the right group:
// X viewed as (L, I_s, ..., I_{N-1}) with L = I_0 ... I_{s-1}, mode 0, gives
// T_L (L x R).  Pass B contracts the left group: X viewed as (I_0, ...,
// I_{s-1}, Rr), mode s, gives T_R (Rr x R).  Each mode's MTTKRP is then a
// leaf of its group's intermediate (k_tree_leaf).  Used only while the
// intermediates (written once, read by every leaf of their group) move fewer
// entries than one pass over X; for N = 3 the split is fixed at s = 2 and
// further needs pass A to plan as the wide right-first kernel (tree_reach_ok).
struct TreePlan {
    bool use = false;
    int s = 0, nA = 0, nB = 0;
    int64_t L = 1, Rr = 1;
    int64_t dA[CPM_MAX_MODES], dB[CPM_MAX_MODES];
};

TreePlan plan_tree(const int64_t *dims, int N, int R) {
    TreePlan t{};
    if (N < 3) return t;
    if (N == 3) {
        // 3-way: modes 0 and 1 from one pass that contracts mode 2 (a
        // right-first pass over the (I_0 I_1, I_2) view, whose wide output
        // is the intermediate), mode 2 from an ordinary pass; taken only
        // when that wide pass plans as one resident chunk per work-group
        // (tree_reach_ok checks the launch)
        // same entry count rule as below: the intermediates (written once,
        // read by each leaf of their group) must move fewer entries than X
        if (((double)dims[0] * dims[1] * 3 + (double)dims[2] * 2) * R > (double)dims[0] * dims[1] * dims[2])
            return t;
        t.use = true;
        t.s = 2;
        t.L = dims[0] * dims[1];
        t.Rr = dims[2];
        t.nA = 2;
        t.dA[0] = t.L;
        t.dA[1] = dims[2];
        t.nB = 3;
        t.dB[0] = dims[0];
        t.dB[1] = dims[1];
        t.dB[2] = dims[2];
        return t;
    }
    int64_t I = 1;
    for (int k = 0; k < N; ++k) I *= dims[k];
    double best = 0.0;
    int bs = 0;
    int64_t L = 1;
    for (int s = 1; s < N; ++s) {
        L *= dims[s - 1];
        const int64_t Rr = I / L;
        const double cost = ((double)L * (1 + s) + (double)Rr * (1 + N - s)) * R;
        if (bs == 0 || cost < best) {
            best = cost;
            bs = s;
        }
    }
    if (best > (double)I) return t;
    t.use = true;
    t.s = bs;
    for (int k = 0; k < bs; ++k) t.L *= dims[k];
    t.Rr = I / t.L;
    t.nA = N - bs + 1;
    t.dA[0] = t.L;
    for (int k = bs; k < N; ++k) t.dA[k - bs + 1] = dims[k];
    t.nB = bs + 1;
    for (int k = 0; k < bs; ++k) t.dB[k] = dims[k];
    t.dB[bs] = t.Rr;
    return t;
}

bool tree_reach_ok(const TreePlan &t, const void *X, int R, cpm_dtype dt) {
    const Plan a = make_plan(t.dA, t.nA, R, 0, dt, X);
    if (t.nA == 2 && t.nB == 3) {
        // the 3-way split: only the float32 wide pass with one j range per
        // wave and the whole contracted mode resident is fast enough
        if (!(a.kind == kRight32 && a.MB == 4 && a.nlc == 1)) return false;
    }
    return a.max_offset < kMaxBufferOffset && make_plan(t.dB, t.nB, R, t.s, dt, X).max_offset < kMaxBufferOffset;
}

// Leaf launch shape for mode t of a group with dims g[0..m).
constexpr int64_t kLeafBlocks = 4096;
constexpr int64_t kLeafMinPairs = 256;
constexpr int64_t kLeafMaxRowBlocks = 65536;
struct LeafShape {
    int64_t Ll, It, pairs, per_split, S, xblocks;
    int rc_shift, ncb;
};

// vec: the float32 form with 4 rank columns per lane (k_tree_leaf4)
LeafShape leaf_shape(const int64_t *g, int m, int t, int R, bool vec) {
    LeafShape q{};
    q.Ll = 1;
    for (int k = 0; k < t; ++k) q.Ll *= g[k];
    q.It = g[t];
    int64_t Lr = 1;
    for (int k = t + 1; k < m; ++k) Lr *= g[k];
    q.pairs = q.Ll * Lr;
    const int lanes = vec ? R / 4 : R;  // lanes a row's columns need
    const int RC = lanes >= 64 ? 64 : pow2_at_least(lanes);
    q.rc_shift = 0;
    while ((1 << q.rc_shift) < RC) ++q.rc_shift;
    q.ncb = (int)ceil_div(lanes, RC);
    q.xblocks = std::min(q.It, kLeafMaxRowBlocks);
    int64_t S = ceil_div(kLeafBlocks, q.xblocks * q.ncb);
    S = std::max<int64_t>(1, std::min(S, ceil_div(q.pairs, kLeafMinPairs)));
    q.per_split = ceil_div(q.pairs, S);
    q.S = ceil_div(q.pairs, q.per_split);
    return q;
}

constexpr int64_t kPairGroups = 512;

// Both leaves of a two-mode group in one pass (k_pair_leaf): the group's
// first mode has B values, its second A.  Float32 intermediates (float32 and
// split-bf16 paths) with R a multiple of 4 up to 128.
struct PairShape {
    bool ok = false;
    int wpw = 0, ta = 0;      // workers per wave, a values per wave
    int64_t gx = 0, gy = 0;   // b tiles (slices of M_a), a tiles (slices of M_b)
    size_t bytes_a = 0, bytes_b = 0;  // partial slices (0 when one slice is the result)
};

PairShape pair_shape(int64_t B, int64_t A, int R, cpm_dtype dt) {
    PairShape q;
    if (dt == CPM_F64 || R % 4 != 0 || R > 128) return q;
    q.wpw = R <= 32 ? 8 : R <= 64 ? 4 : 2;
    q.gx = ceil_div(B, kPairTB);
    // fewer a values per wave (down to one chunk of wpw) while the grid
    // would hold fewer than kPairGroups work-groups
    q.ta = kPairTA;
    while (q.ta > q.wpw && q.gx * ceil_div(A, 4 * q.ta) < kPairGroups) q.ta /= 2;
    q.gy = ceil_div(A, 4 * q.ta);
    if (q.gy > 65535 || (A * B + kPairTB) * R * 4 > (int64_t)kRsrcRange) return q;
    q.bytes_a = q.gx > 1 ? align_up((size_t)q.gx * A * R * sizeof(float)) : 0;
    q.bytes_b = q.gy > 1 ? align_up((size_t)q.gy * B * R * sizeof(float)) : 0;
    q.ok = true;
    return q;
}

size_t leaf_partial_bytes(const int64_t *dims, int N, int R, cpm_dtype dt, const TreePlan &t) {
    size_t b = 0;
    for (int n = 0; n < N; ++n) {
        const int g0 = n < t.s ? 0 : t.s, g1 = n < t.s ? t.s : N;
        for (bool vec : {false, true}) {
            if (vec && (R % 4 != 0 || dt == CPM_F64)) continue;
            const LeafShape q = leaf_shape(dims + g0, g1 - g0, n - g0, R, vec);
            if (q.S > 1) b = std::max(b, (size_t)q.S * q.It * R * dtype_f_bytes(dt));
        }
        if (g1 - g0 == 2) {
            const PairShape pq = pair_shape(dims[g0], dims[g0 + 1], R, dt);
            if (pq.ok) b = std::max(b, pq.bytes_a + pq.bytes_b);
        }
    }
    return b;
}

struct AllWs {
    void *TL, *TR, *leaf, *mws;
    size_t need;
};

// Workspace of the all-mode MTTKRP, carved from base + off (sizes only when
// base is null): the intermediates, the leaf partials and the workspace of
// the largest single MTTKRP (per mode, or either pass).
AllWs layout_all(const int64_t *dims, int N, int R, cpm_dtype dt, char *base, size_t off) {
    AllWs w{};
    const size_t start = off;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    TreePlan t = plan_tree(dims, N, R);
    // the intermediates are reserved whenever a 16-byte aligned tensor
    // would take the split (an unaligned one may then leave them unused)
    t.use = t.use && tree_reach_ok(t, (const void *)(uintptr_t)4096, R, dt);
    size_t m = max_mttkrp_ws(dims, N, R, dt);
    if (t.use) {
        const size_t fz = dtype_f_bytes(dt);
        w.TL = take((size_t)t.L * R * fz);
        w.TR = take((size_t)t.Rr * R * fz);
        w.leaf = take(leaf_partial_bytes(dims, N, R, dt, t));
        m = std::max(m, mttkrp_ws(t.dA, t.nA, R, 0, dt));
        m = std::max(m, mttkrp_ws(t.dB, t.nB, R, t.s, dt));
    }
    w.mws = take(m);
    w.need = off - start;
    return w;
}

// Pass A (left = true: T_L from the right group's factors) or pass B.
// dst, when non-null, receives the intermediate instead of the workspace
// (a one-mode group's intermediate is that mode's MTTKRP).
cpm_status tree_pass(const TreePlan &t, bool left, const void *X, const void *const *factors, int R, cpm_dtype dt,
                     const AllWs &w, hipStream_t st, void *dst = nullptr, SumList *defer = nullptr) {
    const void *f[CPM_MAX_MODES];
    if (left) {
        const int N = t.nA + t.s - 1;
        f[0] = nullptr;
        for (int k = t.s; k < N; ++k) f[k - t.s + 1] = factors[k];
        const Plan p = make_plan(t.dA, t.nA, R, 0, dt, X);
        return run_mttkrp(p, X, t.dA, t.nA, f, R, 0, dst ? dst : w.TL, dt, w.mws, st, defer);
    }
    for (int k = 0; k < t.s; ++k) f[k] = factors[k];
    f[t.s] = nullptr;
    const Plan p = make_plan(t.dB, t.nB, R, t.s, dt, X);
    return run_mttkrp(p, X, t.dB, t.nB, f, R, t.s, dst ? dst : w.TR, dt, w.mws, st, defer);
}

template <typename T>
cpm_status tree_leaf_t(const TreePlan &t, const int64_t *dims, int N, const void *const *factors, int R, int n,
                       const AllWs &w, T *out, hipStream_t st) {
    const bool left = n < t.s;
    const int g0 = left ? 0 : t.s, g1 = left ? t.s : N;
    // the group's other modes in order: the pair index q = b + Ll * a runs
    // over their Khatri-Rao product, first mode fastest
    int om[CPM_MAX_MODES];
    int no = 0;
    for (int k = g0; k < g1; ++k)
        if (k != n) om[no++] = k;
    const Krp<T> kk = krp_of<T>(factors, dims, om, no);
    const T *Tm = reinterpret_cast<const T *>(left ? w.TL : w.TR);
    // 16-byte rows of T and of every factor read: the 4-column form
    bool vec = std::is_same<T, float>::value && R % 4 == 0 && (uintptr_t)Tm % 16 == 0;
    for (int z = 0; z < no; ++z) vec = vec && (uintptr_t)factors[om[z]] % 16 == 0;
    const LeafShape q = leaf_shape(dims + g0, g1 - g0, n - g0, R, vec);
    T *dst = q.S > 1 ? reinterpret_cast<T *>(w.leaf) : out;
    const dim3 grid((unsigned)q.xblocks, (unsigned)q.S, (unsigned)q.ncb);
    if constexpr (std::is_same<T, float>::value) {
        if (vec) {
            hipLaunchKernelGGL(k_tree_leaf4, grid, dim3(kThreads), 0, st, Tm, q.Ll, q.It, q.pairs, q.per_split, kk,
                               R, q.rc_shift, dst);
            LAUNCH_CHECK("k_tree_leaf4");
        }
    }
    if (!vec) {
        hipLaunchKernelGGL(k_tree_leaf<T>, grid, dim3(kThreads), 0, st, Tm, q.Ll, q.It, q.pairs, q.per_split, kk, R,
                           q.rc_shift, dst);
        LAUNCH_CHECK("k_tree_leaf");
    }
    if (q.S > 1) {
        const Krp<T> none{};
        hipLaunchKernelGGL((k_reduce<T, T>), dim3((unsigned)ceil_div(q.It * R, 64)), dim3(kThreads), 0, st, dst,
                           q.S, q.It, q.It, (int64_t)1, none, R, out);
        LAUNCH_CHECK("k_reduce");
    }
    return CPM_OK;
}

cpm_status tree_leaf(const TreePlan &t, const int64_t *dims, int N, const void *const *factors, int R, int n,
                     cpm_dtype dt, const AllWs &w, void *out, hipStream_t st) {
    if (dt == CPM_F64) return tree_leaf_t<double>(t, dims, N, factors, R, n, w, (double *)out, st);
    return tree_leaf_t<float>(t, dims, N, factors, R, n, w, (float *)out, st);
}

// Whether mode n is alone in its group (its intermediate is its MTTKRP).
bool tree_single(const TreePlan &t, int N, int n) { return n < t.s ? t.s == 1 : t.s == N - 1; }

// Both MTTKRPs of a two-mode group [g0, g0 + 2) from one pass over its
// intermediate, into out_fast (mode g0) and out_slow (mode g0 + 1).  Sets
// *done = false, launching nothing, when the shape or an alignment does not
// allow it (the caller then runs the two single-mode leaves).
cpm_status tree_pair_leaf(const TreePlan &t, const int64_t *dims, const void *const *factors, int R, int g0,
                          cpm_dtype dt, const AllWs &w, void *out_fast, void *out_slow, hipStream_t st,
                          bool *done, SumList *defer = nullptr) {
    *done = false;
    const int64_t B = dims[g0], A = dims[g0 + 1];
    const PairShape q = pair_shape(B, A, R, dt);
    const float *Tm = (const float *)(g0 == 0 ? w.TL : w.TR);
    if (!q.ok || !Tm) return CPM_OK;
    float *PA = q.bytes_a ? (float *)w.leaf : (float *)out_slow;
    float *PB = q.bytes_b ? (float *)((char *)w.leaf + q.bytes_a) : (float *)out_fast;
    for (const void *p : {(const void *)Tm, factors[g0], factors[g0 + 1], (const void *)PA})
        if ((uintptr_t)p % 16 != 0) return CPM_OK;
    const dim3 grid((unsigned)q.gx, (unsigned)q.gy);
    const float *Ub = (const float *)factors[g0], *Ua = (const float *)factors[g0 + 1];
#define PAIR_LEAF(W, T) \
    hipLaunchKernelGGL((k_pair_leaf<W, T>), grid, dim3(kThreads), 0, st, Tm, A, B, Ua, Ub, R, PA, PB)
    if (q.wpw == 8) PAIR_LEAF(8, 8);
    else if (q.wpw == 4 && q.ta == 8) PAIR_LEAF(4, 8);
    else if (q.wpw == 4) PAIR_LEAF(4, 4);
    else if (q.ta == 8) PAIR_LEAF(2, 8);
    else if (q.ta == 4) PAIR_LEAF(2, 4);
    else PAIR_LEAF(2, 2);
#undef PAIR_LEAF
    LAUNCH_CHECK("k_pair_leaf");
    // the slice sums: queued on the caller's list, or launched here
    SumList local;
    SumList &L = defer ? *defer : local;
    cpm_status s = CPM_OK;
    if (q.bytes_a) s = sum_add(L, PA, q.gx, A * R, (float *)out_slow, st);
    if (!s && q.bytes_b) s = sum_add(L, PB, q.gy, B * R, (float *)out_fast, st);
    if (!s && !defer) s = sum_flush(L, st);
    if (s) return s;
    *done = true;
    return CPM_OK;
}

// Every requested mode's MTTKRP (arguments validated, workspace laid out):
// the two-group reuse when it pays, otherwise one ordinary MTTKRP per mode.
cpm_status all_enqueue(const void *X, const int64_t *dims, int N, const void *const *factors, int R,
                       void *const *outs, cpm_dtype dt, const AllWs &w, hipStream_t stream) {
    cpm_status s;
    int nwant = 0;
    bool want_left = false, want_right = false;
    TreePlan tree = plan_tree(dims, N, R);
    for (int n = 0; n < N; ++n)
        if (outs[n]) {
            ++nwant;
            (n < tree.s ? want_left : want_right) = true;
        }
    tree.use = tree.use && nwant >= 3 && w.TL && tree_reach_ok(tree, X, R, dt);
    bool done[CPM_MAX_MODES] = {};
    if (tree.use) {
        // A one-mode group's intermediate is that mode's MTTKRP: its pass
        // writes the output directly.  A two-mode group with both modes
        // wanted takes one pass over its intermediate for both, launched
        // right after the pass that wrote it (the intermediate is then
        // still in the last-level cache).
        // When the right group is one mode, the left pair's slice sums wait
        // for the right pass and go out with its split-K sums in one launch
        // (the pair's slices sit in the leaf workspace, which that pass does
        // not touch); otherwise each list is launched where it is filled.
        const bool merge = want_right && tree_single(tree, N, N - 1);
        SumList sums;
        auto pair_of = [&](int g0) -> cpm_status {
            const int g1 = g0 == 0 ? tree.s : N;
            if (g1 - g0 != 2 || !outs[g0] || !outs[g0 + 1] || dt == CPM_F64) return CPM_OK;
            bool pair = false;
            const cpm_status r = tree_pair_leaf(tree, dims, factors, R, g0, dt, w, outs[g0], outs[g0 + 1], stream,
                                                &pair, merge ? &sums : nullptr);
            done[g0] = done[g0 + 1] = pair;
            return r;
        };
        if (want_left) {
            const bool one = tree_single(tree, N, 0);
            s = tree_pass(tree, true, X, factors, R, dt, w, stream, one ? outs[0] : nullptr);
            if (s) return s;
            done[0] = one;
            s = pair_of(0);
            if (s) return s;
        }
        if (want_right) {
            const bool one = tree_single(tree, N, N - 1);
            s = tree_pass(tree, false, X, factors, R, dt, w, stream, one ? outs[N - 1] : nullptr,
                          merge ? &sums : nullptr);
            if (s) return s;
            done[N - 1] = one;
            s = pair_of(tree.s);
            if (s) return s;
        }
        s = sum_flush(sums, stream);
        if (s) return s;
    }
    for (int n = 0; n < N; ++n) {
        if (!outs[n] || done[n]) continue;
        if (tree.use) {
            s = tree_leaf(tree, dims, N, factors, R, n, dt, w, outs[n], stream);
        } else {
            const Plan p = make_plan(dims, N, R, n, dt, X);
            s = run_mttkrp(p, X, dims, N, factors, R, n, outs[n], dt, w.mws, stream);
        }
        if (s) return s;
    }
    return CPM_OK;
}

// ------------------------- symmetric-pair packed storage -------------------
// The packed tensor viewed as an (N-1)-way tensor (P, I_2, ..., I_{N-1}).
struct SymView {
    int64_t n = 0, P = 0, rest = 1;
    int NV = 0;
    int64_t vd[CPM_MAX_MODES];
};

SymView sym_view(const int64_t *dims, int N) {
    SymView v;
    v.n = dims[0];
    v.P = v.n * (v.n + 1) / 2;
    v.NV = N - 1;
    v.vd[0] = v.P;
    for (int k = 2; k < N; ++k) {
        v.vd[k - 1] = dims[k];
        v.rest *= dims[k];
    }
    return v;
}

// Workspace: the pair factor W and the pair intermediate T (P x R each),
// then the view's all-mode workspace.
struct SymWs {
    void *W, *T;
    AllWs all;
    size_t need;
};

SymWs layout_sym(const SymView &v, int R, cpm_dtype dt, char *base) {
    SymWs w{};
    const size_t pr = align_up((size_t)v.P * R * dtype_f_bytes(dt));
    w.W = base;
    w.T = base ? base + pr : nullptr;
    w.all = layout_all(v.vd, v.NV, R, dt, base, 2 * pr);
    w.need = 2 * pr + w.all.need;
    return w;
}

cpm_status check_sym(const int64_t *dims, int N, int R, cpm_dtype dt) {
    int64_t total;
    cpm_status s = check_dtype(dt);
    if (s) return s;
    s = check_shape(dims, N, R, &total, CPM_MAX_RANK);
    if (s) return s;
    if (N < 3) return fail(CPM_EINVAL, "packed symmetric-pair storage needs N >= 3 (N=%d)", N);
    if (dims[0] != dims[1])
        return fail(CPM_EINVAL, "the symmetric pair needs dims[0] == dims[1] (%lld, %lld)", (long long)dims[0],
                    (long long)dims[1]);
    return CPM_OK;
}

// ------------------ the straightforward baseline (Section 2.3) --------------
// X_(n) reordered explicitly (internal modes), the full Khatri-Rao product
// formed explicitly, one hipBLASLt matrix multiplication.
constexpr size_t kGemmWsBytes = (size_t)32 << 20;
constexpr int kMaxDevicesBlas = 64;

struct ExplicitWs {
    void *Y, *K, *gemm;
    size_t need;
};

ExplicitWs layout_explicit(const int64_t *dims, int N, int R, int mode, cpm_dtype dt, char *base) {
    ExplicitWs w{};
    int64_t I = 1;
    for (int k = 0; k < N; ++k) I *= dims[k];
    const size_t fz = dtype_f_bytes(dt);
    const bool internal = mode > 0 && mode < N - 1;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    w.Y = internal ? take((size_t)I * fz) : nullptr;
    w.K = take((size_t)(I / dims[mode]) * R * fz);
    w.gemm = take(kGemmWsBytes);
    w.need = off;
    return w;
}

// hipBLASLt handle per device, created on first use with that device
// current, and the algorithm chosen for each GEMM shape.
std::mutex g_blas_mu;
hipblasLtHandle_t g_blas[kMaxDevicesBlas];
std::map<std::tuple<int, int, int, int64_t, int64_t, int>, hipblasLtMatmulAlgo_t> g_algo;

cpm_status blas_handle(int dev, hipblasLtHandle_t *h) {
    if (dev < 0 || dev >= kMaxDevicesBlas) return fail(CPM_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevicesBlas);
    if (!g_blas[dev]) {
        hipblasLtHandle_t nh = nullptr;
        if (hipblasLtCreate(&nh) != HIPBLAS_STATUS_SUCCESS || !nh) return fail(CPM_EHIP, "hipblasLtCreate failed");
        g_blas[dev] = nh;
    }
    *h = g_blas[dev];
    return CPM_OK;
}

// D (R x In, column-major, ld R: M row-major) = K^T (R x J, ld R) * op(B):
// rowmajor = false: B is X_(n) column-major (In x J, ld In), op = transpose;
// rowmajor = true: B is X_(n) row-major, i.e. (J x In, ld J), op = none.
cpm_status gemm_mttkrp(const void *K, const void *B, bool rowmajor, int64_t In, int64_t J, int R, cpm_dtype dt,
                       void *out, void *gws, hipStream_t st) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const hipDataType ty = dt == CPM_F64 ? HIP_R_64F : HIP_R_32F;
    const hipblasComputeType_t ct = dt == CPM_F64 ? HIPBLAS_COMPUTE_64F : HIPBLAS_COMPUTE_32F;
    std::lock_guard<std::mutex> lock(g_blas_mu);
    hipblasLtHandle_t h;
    cpm_status s = blas_handle(dev, &h);
    if (s) return s;
    hipblasLtMatmulDesc_t op = nullptr;
    hipblasLtMatrixLayout_t la = nullptr, lb = nullptr, lc = nullptr;
    hipblasLtMatmulPreference_t pref = nullptr;
    auto cleanup = [&]() {
        if (pref) hipblasLtMatmulPreferenceDestroy(pref);
        if (lc) hipblasLtMatrixLayoutDestroy(lc);
        if (lb) hipblasLtMatrixLayoutDestroy(lb);
        if (la) hipblasLtMatrixLayoutDestroy(la);
        if (op) hipblasLtMatmulDescDestroy(op);
    };
    const hipblasOperation_t ta = HIPBLAS_OP_N, tb = rowmajor ? HIPBLAS_OP_N : HIPBLAS_OP_T;
    bool ok = hipblasLtMatmulDescCreate(&op, ct, ty) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatmulDescSetAttribute(op, HIPBLASLT_MATMUL_DESC_TRANSA, &ta, sizeof(ta)) ==
                  HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatmulDescSetAttribute(op, HIPBLASLT_MATMUL_DESC_TRANSB, &tb, sizeof(tb)) ==
                  HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatrixLayoutCreate(&la, ty, (uint64_t)R, (uint64_t)J, R) == HIPBLAS_STATUS_SUCCESS &&
              (rowmajor ? hipblasLtMatrixLayoutCreate(&lb, ty, (uint64_t)J, (uint64_t)In, J)
                        : hipblasLtMatrixLayoutCreate(&lb, ty, (uint64_t)In, (uint64_t)J, In)) ==
                  HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatrixLayoutCreate(&lc, ty, (uint64_t)R, (uint64_t)In, R) == HIPBLAS_STATUS_SUCCESS;
    if (!ok) {
        cleanup();
        return fail(CPM_EHIP, "hipBLASLt descriptor set-up failed");
    }
    const auto key = std::make_tuple(dev, (int)dt, R, In, J, (int)rowmajor);
    auto it = g_algo.find(key);
    if (it == g_algo.end()) {
        const uint64_t wsb = kGemmWsBytes;
        hipblasLtMatmulHeuristicResult_t res[1];
        int count = 0;
        ok = hipblasLtMatmulPreferenceCreate(&pref) == HIPBLAS_STATUS_SUCCESS &&
             hipblasLtMatmulPreferenceSetAttribute(pref, HIPBLASLT_MATMUL_PREF_MAX_WORKSPACE_BYTES, &wsb,
                                                   sizeof(wsb)) == HIPBLAS_STATUS_SUCCESS &&
             hipblasLtMatmulAlgoGetHeuristic(h, op, la, lb, lc, lc, pref, 1, res, &count) ==
                 HIPBLAS_STATUS_SUCCESS &&
             count > 0;
        if (!ok) {
            cleanup();
            return fail(CPM_EUNSUPPORTED, "hipBLASLt has no algorithm for this %s GEMM (%d x %lld x %lld)",
                        dt == CPM_F64 ? "float64" : "float32", R, (long long)In, (long long)J);
        }
        it = g_algo.emplace(key, res[0].algo).first;
    }
    const double a64 = 1.0, b64 = 0.0;
    const float a32 = 1.f, b32 = 0.f;
    const void *alpha = dt == CPM_F64 ? (const void *)&a64 : (const void *)&a32;
    const void *beta = dt == CPM_F64 ? (const void *)&b64 : (const void *)&b32;
    const hipblasStatus_t bs =
        hipblasLtMatmul(h, op, alpha, K, la, B, lb, beta, out, lc, out, lc, &it->second, gws, kGemmWsBytes, st);
    cleanup();
    if (bs != HIPBLAS_STATUS_SUCCESS) return fail(CPM_EHIP, "hipblasLtMatmul failed (status %d)", (int)bs);
    return CPM_OK;
}

// ------------------------------ residual ------------------------------------
// X viewed as Rr rows (modes s..N-1) of L contiguous entries (modes 0..s-1);
// s maximises the used part of a work-group's 128 x 32 output tile,
// min(Rr, 128) * min(L, 32), and among equals takes the longest rows.  K_L is split as in
// the MTTKRP kernels: an inner group of the fastest modes (up to a 128-entry
// chunk) and an outer scale.
constexpr int kResChunk = 128;
constexpr int64_t kCus = 256;            // compute units of the MI355X
constexpr size_t kLdsPerCu = 160 * 1024; // LDS bytes per compute unit
constexpr size_t kResStaticLds = kThreads * sizeof(double);
// longest row of the view: 32 rows of it must stay within one buffer
// resource's 32-bit offsets (128 L bytes below kRsrcRange)
constexpr int64_t kResMaxL = 33554430;
struct ResPlan {
    int s = 0, q = 0, LC = 32, RP = 32;
    int64_t Rr = 1, L = 1, G_in = 1, n_outer = 1, ntiles = 1, nlc = 1, S = 1, bps = 1;
    size_t lds = 0;
};

ResPlan plan_residual(const int64_t *dims, int N, int R) {
    ResPlan p;
    int64_t I = 1;
    for (int k = 0; k < N; ++k) I *= dims[k];
    // used part of a work-group's 128 x 32 output tile; among equals the
    // longest rows
    int64_t best = -1, L = 1;
    for (int s = 0; s <= N; ++s) {
        if (s > 0) L *= dims[s - 1];
        if (L > kResMaxL) break;
        const int64_t eff = std::min<int64_t>(I / L, kResRows) * std::min<int64_t>(L, 32);
        if (eff >= best) {
            best = eff;
            p.s = s;
        }
    }
    p.L = 1;
    for (int k = 0; k < p.s; ++k) p.L *= dims[k];
    p.Rr = I / p.L;
    p.q = 0;
    p.G_in = 1;
    while (p.q < p.s && p.G_in < kResChunk) p.G_in *= dims[p.q++];
    p.LC = (int)std::min<int64_t>(kResChunk, ceil_div(p.G_in, 32) * 32);
    p.nlc = ceil_div(p.G_in, p.LC);
    p.n_outer = p.L / p.G_in;
    p.ntiles = ceil_div(p.Rr, kResRows);
    p.RP = R <= 32 ? 32 : (R <= 64 ? 64 : 128);
    p.lds = p.RP == 32 ? residual_lds_bytes<32>(p.LC)
                       : (p.RP == 64 ? residual_lds_bytes<64>(p.LC) : residual_lds_bytes<128>(p.LC));
    // one round of resident work-groups (LDS decides how many fit a CU)
    const int64_t per_cu = std::max<int64_t>(1, (int64_t)kLdsPerCu / (int64_t)(p.lds + kResStaticLds));
    const int64_t groups = kCus * per_cu;
    int64_t S = std::max<int64_t>(1, groups / (p.ntiles * p.nlc));
    S = std::min(S, p.n_outer);
    p.bps = ceil_div(p.n_outer, S);
    p.S = ceil_div(p.n_outer, p.bps);
    return p;
}

size_t residual_ws(const int64_t *dims, int N, int R) {
    const ResPlan p = plan_residual(dims, N, R);
    return align_up((size_t)(p.ntiles * p.nlc * p.S) * sizeof(double));
}

template <int RP, bool BF>
cpm_status launch_residual(const ResPlan &p, const void *X, int64_t I, const Krp<float> &kr,
                           const Krp<float> &kin, const Krp<float> &kout, int R, double *part, hipStream_t st) {
    const void *fn = (const void *)k_residual32<RP, BF>;
    if (p.lds > 65536) HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds));
    const int64_t blocks = p.ntiles * p.nlc * p.S;
    hipLaunchKernelGGL((k_residual32<RP, BF>), dim3((unsigned)blocks), dim3(kThreads), p.lds, st, X, I, p.Rr, p.L,
                       p.G_in, p.n_outer, kr, kin, kout, R, p.LC, p.ntiles, p.nlc, p.bps, part);
    LAUNCH_CHECK("k_residual32");
    return CPM_OK;
}

cpm_status residual_enqueue(const void *X, const int64_t *dims, int N, const void *const *factors, int R,
                            cpm_dtype dt, double *part, double *out, hipStream_t st) {
    const ResPlan p = plan_residual(dims, N, R);
    int in_modes[CPM_MAX_MODES], out_modes[CPM_MAX_MODES], r_modes[CPM_MAX_MODES];
    int nin = 0, nout = 0, nr = 0;
    for (int k = 0; k < p.q; ++k) in_modes[nin++] = k;
    for (int k = p.q; k < p.s; ++k) out_modes[nout++] = k;
    for (int k = p.s; k < N; ++k) r_modes[nr++] = k;
    const Krp<float> kin = krp_of<float>(factors, dims, in_modes, nin);
    const Krp<float> kout = krp_of<float>(factors, dims, out_modes, nout);
    const Krp<float> kr = krp_of<float>(factors, dims, r_modes, nr);
    const int64_t I = p.L * p.Rr;
    const bool bf = dt == CPM_BF16X2;
    cpm_status s;
    if (p.RP == 32)
        s = bf ? launch_residual<32, true>(p, X, I, kr, kin, kout, R, part, st)
               : launch_residual<32, false>(p, X, I, kr, kin, kout, R, part, st);
    else if (p.RP == 64)
        s = bf ? launch_residual<64, true>(p, X, I, kr, kin, kout, R, part, st)
               : launch_residual<64, false>(p, X, I, kr, kin, kout, R, part, st);
    else
        s = bf ? launch_residual<128, true>(p, X, I, kr, kin, kout, R, part, st)
               : launch_residual<128, false>(p, X, I, kr, kin, kout, R, part, st);
    if (s) return s;
    const int64_t n = p.ntiles * p.nlc * p.S;
    hipLaunchKernelGGL(k_sum_vector, dim3(1), dim3(kThreads), 0, st, part, (int)n, out);
    LAUNCH_CHECK("k_sum_vector");
    return CPM_OK;
}

// ---------------------------- ALS / gradient -------------------------------
struct SolveWs {
    int *status;
    double *xnorm2, *inner, *result;
    double *grams, *gpart, *H, *L, *Lt, *hpart;
    void *M, *M2, *snap, *sumsq;  // M2: the second output of a two-mode leaf (gradient only)
    AllWs all;  // intermediates of the all-mode MTTKRP and the MTTKRP workspace
    size_t need;
};

// Gram partials: about 32 rows per work-group, at most kGramBlocks slices.
constexpr int64_t kGramRows = 32;
constexpr int64_t kGramBlocks = 64;
int64_t gram_blocks(int64_t I) { return std::min(kGramBlocks, ceil_div(I, kGramRows)); }
constexpr int kSumsqBlocks = 1024;
constexpr int kHadsumBlocks = 64;

// f (or the fit) from ||X||^2, <M_{N-1}, U_{N-1}> and the Grams.
cpm_status loss_enqueue(const double *xnorm2, const double *inner, const double *grams, int N, int R,
                        double *hpart, int want_fit, double *out, hipStream_t st) {
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kHadsumBlocks, ceil_div((int64_t)R * R, kThreads)));
    hipLaunchKernelGGL(k_hadsum_partial, dim3(blocks), dim3(kThreads), 0, st, grams, N, R, hpart);
    LAUNCH_CHECK("k_hadsum_partial");
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(64), 0, st, xnorm2, inner, hpart, blocks, want_fit, out);
    LAUNCH_CHECK("k_loss");
    return CPM_OK;
}

SolveWs layout_solve(const int64_t *dims, int N, int R, cpm_dtype dt, char *base, bool snapshot) {
    SolveWs w{};
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    int64_t maxI = 0, sumI = 0, maxblocks = 1;
    for (int k = 0; k < N; ++k) {
        maxI = std::max(maxI, dims[k]);
        sumI += dims[k];
        maxblocks = std::max(maxblocks, gram_blocks(dims[k]));
    }
    const size_t fz = dtype_f_bytes(dt);
    w.status = (int *)take(sizeof(int));
    w.xnorm2 = (double *)take(sizeof(double));
    w.inner = (double *)take(sizeof(double));
    w.result = (double *)take(sizeof(double));
    w.grams = (double *)take((size_t)N * R * R * sizeof(double));
    w.gpart = (double *)take((size_t)maxblocks * R * R * sizeof(double));
    w.H = (double *)take((size_t)R * R * sizeof(double));
    w.L = (double *)take((size_t)R * R * sizeof(double));
    w.Lt = (double *)take((size_t)R * R * sizeof(double));
    w.hpart = (double *)take((size_t)kHadsumBlocks * sizeof(double));
    w.M = take((size_t)maxI * R * fz);
    w.M2 = snapshot ? nullptr : take((size_t)maxI * R * fz);
    w.snap = snapshot ? take((size_t)sumI * R * fz) : nullptr;
    w.sumsq = take((size_t)kSumsqBlocks * sizeof(double));
    w.all = layout_all(dims, N, R, dt, base, off);
    w.need = off + w.all.need;
    return w;
}

template <typename T>
cpm_status gram_t(const T *U, int64_t I, int R, double *gpart, double *G, hipStream_t st) {
    const int64_t blocks = gram_blocks(I);
    const int64_t rows = ceil_div(I, blocks);
    const int tr = (R + 3) / 4;
    const unsigned tiles = (unsigned)ceil_div((int64_t)tr * tr, kThreads);
    hipLaunchKernelGGL((k_gram_partial<T>), dim3((unsigned)blocks, tiles), dim3(kThreads), 0, st, U, I, R, rows,
                       gpart);
    LAUNCH_CHECK("k_gram_partial");
    hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)ceil_div((int64_t)R * R, kThreads)), dim3(kThreads), 0, st,
                       gpart, blocks, (int64_t)R * R, G);
    LAUNCH_CHECK("k_sum_slices");
    return CPM_OK;
}

cpm_status gram(const void *U, int64_t I, int R, cpm_dtype dt, double *gpart, double *G, hipStream_t st) {
    if (dt == CPM_F64) return gram_t<double>((const double *)U, I, R, gpart, G, st);
    return gram_t<float>((const float *)U, I, R, gpart, G, st);
}

cpm_status xnorm2_enqueue(const void *X, int64_t total, cpm_dtype dt, double *part, double *out, hipStream_t st) {
    const int blocks = (int)std::min<int64_t>(kSumsqBlocks, ceil_div(total, kThreads));
    const int vec = ((uintptr_t)X % 16 == 0 && total % 8 == 0) ? 1 : 0;
    if (dt == CPM_F32)
        hipLaunchKernelGGL(k_sumsq_partial<CPM_F32>, dim3(blocks), dim3(kThreads), 0, st, X, total, vec, part);
    else if (dt == CPM_F64)
        hipLaunchKernelGGL(k_sumsq_partial<CPM_F64>, dim3(blocks), dim3(kThreads), 0, st, X, total, 0, part);
    else
        hipLaunchKernelGGL(k_sumsq_partial<CPM_BF16X2>, dim3(blocks), dim3(kThreads), 0, st, X, total, vec, part);
    LAUNCH_CHECK("k_sumsq_partial");
    hipLaunchKernelGGL(k_sum_vector, dim3(1), dim3(kThreads), 0, st, part, blocks, out);
    LAUNCH_CHECK("k_sum_vector");
    return CPM_OK;
}

cpm_status hadamard_except(const double *grams, int N, int R, int skip, double *H, hipStream_t st) {
    hipLaunchKernelGGL(k_hadamard_except, dim3((unsigned)ceil_div((int64_t)R * R, kThreads)), dim3(kThreads), 0,
                       st, grams, N, R, skip, H);
    LAUNCH_CHECK("k_hadamard_except");
    return CPM_OK;
}

// *out = <a, b> in float64: fixed-split partials into part (kDotBlocks
// doubles), summed in order.
constexpr int kDotBlocks = 64;
cpm_status dot_enqueue(const void *a, const void *b, int64_t n, cpm_dtype dt, double *part, double *out,
                       hipStream_t st) {
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, ceil_div(n, kThreads)));
    if (dt == CPM_F64)
        hipLaunchKernelGGL(k_dot_partial<double>, dim3(blocks), dim3(kThreads), 0, st, (const double *)a,
                           (const double *)b, n, part);
    else
        hipLaunchKernelGGL(k_dot_partial<float>, dim3(blocks), dim3(kThreads), 0, st, (const float *)a,
                           (const float *)b, n, part);
    LAUNCH_CHECK("k_dot_partial");
    hipLaunchKernelGGL(k_sum_vector, dim3(1), dim3(kThreads), 0, st, part, blocks, out);
    LAUNCH_CHECK("k_sum_vector");
    return CPM_OK;
}

cpm_status check_lds_for_cholesky(int R) {
    int dev = 0, lds = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t need = (size_t)R * R * sizeof(double) + 64;
    if ((size_t)lds < need)
        return fail(CPM_EUNSUPPORTED, "R=%d needs %zu bytes of LDS for the Cholesky factorisation, device has %d",
                    R, need, lds);
    return CPM_OK;
}

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and cached.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

cpm_status scratch_ptr(void **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CPM_EUNSUPPORTED, "device %d beyond %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(CPM_EHIP, "hipGetSymbolAddress gave a null address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return CPM_OK;
}

}  // namespace

// ================================ C-ABI ====================================
extern "C" {

int cpm_version(void) { return 10000; }

const char *cpm_last_error(void) { return g_last_error.c_str(); }

size_t cpm_mttkrp_workspace_bytes(const int64_t *dims, int N, int R, int mode, cpm_dtype dt) {
    int64_t total;
    std::string saved = g_last_error;
    if (check_dtype(dt) || check_shape(dims, N, R, &total, CPM_MAX_RANK) || mode < 0 || mode >= N) {
        g_last_error = saved;
        return 0;
    }
    return mttkrp_ws(dims, N, R, mode, dt);
}

cpm_status mttkrp(const void *X, const int64_t *dims, int N, const void *const *factors, int R, int mode,
                  void *out, cpm_dtype dt, void *workspace, size_t ws_bytes, hipStream_t stream) {
    int64_t total;
    cpm_status s = validate_mttkrp(X, dims, N, factors, R, mode, out, dt, &total);
    if (s) return s;
    Plan p = make_plan(dims, N, R, mode, dt, X);
    if (p.max_offset >= kMaxBufferOffset)
        return fail(CPM_EUNSUPPORTED, "mode %d: entries %lld apart along mode %d exceed the 4 GiB reach of one "
                    "buffer resource", mode, (long long)p.IL, mode);
    const size_t need = align_up(p.partial_bytes);
    if (need > 0 && (!workspace || ws_bytes < need))
        return fail(CPM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    return run_mttkrp(p, X, dims, N, factors, R, mode, out, dt, workspace, stream);
}

int cpm_mttkrp_describe(const int64_t *dims, int N, int R, int mode, cpm_dtype dt, const void *X, char *buf,
                        size_t len) {
    int64_t total;
    cpm_status s = check_dtype(dt);
    if (s) return s;
    s = check_shape(dims, N, R, &total, CPM_MAX_RANK);
    if (s) return s;
    if (mode < 0 || mode >= N) return fail(CPM_EINVAL, "mode=%d outside [0, %d)", mode, N);
    if (!buf || len == 0) return fail(CPM_EINVAL, "buf is null or empty");
    const Plan p = make_plan(dims, N, R, mode, dt, X);
    char name[96];
    switch (p.kind) {
    case kLeft32: snprintf(name, sizeof(name), "k_left32<NC=%d,WM=%d>", p.NB, p.MB); break;
    case kRight32: snprintf(name, sizeof(name), "k_right32<NC=%d,TJ=%d,WJ=%d>", p.NB, p.Q, p.MB); break;
    case kLeft:
        snprintf(name, sizeof(name), "k_contract_left<%s,NB=%d,MB=%d,V4=%d,Q=%d>", dt == CPM_F64 ? "f64" : "f32",
                 p.NB, p.MB, (int)p.v4, p.Q);
        break;
    case kRight:
        snprintf(name, sizeof(name), "k_contract_right<%s,NB=%d,MJ=1,V4=%d>", dt == CPM_F64 ? "f64" : "f32",
                 p.NB, (int)p.v4);
        break;
    case kBf16Left:
        snprintf(name, sizeof(name), "k_contract_left_bf16<NB=%d,MB=%d,Q=%d,V8=%d,WM=%d>", p.NB, p.MB, p.Q,
                 (int)p.v4, p.WMg);
        break;
    default: snprintf(name, sizeof(name), "k_contract_right_bf16<NB=%d,V8=%d>", p.NB, (int)p.v4); break;
    }
    snprintf(buf, len, "%s grid=(%lld,%lld,%d) lds=%zu chunk=%d steps_per_block=%d inner=%lld outer_blocks=%lld "
             "splits=%lld chunks=%lld reduce=%d",
             name, (long long)p.ntiles, (long long)(p.S * p.nlc), p.ncb, p.lds, p.LC, p.SPB, (long long)p.G_in,
             (long long)p.n_outer, (long long)p.S, (long long)p.nlc, (int)p.reduce);
    return CPM_OK;
}

cpm_status mttkrp_scratch(const void *X, const int64_t *dims, int N, const void *const *factors, int R, int mode,
                          void *out, cpm_dtype dt, hipStream_t stream) {
    int64_t total;
    cpm_status s = validate_mttkrp(X, dims, N, factors, R, mode, out, dt, &total);
    if (s) return s;
    Plan p = make_plan(dims, N, R, mode, dt, X);
    if (p.max_offset >= kMaxBufferOffset)
        return fail(CPM_EUNSUPPORTED, "mode %d: entries %lld apart along mode %d exceed the 4 GiB reach of one "
                    "buffer resource", mode, (long long)p.IL, mode);
    const size_t need = align_up(p.partial_bytes);
    if (need > (size_t)CPM_SCRATCH_BYTES)
        return fail(CPM_EUNSUPPORTED, "this MTTKRP needs %zu bytes of partial results, above the %zu-byte scratch "
                    "array; call mttkrp with a workspace", need, (size_t)CPM_SCRATCH_BYTES);
    void *ws = nullptr;
    if (need > 0) {
        s = scratch_ptr(&ws);
        if (s) return s;
    }
    return run_mttkrp(p, X, dims, N, factors, R, mode, out, dt, ws, stream);
}

size_t cpm_mttkrp_all_workspace_bytes(const int64_t *dims, int N, int R, cpm_dtype dt) {
    int64_t total;
    std::string saved = g_last_error;
    if (check_dtype(dt) || check_shape(dims, N, R, &total, CPM_MAX_RANK)) {
        g_last_error = saved;
        return 0;
    }
    return layout_all(dims, N, R, dt, nullptr, 0).need;
}

cpm_status mttkrp_all(const void *X, const int64_t *dims, int N, const void *const *factors, int R,
                      void *const *outs, cpm_dtype dt, void *workspace, size_t ws_bytes, hipStream_t stream) {
    int64_t total;
    cpm_status s = check_dtype(dt);
    if (s) return s;
    s = check_shape(dims, N, R, &total, CPM_MAX_RANK);
    if (s) return s;
    if (!X) return fail(CPM_EINVAL, "X is null");
    if (!factors) return fail(CPM_EINVAL, "factors is null");
    if (!outs) return fail(CPM_EINVAL, "outs is null");
    for (int k = 0; k < N; ++k)
        if (!factors[k]) return fail(CPM_EINVAL, "factors[%d] is null", k);
    s = check_factor_reach(dims, N, R, dt, -1);
    if (s) return s;
    const size_t need = layout_all(dims, N, R, dt, nullptr, 0).need;
    if (need > 0 && (!workspace || ws_bytes < need))
        return fail(CPM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    s = check_reach(X, dims, N, R, dt);
    if (s) return s;
    return all_enqueue(X, dims, N, factors, R, outs, dt, layout_all(dims, N, R, dt, (char *)workspace, 0), stream);
}

size_t cpm_sympair_workspace_bytes(const int64_t *dims, int N, int R, cpm_dtype dt) {
    std::string saved = g_last_error;
    if (check_sym(dims, N, R, dt)) {
        g_last_error = saved;
        return 0;
    }
    return layout_sym(sym_view(dims, N), R, dt, nullptr).need;
}

cpm_status mttkrp_sympair(const void *Xp, const int64_t *dims, int N, const void *const *factors, int R,
                          void *const *outs, cpm_dtype dt, void *workspace, size_t ws_bytes, hipStream_t stream) {
    cpm_status s = check_sym(dims, N, R, dt);
    if (s) return s;
    if (!Xp) return fail(CPM_EINVAL, "Xp is null");
    if (!factors) return fail(CPM_EINVAL, "factors is null");
    if (!outs) return fail(CPM_EINVAL, "outs is null");
    for (int k = 0; k < N; ++k)
        if (!factors[k]) return fail(CPM_EINVAL, "factors[%d] is null", k);
    s = check_factor_reach(dims, N, R, dt, -1);
    if (s) return s;
    const SymView v = sym_view(dims, N);
    s = check_factor_reach(v.vd, 1, R, dt, -1);  // the pair factor W
    if (s) return s;
    const size_t need = layout_sym(v, R, dt, nullptr).need;
    if (!workspace || ws_bytes < need)
        return fail(CPM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    s = check_reach(Xp, v.vd, v.NV, R, dt);
    if (s) return s;
    const SymWs w = layout_sym(v, R, dt, (char *)workspace);
    const bool want_pair = outs[0] || outs[1];
    bool want_rest = false;
    for (int k = 2; k < N; ++k) want_rest = want_rest || outs[k];
    if (!want_pair && !want_rest) return CPM_OK;
    const size_t fz = dtype_f_bytes(dt);
    if (want_rest) {
        const unsigned blocks = (unsigned)std::min<int64_t>(4096, ceil_div(v.P * R, kThreads));
        if (fz == 8)
            hipLaunchKernelGGL(k_sympair_rows<double>, dim3(blocks), dim3(kThreads), 0, stream,
                               (const double *)factors[0], (const double *)factors[1], v.P, R, (double *)w.W);
        else
            hipLaunchKernelGGL(k_sympair_rows<float>, dim3(blocks), dim3(kThreads), 0, stream,
                               (const float *)factors[0], (const float *)factors[1], v.P, R, (float *)w.W);
        LAUNCH_CHECK("k_sympair_rows");
    }
    // the view: factors (W, U_2, ...), outputs (T, M_2, ...)
    const void *vf[CPM_MAX_MODES];
    void *vo[CPM_MAX_MODES];
    vf[0] = want_rest ? w.W : nullptr;
    vo[0] = want_pair ? w.T : nullptr;
    for (int k = 2; k < N; ++k) {
        vf[k - 1] = factors[k];
        vo[k - 1] = outs[k];
    }
    s = all_enqueue(Xp, v.vd, v.NV, vf, R, vo, dt, w.all, stream);
    if (s) return s;
    for (int m = 0; m < 2; ++m) {
        if (!outs[m]) continue;
        const dim3 grid((unsigned)v.n, (unsigned)ceil_div(R, 64));
        const void *other = factors[1 - m];
        if (fz == 8)
            hipLaunchKernelGGL(k_sympair_leaf<double>, grid, dim3(kThreads), 0, stream, (const double *)w.T,
                               (const double *)other, v.n, R, (double *)outs[m]);
        else
            hipLaunchKernelGGL(k_sympair_leaf<float>, grid, dim3(kThreads), 0, stream, (const float *)w.T,
                               (const float *)other, v.n, R, (float *)outs[m]);
        LAUNCH_CHECK("k_sympair_leaf");
    }
    return CPM_OK;
}

cpm_status cpm_pack_sympair(const void *X, const int64_t *dims, int N, cpm_dtype dt, void *Xp, hipStream_t stream) {
    cpm_status s = check_sym(dims, N, 1, dt);
    if (s) return s;
    if (!X || !Xp) return fail(CPM_EINVAL, "X or Xp is null");
    const SymView v = sym_view(dims, N);
    const dim3 grid((unsigned)ceil_div(v.P, kThreads), (unsigned)std::min<int64_t>(v.rest, 1024),
                    dt == CPM_BF16X2 ? 2u : 1u);
    if (dt == CPM_F64)
        hipLaunchKernelGGL(k_pack_sympair<uint64_t>, grid, dim3(kThreads), 0, stream, (const uint64_t *)X, v.n,
                           v.rest, (uint64_t *)Xp);
    else if (dt == CPM_F32)
        hipLaunchKernelGGL(k_pack_sympair<uint32_t>, grid, dim3(kThreads), 0, stream, (const uint32_t *)X, v.n,
                           v.rest, (uint32_t *)Xp);
    else
        hipLaunchKernelGGL(k_pack_sympair<uint16_t>, grid, dim3(kThreads), 0, stream, (const uint16_t *)X, v.n,
                           v.rest, (uint16_t *)Xp);
    LAUNCH_CHECK("k_pack_sympair");
    return CPM_OK;
}

size_t cpm_explicit_workspace_bytes(const int64_t *dims, int N, int R, int mode, cpm_dtype dt) {
    int64_t total;
    std::string saved = g_last_error;
    if (check_dtype(dt) || dt == CPM_BF16X2 || check_shape(dims, N, R, &total, CPM_MAX_RANK) || mode < 0 ||
        mode >= N) {
        g_last_error = saved;
        return 0;
    }
    return layout_explicit(dims, N, R, mode, dt, nullptr).need;
}

cpm_status mttkrp_explicit(const void *X, const int64_t *dims, int N, const void *const *factors, int R, int mode,
                           void *out, cpm_dtype dt, void *workspace, size_t ws_bytes, hipStream_t stream) {
    int64_t total;
    cpm_status s = validate_mttkrp(X, dims, N, factors, R, mode, out, dt, &total);
    if (s) return s;
    if (dt == CPM_BF16X2) return fail(CPM_EUNSUPPORTED, "mttkrp_explicit takes float32 or float64 tensors");
    const size_t need = layout_explicit(dims, N, R, mode, dt, nullptr).need;
    if (!workspace || ws_bytes < need)
        return fail(CPM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    const ExplicitWs w = layout_explicit(dims, N, R, mode, dt, (char *)workspace);
    int64_t IL = 1, IR = 1;
    for (int k = 0; k < mode; ++k) IL *= dims[k];
    for (int k = mode + 1; k < N; ++k) IR *= dims[k];
    const int64_t In = dims[mode], J = IL * IR;
    // 1. X_(n): reordered for internal modes; the tensor itself otherwise
    const void *B = X;
    const bool rowmajor = mode == N - 1 && N > 1;
    if (w.Y) {
        const int64_t tiles = ceil_div(IL, 64) * ceil_div(In, 64) * IR;
        const unsigned blocks = (unsigned)std::min<int64_t>(tiles, 65536);
        if (dt == CPM_F64)
            hipLaunchKernelGGL(k_unfold<uint64_t>, dim3(blocks), dim3(kThreads), 0, stream, (const uint64_t *)X, IL,
                               In, IR, (uint64_t *)w.Y);
        else
            hipLaunchKernelGGL(k_unfold<uint32_t>, dim3(blocks), dim3(kThreads), 0, stream, (const uint32_t *)X, IL,
                               In, IR, (uint32_t *)w.Y);
        LAUNCH_CHECK("k_unfold");
        B = w.Y;
    }
    // 2. the full Khatri-Rao product, rows in the natural order of the other
    // modes (mode 0 fastest): U_{N-1} kr ... kr U_{n+1} kr U_{n-1} kr ... kr U_0
    int om[CPM_MAX_MODES];
    int no = 0;
    for (int k = 0; k < N; ++k)
        if (k != mode) om[no++] = k;
    const int RP = (R + 15) / 16 * 16;
    const unsigned kblocks = (unsigned)ceil_div(J, 64);
    if (dt == CPM_F64) {
        const Krp<double> k = krp_of<double>(factors, dims, om, no);
        hipLaunchKernelGGL(k_krp_rows<double>, dim3(kblocks), dim3(kThreads), 0, stream, k, R, RP, (int64_t)0, J,
                           (double *)w.K);
    } else {
        const Krp<float> k = krp_of<float>(factors, dims, om, no);
        hipLaunchKernelGGL(k_krp_rows<float>, dim3(kblocks), dim3(kThreads), 0, stream, k, R, RP, (int64_t)0, J,
                           (float *)w.K);
    }
    LAUNCH_CHECK("k_krp_rows");
    // 3. one GEMM
    return gemm_mttkrp(w.K, B, rowmajor, In, J, R, dt, out, w.gemm, stream);
}

size_t cpm_residual2_workspace_bytes(const int64_t *dims, int N, int R, cpm_dtype dt) {
    int64_t total;
    std::string saved = g_last_error;
    if (check_dtype(dt) || dt == CPM_F64 || check_shape(dims, N, R, &total, CPM_MAX_RANK_SOLVE)) {
        g_last_error = saved;
        return 0;
    }
    return residual_ws(dims, N, R);
}

cpm_status cpm_residual2(const void *X, const int64_t *dims, int N, const void *const *factors, int R,
                         cpm_dtype dt, double *out_dev, void *workspace, size_t ws_bytes, hipStream_t stream) {
    int64_t total;
    cpm_status s = check_dtype(dt);
    if (s) return s;
    if (dt == CPM_F64) return fail(CPM_EUNSUPPORTED, "cpm_residual2 takes float32 or split-bf16 tensors");
    s = check_shape(dims, N, R, &total, CPM_MAX_RANK_SOLVE);
    if (s) return s;
    if (!X) return fail(CPM_EINVAL, "X is null");
    if (!out_dev) return fail(CPM_EINVAL, "out_dev is null");
    if (!factors) return fail(CPM_EINVAL, "factors is null");
    for (int k = 0; k < N; ++k)
        if (!factors[k]) return fail(CPM_EINVAL, "factors[%d] is null", k);
    s = check_factor_reach(dims, N, R, dt, -1);
    if (s) return s;
    const size_t need = residual_ws(dims, N, R);
    if (!workspace || ws_bytes < need)
        return fail(CPM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    return residual_enqueue(X, dims, N, factors, R, dt, (double *)workspace, out_dev, stream);
}

size_t cpm_cp_als_workspace_bytes(const int64_t *dims, int N, int R, cpm_dtype dt) {
    int64_t total;
    std::string saved = g_last_error;
    if (check_dtype(dt) || check_shape(dims, N, R, &total, CPM_MAX_RANK_SOLVE)) {
        g_last_error = saved;
        return 0;
    }
    return layout_solve(dims, N, R, dt, nullptr, true).need;
}

size_t cpm_cp_grad_workspace_bytes(const int64_t *dims, int N, int R, cpm_dtype dt) {
    int64_t total;
    std::string saved = g_last_error;
    if (check_dtype(dt) || check_shape(dims, N, R, &total, CPM_MAX_RANK)) {
        g_last_error = saved;
        return 0;
    }
    return layout_solve(dims, N, R, dt, nullptr, false).need;
}

cpm_status cp_als_step(const void *X, const int64_t *dims, int N, void *const *factors, int R, cpm_dtype dt,
                       double xnorm2, double *fit_out, void *workspace, size_t ws_bytes, hipStream_t stream) {
    int64_t total;
    cpm_status s = check_dtype(dt);
    if (s) return s;
    s = check_shape(dims, N, R, &total, CPM_MAX_RANK_SOLVE);
    if (s) return s;
    if (!X) return fail(CPM_EINVAL, "X is null");
    if (!factors) return fail(CPM_EINVAL, "factors is null");
    for (int k = 0; k < N; ++k)
        if (!factors[k]) return fail(CPM_EINVAL, "factors[%d] is null", k);
    s = check_factor_reach(dims, N, R, dt, -1);
    if (s) return s;
    const size_t need = layout_solve(dims, N, R, dt, nullptr, true).need;
    if (!workspace || ws_bytes < need)
        return fail(CPM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    s = check_reach(X, dims, N, R, dt);
    if (s) return s;
    s = check_lds_for_cholesky(R);
    if (s) return s;
    SolveWs w = layout_solve(dims, N, R, dt, (char *)workspace, true);
    const size_t fz = dtype_f_bytes(dt);

    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, stream, w.status);
    LAUNCH_CHECK("k_clear_status");
    size_t off = 0;
    for (int k = 0; k < N; ++k) {
        HIP_TRY(hipMemcpyAsync((char *)w.snap + off, factors[k], (size_t)dims[k] * R * fz, hipMemcpyDeviceToDevice,
                               stream));
        off += (size_t)dims[k] * R * fz;
    }
    for (int k = 0; k < N; ++k) {
        s = gram(factors[k], dims[k], R, dt, w.gpart, w.grams + (size_t)k * R * R, stream);
        if (s) return s;
    }
    const size_t lds_chol = (size_t)R * R * sizeof(double);
    // With the cross-mode reuse, T_L depends only on the right group's
    // factors, which are not updated before mode s, and T_R is formed after
    // the left group's updates: the sweep stays Gauss-Seidel.
    TreePlan tree = plan_tree(dims, N, R);
    tree.use = tree.use && w.all.TL && tree_reach_ok(tree, X, R, dt);
    const void *const *cf = (const void *const *)factors;
    for (int n = 0; n < N; ++n) {
        if (tree.use) {
            const bool one = tree_single(tree, N, n);
            if (n == 0 || n == tree.s) {
                s = tree_pass(tree, n == 0, X, cf, R, dt, w.all, stream, one ? w.M : nullptr);
                if (s) return s;
            }
            if (!one) s = tree_leaf(tree, dims, N, cf, R, n, dt, w.all, w.M, stream);
        } else {
            Plan p = make_plan(dims, N, R, n, dt, X);
            s = run_mttkrp(p, X, dims, N, cf, R, n, w.M, dt, w.all.mws, stream);
        }
        if (s) return s;
        if (n == 0 && lds_chol > 65536)
            HIP_TRY(hipFuncSetAttribute((const void *)k_cholesky, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)lds_chol));
        hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(kThreads), lds_chol, stream, w.grams, N, n, R, w.L, w.Lt,
                           w.status);
        LAUNCH_CHECK("k_cholesky");
        // L and L^T go to LDS when they fit 64 KB (R <= 64); one row per wave.
        const bool lds_l = R <= 64;
        const int rpw = 1;
        const unsigned blocks = (unsigned)ceil_div(dims[n], 4 * rpw);
        const size_t lds_solve = lds_l ? (size_t)2 * R * R * sizeof(double) : 0;
        if (dt == CPM_F64) {
            if (lds_l)
                hipLaunchKernelGGL((k_chol_solve_rows<double, true>), dim3(blocks), dim3(kThreads), lds_solve, stream,
                                   w.L, w.Lt, w.status, (const double *)w.M, dims[n], R, rpw, (double *)factors[n]);
            else
                hipLaunchKernelGGL((k_chol_solve_rows<double, false>), dim3(blocks), dim3(kThreads), 0, stream, w.L,
                                   w.Lt, w.status, (const double *)w.M, dims[n], R, rpw, (double *)factors[n]);
        } else {
            if (lds_l)
                hipLaunchKernelGGL((k_chol_solve_rows<float, true>), dim3(blocks), dim3(kThreads), lds_solve, stream,
                                   w.L, w.Lt, w.status, (const float *)w.M, dims[n], R, rpw, (float *)factors[n]);
            else
                hipLaunchKernelGGL((k_chol_solve_rows<float, false>), dim3(blocks), dim3(kThreads), 0, stream, w.L,
                                   w.Lt, w.status, (const float *)w.M, dims[n], R, rpw, (float *)factors[n]);
        }
        LAUNCH_CHECK("k_chol_solve_rows");
        s = gram(factors[n], dims[n], R, dt, w.gpart, w.grams + (size_t)n * R * R, stream);
        if (s) return s;
    }
    if (fit_out) {
        if (xnorm2 >= 0.0) {
            hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, stream, w.xnorm2, xnorm2);
            LAUNCH_CHECK("k_set_scalar");
        } else {
            s = xnorm2_enqueue(X, total, dt, (double *)w.sumsq, w.xnorm2, stream);
            if (s) return s;
        }
        s = dot_enqueue(w.M, factors[N - 1], dims[N - 1] * R, dt, (double *)w.sumsq, w.inner, stream);
        if (s) return s;
        s = loss_enqueue(w.xnorm2, w.inner, w.grams, N, R, w.hpart, 1, w.result, stream);
        if (s) return s;
    }
    int status_h = 0;
    double result_h = 0.0;
    HIP_TRY(hipMemcpyAsync(&status_h, w.status, sizeof(int), hipMemcpyDeviceToHost, stream));
    if (fit_out) HIP_TRY(hipMemcpyAsync(&result_h, w.result, sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (status_h) {
        // the modes before the failing one were updated: every factor goes
        // back to its snapshot (only on this path, after the status is known)
        off = 0;
        for (int k = 0; k < N; ++k) {
            const size_t bytes = (size_t)dims[k] * R * fz;
            HIP_TRY(hipMemcpyAsync(factors[k], (char *)w.snap + off, bytes, hipMemcpyDeviceToDevice, stream));
            off += bytes;
        }
        HIP_TRY(hipStreamSynchronize(stream));
        return fail(CPM_ENOTPD, "Hadamard product of Grams is not positive definite; factors restored");
    }
    if (fit_out) *fit_out = result_h;
    return CPM_OK;
}

cpm_status cp_grad(const void *X, const int64_t *dims, int N, const void *const *factors, int R,
                   void *const *grads, double xnorm2, double *loss_dev, cpm_dtype dt, void *workspace,
                   size_t ws_bytes, hipStream_t stream) {
    int64_t total;
    cpm_status s = check_dtype(dt);
    if (s) return s;
    s = check_shape(dims, N, R, &total, CPM_MAX_RANK);
    if (s) return s;
    if (!X) return fail(CPM_EINVAL, "X is null");
    if (!factors) return fail(CPM_EINVAL, "factors is null");
    for (int k = 0; k < N; ++k)
        if (!factors[k]) return fail(CPM_EINVAL, "factors[%d] is null", k);
    s = check_factor_reach(dims, N, R, dt, -1);
    if (s) return s;
    const size_t need = layout_solve(dims, N, R, dt, nullptr, false).need;
    if (!workspace || ws_bytes < need)
        return fail(CPM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    s = check_reach(X, dims, N, R, dt);
    if (s) return s;
    SolveWs w = layout_solve(dims, N, R, dt, (char *)workspace, false);
    for (int k = 0; k < N; ++k) {
        s = gram(factors[k], dims[k], R, dt, w.gpart, w.grams + (size_t)k * R * R, stream);
        if (s) return s;
    }
    auto wanted = [&](int n) { return (grads && grads[n]) || (loss_dev && n == N - 1); };
    int nwant = 0;
    bool want_left = false, want_right = false;
    TreePlan tree = plan_tree(dims, N, R);
    for (int n = 0; n < N; ++n)
        if (wanted(n)) {
            ++nwant;
            (n < tree.s ? want_left : want_right) = true;
        }
    // the reuse pays once three or more modes are wanted
    tree.use = tree.use && nwant >= 3 && w.all.TL && tree_reach_ok(tree, X, R, dt);
    if (tree.use) {
        if (want_left) {
            s = tree_pass(tree, true, X, factors, R, dt, w.all, stream);
            if (s) return s;
        }
        if (want_right) {
            s = tree_pass(tree, false, X, factors, R, dt, w.all, stream);
            if (s) return s;
        }
    }
    int in_m2 = -1;  // the mode whose MTTKRP a two-mode leaf left in M2
    for (int n = 0; n < N; ++n) {
        const bool want_grad = grads && grads[n];
        const bool want_inner = loss_dev && n == N - 1;
        if (!want_grad && !want_inner) continue;
        void *M = w.M;
        if (tree.use) {
            // a one-mode group's intermediate is its MTTKRP; a two-mode
            // group forms both of its MTTKRPs in one pass (the second in M2)
            const int g0 = n < tree.s ? 0 : tree.s, g1 = n < tree.s ? tree.s : N;
            if (g1 - g0 == 1) {
                M = n < tree.s ? w.all.TL : w.all.TR;
            } else if (n == in_m2) {
                M = w.M2;
            } else {
                bool pair = false;
                if (n == g0 && g1 - g0 == 2 && wanted(n + 1) && dt != CPM_F64) {
                    s = tree_pair_leaf(tree, dims, factors, R, g0, dt, w.all, w.M, w.M2, stream, &pair);
                    if (s) return s;
                    if (pair) in_m2 = n + 1;
                }
                if (!pair) s = tree_leaf(tree, dims, N, factors, R, n, dt, w.all, w.M, stream);
            }
        } else {
            Plan p = make_plan(dims, N, R, n, dt, X);
            s = run_mttkrp(p, X, dims, N, factors, R, n, w.M, dt, w.all.mws, stream);
        }
        if (s) return s;
        if (want_inner) {
            s = dot_enqueue(M, factors[n], dims[n] * R, dt, (double *)w.sumsq, w.inner, stream);
            if (s) return s;
        }
        if (want_grad) {
            s = hadamard_except(w.grams, N, R, n, w.H, stream);
            if (s) return s;
            const unsigned blocks = (unsigned)ceil_div(dims[n] * R, 64);
            if (dt == CPM_F64)
                hipLaunchKernelGGL(k_grad<double>, dim3(blocks), dim3(kThreads), 0, stream,
                                   (const double *)factors[n], w.H, (const double *)M, dims[n], R,
                                   (double *)grads[n]);
            else
                hipLaunchKernelGGL(k_grad<float>, dim3(blocks), dim3(kThreads), 0, stream, (const float *)factors[n],
                                   w.H, (const float *)M, dims[n], R, (float *)grads[n]);
            LAUNCH_CHECK("k_grad");
        }
    }
    if (loss_dev) {
        if (xnorm2 >= 0.0) {
            hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, stream, w.xnorm2, xnorm2);
            LAUNCH_CHECK("k_set_scalar");
        } else {
            s = xnorm2_enqueue(X, total, dt, (double *)w.sumsq, w.xnorm2, stream);
            if (s) return s;
        }
        s = loss_enqueue(w.xnorm2, w.inner, w.grams, N, R, w.hpart, 0, loss_dev, stream);
        if (s) return s;
    }
    return CPM_OK;
}

size_t cpm_xnorm2_workspace_bytes(const int64_t *dims, int N, cpm_dtype dt) {
    (void)dims;
    (void)N;
    (void)dt;
    return align_up((size_t)kSumsqBlocks * sizeof(double));
}

cpm_status cpm_xnorm2(const void *X, const int64_t *dims, int N, cpm_dtype dt, double *out_dev, void *workspace,
                      size_t ws_bytes, hipStream_t stream) {
    int64_t total;
    cpm_status s = check_dtype(dt);
    if (s) return s;
    s = check_shape(dims, N, 1, &total, CPM_MAX_RANK);
    if (s) return s;
    if (!X || !out_dev) return fail(CPM_EINVAL, "X or out_dev is null");
    const size_t need = cpm_xnorm2_workspace_bytes(dims, N, dt);
    if (!workspace || ws_bytes < need)
        return fail(CPM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    return xnorm2_enqueue(X, total, dt, (double *)workspace, out_dev, stream);
}

cpm_status cpm_split_bf16(const float *x, int64_t count, uint16_t *planes, hipStream_t stream) {
    if (!x || !planes) return fail(CPM_EINVAL, "x or planes is null");
    if (count < 0) return fail(CPM_EINVAL, "count < 0");
    if (count == 0) return CPM_OK;
    const unsigned blocks = (unsigned)std::min<int64_t>(4096, ceil_div(count, kThreads));
    const int vec8 = ((uintptr_t)x % 16 == 0 && (uintptr_t)planes % 16 == 0 && count % 8 == 0) ? 1 : 0;
    hipLaunchKernelGGL(k_split_bf16, dim3(blocks), dim3(kThreads), 0, stream, x, count, vec8, planes);
    LAUNCH_CHECK("k_split_bf16");
    return CPM_OK;
}

cpm_status cpm_krp_rows(const void *const *mats, const int64_t *J, int Z, int R, int64_t j0, int64_t nrows,
                        void *out, cpm_dtype dt, hipStream_t stream) {
    if (dt != CPM_F32 && dt != CPM_F64) return fail(CPM_EINVAL, "cpm_krp_rows takes CPM_F32 or CPM_F64");
    if (!mats || !J || !out) return fail(CPM_EINVAL, "null argument");
    if (Z < 1 || Z > CPM_MAX_MODES) return fail(CPM_EINVAL, "Z=%d outside [1, %d]", Z, CPM_MAX_MODES);
    if (R < 1 || R > CPM_MAX_RANK) return fail(R < 1 ? CPM_EINVAL : CPM_EUNSUPPORTED, "R=%d outside [1, %d]", R,
                                              CPM_MAX_RANK);
    int64_t rows = 1;
    for (int z = 0; z < Z; ++z) {
        if (!mats[z]) return fail(CPM_EINVAL, "mats[%d] is null", z);
        if (J[z] < 1) return fail(CPM_EINVAL, "J[%d] < 1", z);
        if (rows > ((int64_t)1 << 62) / J[z]) return fail(CPM_EUNSUPPORTED, "too many rows");
        rows *= J[z];
    }
    if (j0 < 0 || nrows < 0 || j0 + nrows > rows) return fail(CPM_EINVAL, "row range outside the product");
    if (nrows == 0) return CPM_OK;
    if (ceil_div(nrows, 64) > INT32_MAX) return fail(CPM_EUNSUPPORTED, "nrows too large");
    // mats[0] kr ... kr mats[Z-1]: the last matrix is the fastest index.
    const int RP = (R + 15) / 16 * 16;
    const unsigned blocks = (unsigned)ceil_div(nrows, 64);
    if (dt == CPM_F32) {
        Krp<float> k{};
        k.rows = 1;
        for (int z = Z - 1; z >= 0; --z) {
            k.J[k.Z] = J[z];
            k.stride[k.Z] = k.rows;
            k.U[k.Z] = (const float *)mats[z];
            k.rows *= J[z];
            ++k.Z;
        }
        hipLaunchKernelGGL(k_krp_rows<float>, dim3(blocks), dim3(kThreads), 0, stream, k, R, RP, j0, nrows,
                           (float *)out);
    } else {
        Krp<double> k{};
        k.rows = 1;
        for (int z = Z - 1; z >= 0; --z) {
            k.J[k.Z] = J[z];
            k.stride[k.Z] = k.rows;
            k.U[k.Z] = (const double *)mats[z];
            k.rows *= J[z];
            ++k.Z;
        }
        hipLaunchKernelGGL(k_krp_rows<double>, dim3(blocks), dim3(kThreads), 0, stream, k, R, RP, j0, nrows,
                           (double *)out);
    }
    LAUNCH_CHECK("k_krp_rows");
    return CPM_OK;
}

}  // extern "C"
