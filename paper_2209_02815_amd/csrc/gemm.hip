// Capacitance matrix S = alpha*I + J Z^T (Algorithm 3, second step) on the
// FP64 matrix cores: J is m x N (FP64), Z is m x N (FP64, or FP32 converted
// exactly to FP64 on load), both row-major with K = N contiguous.
//
// The product has a long inner dimension (N up to 1.7e7) and a small output
// (m <= a few thousand), so the K range is split over work-groups: work-group
// (tile, split) accumulates a 128 x 128 output tile over K range `split` and
// writes it to partial[split]; a second kernel sums the splits in a fixed
// order (deterministic) and adds alpha on the diagonal. When S is known to be
// symmetric (FP64 Z), only tiles on or below the diagonal are computed and
// the upper triangle is mirrored. The product is general rectangular
// (m rows of J against m2 <= m rows of Z), which also serves a capacitance
// built from Z in row chunks when Z does not fit next to J: there the block
// S[c0:, c0:c0+m2] starts on the diagonal, and its lower mode skips the tiles
// (and 64 x 64 wave quadrants) strictly above it in the same way.
//
// Each wave owns a 64 x 64 sub-tile = 4 x 4 blocks of v_mfma_f64_16x16x4_f64
// whose operands come from LDS copies of the work-group's 128-row tiles of J
// and Z (each element is read from HBM once per work-group, not once per
// wave). Accumulator layout of the FP64 16x16 block: lane l, element v holds
// row (l/16) + 4v, column l%16.
//
// Launch: one work-group per (tile, split), two resident per CU.
// Work items are ordered split-major and dealt to the 8 XCDs in contiguous
// ranges (work-group ids go round-robin over XCDs), so the tiles that share a
// K range share one XCD's L2.
#include <algorithm>

#include "devutil.h"
#include "internal.h"

namespace h1w {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kTileMN = 128;
constexpr int kGemmThreads = 256;
constexpr int kResidentWG = 512;  // 256 CUs x 2 work-groups
constexpr size_t kMaxPartialBytes = size_t(1) << 30;
// rounds of resident work-groups a product is planned for (shorter K ranges
// per work item with more rounds): at 257^3 (m = 1024, 256-row blocks of Z)
// 8 rounds gave 48.3 TF/s against 47.3 with 4, 48.4 with 16 and 46.9 with 2
// in one process; the HBM traffic did not drop (FETCH_SIZE rose 5%)
constexpr int kRounds = 8;

// K is consumed in chunks of KB = 16: the 256 threads copy the 128 x KB
// tiles of J and Z into LDS (double-buffered; rows padded to an odd stride so
// the MFMA operand reads do not collide on banks), then each wave runs its
// 4 x 4 MFMA blocks over the chunk (4 k-steps). The global loads of chunk
// c+1 are in flight while chunk c is computed; one barrier per chunk.
// Loader mapping: thread t owns column k = t % 16 of rows t/16 + 16u
// (u = 0..7), so one load instruction of a wave reads 4 whole 128-byte row
// segments.
constexpr int KB = 16;
constexpr int LDT = KB + 1;  // LDS row stride (doubles)

// One work item of the product: the 128 x 128 output tile (tr, tc) of
// J (m rows) times Z^T (m2 rows) over the K range [k0, k1), stored into P
// (m x m2, row-major). lower: the product is the lower triangle of a
// symmetric one (the wave quadrant strictly above a diagonal tile idles).
template <typename TZ>
__device__ __forceinline__ void cap_tile(int m, int m2, const double* __restrict__ J, int64_t ldj,
                                         const TZ* __restrict__ Z, int64_t ldz, int tr, int tc, bool lower,
                                         int64_t k0, int64_t k1, double* __restrict__ P) {
    __shared__ double sA[2][kTileMN * LDT];
    __shared__ double sB[2][kTileMN * LDT];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int l16 = lane & 15, g = lane >> 4;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    const int arow0 = tr * kTileMN, brow0 = tc * kTileMN;
    // on a diagonal tile of the lower-triangle product the wave at rows 0-63,
    // columns 64-127 lies strictly above the diagonal, whose entries the
    // reduction never reads; on a ragged tile a wave's quadrant can lie past
    // the last row or column. Such a wave keeps loading and synchronising
    // with the group but skips its MFMAs (its SIMD time goes to the
    // co-resident group)
    const bool idle = (lower && tr == tc && wr < wc) || arow0 + wr >= m || brow0 + wc >= m2;

    // loader: column lk of rows lr + 16 q, q = 0..7. Rows past the end of J
    // or Z read row 0 instead: they only feed output rows (columns) that are
    // never stored. Columns past the K range are zeroed, at the LDS store:
    // the loaded registers are first used there, after the chunk's MFMAs,
    // so the loads stay in flight during the compute (a select right after
    // the load would make the wave wait for them at once).
    const int lk = tid & 15, lr = tid >> 4;
    const double* pa[8];
    const TZ* pb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int r = arow0 + lr + 16 * q;
        pa[q] = J + (int64_t)(r < m ? r : 0) * ldj;
        const int c = brow0 + lr + 16 * q;
        pb[q] = Z + (int64_t)(c < m2 ? c : 0) * ldz;
    }
    const int nchunk = (int)((k1 - k0 + KB - 1) / KB);
    double ra[8];
    TZ rb[8];
    bool kin = false;
    auto gload = [&](int c) {
        const int64_t k = k0 + (int64_t)c * KB + lk;
        kin = k < k1;
        const int64_t kc = kin ? k : k0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            ra[q] = pa[q][kc];
            rb[q] = pb[q][kc];
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            sA[buf][(lr + 16 * q) * LDT + lk] = kin ? ra[q] : 0.0;
            sB[buf][(lr + 16 * q) * LDT + lk] = kin ? double(rb[q]) : 0.0;
        }
    };
    d4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    if (nchunk > 0) {
        gload(0);
        lstore(0);
    }
    __syncthreads();
    for (int c = 0; c < nchunk; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunk) gload(c + 1);
        const double* A = sA[buf];
        const double* B = sB[buf];
#pragma unroll
        for (int s4 = 0; s4 < KB / 4 && !idle; ++s4) {
            const int kk = 4 * s4 + g;
            double a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                a[r] = A[(wr + 16 * r + l16) * LDT + kk];
                b[r] = B[(wc + 16 * r + l16) * LDT + kk];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int cc = 0; cc < 4; ++cc)
                    acc[r][cc] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r], b[cc], acc[r][cc], 0, 0, 0);
        }
        if (c + 1 < nchunk) lstore(buf ^ 1);
        __syncthreads();
    }
    if (idle) return;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = arow0 + wr + r * 16 + g + 4 * v;
                const int col = brow0 + wc + c * 16 + l16;
                if (row < m && col < m2) P[(int64_t)row * m2 + col] = acc[r][c][v];
            }
}

template <typename TZ>
__global__ __launch_bounds__(kGemmThreads, 2) void k_cap_gemm(int m, int m2, int64_t N, const double* __restrict__ J,
                                                              int64_t ldj, const TZ* __restrict__ Z, int64_t ldz,
                                                              int T, int T2, int ntile, int lower, int total,
                                                              int64_t kper, double* __restrict__ partial) {
    const int bid = blockIdx.x;
    const int per = (total + 7) / 8;
    const int u = (bid & 7) * per + (bid >> 3);
    if (u >= total) return;
    const int split = u / ntile;
    const int tile = u - split * ntile;
    int tr, tc;
    if (lower) {
        // row tile r holds min(r + 1, T2) tiles: a triangle of T2 (T2 + 1) / 2
        // tiles, then full rows of T2
        const int tri = T2 * (T2 + 1) / 2;
        if (tile < tri) {
            tr = 0;
            while ((tr + 1) * (tr + 2) / 2 <= tile) ++tr;
            tc = tile - tr * (tr + 1) / 2;
        } else {
            tr = T2 + (tile - tri) / T2;
            tc = (tile - tri) - (tr - T2) * T2;
        }
    } else {
        tr = tile / T2;
        tc = tile - tr * T2;
    }
    const int64_t k0 = (int64_t)split * kper;
    cap_tile<TZ>(m, m2, J, ldj, Z, ldz, tr, tc, lower != 0, k0, std::min<int64_t>(N, k0 + kper),
                 partial + (int64_t)split * m * m2);
}

// Grouped products of a lock-step batch: work item u is split u - io[g] of
// instance g (m[g] <= 128 rows, one 128 x 128 tile), found by bisection over
// io; the items go to the 8 XCDs in contiguous ranges as above.
__global__ __launch_bounds__(kGemmThreads, 2) void k_grp_gemm(GrpGemm t, int64_t N, const double* __restrict__ J,
                                                              int64_t ldj, const double* __restrict__ Z,
                                                              int64_t ldz, double* __restrict__ partial) {
    const int bid = blockIdx.x;
    const int per = (t.total + 7) / 8;
    const int u = (bid & 7) * per + (bid >> 3);
    if (u >= t.total) return;
    int lo = 0, hi = t.G - 1;  // the last g with io[g] <= u
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.io[mid] <= u) lo = mid;
        else hi = mid - 1;
    }
    const int g = lo, m = t.m[g];
    const int64_t kp = t.kper[g];
    const int64_t k0 = (int64_t)(u - t.io[g]) * kp;
    cap_tile<double>(m, m, J + (int64_t)t.ro[g] * ldj, ldj, Z + (int64_t)t.ro[g] * ldz, ldz, 0, 0, false, k0,
                     std::min<int64_t>(N, k0 + kp), partial + t.poff[g] + (int64_t)(u - t.io[g]) * m * m);
}

// S_g = alpha_g I + the sum of instance g's partials in item order
__global__ __launch_bounds__(kBlock) void k_grp_reduce(GrpGemm t, const double* __restrict__ partial,
                                                       double* __restrict__ S) {
    const int g = blockIdx.y, m = t.m[g];
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= m * m) return;
    const int ns = t.io[g + 1] - t.io[g];
    const double* p = partial + t.poff[g] + idx;
    double acc = 0.0;
    for (int sp = 0; sp < ns; ++sp) acc += p[(int64_t)sp * m * m];
    const int i = idx / m, j = idx - i * m;
    if (i == j) acc += t.alpha[g];
    S[t.soff[g] + idx] = acc;
}

// FP32-accumulated variant (opt-in, MIXED contexts): the same work items and
// K splits, but the operands are FP32 (J rounded to FP32 as it is loaded, Z
// stored FP32) and the product runs on the FP32 matrix cores,
// v_mfma_f32_16x16x4_f32, accumulating in FP32 over the work-group's whole K
// range; only the split partials are summed in FP64 (k_cap_reduce). The
// result differs from J Z^T by about eps32 * sqrt(K range) * |J||Z| per entry,
// which the Woodbury correction cannot absorb when ||S|| / alpha is large:
// the mode exists to measure that, the FP64-accumulated product is the default.
// Accumulator layout of the FP32 16x16 block: lane l, element v holds row
// 4 (l/16) + v, column l%16 (the FP64 block above has row (l/16) + 4v).
// K is consumed in chunks of 32 (one 128-byte FP32 row segment); loader
// mapping: thread t owns column k = t % 32 of rows t/32 + 8u (u = 0..15).
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int KB32 = 32;
constexpr int LDT32 = KB32 + 1;  // LDS row stride (floats)

__global__ __launch_bounds__(kGemmThreads, 2) void k_cap_gemm32(int m, int m2, int64_t N,
                                                                const double* __restrict__ J, int64_t ldj,
                                                                const float* __restrict__ Z, int64_t ldz, int T2,
                                                                int ntile, int total, int64_t kper,
                                                                double* __restrict__ partial) {
    __shared__ float sA[2][kTileMN * LDT32];
    __shared__ float sB[2][kTileMN * LDT32];
    const int bid = blockIdx.x;
    const int per = (total + 7) / 8;
    const int u = (bid & 7) * per + (bid >> 3);
    if (u >= total) return;
    const int split = u / ntile;
    const int tile = u - split * ntile;
    const int tr = tile / T2, tc = tile - (tile / T2) * T2;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int l16 = lane & 15, g = lane >> 4;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    const int arow0 = tr * kTileMN, brow0 = tc * kTileMN;

    // rows past the ends read row 0 and K columns past the range are zeroed
    // at the LDS store, as in k_cap_gemm (loads stay in flight over the MFMAs)
    const int lk = tid & 31, lr = tid >> 5;
    const double* pa[16];
    const float* pb[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int r = arow0 + lr + 8 * q;
        pa[q] = J + (int64_t)(r < m ? r : 0) * ldj;
        const int c = brow0 + lr + 8 * q;
        pb[q] = Z + (int64_t)(c < m2 ? c : 0) * ldz;
    }
    const int64_t k0 = (int64_t)split * kper;
    const int64_t k1 = std::min<int64_t>(N, k0 + kper);
    const int nchunk = (int)((k1 - k0 + KB32 - 1) / KB32);
    double ra[16];
    float rb[16];
    bool kin = false;
    auto gload = [&](int c) {
        const int64_t k = k0 + (int64_t)c * KB32 + lk;
        kin = k < k1;
        const int64_t kc = kin ? k : k0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            ra[q] = pa[q][kc];
            rb[q] = pb[q][kc];
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            sA[buf][(lr + 8 * q) * LDT32 + lk] = kin ? (float)ra[q] : 0.0f;
            sB[buf][(lr + 8 * q) * LDT32 + lk] = kin ? rb[q] : 0.0f;
        }
    };
    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    if (nchunk > 0) {
        gload(0);
        lstore(0);
    }
    __syncthreads();
    for (int c = 0; c < nchunk; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunk) gload(c + 1);
        const float* A = sA[buf];
        const float* B = sB[buf];
#pragma unroll
        for (int s4 = 0; s4 < KB32 / 4; ++s4) {
            const int kk = 4 * s4 + g;
            float a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                a[r] = A[(wr + 16 * r + l16) * LDT32 + kk];
                b[r] = B[(wc + 16 * r + l16) * LDT32 + kk];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int cc = 0; cc < 4; ++cc)
                    acc[r][cc] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r], b[cc], acc[r][cc], 0, 0, 0);
        }
        if (c + 1 < nchunk) lstore(buf ^ 1);
        __syncthreads();
    }
    double* P = partial + (int64_t)split * m * m2;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = arow0 + wr + r * 16 + 4 * g + v;
                const int col = brow0 + wc + c * 16 + l16;
                if (row < m && col < m2) P[(int64_t)row * m2 + col] = (double)acc[r][c][v];
            }
}

// S[i][j] (block of m x m2 at S, leading dimension lds) = sum over splits of
// the partials (+ alpha where i == j + diag_off: the global diagonal of a
// block that starts diag_off columns right of it). lower: the square
// product was computed on and below the diagonal only; S[i][j] for i < j is
// taken from the partial at (j, i). A work-group takes kRedOut consecutive
// outputs; its kRedGroups thread groups sum the splits g, g + kRedGroups, ...
// and the group sums are added in group order (a fixed order, so the result
// does not depend on timing).
constexpr int kRedGroups = 8;
constexpr int kRedOut = kBlock / kRedGroups;

__global__ __launch_bounds__(kBlock) void k_cap_reduce(int m, int m2, int splits, const double* __restrict__ partial,
                                                       int lower, double alpha, int diag_off, double* __restrict__ S,
                                                       int64_t lds) {
    __shared__ double sh[kRedGroups][kRedOut];
    const int g = threadIdx.x / kRedOut, q = threadIdx.x % kRedOut;
    const int64_t idx = (int64_t)blockIdx.x * kRedOut + q;
    const bool ok = idx < (int64_t)m * m2;
    const int i = ok ? (int)(idx / m2) : 0, j = ok ? (int)(idx - (int64_t)i * m2) : 0;
    double acc = 0.0;
    if (ok) {
        const int si = (lower && i < j) ? j : i;
        const int sj = (lower && i < j) ? i : j;
        const double* p = partial + (int64_t)si * m2 + sj;
        for (int s = g; s < splits; s += kRedGroups) acc += p[(int64_t)s * m * m2];
    }
    sh[g][q] = acc;
    __syncthreads();
    if (g == 0 && ok) {
        double t = sh[0][q];
#pragma unroll
        for (int h = 1; h < kRedGroups; ++h) t += sh[h][q];
        if (i == j + diag_off) t += alpha;
        S[(int64_t)i * lds + j] = t;
    }
}

// S[i][j] = S[j][i] for i < j (upper triangle from the lower one)
__global__ __launch_bounds__(kBlock) void k_mirror_lower(int m, double* __restrict__ S) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (int64_t)m * m) return;
    const int i = (int)(idx / m), j = (int)(idx - (int64_t)i * m);
    if (i < j) S[(int64_t)i * m + j] = S[(int64_t)j * m + i];
}

struct GemmPlan {
    int T, T2, ntile, splits;
    int64_t kper;
};

GemmPlan plan(int m, int m2, int64_t N, bool lower) {
    GemmPlan p;
    p.T = (int)cdiv(m, kTileMN);
    p.T2 = (int)cdiv(m2, kTileMN);
    p.ntile = lower ? p.T2 * (p.T2 + 1) / 2 + (p.T - p.T2) * p.T2 : p.T * p.T2;
    // splits: about kRounds rounds of resident work-groups, the count in
    // [s0, 4 s0] whose last round is the fullest (fewest idle slots while the
    // slowest groups finish); bounded by the partial buffer and by K
    const size_t per_split = (size_t)m * m2 * sizeof(double);
    const int smax_mem = (int)std::max<size_t>(1, kMaxPartialBytes / per_split);
    const int smax_k = (int)std::max<int64_t>(1, cdiv(N, 256));
    const int s0 = std::max(1, (int)cdiv(kRounds * kResidentWG, p.ntile) / 2);
    int splits = 1;
    double best = 1e30;
    for (int sp = s0; sp <= 4 * s0; ++sp) {
        const int spc = std::min({sp, smax_mem, smax_k});
        const double tot = (double)p.ntile * spc;
        const double waste = std::ceil(tot / kResidentWG) * kResidentWG / tot;
        if (waste < best - 1e-9) {
            best = waste;
            splits = spc;
        }
    }
    p.kper = cdiv(cdiv(N, splits), KB) * KB;
    p.splits = (int)cdiv(N, p.kper);
    return p;
}

}  // namespace

size_t gemm_partial_elems(int m, int m2, int64_t N) {
    const GemmPlan p = plan(m, m2, N, false);
    size_t e = (size_t)p.splits * m * m2;
    if (m >= m2) e = std::max(e, (size_t)plan(m, m2, N, true).splits * m * m2);
    return e;
}

template <typename TZ>
int launch_capacitance_partial(hipStream_t s, int m, int m2, int64_t N, const double* J, int64_t ldj, const TZ* Z,
                               int64_t ldz, bool lower_only, double* partial, size_t partial_elems) {
    if (m <= 0 || m2 <= 0) return 0;
    if (lower_only && m < m2) throw Error{H1W_EINVAL, "internal: lower-triangle GEMM needs m >= m2"};
    const GemmPlan p = plan(m, m2, N, lower_only);
    if ((size_t)p.splits * m * m2 > partial_elems) throw Error{H1W_EINVAL, "internal: GEMM partial buffer too small"};
    const int total = p.ntile * p.splits;
    const int grid = 8 * ((total + 7) / 8);
    hipLaunchKernelGGL((k_cap_gemm<TZ>), dim3(grid), dim3(kGemmThreads), 0, s, m, m2, N, J, ldj, Z, ldz, p.T, p.T2,
                       p.ntile, (int)lower_only, total, p.kper, partial);
    H1W_LAUNCHED();
    return p.splits;
}

int launch_capacitance_partial_f32acc(hipStream_t s, int m, int m2, int64_t N, const double* J, int64_t ldj,
                                      const float* Z, int64_t ldz, double* partial, size_t partial_elems) {
    if (m <= 0 || m2 <= 0) return 0;
    const GemmPlan p = plan(m, m2, N, false);
    if ((size_t)p.splits * m * m2 > partial_elems) throw Error{H1W_EINVAL, "internal: GEMM partial buffer too small"};
    const int total = p.ntile * p.splits;
    const int grid = 8 * ((total + 7) / 8);
    hipLaunchKernelGGL(k_cap_gemm32, dim3(grid), dim3(kGemmThreads), 0, s, m, m2, N, J, ldj, Z, ldz, p.T2, p.ntile,
                       total, p.kper, partial);
    H1W_LAUNCHED();
    return p.splits;
}

void launch_capacitance_reduce(hipStream_t s, int m, int m2, int splits, const double* partial, bool lower_only,
                               double alpha, int diag_off, double* S, int64_t lds) {
    if (m <= 0 || m2 <= 0) return;
    hipLaunchKernelGGL(k_cap_reduce, dim3((unsigned)cdiv((int64_t)m * m2, kRedOut)), dim3(kBlock), 0, s, m, m2,
                       splits, partial, (int)lower_only, alpha, diag_off, S, lds);
    H1W_LAUNCHED();
}

void launch_grp_gemm_partial(hipStream_t s, const GrpGemm& t, int64_t N, const double* J, int64_t ldj,
                             const double* Z, int64_t ldz, double* partial) {
    if (t.total <= 0) return;
    hipLaunchKernelGGL(k_grp_gemm, dim3((unsigned)(8 * cdiv(t.total, 8))), dim3(kGemmThreads), 0, s, t, N, J, ldj, Z,
                       ldz, partial);
    H1W_LAUNCHED();
}

void launch_grp_gemm_reduce(hipStream_t s, const GrpGemm& t, const double* partial, double* S) {
    if (t.G <= 0) return;
    hipLaunchKernelGGL(k_grp_reduce, dim3((unsigned)cdiv(128 * 128, kBlock), (unsigned)t.G), dim3(kBlock), 0, s, t,
                       partial, S);
    H1W_LAUNCHED();
}

void launch_mirror_lower(hipStream_t s, int m, double* S) {
    hipLaunchKernelGGL(k_mirror_lower, dim3((unsigned)cdiv((int64_t)m * m, kBlock)), dim3(kBlock), 0, s, m, S);
    H1W_LAUNCHED();
}

template int launch_capacitance_partial<double>(hipStream_t, int, int, int64_t, const double*, int64_t,
                                                const double*, int64_t, bool, double*, size_t);
template int launch_capacitance_partial<float>(hipStream_t, int, int, int64_t, const double*, int64_t, const float*,
                                               int64_t, bool, double*, size_t);

}  // namespace h1w
