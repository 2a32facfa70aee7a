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
// (m rows of J against m2 rows of Z), which also serves a capacitance built
// from Z in row chunks when Z does not fit next to J.
//
// Each wave owns a 64 x 64 sub-tile = 4 x 4 blocks of v_mfma_f64_16x16x4_f64.
// The MFMA contracts 4 k-values held by the 4 groups of 16 lanes; any
// assignment of physical k to (lane group, step) gives the same sum, so lane
// group g walks KL consecutive k-values per step: lanes read 8-byte words of
// contiguous rows straight from global memory (no LDS), and one step covers
// 4*KL = 16 k-values. Accumulator layout of the FP64 16x16 block: lane l,
// element v holds row (l/16) + 4v, column l%16.
//
// Launch: one work-group per (tile, split), at most ~2 resident per CU.
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
constexpr int KL = 4;
constexpr int KSTEP = 4 * KL;
constexpr int kGemmThreads = 256;
constexpr int kResidentWG = 256;  // 256 CUs x 1 work-group (occupancy 1 wave/SIMD)
constexpr size_t kMaxPartialBytes = size_t(256) << 20;

template <typename TZ>
__global__ __launch_bounds__(kGemmThreads) void k_cap_gemm(int m, int m2, int64_t N, const double* __restrict__ J,
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
        tr = 0;
        while ((tr + 1) * (tr + 2) / 2 <= tile) ++tr;
        tc = tile - tr * (tr + 1) / 2;
    } else {
        tr = tile / T2;
        tc = tile - tr * T2;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int l16 = lane & 15, g = lane >> 4;
    const int row0 = tr * kTileMN + (wave >> 1) * 64;
    const int col0 = tc * kTileMN + (wave & 1) * 64;

    const double* pa[4];
    const TZ* pb[4];
    bool va[4], vb[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int r = row0 + b * 16 + l16;
        va[b] = r < m;
        pa[b] = J + (int64_t)(va[b] ? r : 0) * ldj;
        const int c = col0 + b * 16 + l16;
        vb[b] = c < m2;
        pb[b] = Z + (int64_t)(vb[b] ? c : 0) * ldz;
    }
    d4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    const int64_t k0 = (int64_t)split * kper;
    const int64_t k1 = std::min<int64_t>(N, k0 + kper);
    // Operands for one k-step: KL consecutive k-values per lane for 4 row
    // blocks of J and 4 of Z. Two register sets alternate so that the loads of
    // step s+1 are in flight while the MFMAs of step s run.
    auto load = [&](int64_t k, double (&a)[4][KL], double (&b)[4][KL]) {
        const int64_t kk = k + g * KL;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int t = 0; t < KL; ++t) {
                const double x = pa[r][kk + t];
                a[r][t] = va[r] ? x : 0.0;
                const double y = double(pb[r][kk + t]);
                b[r][t] = vb[r] ? y : 0.0;
            }
    };
    auto mma = [&](const double (&a)[4][KL], const double (&b)[4][KL]) {
#pragma unroll
        for (int t = 0; t < KL; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r][t], b[c][t], acc[r][c], 0, 0, 0);
    };
    const int64_t nfull = (k1 - k0) / KSTEP;  // full k-steps in this split
    int64_t k = k0;
    if (nfull > 0) {
        double a0[4][KL], b0[4][KL], a1[4][KL], b1[4][KL];
        load(k, a0, b0);
        int64_t s = 0;
        for (; s + 2 <= nfull; s += 2) {
            load(k + KSTEP, a1, b1);
            mma(a0, b0);
            if (s + 2 < nfull) load(k + 2 * KSTEP, a0, b0);
            mma(a1, b1);
            k += 2 * KSTEP;
        }
        if (s < nfull) {  // one full step left, already loaded in a0/b0
            mma(a0, b0);
            k += KSTEP;
        }
    }
    if (k < k1) {  // ragged tail: k-values at or beyond k1 contribute zero
        const int64_t kk = k + g * KL;
        double a[4][KL], b[4][KL];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int t = 0; t < KL; ++t) {
                const bool in = kk + t < k1;
                const int64_t kc = in ? kk + t : k0;
                const double x = pa[r][kc];
                a[r][t] = (va[r] && in) ? x : 0.0;
                const double y = double(pb[r][kc]);
                b[r][t] = (vb[r] && in) ? y : 0.0;
            }
        mma(a, b);
    }
    double* P = partial + (int64_t)split * m * m2;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = row0 + r * 16 + g + 4 * v;
                const int col = col0 + c * 16 + l16;
                if (row < m && col < m2) P[(int64_t)row * m2 + col] = acc[r][c][v];
            }
}

// S[i][j] (block of m x m2 at S, leading dimension lds) = sum over splits of
// the partials (+ alpha on the block diagonal i == j). lower: the square
// product was computed on and below the diagonal only; S[i][j] for i < j is
// taken from the partial at (j, i).
__global__ __launch_bounds__(kBlock) void k_cap_reduce(int m, int m2, int splits, const double* __restrict__ partial,
                                                       int lower, double alpha, double* __restrict__ S,
                                                       int64_t lds) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (int64_t)m * m2) return;
    const int i = (int)(idx / m2), j = (int)(idx - (int64_t)i * m2);
    const int si = (lower && i < j) ? j : i;
    const int sj = (lower && i < j) ? i : j;
    const double* p = partial + (int64_t)si * m2 + sj;
    double acc = 0.0;
    for (int s = 0; s < splits; ++s) acc += p[(int64_t)s * m * m2];
    if (i == j) acc += alpha;
    S[(int64_t)i * lds + j] = acc;
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
    p.ntile = lower ? p.T * (p.T + 1) / 2 : p.T * p.T2;
    const size_t per_split = (size_t)m * m2 * sizeof(double);
    int splits = std::max(1, kResidentWG / p.ntile);
    splits = (int)std::min<int64_t>(splits, std::max<int64_t>(1, cdiv(N, 256)));
    splits = (int)std::max<size_t>(1, std::min<size_t>(splits, kMaxPartialBytes / per_split));
    p.kper = cdiv(cdiv(N, splits), KSTEP) * KSTEP;
    p.splits = (int)cdiv(N, p.kper);
    return p;
}

}  // namespace

size_t gemm_partial_elems(int m, int m2, int64_t N) {
    const GemmPlan p = plan(m, m2, N, false);
    size_t e = (size_t)p.splits * m * m2;
    if (m == m2) e = std::max(e, (size_t)plan(m, m, N, true).splits * m * m);
    return e;
}

template <typename TZ>
int launch_capacitance_partial(hipStream_t s, int m, int m2, int64_t N, const double* J, int64_t ldj, const TZ* Z,
                               int64_t ldz, bool lower_only, double* partial, size_t partial_elems) {
    if (m <= 0 || m2 <= 0) return 0;
    if (lower_only && m != m2) throw Error{H1W_EINVAL, "internal: lower-triangle GEMM needs a square output"};
    const GemmPlan p = plan(m, m2, N, lower_only);
    if ((size_t)p.splits * m * m2 > partial_elems) throw Error{H1W_EINVAL, "internal: GEMM partial buffer too small"};
    const int total = p.ntile * p.splits;
    const int grid = 8 * ((total + 7) / 8);
    hipLaunchKernelGGL((k_cap_gemm<TZ>), dim3(grid), dim3(kGemmThreads), 0, s, m, m2, N, J, ldj, Z, ldz, p.T, p.T2,
                       p.ntile, (int)lower_only, total, p.kper, partial);
    H1W_LAUNCHED();
    return p.splits;
}

void launch_capacitance_reduce(hipStream_t s, int m, int m2, int splits, const double* partial, bool lower_only,
                               double alpha, double* S, int64_t lds) {
    if (m <= 0 || m2 <= 0) return;
    hipLaunchKernelGGL(k_cap_reduce, dim3((unsigned)cdiv((int64_t)m * m2, kBlock)), dim3(kBlock), 0, s, m, m2,
                       splits, partial, (int)lower_only, alpha, S, lds);
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
