// Lock-step solve of many GN systems on one grid (the batch's grouped mode;
// Algorithm 3 for each instance, all instances advanced together).
//
// The G instances share the grid, so their vectors are stacked (pitch P) and
// one launch serves the whole group: the V-cycles of all right-hand sides,
// the operator apply, the dot products, the step lengths and updates with
// per-instance scalars and activity masks (the batched kernels of the
// MG-PCG). The rows of every J_g are stacked into one M x P array (M = sum
// m_g), so J v (a work-group per row) and J^T u (a work-group per instance
// and node block) over all instances are single launches too; Z = B J^T is
// one batched V-cycle over the M rows. Each
// instance has m_g <= 128 rows, so its capacitance S_g = alpha_g I + J_g Z_g^T
// is one 128 x 128 product tile (split over K into work items of the grouped
// MFMA product) and is inverted by Gauss-Jordan elimination in one
// work-group's LDS; the preconditioner then multiplies by S_g^{-1}.
//
// Per instance the iteration is preconditioned CG with the Woodbury apply in
// its stored form,
//     y = B r,  t = J y,  w = S^{-1} t,  z = (y - Z^T w) / alpha,
// G p = alpha A p + J^T (J p), and the flexible (Polak-Ribiere) direction
// coefficient, which covers the FP32 cycles of a MIXED context (there the
// cycles of Z and of every y are the FP32 V-cycle with its constant mode
// handled in FP64, S is formed in FP64 from the same Z, and everything else
// is FP64). An instance stops when its
// recursive residual reaches rtol; the true residual b - G x is then checked
// and an instance that misses rtol restarts from its x. Converged instances
// drop out of the passes over J (masked work-groups) and, once a quarter of
// the group has converged, out of the V-cycles (the active right-hand sides
// are compacted), so the group's slowest instances do not make every
// instance pay for their extra iterations. Each instance ends with a status
// of its own: non-finite values or a breakdown stop only that instance.
#include <algorithm>
#include <cmath>
#include <vector>

#include "context.h"

namespace h1w {

namespace {

constexpr int kGrpRows = Ctx::kGroupMaxRows;
constexpr int kGJThreadsG = 1024;

// Activity masks: act[g] = 0 marks an instance that has converged; the
// kernels below skip its rows and vectors (act == nullptr: every instance),
// so a step costs about what its active instances need.

// out[i] = J_i . v_g for the M stacked rows (g = rowg[i], the instance of row
// i): one work-group per row, eight independent partial sums per thread,
// combined in a fixed tree order
__global__ __launch_bounds__(kBlock) void k_grp_rows_dot(int64_t N, const double* __restrict__ A, int64_t lda,
                                                          const double* __restrict__ V, int64_t ldv,
                                                          const int* __restrict__ rowg,
                                                          const int* __restrict__ act, double* __restrict__ out) {
    __shared__ double sh[kBlock / 64];
    const int64_t i = blockIdx.x;
    const int lo = rowg[i];
    if (act && !act[lo]) return;
    const double* a = A + i * lda;
    const double* v = V + (int64_t)lo * ldv;
    constexpr int U = 8;  // independent partial sums: eight loads of the row in flight per thread
    double acc[U];
#pragma unroll
    for (int q = 0; q < U; ++q) acc[q] = 0.0;
    int64_t n = threadIdx.x;
    for (; n + (U - 1) * kBlock < N; n += U * kBlock) {
#pragma unroll
        for (int q = 0; q < U; ++q) acc[q] = fma(a[n + q * kBlock], v[n + q * kBlock], acc[q]);
    }
    for (int q = 0; n < N; n += kBlock, ++q) acc[q] = fma(a[n], v[n], acc[q]);
#pragma unroll
    for (int w = U / 2; w > 0; w /= 2)
#pragma unroll
        for (int q = 0; q < w; ++q) acc[q] += acc[q + w];
    const double s = block_sum<kBlock>(acc[0], sh);
    if (threadIdx.x == 0) out[i] = s;
}

// stacked rows: Out[r, :] = src[r][:] (r < rows; pointer table src), and the
// reverse for the solution vectors (Out[g] = X[g, :] into dst[g])
__global__ __launch_bounds__(kBlock) void k_grp_gather(int64_t N, const double* const* __restrict__ src,
                                                       double* __restrict__ Out, int64_t ldo) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    const int r = blockIdx.y;
    Out[r * ldo + n] = src[r][n];
}

__global__ __launch_bounds__(kBlock) void k_grp_scatter(int64_t N, const double* __restrict__ X, int64_t ldx,
                                                        double* const* __restrict__ dst) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    const int g = blockIdx.y;
    dst[g][n] = X[g * ldx + n];
}

// compaction of the active vectors (idx: the active instances in order):
// Dst[r] = Src[idx[r]] (TO_COMPACT) or Dst[idx[r]] = Src[r], r < the grid's y
template <bool TO_COMPACT>
__global__ __launch_bounds__(kBlock) void k_grp_compact(int64_t N, const double* __restrict__ Src, int64_t lds,
                                                        const int* __restrict__ idx, double* __restrict__ Dst,
                                                        int64_t ldd) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    const int r = blockIdx.y;
    const int64_t s = TO_COMPACT ? idx[r] : r, d = TO_COMPACT ? r : idx[r];
    Dst[d * ldd + n] = Src[s * lds + n];
}

// sum over instance g's rows of A[i, n] c[i], combined per MODE:
//   0: Out[g, n] = alpha_g Out[g, n] + sum     (G p, with Out holding A p)
//   1: Out[g, n] = (Y[g, n] - sum) / alpha_g   (the Woodbury apply)
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_grp_jt(int64_t N, const double* __restrict__ A, int64_t lda,
                                                   const int* __restrict__ ro, const double* __restrict__ c,
                                                   const double* __restrict__ alpha, const double* __restrict__ Y,
                                                   int64_t ldy, const int* __restrict__ act, double* __restrict__ Out,
                                                   int64_t ldo) {
    __shared__ double cs[kGrpRows];
    const int g = blockIdx.y;
    if (act && !act[g]) return;
    const int r0 = ro[g], m = ro[g + 1] - r0;
    for (int t = threadIdx.x; t < m; t += kBlock) cs[t] = c[r0 + t];
    __syncthreads();
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    const double* a = A + (int64_t)r0 * lda + n;
    double s = 0.0;
    for (int i = 0; i < m; ++i) s = fma(a[(int64_t)i * lda], cs[i], s);
    double* o = Out + (int64_t)g * ldo + n;
    if (MODE == 0)
        *o = alpha[g] * *o + s;
    else
        *o = (Y[(int64_t)g * ldy + n] - s) / alpha[g];
}

// In-place Gauss-Jordan inverse of S_g (m_g <= 128) without pivoting, in
// LDS, one work-group per instance; writes the inverse transposed
// (SinvT[j m + i] = S^{-1}[i][j]); flag[0] = 1 on a zero or non-finite pivot.
__global__ __launch_bounds__(kGJThreadsG) void k_grp_inverse(const int* __restrict__ ro,
                                                             const int64_t* __restrict__ soff,
                                                             const double* __restrict__ S,
                                                             double* __restrict__ SinvT, int* __restrict__ flag) {
    __shared__ double a[kGrpRows * kGrpRows];
    __shared__ double prow[kGrpRows], pcol[kGrpRows];
    const int g = blockIdx.x;
    const int m = ro[g + 1] - ro[g];
    if (m == 0) return;
    const double* Sg = S + soff[g];
    const int tid = threadIdx.x;
    for (int t = tid; t < m * m; t += kGJThreadsG) a[t] = Sg[t];
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        double piv = a[k * m + k];
        if (!(std::fabs(piv) > 0.0 && std::fabs(piv) <= 1.79e308)) {
            if (tid == 0) flag[0] = 1;
            piv = 1.0;
        }
        const double inv = 1.0 / piv;
        for (int t = tid; t < m; t += kGJThreadsG) {
            prow[t] = a[k * m + t] * inv;
            pcol[t] = a[t * m + k];
        }
        __syncthreads();
        for (int t = tid; t < m * m; t += kGJThreadsG) {
            const int i = t / m, j = t - i * m;
            if (i == k)
                a[t] = (j == k) ? inv : prow[j];
            else
                a[t] = (j == k) ? -pcol[i] * inv : a[t] - pcol[i] * prow[j];
        }
        __syncthreads();
    }
    double* out = SinvT + soff[g];
    for (int t = tid; t < m * m; t += kGJThreadsG) {
        const int i = t / m, j = t - i * m;
        out[(int64_t)j * m + i] = a[t];
    }
}

// w[ro_g + i] = sum_j S_g^{-1}[i][j] t[ro_g + j], one work-group per instance
__global__ __launch_bounds__(kGrpRows) void k_grp_matvec(const int* __restrict__ ro, const int64_t* __restrict__ soff,
                                                         const double* __restrict__ SinvT,
                                                         const double* __restrict__ t, const int* __restrict__ act,
                                                         double* __restrict__ w) {
    __shared__ double ts[kGrpRows];
    const int g = blockIdx.x;
    if (!act[g]) return;
    const int r0 = ro[g], m = ro[g + 1] - r0;
    const int i = threadIdx.x;
    if (i < m) ts[i] = t[r0 + i];
    __syncthreads();
    if (i >= m) return;
    const double* col = SinvT + soff[g];
    double s = 0.0;
    for (int j = 0; j < m; ++j) s = fma(col[(int64_t)j * m + i], ts[j], s);
    w[r0 + i] = s;
}

// R[g] = B[g] - Q[g] for the G stacked vectors
__global__ __launch_bounds__(kBlock) void k_grp_sub(int64_t N, const double* __restrict__ B, const double* __restrict__ Q,
                                                    double* __restrict__ R, int64_t ld) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    const int64_t o = (int64_t)blockIdx.y * ld + n;
    R[o] = B[o] - Q[o];
}

// Constant-mode deflation of batched FP32 V-cycles (MIXED contexts), the
// single-vector steps of vcycle_B applied to k vectors at once:
// Y_g = float(F_g - c_g w) with c_g = sum(F_g) / sum(w) ...
__global__ __launch_bounds__(kBlock) void k_grp_defl_in(int64_t N, const double* __restrict__ F, int64_t ldf,
                                                        const double* __restrict__ fsum, double inv_w,
                                                        const double* __restrict__ wv, float* __restrict__ Y,
                                                        int64_t ldy) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    const int g = blockIdx.y;
    Y[g * ldy + n] = float(F[g * ldf + n] - (fsum[g] * inv_w) * wv[n]);
}

// ... partial sums of w . X_g (X_g the FP32 cycle's output) in the layout of
// the batched dot products ...
__global__ __launch_bounds__(kBlock) void k_grp_wdot(int64_t N, const double* __restrict__ wv,
                                                     const float* __restrict__ X, int64_t ldx,
                                                     double* __restrict__ partial) {
    __shared__ double sh[kBlock / 64];
    const int g = blockIdx.y;
    const float* x = X + g * ldx;
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x; n < N; n += (int64_t)gridDim.x * kBlock)
        acc += wv[n] * double(x[n]);
    const double sm = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t)g * gridDim.x + blockIdx.x] = sm;
}

// ... and Y_g = X_g - mu_g + c_g v with mu_g = (w . X_g) / sum(w), v = B w in FP64
__global__ __launch_bounds__(kBlock) void k_grp_defl_out(int64_t N, const float* __restrict__ X, int64_t ldx,
                                                         const double* __restrict__ fsum,
                                                         const double* __restrict__ wsx, double inv_w,
                                                         const double* __restrict__ v, double* __restrict__ Y,
                                                         int64_t ldy) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    const int g = blockIdx.y;
    Y[g * ldy + n] = double(X[g * ldx + n]) - wsx[g] * inv_w + (fsum[g] * inv_w) * v[n];
}

}  // namespace

// one V-cycle per right-hand side for a group: FP64 cycles, or FP32 cycles
// with the constant mode handled in FP64 as in vcycle_B
void Ctx::vcycle_group(int k, const double* F, int64_t ldf, double* X, int64_t ldx) {
    if (!fp32) {
        vcycle<double>(k, F, ldf, X, ldx);
        return;
    }
    ensure_deflation_vectors();
    const int64_t n = N(), P = pitch[0];
    const double inv_w = 1.0 / wsum;
    grpDefl.reserve((size_t)(2 + 64) * chunk * sizeof(double));
    double* fsum = grpDefl.as<double>();
    double* wsx = fsum + chunk;
    double* pp = wsx + chunk;
    const int nb = (int)std::min<int64_t>(64, cdiv(n, kBlock * 4));
    for (int r0 = 0; r0 < k; r0 += chunk) {
        const int kk = std::min(chunk, k - r0);
        stage.reserve((size_t)2 * kk * P * sizeof(float));
        float* fin = stage.as<float>();
        float* fout = fin + (size_t)kk * P;
        const double* Fc = F + (int64_t)r0 * ldf;
        launch_batched_dots(stream, kk, n, ones.as<double>(), 0, Fc, ldf, pp, fsum);
        const dim3 grid((unsigned)cdiv(n, kBlock), (unsigned)kk);
        hipLaunchKernelGGL(k_grp_defl_in, grid, dim3(kBlock), 0, stream, n, Fc, ldf, (const double*)fsum, inv_w,
                           (const double*)wvec.p, fin, P);
        H1W_LAUNCHED();
        vcycle_chunk<float>(kk, fin, P, fout, P);
        hipLaunchKernelGGL(k_grp_wdot, dim3((unsigned)nb, (unsigned)kk), dim3(kBlock), 0, stream, n,
                           (const double*)wvec.p, (const float*)fout, P, pp);
        H1W_LAUNCHED();
        launch_reduce_parts(stream, kk, nb, pp, wsx);
        hipLaunchKernelGGL(k_grp_defl_out, grid, dim3(kBlock), 0, stream, n, (const float*)fout, P,
                           (const double*)fsum, (const double*)wsx, inv_w, (const double*)vdef.p,
                           X + (int64_t)r0 * ldx, ldx);
        H1W_LAUNCHED();
    }
}

void Ctx::gn_group_solve(int G, const GroupItem* items, const h1w_solve_opts& so, h1w_info* infos,
                         h1w_status* status) {
    require(!ert, "grouped solves need an H1 context");
    require(G >= 1, "internal: empty group");
    const int64_t n = N(), P = pitch[0];
    const double rtol = so.rtol > 0.0 ? so.rtol : 1e-10;
    const int maxit = so.maxit > 0 ? so.maxit : 500;

    // instance tables (host), then one upload
    std::vector<int> ro(G + 1, 0), io(G + 1, 0), mm(G);
    std::vector<int64_t> soff(G + 1, 0), poff(G + 1, 0), kper(G, 0);
    std::vector<double> alph(G);
    for (int g = 0; g < G; ++g) {
        const GroupItem& it = items[g];
        require(it.m >= 0 && it.m <= kGroupMaxRows, "grouped solves take at most 128 rows per instance");
        require(std::isfinite(it.alpha) && it.alpha > 0.0, "item alpha must be finite and > 0");
        require(it.b != nullptr && it.x != nullptr && (it.m == 0 || (it.J != nullptr && it.ldj >= n)),
                "item b, x (and J with ldj >= N when m > 0) must be given");
        mm[g] = it.m;
        alph[g] = it.alpha;
        ro[g + 1] = ro[g] + it.m;
        soff[g + 1] = soff[g] + (int64_t)it.m * it.m;
        int ns = 0;
        if (it.m > 0) {
            // K cut into ranges of about 2048 values (at most 64 of them)
            const int64_t s0 = std::clamp<int64_t>(cdiv(n, 2048), 1, 64);
            kper[g] = cdiv(cdiv(n, s0), 16) * 16;
            ns = (int)cdiv(n, kper[g]);
        }
        io[g + 1] = io[g] + ns;
        poff[g + 1] = poff[g] + (int64_t)ns * it.m * it.m;
    }
    const int M = ro[G];
    const size_t rows = (size_t)std::max(M, 1);

    // device tables: int64 block (soff, poff, kper, then the row, b and x
    // pointers), int block (ro, io, m, the instance of each row; padded to an
    // even count so that alpha stays 8-byte aligned), alpha
    const size_t nptr = rows + 2 * (size_t)G;
    const size_t n64 = (size_t)(G + 1) * 2 + G + nptr, nint = ((size_t)(G + 1) * 2 + G + rows + 1) / 2 * 2;
    std::vector<char> host(n64 * 8 + nint * 4 + (size_t)G * 8);
    {
        const void** hp = (const void**)(host.data() + ((size_t)(G + 1) * 2 + G) * 8);
        for (int g = 0; g < G; ++g) {
            for (int r = 0; r < items[g].m; ++r) hp[ro[g] + r] = items[g].J + (int64_t)r * items[g].ldj;
            hp[rows + g] = items[g].b;
            hp[rows + G + g] = items[g].x;
        }
        if (M == 0) hp[0] = items[0].b;  // the unused row slot
        int64_t* h64 = (int64_t*)host.data();
        std::copy(soff.begin(), soff.end(), h64);
        std::copy(poff.begin(), poff.end(), h64 + (G + 1));
        std::copy(kper.begin(), kper.end(), h64 + 2 * (G + 1));
        int* hi = (int*)(host.data() + n64 * 8);
        std::copy(ro.begin(), ro.end(), hi);
        std::copy(io.begin(), io.end(), hi + (G + 1));
        std::copy(mm.begin(), mm.end(), hi + 2 * (G + 1));
        int* hrow = hi + 2 * (G + 1) + G;
        hrow[0] = 0;
        for (int g = 0; g < G; ++g)
            for (int r = ro[g]; r < ro[g + 1]; ++r) hrow[r] = g;
        std::copy(alph.begin(), alph.end(), (double*)(host.data() + n64 * 8 + nint * 4));
    }
    grpTab.reserve(host.size());
    H1W_HIP(hipMemcpyAsync(grpTab.p, host.data(), host.size(), hipMemcpyHostToDevice, stream));
    const int64_t* d_soff = grpTab.as<int64_t>();
    const int64_t* d_poff = d_soff + (G + 1);
    const int64_t* d_kper = d_soff + 2 * (G + 1);
    const int* d_ro = (const int*)((const char*)grpTab.p + n64 * 8);
    const int* d_io = d_ro + (G + 1);
    const int* d_m = d_io + (G + 1);
    const int* d_rowg = d_m + G;
    const double* d_alpha = (const double*)((const char*)grpTab.p + n64 * 8 + nint * 4);
    const double* const* d_rowp = (const double* const*)(d_soff + (G + 1) * 2 + G);
    const double* const* d_bp = d_rowp + rows;
    double* const* d_xp = (double* const*)(d_bp + G);

    // stacked rows of J and Z = B J^T
    grpJ.reserve(rows * P * sizeof(double));
    grpZ.reserve(rows * P * sizeof(double));
    double* Jall = grpJ.as<double>();
    double* Zall = grpZ.as<double>();
    if (M > 0) {
        hipLaunchKernelGGL(k_grp_gather, dim3((unsigned)cdiv(n, kBlock), (unsigned)M), dim3(kBlock), 0, stream, n,
                           d_rowp, Jall, P);
        H1W_LAUNCHED();
    }
    if (M > 0) vcycle_group(M, Jall, P, Zall, P);

    // S_g = alpha_g I + J_g Z_g^T and their inverses
    GrpGemm t{G, io[G], d_m, d_ro, d_io, d_kper, d_poff, d_soff, d_alpha};
    grpPart.reserve((size_t)std::max<int64_t>(poff[G], 1) * sizeof(double));
    grpS.reserve((size_t)std::max<int64_t>(soff[G], 1) * sizeof(double));
    grpSinv.reserve((size_t)std::max<int64_t>(soff[G], 1) * sizeof(double));
    launch_grp_gemm_partial(stream, t, n, Jall, P, Zall, P, grpPart.as<double>());
    launch_grp_gemm_reduce(stream, t, grpPart.as<double>(), grpS.as<double>());

    // vectors: B, X, R, Z, P, Q, Y and the compacted Rc, Yc (G x P each);
    // M-vectors t (J y or J p) and w = S^{-1} t; scalars
    grpVec.reserve((size_t)9 * G * P * sizeof(double) + (size_t)2 * rows * sizeof(double));
    double* Bv = grpVec.as<double>();
    double* X = Bv + (size_t)G * P;
    double* R = X + (size_t)G * P;
    double* Zv = R + (size_t)G * P;
    double* Pv = Zv + (size_t)G * P;
    double* Q = Pv + (size_t)G * P;
    double* Y = Q + (size_t)G * P;
    double* Rc = Y + (size_t)G * P;
    double* Yc = Rc + (size_t)G * P;
    double* tv = Yc + (size_t)G * P;
    double* wv = tv + rows;
    grpScal.reserve((size_t)(7 * G + 64 * G) * sizeof(double) + (size_t)(2 * G + 8) * sizeof(int));
    double* dnrm = grpScal.as<double>();
    double* drz = dnrm + G;
    double* dpq = drz + G;
    double* da = dpq + G;
    double* db = da + G;
    double* dzq = db + G;
    double* drzn = dzq + G;
    double* pp = drzn + G;  // 64 G dot-product partials
    int* dact = (int*)(pp + 64 * G);
    int* didx = dact + G;  // the active instances, in order
    int* dflag = didx + G;
    H1W_HIP(hipMemsetAsync(dflag, 0, 8 * sizeof(int), stream));
    if (M > 0)
        hipLaunchKernelGGL(k_grp_inverse, dim3((unsigned)G), dim3(kGJThreadsG), 0, stream, d_ro, d_soff,
                           (const double*)grpS.p, grpSinv.as<double>(), dflag);
    H1W_LAUNCHED();

    hipLaunchKernelGGL(k_grp_gather, dim3((unsigned)cdiv(n, kBlock), (unsigned)G), dim3(kBlock), 0, stream, n, d_bp,
                       Bv, P);
    H1W_LAUNCHED();
    H1W_HIP(hipMemset2DAsync(X, P * sizeof(double), 0, n * sizeof(double), G, stream));
    // Z, P, Q, Y start at zero: the rows of an instance that never runs (b = 0)
    // are then read as zeros by the unmasked kernels
    H1W_HIP(hipMemsetAsync(Zv, 0, (size_t)4 * G * P * sizeof(double), stream));

    const dim3 gridNG((unsigned)cdiv(n, kBlock), (unsigned)G);
    // host copies of the activity mask and of the active instances' indices
    std::vector<double> rr(G), nb(G);
    std::vector<int> act(G, 0), iters(G, 0), hidx(G, 0);
    int nact = 0;
    // out[i] = J_i . V[instance of i] for the M stacked rows (mask: nullptr or dact)
    auto rows_dot = [&](const double* V, double* out, const int* mask) {
        hipLaunchKernelGGL(k_grp_rows_dot, dim3((unsigned)M), dim3(kBlock), 0, stream, n, (const double*)Jall, P, V, P,
                           d_rowg, mask, out);
        H1W_LAUNCHED();
    };
    // z = P^{-1} r for the active instances. With a quarter or more of the
    // group converged, their right-hand sides are compacted first, so the
    // V-cycles run on the active ones only (two extra vector copies each).
    auto precond = [&](const double* Rin, double* Zout) {
        if (nact * 4 > G * 3) {
            vcycle_group(G, Rin, P, Y, P);
        } else if (nact > 0) {
            const dim3 gc((unsigned)cdiv(n, kBlock), (unsigned)nact);
            hipLaunchKernelGGL(k_grp_compact<true>, gc, dim3(kBlock), 0, stream, n, Rin, P, (const int*)didx, Rc, P);
            H1W_LAUNCHED();
            vcycle_group(nact, Rc, P, Yc, P);
            hipLaunchKernelGGL(k_grp_compact<false>, gc, dim3(kBlock), 0, stream, n, (const double*)Yc, P,
                               (const int*)didx, Y, P);
            H1W_LAUNCHED();
        }
        if (M > 0) {
            rows_dot(Y, tv, dact);
            hipLaunchKernelGGL(k_grp_matvec, dim3((unsigned)G), dim3(kGrpRows), 0, stream, d_ro, d_soff,
                               (const double*)grpSinv.p, (const double*)tv, (const int*)dact, wv);
        }
        hipLaunchKernelGGL(k_grp_jt<1>, gridNG, dim3(kBlock), 0, stream, n, (const double*)Zall, P, d_ro,
                           (const double*)wv, d_alpha, (const double*)Y, P, (const int*)dact, Zout, P);
        H1W_LAUNCHED();
    };
    // Q = G X = alpha A X + J^T (J X) (mask: nullptr, every instance, or dact)
    auto applyG = [&](const double* Pin, double* Qout, const int* mask) {
        launch_apply<double>(stream, dim, lv[0], G, Pin, P, Qout, P, 1.0);
        if (M > 0) rows_dot(Pin, tv, mask);
        hipLaunchKernelGGL(k_grp_jt<0>, gridNG, dim3(kBlock), 0, stream, n, (const double*)Jall, P, d_ro,
                           (const double*)tv, d_alpha, (const double*)nullptr, 0, mask, Qout, P);
        H1W_LAUNCHED();
    };
    int hflag[2] = {0, 0};
    auto fetch = [&](const double* d, std::vector<double>& h) {
        H1W_HIP(hipMemcpyAsync(h.data(), d, G * sizeof(double), hipMemcpyDeviceToHost, stream));
        H1W_HIP(hipMemcpyAsync(hflag, dflag, 2 * sizeof(int), hipMemcpyDeviceToHost, stream));
        sync();
    };
    // uploads the mask and the active list (the host copies change only after
    // the next fetch has synchronised the stream)
    auto put_act = [&]() {
        nact = 0;
        for (int g = 0; g < G; ++g)
            if (act[g]) hidx[nact++] = g;
        H1W_HIP(hipMemcpyAsync(dact, act.data(), G * sizeof(int), hipMemcpyHostToDevice, stream));
        H1W_HIP(hipMemcpyAsync(didx, hidx.data(), G * sizeof(int), hipMemcpyHostToDevice, stream));
    };

    // ||b||, and r = b (x = 0)
    H1W_HIP(hipMemcpy2DAsync(R, P * sizeof(double), Bv, P * sizeof(double), n * sizeof(double), G,
                             hipMemcpyDeviceToDevice, stream));
    launch_batched_dots(stream, G, n, R, P, R, P, pp, dnrm);
    fetch(dnrm, rr);
    if (hflag[0]) throw Error{H1W_ENUMERIC, "capacitance matrix of a grouped instance has a zero or non-finite pivot"};
    // per-instance outcome: an instance with non-finite values or a CG
    // breakdown stops alone (ENUMERIC), one that misses rtol within maxit
    // iterations and the restarts is ENOCONV; the others are unaffected
    for (int g = 0; g < G; ++g) status[g] = H1W_OK;
    for (int g = 0; g < G; ++g) {
        nb[g] = std::sqrt(rr[g]);
        if (!std::isfinite(rr[g])) status[g] = H1W_ENUMERIC;
        act[g] = status[g] == H1W_OK && nb[g] > 0.0;
    }
    std::vector<double> relres(G, 0.0), hpq(G);
    int total_it = 0;
    bool out_of_iters = false;
    for (int cycle = 0; cycle < 3 && !out_of_iters; ++cycle) {
        if (std::none_of(act.begin(), act.end(), [](int v) { return v; })) break;
        put_act();
        // z = P^{-1} r, p = z, rz = r.z
        precond(R, Zv);
        H1W_HIP(hipMemcpy2DAsync(Pv, P * sizeof(double), Zv, P * sizeof(double), n * sizeof(double), G,
                                 hipMemcpyDeviceToDevice, stream));
        launch_batched_dots(stream, G, n, R, P, Zv, P, pp, drz);
        for (;;) {
            if (total_it >= maxit) {
                out_of_iters = true;
                break;
            }
            applyG(Pv, Q, dact);
            launch_batched_dots(stream, G, n, Pv, P, Q, P, pp, dpq);
            launch_pcg_alpha(stream, G, drz, dpq, dact, da, dflag + 1);
            launch_batched_cg_xr(stream, G, n, da, Pv, P, Q, P, X, P, R, P, dact);
            launch_batched_dots(stream, G, n, R, P, R, P, pp, dnrm);
            fetch(dnrm, rr);
            if (hflag[1]) {
                // p.Gp <= 0 or not finite for some active instance (its step
                // was 0): find it, stop it, clear the flag
                fetch(dpq, hpq);
                for (int g = 0; g < G; ++g)
                    if (act[g] && !(hpq[g] > 0.0 && hpq[g] <= 1.79e308)) {
                        status[g] = H1W_ENUMERIC;
                        act[g] = 0;
                    }
                H1W_HIP(hipMemsetAsync(dflag + 1, 0, sizeof(int), stream));
                hflag[1] = 0;
            }
            ++total_it;
            bool any = false;
            for (int g = 0; g < G; ++g) {
                if (!act[g]) continue;
                if (!std::isfinite(rr[g])) {
                    status[g] = H1W_ENUMERIC;
                    act[g] = 0;
                    continue;
                }
                ++iters[g];
                if (std::sqrt(rr[g]) <= rtol * nb[g]) act[g] = 0;
                any = any || act[g];
            }
            put_act();
            if (!any) break;
            precond(R, Zv);
            launch_batched_dots(stream, G, n, R, P, Zv, P, pp, drzn);
            launch_batched_dots(stream, G, n, Zv, P, Q, P, pp, dzq);
            launch_pcg_beta(stream, G, drzn, drz, dzq, da, dact, db);
            launch_batched_p(stream, G, n, db, Zv, P, Pv, P, dact);
        }
        // true residuals r = b - G x (every instance); one that misses rtol
        // restarts from x
        applyG(X, Q, nullptr);
        hipLaunchKernelGGL(k_grp_sub, gridNG, dim3(kBlock), 0, stream, n, (const double*)Bv, (const double*)Q, R, P);
        H1W_LAUNCHED();
        launch_batched_dots(stream, G, n, R, P, R, P, pp, dnrm);
        fetch(dnrm, rr);
        for (int g = 0; g < G; ++g) {
            relres[g] = nb[g] > 0.0 ? std::sqrt(rr[g]) / nb[g] : 0.0;
            act[g] = status[g] == H1W_OK && !(relres[g] <= rtol);
        }
    }
    hipLaunchKernelGGL(k_grp_scatter, dim3((unsigned)cdiv(n, kBlock), (unsigned)G), dim3(kBlock), 0, stream, n,
                       (const double*)X, P, d_xp);
    H1W_LAUNCHED();
    for (int g = 0; g < G; ++g) {
        infos[g].iters = iters[g];
        infos[g].relres_true = relres[g];
        infos[g].relres_rec = relres[g];
        infos[g].nlevels = (int)lv.size();
    }
    sync();
    for (int g = 0; g < G; ++g)
        if (status[g] == H1W_OK && !(relres[g] <= rtol)) status[g] = H1W_ENOCONV;
}

}  // namespace h1w
