// Dense m x m kernels for the capacitance system (Algorithm 3, third step and
// the two triangular solves of the preconditioner apply): the LU with partial
// pivoting used when the blocked factorisation meets a vanishing pivot, its
// triangular solves, the transpose, the asymmetry measure and the J-space
// update of the CG recurrences. One work-group of 1024 threads walks the columns; m is at most
// a few thousand, so these are latency-bound and small next to the V-cycles
// and the GEMM. All matrices are row-major with leading dimension m.
#include <algorithm>

#include "devutil.h"
#include "internal.h"

namespace h1w {

namespace {

constexpr int kDense = 1024;
constexpr int kMaxSolveM = 4096;  // x is staged in LDS (32 KB)

// LU with partial pivoting, in place: P A = L U with unit-lower L below the
// diagonal. piv[k] = row swapped with k at step k. info[0] = -1 on success,
// else the first zero (or non-finite) pivot column.
__global__ __launch_bounds__(kDense) void k_lu(int m, double* __restrict__ A, int* __restrict__ piv,
                                               int* __restrict__ info) {
    __shared__ double sval[kDense / 64];
    __shared__ int sidx[kDense / 64];
    __shared__ int sp;
    __shared__ int sfail;
    if (threadIdx.x == 0) sfail = -1;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < m; ++k) {
        // pivot search: largest |A[i][k]|, i >= k, smallest index on ties
        double best = -1.0;
        int bi = m;
        for (int i = k + threadIdx.x; i < m; i += kDense) {
            const double v = fabs(A[(int64_t)i * m + k]);
            if (v > best) { best = v; bi = i; }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_down(best, off, 64);
            const int oi = __shfl_down(bi, off, 64);
            if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
        }
        if (lane == 0) { sval[wid] = best; sidx[wid] = bi; }
        __syncthreads();
        if (threadIdx.x == 0) {
            double b = sval[0];
            int ii = sidx[0];
            for (int w = 1; w < kDense / 64; ++w)
                if (sval[w] > b || (sval[w] == b && sidx[w] < ii)) { b = sval[w]; ii = sidx[w]; }
            if (!(b > 0.0) || !isfinite(b) || ii >= m) { sfail = k; ii = k; }
            sp = ii;
            piv[k] = ii;
        }
        __syncthreads();
        if (sfail >= 0) break;
        const int p = sp;
        if (p != k) {
            double* rk = A + (int64_t)k * m;
            double* rp = A + (int64_t)p * m;
            for (int j = threadIdx.x; j < m; j += kDense) {
                const double t = rk[j];
                rk[j] = rp[j];
                rp[j] = t;
            }
        }
        __syncthreads();
        const double* rk = A + (int64_t)k * m;
        const double inv = 1.0 / rk[k];
        for (int i = k + 1 + threadIdx.x; i < m; i += kDense) A[(int64_t)i * m + k] *= inv;
        __syncthreads();
        for (int i = k + 1; i < m; ++i) {
            double* ri = A + (int64_t)i * m;
            const double l = ri[k];
            for (int j = k + 1 + threadIdx.x; j < m; j += kDense) ri[j] -= l * rk[j];
        }
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x == 0) info[0] = sfail;
}

__global__ __launch_bounds__(kBlock) void k_transpose(int m, const double* __restrict__ A, double* __restrict__ At) {
    __shared__ double tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int i = by + r, j = bx + tx;
        if (i < m && j < m) tile[r][tx] = A[(int64_t)i * m + j];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = bx + r, j = by + tx;
        if (i < m && j < m) At[(int64_t)i * m + j] = tile[tx][r];
    }
}

// Solve T y = b in place for triangular T given column by column: C holds
// row k = column k of T (i.e. C is T stored column-major). Column-oriented
// substitution, two barriers per column.
__device__ void trsv_cols(int m, const double* __restrict__ C, bool lower, bool unit, double* sx) {
    if (lower) {
        for (int k = 0; k < m; ++k) {
            __syncthreads();
            const double* ck = C + (int64_t)k * m;
            const double xk = unit ? sx[k] : sx[k] / ck[k];
            __syncthreads();
            if (threadIdx.x == 0) sx[k] = xk;
            for (int i = k + 1 + threadIdx.x; i < m; i += kDense) sx[i] -= ck[i] * xk;
        }
    } else {
        for (int k = m - 1; k >= 0; --k) {
            __syncthreads();
            const double* ck = C + (int64_t)k * m;
            const double xk = unit ? sx[k] : sx[k] / ck[k];
            __syncthreads();
            if (threadIdx.x == 0) sx[k] = xk;
            for (int i = threadIdx.x; i < k; i += kDense) sx[i] -= ck[i] * xk;
        }
    }
    __syncthreads();
}

// P S = L U (LU in place, LUt its transpose = the factors stored column-major).
__global__ __launch_bounds__(kDense) void k_lu_solve(int m, const double* __restrict__ LUt,
                                                     const int* __restrict__ piv, double* __restrict__ x) {
    __shared__ double sx[kMaxSolveM];
    for (int i = threadIdx.x; i < m; i += kDense) sx[i] = x[i];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < m; ++k) {
            const int p = piv[k];
            if (p != k) {
                const double t = sx[k];
                sx[k] = sx[p];
                sx[p] = t;
            }
        }
    trsv_cols(m, LUt, true, true, sx);
    trsv_cols(m, LUt, false, false, sx);
    for (int i = threadIdx.x; i < m; i += kDense) x[i] = sx[i];
}

// Jz_i = (Jy_i - sum_j S_ij w_j + alpha w_i) / alpha ;  Jp_i = Jz_i + beta Jp_i.
// One wave per row.
__global__ __launch_bounds__(kBlock) void k_jz_update(int m, const double* __restrict__ S, double alpha,
                                                      const double* __restrict__ Jy, const double* __restrict__ w,
                                                      const double* __restrict__ bdev,
                                                      double* __restrict__ Jz, double* __restrict__ Jp) {
    const double beta = *bdev;
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= m) return;
    const double* s = S + (int64_t)row * m;
    double acc = 0.0;
    for (int j = lane; j < m; j += 64) acc += s[j] * w[j];
    acc = wave_sum(acc);
    if (lane == 0) {
        const double jz = (Jy[row] - acc + alpha * w[row]) / alpha;
        Jz[row] = jz;
        Jp[row] = beta == 0.0 ? jz : jz + beta * Jp[row];
    }
}

// out[0] = max_ij |S_ij - S_ji|
__global__ __launch_bounds__(kDense) void k_asym(int m, const double* __restrict__ S, double* __restrict__ out) {
    __shared__ double sh[kDense / 64];
    double mx = 0.0;
    for (int64_t idx = threadIdx.x; idx < (int64_t)m * m; idx += kDense) {
        const int i = (int)(idx / m), j = (int)(idx - (int64_t)i * m);
        if (j > i) mx = fmax(mx, fabs(S[(int64_t)i * m + j] - S[(int64_t)j * m + i]));
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int w = 0; w < kDense / 64; ++w) r = fmax(r, sh[w]);
        out[0] = r;
    }
}

// out[0..3] = max S_ii, min S_ii, max |F_ii|, min |F_ii| (S and its factor,
// whose diagonal holds the pivots u_ii of S = U^T U or S = L U)
__global__ __launch_bounds__(kDense) void k_diag_stats(int m, const double* __restrict__ S,
                                                       const double* __restrict__ F, double* __restrict__ out) {
    __shared__ double sh[4][kDense / 64];
    double smax = -INFINITY, smin = INFINITY, fmax_ = 0.0, fmin_ = INFINITY;
    for (int i = threadIdx.x; i < m; i += kDense) {
        const double sv = S[(int64_t)i * m + i], fv = fabs(F[(int64_t)i * m + i]);
        smax = fmax(smax, sv);
        smin = fmin(smin, sv);
        fmax_ = fmax(fmax_, fv);
        fmin_ = fmin(fmin_, fv);
    }
    for (int off = 32; off > 0; off >>= 1) {
        smax = fmax(smax, __shfl_down(smax, off, 64));
        smin = fmin(smin, __shfl_down(smin, off, 64));
        fmax_ = fmax(fmax_, __shfl_down(fmax_, off, 64));
        fmin_ = fmin(fmin_, __shfl_down(fmin_, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = smax;
        sh[1][threadIdx.x >> 6] = smin;
        sh[2][threadIdx.x >> 6] = fmax_;
        sh[3][threadIdx.x >> 6] = fmin_;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kDense / 64; ++w) {
            sh[0][0] = fmax(sh[0][0], sh[0][w]);
            sh[1][0] = fmin(sh[1][0], sh[1][w]);
            sh[2][0] = fmax(sh[2][0], sh[2][w]);
            sh[3][0] = fmin(sh[3][0], sh[3][w]);
        }
        for (int k = 0; k < 4; ++k) out[k] = sh[k][0];
    }
}

}  // namespace

void launch_diag_stats(hipStream_t s, int m, const double* S, const double* F, double* out) {
    hipLaunchKernelGGL(k_diag_stats, dim3(1), dim3(kDense), 0, s, m, S, F, out);
    H1W_LAUNCHED();
}

void launch_lu(hipStream_t s, int m, double* A, int* piv, int* info) {
    hipLaunchKernelGGL(k_lu, dim3(1), dim3(kDense), 0, s, m, A, piv, info);
    H1W_LAUNCHED();
}

void launch_transpose(hipStream_t s, int m, const double* A, double* At) {
    const dim3 grid((unsigned)cdiv(m, 32), (unsigned)cdiv(m, 32));
    hipLaunchKernelGGL(k_transpose, grid, dim3(kBlock), 0, s, m, A, At);
    H1W_LAUNCHED();
}

void launch_lu_solve(hipStream_t s, int m, const double* LUt, const double* /*LU*/, const int* piv, double* x) {
    if (m > kMaxSolveM) throw Error{H1W_EINVAL, "m too large for the triangular solve"};
    hipLaunchKernelGGL(k_lu_solve, dim3(1), dim3(kDense), 0, s, m, LUt, piv, x);
    H1W_LAUNCHED();
}

void launch_jz_update_dev(hipStream_t s, int m, const double* S, double alpha, const double* Jy, const double* w,
                          const double* bdev, double* Jz, double* Jp) {
    hipLaunchKernelGGL(k_jz_update, dim3((unsigned)cdiv(m, kBlock / 64)), dim3(kBlock), 0, s, m, S, alpha, Jy, w,
                       bdev, Jz, Jp);
    H1W_LAUNCHED();
}

void launch_asym(hipStream_t s, int m, const double* S, double* out) {
    hipLaunchKernelGGL(k_asym, dim3(1), dim3(kDense), 0, s, m, S, out);
    H1W_LAUNCHED();
}

}  // namespace h1w
