// Blocked factorisations of the m x m capacitance matrix S (Algorithm 3,
// third step) and the triangular solves of the preconditioner apply.
//
// Right-looking, block size NB = 64, three launches per block column kb:
//   diag   one work-group of 16 waves factors the NB x NB diagonal block
//          held in registers (Cholesky S_kk = U^T U, or LU without pivoting)
//          and writes the explicit inverses of its triangular factors
//          (Dinv_fwd, Dinv_bwd)
//   panel  Cholesky: U[kb, jb] = U_kk^{-T} A[kb, jb]                (jb > kb)
//          LU:       U[kb, jb] = L_kk^{-1} A[kb, jb], L[ib, kb] = A[ib, kb] U_kk^{-1}
//   update Cholesky: A[ib, jb] -= U[kb, ib]^T U[kb, jb]             (kb < ib <= jb)
//          LU:       A[ib, jb] -= L[ib, kb] U[kb, jb]               (ib, jb > kb)
// The NB x NB block products run on v_mfma_f64_16x16x4_f64: 4 waves, each a
// 32 x 32 quadrant = 2 x 2 MFMA blocks, K = NB in 16 steps, operands read
// straight from global memory (S is at most a few MB and stays in L2).
// A failed pivot stops the factorisation: info[0] is set and every later
// launch returns immediately.
//
// Triangular solves with a factor T run in one work-group: block by block,
// the right-hand side is updated with the already-solved part (T accessed
// through its transpose C, C[j][i] = T[i][j], so reads are coalesced) and
// multiplied by the explicit inverse of the diagonal block.
#include <algorithm>

#include "devutil.h"
#include "internal.h"

namespace h1w {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NB = 64;

__device__ __forceinline__ double ld_blk(const double* A, int m, int r, int c) {
    return (r < m && c < m) ? A[(int64_t)r * m + c] : 0.0;
}

// acc (this wave's 32x32 quadrant as 2x2 MFMA blocks) += op(X) * Y over K = NB.
// op(X)[r][k] = X[r0 + r][k0 + k]  (tx = false) or X[k0 + k][r0 + r] (tx = true);
// Y[k][c] = Y[y0 + k][c0 + c]. Out-of-range entries read as zero.
__device__ __forceinline__ void mfma_block(const double* X, int xr0, int xk0, bool tx, const double* Y, int yk0,
                                           int yc0, int m, d4 acc[2][2]) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int l16 = lane & 15, g = lane >> 4;
    const int qr = (wave >> 1) * 32, qc = (wave & 1) * 32;
#pragma unroll 4
    for (int s = 0; s < NB / 4; ++s) {
        const int k = 4 * s + g;
        double a[2], b[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int r = qr + 16 * t + l16;
            a[t] = tx ? ld_blk(X, m, xk0 + k, xr0 + r) : ld_blk(X, m, xr0 + r, xk0 + k);
            const int c = qc + 16 * t + l16;
            b[t] = ld_blk(Y, m, yk0 + k, yc0 + c);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
}

// Element (row, col) of the quadrant held by (lane, i, j, v): FP64 16x16 MFMA
// accumulator layout is row = (lane/16) + 4v, col = lane%16.
__device__ __forceinline__ void quad_pos(int i, int j, int v, int& r, int& c) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    r = (wave >> 1) * 32 + 16 * i + (lane >> 4) + 4 * v;
    c = (wave & 1) * 32 + 16 * j + (lane & 15);
}

// v of lane `lane` (wave-uniform) of the calling wave
__device__ __forceinline__ double lane_value(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------- diag
// mode 0: Cholesky (upper), mode 1: LU without pivoting.
// Lane j of wave w (16 waves) holds column j of the block rows 4w .. 4w + 3
// in registers (d[t] = row 4w + t) for the whole kernel. The elimination
// runs in 16 panel steps of 4 columns: the wave holding the panel's 4 rows
// eliminates them among themselves (pivots and multipliers from lane k by
// readlane), publishes them in LDS, and after one barrier every later wave
// applies the 4 eliminations to its rows in the same order. Each entry sees
// the same operations in the same order as in column-by-column elimination.
// The explicit inverses of the triangular factors are computed the same way
// by back (and, for LU, forward) substitution on all NB columns of the
// identity at once.
constexpr int kDiagThreads = 1024;
constexpr int kPanel = 4;   // rows per wave = columns per panel step
static_assert(kDiagThreads / 64 * kPanel == NB, "16 waves of 4 rows");

__device__ __forceinline__ bool bad_pivot(int mode, double p) {
    return mode == 0 ? !(p > 0.0) || !isfinite(p) : !(p != 0.0) || !isfinite(p);
}

__global__ __launch_bounds__(kDiagThreads) void k_blk_diag(int m, double* __restrict__ A, int kb, int mode,
                                                           double* __restrict__ Dfwd, double* __restrict__ Dbwd,
                                                           int* __restrict__ info) {
    __shared__ double pan[2][kPanel][NB];
    __shared__ int pfail[2];
    __shared__ double X[NB][NB + 1];
    if (info[0] >= 0) return;
    const int o = kb * NB;
    const int tid = threadIdx.x;
    const int j = tid & 63, w = tid >> 6;
    const int r0 = kPanel * w;  // first row of this wave
    double d[kPanel];
#pragma unroll
    for (int t = 0; t < kPanel; ++t) {
        const int i = r0 + t;
        d[t] = (o + i < m && o + j < m) ? A[(int64_t)(o + i) * m + o + j] : (i == j ? 1.0 : 0.0);
    }
    // Cholesky S = U^T U: u_kk = sqrt(p), u_kj = d_kj / u_kk, and the upper
    // trailing entries lose u_ki u_kj (p = d_kk before step k); the lower
    // triangle is left as it was. LU: l_ik = d_ik / p in place of d_ik, and
    // d_ij -= l_ik d_kj for i, j > k. The first bad pivot goes through LDS
    // to every thread, so all of them stop together.
    int fail = -1;
    for (int kp = 0; kp < NB / kPanel; ++kp) {
        const int k0 = kPanel * kp;
        double (*P)[NB] = pan[kp & 1];
        if (w == kp) {
            int f = -1;
#pragma unroll
            for (int t = 0; t < kPanel; ++t) {
                const int k = k0 + t;
                const double p = lane_value(d[t], k);
                if (f < 0 && bad_pivot(mode, p)) f = o + k;
                if (mode == 0) {
                    const double sk = sqrt(p);
                    const double u = d[t] / sk;
#pragma unroll
                    for (int t2 = t + 1; t2 < kPanel; ++t2) {
                        const double ui = lane_value(u, k0 + t2);
                        if (j >= k0 + t2) d[t2] -= ui * u;
                    }
                    P[t][j] = u;
                    if (j >= k) d[t] = j == k ? sk : u;
                } else {
#pragma unroll
                    for (int t2 = t + 1; t2 < kPanel; ++t2) {
                        const double l = lane_value(d[t2], k) / p;
                        d[t2] = j > k ? d[t2] - l * d[t] : (j == k ? l : d[t2]);
                    }
                    P[t][j] = d[t];
                }
            }
            if (j == 0) pfail[kp & 1] = f;
        }
        __syncthreads();
        fail = pfail[kp & 1];
        if (fail >= 0) break;
        if (w > kp) {
#pragma unroll
            for (int t = 0; t < kPanel; ++t) {
                const int k = k0 + t;
                const double ukj = P[t][j];
                if (mode == 0) {
#pragma unroll
                    for (int q = 0; q < kPanel; ++q) {
                        const double nv = d[q] - P[t][r0 + q] * ukj;
                        d[q] = j >= r0 + q ? nv : d[q];
                    }
                } else {
                    const double p = P[t][k];
#pragma unroll
                    for (int q = 0; q < kPanel; ++q) {
                        const double l = lane_value(d[q], k) / p;
                        d[q] = j > k ? d[q] - l * ukj : (j == k ? l : d[q]);
                    }
                }
            }
        }
    }
    if (fail >= 0) {
        if (tid == 0) info[0] = fail;
        return;
    }
    __syncthreads();  // the last panel's readers are done before pan[1] is reused
    // U X = I by back substitution: x_kj = b_kj / u_kk, then b_ij -= u_ik x_kj
    // for the rows i < k, k descending
    double x[kPanel];
#pragma unroll
    for (int t = 0; t < kPanel; ++t) x[t] = (r0 + t == j) ? 1.0 : 0.0;
    for (int kp = NB / kPanel - 1; kp >= 0; --kp) {
        const int k0 = kPanel * kp;
        double (*P)[NB] = pan[kp & 1];
        if (w == kp) {
#pragma unroll
            for (int t = kPanel - 1; t >= 0; --t) {
                const int k = k0 + t;
                x[t] = x[t] / lane_value(d[t], k);
#pragma unroll
                for (int t2 = 0; t2 < t; ++t2) x[t2] -= lane_value(d[t2], k) * x[t];
            }
#pragma unroll
            for (int t = 0; t < kPanel; ++t) P[t][j] = x[t];
        }
        __syncthreads();
        if (w < kp) {
#pragma unroll
            for (int t = kPanel - 1; t >= 0; --t) {
                const double xk = P[t][j];
#pragma unroll
                for (int q = 0; q < kPanel; ++q) x[q] -= lane_value(d[q], k0 + t) * xk;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < kPanel; ++t) X[r0 + t][j] = x[t];
    __syncthreads();
    double* Fw = Dfwd + (int64_t)kb * NB * NB;
    double* Bw = Dbwd + (int64_t)kb * NB * NB;
    for (int e = tid; e < NB * NB; e += kDiagThreads) {
        const int r = e / NB, c = e % NB;
        Bw[e] = r <= c ? X[r][c] : 0.0;
        if (mode == 0) Fw[e] = c <= r ? X[c][r] : 0.0;  // (U^T)^{-1} = (U^{-1})^T
    }
    if (mode == 1) {  // L X = I by forward substitution (unit diagonal): b_ij -= l_ik x_kj, i > k
#pragma unroll
        for (int t = 0; t < kPanel; ++t) x[t] = (r0 + t == j) ? 1.0 : 0.0;
        for (int kp = 0; kp < NB / kPanel; ++kp) {
            const int k0 = kPanel * kp;
            double (*P)[NB] = pan[kp & 1];
            if (w == kp) {
#pragma unroll
                for (int t = 0; t < kPanel; ++t) {
#pragma unroll
                    for (int t2 = t + 1; t2 < kPanel; ++t2) x[t2] -= lane_value(d[t2], k0 + t) * x[t];
                    P[t][j] = x[t];
                }
            }
            __syncthreads();
            if (w > kp) {
#pragma unroll
                for (int t = 0; t < kPanel; ++t) {
                    const double xk = P[t][j];
#pragma unroll
                    for (int q = 0; q < kPanel; ++q) x[q] -= lane_value(d[q], k0 + t) * xk;
                }
            }
        }
#pragma unroll
        for (int t = 0; t < kPanel; ++t) {
            const int i = r0 + t;
            Fw[i * NB + j] = i >= j ? x[t] : 0.0;
        }
    }
#pragma unroll
    for (int t = 0; t < kPanel; ++t) {
        const int i = r0 + t;
        if (o + i < m && o + j < m) A[(int64_t)(o + i) * m + o + j] = d[t];
    }
}

// ---------------------------------------------------------------- panel
// blockIdx.x enumerates the blocks to the right of (and, for LU, below) kb.
__global__ __launch_bounds__(256) void k_blk_panel(int m, double* __restrict__ A, int kb, int mode,
                                                   const double* __restrict__ Dfwd, const double* __restrict__ Dbwd,
                                                   const int* __restrict__ info) {
    if (info[0] >= 0) return;
    const int nb = (m + NB - 1) / NB;
    const int rest = nb - kb - 1;
    int b = blockIdx.x;
    const bool row_panel = b < rest;  // U[kb, jb]
    const int other = kb + 1 + (row_panel ? b : b - rest);
    const int o = kb * NB;
    d4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = d4{0, 0, 0, 0};
    const double* F = Dfwd + (int64_t)kb * NB * NB;
    const double* Bk = Dbwd + (int64_t)kb * NB * NB;
    // block inverse stored as a full NB x NB row-major tile: index it as an
    // m' = NB matrix with no bounds (pass m = NB to the loader).
    if (row_panel) {
        // out = Dfwd[kb] (NB x NB) * A[kb rows, other cols]
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int l16 = lane & 15, g = lane >> 4;
        const int qr = (wave >> 1) * 32, qc = (wave & 1) * 32;
        for (int s = 0; s < NB / 4; ++s) {
            const int k = 4 * s + g;
            double a[2], bb[2];
            for (int t = 0; t < 2; ++t) {
                a[t] = F[(qr + 16 * t + l16) * NB + k];
                bb[t] = ld_blk(A, m, o + k, other * NB + qc + 16 * t + l16);
            }
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();  // every wave has read the input block before it is overwritten
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int v = 0; v < 4; ++v) {
                    int r, c;
                    quad_pos(i, j, v, r, c);
                    const int R = o + r, Cc = other * NB + c;
                    if (R < m && Cc < m) A[(int64_t)R * m + Cc] = acc[i][j][v];
                }
    } else {
        // out = A[other rows, kb cols] (NB x NB) * Dbwd[kb]
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int l16 = lane & 15, g = lane >> 4;
        const int qr = (wave >> 1) * 32, qc = (wave & 1) * 32;
        for (int s = 0; s < NB / 4; ++s) {
            const int k = 4 * s + g;
            double a[2], bb[2];
            for (int t = 0; t < 2; ++t) {
                a[t] = ld_blk(A, m, other * NB + qr + 16 * t + l16, o + k);
                bb[t] = Bk[k * NB + qc + 16 * t + l16];
            }
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int v = 0; v < 4; ++v) {
                    int r, c;
                    quad_pos(i, j, v, r, c);
                    const int R = other * NB + r, Cc = o + c;
                    if (R < m && Cc < m) A[(int64_t)R * m + Cc] = acc[i][j][v];
                }
    }
}

// ---------------------------------------------------------------- trailing update
__global__ __launch_bounds__(256) void k_blk_update(int m, double* __restrict__ A, int kb, int mode,
                                                    const int* __restrict__ info) {
    if (info[0] >= 0) return;
    const int nb = (m + NB - 1) / NB;
    const int rest = nb - kb - 1;
    int ib, jb;
    if (mode == 0) {  // upper-triangle blocks kb < ib <= jb, enumerated row by row
        int t = blockIdx.x, i = 0;
        while (t >= rest - i) {
            t -= rest - i;
            ++i;
        }
        ib = kb + 1 + i;
        jb = ib + t;
    } else {
        ib = kb + 1 + blockIdx.x / rest;
        jb = kb + 1 + blockIdx.x % rest;
    }
    const int o = kb * NB;
    d4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = d4{0, 0, 0, 0};
    if (mode == 0)
        mfma_block(A, ib * NB, o, /*tx=*/true, A, o, jb * NB, m, acc);   // U[kb, ib]^T U[kb, jb]
    else
        mfma_block(A, ib * NB, o, /*tx=*/false, A, o, jb * NB, m, acc);  // L[ib, kb] U[kb, jb]
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int v = 0; v < 4; ++v) {
                int r, c;
                quad_pos(i, j, v, r, c);
                const int R = ib * NB + r, Cc = jb * NB + c;
                if (R < m && Cc < m) A[(int64_t)R * m + Cc] -= acc[i][j][v];
            }
}

// ---------------------------------------------------------------- solves
// Solve T x = b in place on the LDS vector sx (m entries) for block-triangular
// T given by C[j][i] = T[i][j] (row-major, ld m) and the inverses Dinv of its
// diagonal blocks; lower: forward substitution, else backward. All threads of
// the group take part; sx is final at return.
constexpr int kSolveThreads = 1024;
constexpr int kMaxM = 4096;

__device__ void blk_trsv_lds(int m, const double* __restrict__ C, const double* __restrict__ Dinv, bool lower,
                             double* sx, double (*part)[NB + 1], double* tvec) {
    const int tid = threadIdx.x;
    const int li = tid & 63, grp = tid >> 6;  // 64 entries x 16 groups
    const int nb = (m + NB - 1) / NB;
    for (int s = 0; s < nb; ++s) {
        const int kb = lower ? s : nb - 1 - s;
        const int o = kb * NB;
        const int i = o + li;
        // t_i = x_i - sum over solved j of C[j][i] x_j
        double acc = 0.0;
        if (i < m) {
            if (lower) {
                for (int j = grp; j < o; j += 16) acc += C[(int64_t)j * m + i] * sx[j];
            } else {
                for (int j = o + NB + grp; j < m; j += 16) acc += C[(int64_t)j * m + i] * sx[j];
            }
        }
        part[grp][li] = acc;
        __syncthreads();
        if (tid < NB) {
            double t = 0.0;
            for (int q = 0; q < 16; ++q) t += part[q][tid];
            tvec[tid] = (o + tid < m) ? sx[o + tid] - t : 0.0;
        }
        __syncthreads();
        // x_block = Dinv[kb] t
        const double* Dk = Dinv + (int64_t)kb * NB * NB;
        double y = 0.0;
        for (int q = grp; q < NB; q += 16) y += Dk[li * NB + q] * tvec[q];
        part[grp][li] = y;
        __syncthreads();
        if (tid < NB && o + tid < m) {
            double t = 0.0;
            for (int q = 0; q < 16; ++q) t += part[q][tid];
            sx[o + tid] = t;
        }
        __syncthreads();
    }
}

// out = T2^{-1} T1^{-1} in: the two triangular solves of S = T1 T2 in one
// launch, the vector staying in LDS between them (out may equal in)
__global__ __launch_bounds__(kSolveThreads) void k_blk_solve2(int m, const double* __restrict__ C1,
                                                              const double* __restrict__ D1, int lower1,
                                                              const double* __restrict__ C2,
                                                              const double* __restrict__ D2, int lower2,
                                                              const double* in, double* out) {
    __shared__ double sx[kMaxM];
    __shared__ double part[16][NB + 1];
    __shared__ double tvec[NB];
    for (int i = threadIdx.x; i < m; i += kSolveThreads) sx[i] = in[i];
    __syncthreads();
    blk_trsv_lds(m, C1, D1, lower1 != 0, sx, part, tvec);
    blk_trsv_lds(m, C2, D2, lower2 != 0, sx, part, tvec);
    for (int i = threadIdx.x; i < m; i += kSolveThreads) out[i] = sx[i];
}

}  // namespace

size_t blocked_inv_elems(int m) { return (size_t)((m + NB - 1) / NB) * NB * NB; }

void launch_blocked_factor(hipStream_t s, int m, double* A, int mode, double* Dfwd, double* Dbwd, int* info) {
    H1W_HIP(hipMemsetAsync(info, 0xff, sizeof(int), s));  // info = -1
    const int nb = (m + NB - 1) / NB;
    for (int kb = 0; kb < nb; ++kb) {
        hipLaunchKernelGGL(k_blk_diag, dim3(1), dim3(kDiagThreads), 0, s, m, A, kb, mode, Dfwd, Dbwd, info);
        H1W_LAUNCHED();
        const int rest = nb - kb - 1;
        if (rest == 0) break;
        const int npanel = mode == 0 ? rest : 2 * rest;
        hipLaunchKernelGGL(k_blk_panel, dim3(npanel), dim3(256), 0, s, m, A, kb, mode, Dfwd, Dbwd, info);
        H1W_LAUNCHED();
        const int nupd = mode == 0 ? rest * (rest + 1) / 2 : rest * rest;
        hipLaunchKernelGGL(k_blk_update, dim3(nupd), dim3(256), 0, s, m, A, kb, mode, info);
        H1W_LAUNCHED();
    }
}

void launch_blocked_solve2(hipStream_t s, int m, const double* C1, const double* D1, bool lower1, const double* C2,
                           const double* D2, bool lower2, const double* in, double* out) {
    if (m > kMaxM) throw Error{H1W_EINVAL, "m too large for the triangular solve"};
    hipLaunchKernelGGL(k_blk_solve2, dim3(1), dim3(kSolveThreads), 0, s, m, C1, D1, (int)lower1, C2, D2,
                       (int)lower2, in, out);
    H1W_LAUNCHED();
}

}  // namespace h1w
