// Vector kernels of the Krylov loop and the passes over the dense m x N
// matrices J (sensitivities) and Z (= B J^T). All reductions are two-stage
// with a fixed order (per-block partial sums, then one block per output), so
// a rerun with the same launch shapes is bitwise identical.
#include <algorithm>

#include "devutil.h"
#include "internal.h"

namespace h1w {

namespace {

constexpr int kDotBlocks = 1024;   // max blocks of a dot-product pass
constexpr int kRowChunk = kBlock * 8;   // nodes per block in J v
constexpr int kTile = 256;         // rows of J staged in LDS per sweep in J^T v

struct DotArgs {
    const double* x[4];
    const double* y[4];
};

template <int NP>
__global__ __launch_bounds__(kBlock) void k_dots_partial(int64_t N, DotArgs a,
                                                         double* __restrict__ partial) {
    __shared__ double sh[kBlock / 64];
    double acc[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) acc[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * kBlock) {
#pragma unroll
        for (int q = 0; q < NP; ++q) acc[q] += a.x[q][i] * a.y[q][i];
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const double s = block_sum<kBlock>(acc[q], sh);
        if (threadIdx.x == 0) partial[q * gridDim.x + blockIdx.x] = s;
    }
}

// out[v] = sum_b partial[v*nparts + b]; one block per output value.
__global__ __launch_bounds__(kBlock) void k_reduce_parts(int nparts, const double* __restrict__ partial,
                                                         double* __restrict__ out) {
    __shared__ double sh[kBlock / 64];
    const double* p = partial + (int64_t)blockIdx.x * nparts;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) acc += p[b];
    const double s = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// partial[i*nchunk + c] = sum over chunk c of M[i, n] v[n] for every row i.
// Block (c, g) takes chunk c of kRowChunk nodes and the rows of group g
// (rows_per consecutive rows; one group of all m rows on large grids, where
// the chunks alone fill the GPU): each wave takes rows wid, wid + 4, ... of
// the group and reduces each row's chunk itself (lane l holds nodes
// c0 + 2 l + 128 e, e < 16, as 16-byte pairs; fixed order: lane sums over e,
// then the wave sum), so v's slice is read once per block and every row
// piece is a 16 KB (FP64) run.
template <typename TM>
__global__ __launch_bounds__(kBlock) void k_rows_dot(int m, int rows_per, int64_t N, const TM* __restrict__ M,
                                                     int64_t ldm, const double* __restrict__ v,
                                                     double* __restrict__ partial) {
    constexpr int E = kRowChunk / 128;  // node pairs per lane
    const int nchunk = gridDim.x;
    const int64_t base = (int64_t)blockIdx.x * kRowChunk;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double v0[E], v1[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t n = base + 128 * e + 2 * lane;
        v0[e] = n < N ? v[n] : 0.0;
        v1[e] = n + 1 < N ? v[n + 1] : 0.0;
    }
    const bool tail = base + kRowChunk > N;
    const int i0 = blockIdx.y * rows_per, i1 = min(m, i0 + rows_per);
    for (int i = i0 + wid; i < i1; i += kBlock / 64) {
        const TM* row = M + (int64_t)i * ldm;
        double acc = 0.0;
        if (!tail) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t n = base + 128 * e + 2 * lane;
                acc = fma(double(row[n]), v0[e], acc);
                acc = fma(double(row[n + 1]), v1[e], acc);
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t n = base + 128 * e + 2 * lane;
                const double x0 = n < N ? double(row[n]) : 0.0;
                const double x1 = n + 1 < N ? double(row[n + 1]) : 0.0;
                acc = fma(x0, v0[e], acc);
                acc = fma(x1, v1[e], acc);
            }
        }
        acc = wave_sum(acc);
        if (lane == 0) partial[(int64_t)i * nchunk + blockIdx.x] = acc;
    }
}

// Two products in one pass over M: partial sums of M[i,:].v1 and M[i,:].v2,
// in the layout and order of k_rows_dot (block (chunk, row group), a wave per
// row, lane pairs of nodes).
__global__ __launch_bounds__(kBlock) void k_rows_dot2(int m, int rows_per, int64_t N, const double* __restrict__ M,
                                                      int64_t ldm, const double* __restrict__ v1,
                                                      const double* __restrict__ v2, double* __restrict__ part1,
                                                      double* __restrict__ part2) {
    constexpr int E = kRowChunk / 128;
    const int nchunk = gridDim.x;
    const int64_t base = (int64_t)blockIdx.x * kRowChunk;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double a0[E], a1[E], b0[E], b1[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t n = base + 128 * e + 2 * lane;
        a0[e] = n < N ? v1[n] : 0.0;
        a1[e] = n + 1 < N ? v1[n + 1] : 0.0;
        b0[e] = n < N ? v2[n] : 0.0;
        b1[e] = n + 1 < N ? v2[n + 1] : 0.0;
    }
    const bool tail = base + kRowChunk > N;
    const int i0 = blockIdx.y * rows_per, i1 = min(m, i0 + rows_per);
    for (int i = i0 + wid; i < i1; i += kBlock / 64) {
        const double* row = M + (int64_t)i * ldm;
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t n = base + 128 * e + 2 * lane;
            const double x0 = (!tail || n < N) ? row[n] : 0.0;
            const double x1 = (!tail || n + 1 < N) ? row[n + 1] : 0.0;
            s1 = fma(x0, a0[e], s1);
            s1 = fma(x1, a1[e], s1);
            s2 = fma(x0, b0[e], s2);
            s2 = fma(x1, b1[e], s2);
        }
        s1 = wave_sum(s1);
        s2 = wave_sum(s2);
        if (lane == 0) {
            part1[(int64_t)i * nchunk + blockIdx.x] = s1;
            part2[(int64_t)i * nchunk + blockIdx.x] = s2;
        }
    }
}

// u = (r - J^T w) * inv_alpha ;  t = J^T jp
__global__ __launch_bounds__(kBlock) void k_jt_u_t(int m, int64_t N, const double* __restrict__ J,
                                                   int64_t ldj, const double* __restrict__ w,
                                                   const double* __restrict__ jp,
                                                   const double* __restrict__ r, double inv_alpha,
                                                   double* __restrict__ u, double* __restrict__ t) {
    __shared__ double sw[kTile], sj[kTile];
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double aw = 0.0, aj = 0.0;
    for (int i0 = 0; i0 < m; i0 += kTile) {
        const int cnt = std::min(kTile, m - i0);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt; q += kBlock) {
            sw[q] = w[i0 + q];
            sj[q] = jp[i0 + q];
        }
        __syncthreads();
        if (n < N) {
            const double* col = J + (int64_t)i0 * ldj + n;
#pragma unroll 8
            for (int q = 0; q < cnt; ++q) {
                const double jv = col[(int64_t)q * ldj];
                aw += jv * sw[q];
                aj += jv * sj[q];
            }
        }
    }
    if (n < N) {
        u[n] = (r[n] - aw) * inv_alpha;
        t[n] = aj;
    }
}

// out = J^T v + add_coef * add   (add may be null, or equal to out: each
// thread reads add[n] before it writes out[n], so out and add carry no
// __restrict__)
__global__ __launch_bounds__(kBlock) void k_jt_plain(int m, int64_t N, const double* __restrict__ J,
                                                     int64_t ldj, const double* __restrict__ v,
                                                     double* out, const double* add, double add_coef) {
    __shared__ double sv[kTile];
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double acc = 0.0;
    for (int i0 = 0; i0 < m; i0 += kTile) {
        const int cnt = std::min(kTile, m - i0);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt; q += kBlock) sv[q] = v[i0 + q];
        __syncthreads();
        if (n < N) {
            const double* col = J + (int64_t)i0 * ldj + n;
#pragma unroll 8
            for (int q = 0; q < cnt; ++q) acc += col[(int64_t)q * ldj] * sv[q];
        }
    }
    if (n < N) out[n] = add ? acc + add_coef * add[n] : acc;
}

// z = (y - Z^T w - (c0 v - c1)) * inv_alpha, the last term only with v
// (the rank-one parts of a deflated FP32 Z). c0, c1 = s.w, mu.w are read
// from cptr, or, with sd and md given (m <= kBlock * 4), computed here by
// every work-group in the order of k_dots_partial<2> (one block) followed by
// k_reduce_parts, so the values are the same as from those two kernels.
template <typename TZ>
__global__ __launch_bounds__(kBlock) void k_z_stored(int m, int64_t N, const TZ* __restrict__ Z,
                                                     int64_t ldz, const double* __restrict__ w,
                                                     const double* __restrict__ y, double inv_alpha,
                                                     const double* __restrict__ v, const double* __restrict__ cptr,
                                                     const double* __restrict__ sd, const double* __restrict__ md,
                                                     double* __restrict__ z) {
    __shared__ double sw[kTile];
    __shared__ double sh[kBlock / 64];
    __shared__ double sc[2];
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double c0 = 0.0, c1 = 0.0;
    if (v && sd) {
        double a0 = 0.0, a1 = 0.0;
        for (int i = threadIdx.x; i < m; i += kBlock) {
            a0 += sd[i] * w[i];
            a1 += md[i] * w[i];
        }
        const double s0 = block_sum<kBlock>(a0, sh);
        const double s1 = block_sum<kBlock>(a1, sh);
        if (threadIdx.x == 0) {
            sc[0] = s0;
            sc[1] = s1;
        }
        __syncthreads();
        c0 = sc[0];
        c1 = sc[1];
    } else if (v) {
        c0 = cptr[0];
        c1 = cptr[1];
    }
    double acc = 0.0;
    for (int i0 = 0; i0 < m; i0 += kTile) {
        const int cnt = std::min(kTile, m - i0);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt; q += kBlock) sw[q] = w[i0 + q];
        __syncthreads();
        if (n < N) {
            const TZ* col = Z + (int64_t)i0 * ldz + n;
#pragma unroll 8
            for (int q = 0; q < cnt; ++q) acc += double(col[(int64_t)q * ldz]) * sw[q];
        }
    }
    if (n < N) z[n] = (y[n] - acc - (v ? c0 * v[n] - c1 : 0.0)) * inv_alpha;
}

// S[i][j] += a[i] b[j] + c[i] d[j]  (m x m, row-major)
__global__ __launch_bounds__(kBlock) void k_rank2_add(int m, const double* __restrict__ a, const double* __restrict__ bv,
                                                      const double* __restrict__ c, const double* __restrict__ dv,
                                                      double* __restrict__ S) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (int64_t)m * m) return;
    const int i = (int)(idx / m), j = (int)(idx - (int64_t)i * m);
    S[idx] += a[i] * bv[j] + c[i] * dv[j];
}

// y = s * x  for m entries (tiny vectors)
__global__ __launch_bounds__(kBlock) void k_scale(int m, double s, const double* __restrict__ x, double* __restrict__ y) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < m) y[i] = s * x[i];
}

// p = (y - Z^T w) * inv_alpha + beta * p ;  t = J^T jp
template <typename TZ>
__global__ __launch_bounds__(kBlock) void k_p_stored(int m, int64_t N, const TZ* __restrict__ Z,
                                                     int64_t ldz, const double* __restrict__ w,
                                                     const double* __restrict__ J, int64_t ldj,
                                                     const double* __restrict__ jp,
                                                     const double* __restrict__ y, double inv_alpha,
                                                     double beta, double* __restrict__ p,
                                                     double* __restrict__ t) {
    __shared__ double sw[kTile], sj[kTile];
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double az = 0.0, aj = 0.0;
    for (int i0 = 0; i0 < m; i0 += kTile) {
        const int cnt = std::min(kTile, m - i0);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt; q += kBlock) {
            sw[q] = w[i0 + q];
            sj[q] = jp[i0 + q];
        }
        __syncthreads();
        if (n < N) {
            const TZ* zc = Z + (int64_t)i0 * ldz + n;
            const double* jc = J + (int64_t)i0 * ldj + n;
#pragma unroll 8
            for (int q = 0; q < cnt; ++q) {
                az += double(zc[(int64_t)q * ldz]) * sw[q];
                aj += jc[(int64_t)q * ldj] * sj[q];
            }
        }
    }
    if (n < N) {
        p[n] = (y[n] - az) * inv_alpha + beta * p[n];
        t[n] = aj;
    }
}

__global__ __launch_bounds__(kBlock) void k_axpby(int64_t N, double a, const double* __restrict__ x,
                                                  double b, const double* __restrict__ bdev,
                                                  double* __restrict__ y) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const double bb = bdev ? *bdev : b;
    if (n < N) y[n] = a * x[n] + (bb == 0.0 ? 0.0 : bb * y[n]);
}

__global__ __launch_bounds__(kBlock) void k_sub(int64_t N, const double* __restrict__ b,
                                                const double* __restrict__ v,
                                                double* __restrict__ out) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n < N) out[n] = b[n] - v[n];
}

// x += a p ; r -= a q ; partial sums of r.r
// x += a p, r -= a q with the step length a read from device memory;
// partial sums of r.r
// x += a p, r -= a q and the partial sums of r.r; with psum, also those of
// sum(r) (the grid and order of k_dots_partial<1> against a vector of ones)
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t N, const double* __restrict__ adev,
                                                      const double* __restrict__ p, const double* __restrict__ q,
                                                      double* __restrict__ x, double* __restrict__ r,
                                                      double* __restrict__ partial, double* __restrict__ psum) {
    __shared__ double sh[kBlock / 64];
    const double a = *adev;
    double acc = 0.0, acs = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x; n < N;
         n += (int64_t)gridDim.x * kBlock) {
        x[n] += a * p[n];
        const double rn = r[n] - a * q[n];
        r[n] = rn;
        acc += rn * rn;
        acs += rn;
    }
    const double s = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
    if (psum) {
        const double t = block_sum<kBlock>(acs, sh);
        if (threadIdx.x == 0) psum[blockIdx.x] = t;
    }
}

// per-row dot products of a batch: partial[r*nb + b]
__global__ __launch_bounds__(kBlock) void k_batched_dots(int64_t N, const double* __restrict__ X,
                                                         int64_t ldx, const double* __restrict__ Y,
                                                         int64_t ldy, double* __restrict__ partial) {
    __shared__ double sh[kBlock / 64];
    const int r = blockIdx.y;
    const double* x = X + r * ldx;
    const double* y = Y + r * ldy;
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x; n < N;
         n += (int64_t)gridDim.x * kBlock)
        acc += x[n] * y[n];
    const double s = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t)r * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_batched_cg_xr(int64_t N, const double* __restrict__ a,
                                                          const double* __restrict__ P, int64_t ldp,
                                                          const double* __restrict__ Q, int64_t ldq,
                                                          double* __restrict__ X, int64_t ldx,
                                                          double* __restrict__ R, int64_t ldr,
                                                          const int* __restrict__ active) {
    const int r = blockIdx.y;
    if (!active[r]) return;
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    const double ar = a[r];
    X[r * ldx + n] += ar * P[r * ldp + n];
    R[r * ldr + n] -= ar * Q[r * ldq + n];
}

__global__ __launch_bounds__(kBlock) void k_batched_p(int64_t N, const double* __restrict__ b,
                                                      const double* __restrict__ Z, int64_t ldz,
                                                      double* __restrict__ P, int64_t ldp,
                                                      const int* __restrict__ active) {
    const int r = blockIdx.y;
    if (!active[r]) return;
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    P[r * ldp + n] = Z[r * ldz + n] + b[r] * P[r * ldp + n];
}

// per-row CG step lengths a = rz / pq on the device (0 for finished rows);
// flag[0] = 1 on a non-positive or non-finite p.q of an active row
__global__ void k_pcg_alpha(int k, const double* __restrict__ rz, const double* __restrict__ pq,
                            const int* __restrict__ active, double* __restrict__ a, int* __restrict__ flag) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= k) return;
    double v = 0.0;
    if (active[r]) {
        if (!(pq[r] > 0.0 && pq[r] <= 1.79e308)) flag[0] = 1;
        else v = rz[r] / pq[r];
    }
    a[r] = v;
}

// per-row direction coefficients: b = rz_new / rz (or the flexible
// Polak-Ribiere form -a z.q / rz when zq is given), then rz := rz_new
__global__ void k_pcg_beta(int k, const double* __restrict__ rzn, double* __restrict__ rz,
                           const double* __restrict__ zq, const double* __restrict__ a,
                           const int* __restrict__ active, double* __restrict__ b) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= k) return;
    double v = 0.0;
    if (active[r]) v = zq ? -a[r] * zq[r] / rz[r] : rzn[r] / rz[r];
    b[r] = v;
    rz[r] = rzn[r];
}

int dot_blocks(int64_t N) { return (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, cdiv(N, kBlock * 4))); }

}  // namespace

int launch_dots_partial(hipStream_t s, int64_t N, int npair, const double* const* X,
                        const double* const* Y, double* partial) {
    DotArgs a{};
    for (int q = 0; q < npair; ++q) {
        a.x[q] = X[q];
        a.y[q] = Y[q];
    }
    const int nb = dot_blocks(N);
    switch (npair) {
        case 1: hipLaunchKernelGGL(k_dots_partial<1>, dim3(nb), dim3(kBlock), 0, s, N, a, partial); break;
        case 2: hipLaunchKernelGGL(k_dots_partial<2>, dim3(nb), dim3(kBlock), 0, s, N, a, partial); break;
        case 3: hipLaunchKernelGGL(k_dots_partial<3>, dim3(nb), dim3(kBlock), 0, s, N, a, partial); break;
        case 4: hipLaunchKernelGGL(k_dots_partial<4>, dim3(nb), dim3(kBlock), 0, s, N, a, partial); break;
        default: throw Error{H1W_EINVAL, "internal: npair out of range"};
    }
    H1W_LAUNCHED();
    return nb;
}

void launch_reduce_parts(hipStream_t s, int nvec, int nparts, const double* partial, double* out) {
    hipLaunchKernelGGL(k_reduce_parts, dim3(nvec), dim3(kBlock), 0, s, nparts, partial, out);
    H1W_LAUNCHED();
}

size_t rows_dot_partial_elems(int m, int64_t N) { return (size_t)m * (size_t)cdiv(N, kRowChunk); }

// row groups of the J v pass: enough blocks for about 2048 in all (8 per CU),
// at least 4 rows (one per wave) per group
static int rows_dot_rows_per(int m, int nchunk) {
    const int groups = (int)std::clamp<int64_t>(cdiv(2048, nchunk), 1, cdiv(m, 4));
    return (int)(cdiv(cdiv(m, groups), 4) * 4);
}

int launch_rows_dot_partial(hipStream_t s, int m, int64_t N, const double* M, int64_t ldm, const double* v,
                            double* partial) {
    const int nchunk = (int)cdiv(N, kRowChunk);
    if (m <= 0) return nchunk;
    const int rp = rows_dot_rows_per(m, nchunk);
    hipLaunchKernelGGL((k_rows_dot<double>), dim3(nchunk, (unsigned)cdiv(m, rp)), dim3(kBlock), 0, s, m, rp, N, M,
                       ldm, v, partial);
    H1W_LAUNCHED();
    return nchunk;
}

int launch_rows_dot_partial_f32(hipStream_t s, int m, int64_t N, const float* M, int64_t ldm, const double* v,
                                double* partial) {
    const int nchunk = (int)cdiv(N, kRowChunk);
    if (m <= 0) return nchunk;
    const int rp = rows_dot_rows_per(m, nchunk);
    hipLaunchKernelGGL((k_rows_dot<float>), dim3(nchunk, (unsigned)cdiv(m, rp)), dim3(kBlock), 0, s, m, rp, N, M,
                       ldm, v, partial);
    H1W_LAUNCHED();
    return nchunk;
}

void launch_jt_u_t(hipStream_t s, int m, int64_t N, const double* J, int64_t ldj, const double* w,
                   const double* jp, const double* r, double inv_alpha, double* u, double* t) {
    hipLaunchKernelGGL(k_jt_u_t, dim3((unsigned)cdiv(N, kBlock)), dim3(kBlock), 0, s, m, N, J, ldj,
                       w, jp, r, inv_alpha, u, t);
    H1W_LAUNCHED();
}

void launch_jt_plain(hipStream_t s, int m, int64_t N, const double* J, int64_t ldj, const double* v,
                     double* out, const double* add, double add_coef) {
    hipLaunchKernelGGL(k_jt_plain, dim3((unsigned)cdiv(N, kBlock)), dim3(kBlock), 0, s, m, N, J, ldj,
                       v, out, add, add_coef);
    H1W_LAUNCHED();
}

template <typename TZ>
void launch_z_stored(hipStream_t s, int m, int64_t N, const TZ* Z, int64_t ldz, const double* w,
                     const double* y, double inv_alpha, const double* v, const double* cptr, double* z,
                     const double* sd, const double* md) {
    if (sd && m > kBlock * 4) throw Error{H1W_EINVAL, "internal: in-kernel rank-one dots need m <= 1024"};
    hipLaunchKernelGGL((k_z_stored<TZ>), dim3((unsigned)cdiv(N, kBlock)), dim3(kBlock), 0, s, m, N, Z,
                       ldz, w, y, inv_alpha, v, cptr, sd, md, z);
    H1W_LAUNCHED();
}

int launch_rows_dot2_partial(hipStream_t s, int m, int64_t N, const double* M, int64_t ldm, const double* v1,
                             const double* v2, double* part1, double* part2) {
    const int nchunk = (int)cdiv(N, kRowChunk);
    if (m <= 0) return nchunk;
    const int rp = rows_dot_rows_per(m, nchunk);
    hipLaunchKernelGGL(k_rows_dot2, dim3(nchunk, (unsigned)cdiv(m, rp)), dim3(kBlock), 0, s, m, rp, N, M, ldm, v1,
                       v2, part1, part2);
    H1W_LAUNCHED();
    return nchunk;
}

void launch_rank2_add(hipStream_t s, int m, const double* a, const double* bv, const double* c, const double* dv,
                      double* S) {
    hipLaunchKernelGGL(k_rank2_add, dim3((unsigned)cdiv((int64_t)m * m, kBlock)), dim3(kBlock), 0, s, m, a, bv, c, dv,
                       S);
    H1W_LAUNCHED();
}

__global__ __launch_bounds__(kBlock) void k_fill(int64_t N, double v, double* __restrict__ y) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n < N) y[n] = v;
}

// Zout[i][n] = float(Z1[i][n] - mu_i + s_i v[n])  (full Z of a deflated FP32 capacitance)
__global__ __launch_bounds__(kBlock) void k_zout_deflated(int m, int64_t N, const float* __restrict__ Z1, int64_t ldz,
                                                          const double* __restrict__ sv, const double* __restrict__ mu,
                                                          const double* __restrict__ v, float* __restrict__ out,
                                                          int64_t ldo) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    const double vn = v[n];
    for (int i = blockIdx.y; i < m; i += gridDim.y)
        out[(int64_t)i * ldo + n] = float(double(Z1[(int64_t)i * ldz + n]) - mu[i] + sv[i] * vn);
}

void launch_zout_deflated(hipStream_t s, int m, int64_t N, const float* Z1, int64_t ldz, const double* sv,
                          const double* mu, const double* v, float* out, int64_t ldo) {
    hipLaunchKernelGGL(k_zout_deflated, dim3((unsigned)cdiv(N, kBlock), (unsigned)std::min(m, 65535)), dim3(kBlock), 0,
                       s, m, N, Z1, ldz, sv, mu, v, out, ldo);
    H1W_LAUNCHED();
}

// y = x - mu + c v  (FP64 result of a deflated FP32 V-cycle: x converted from float)
// Deflation steps of the single-vector FP32 V-cycle with the partial sums
// reduced inside the kernel (the same fixed order as k_reduce_parts, so every
// block gets the same value): c = inv_w * sum(part) and Y = float(F - c w)
// (cm[0] = c); then mu = inv_w * sum(part) and y = x - mu + c v (cm[1] = mu).
__device__ __forceinline__ double reduce_parts_block(int nparts, const double* __restrict__ part, double* sh,
                                                     double* bc) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) acc += part[b];
    const double s = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) *bc = s;
    __syncthreads();
    return *bc;
}

__global__ __launch_bounds__(kBlock) void k_deflate_in(int64_t N, const double* __restrict__ F,
                                                       const double* __restrict__ part, int nparts, double inv_w,
                                                       const double* __restrict__ wv, float* __restrict__ Y,
                                                       double* __restrict__ cm) {
    __shared__ double sh[kBlock / 64];
    __shared__ double bc;
    const double c = reduce_parts_block(nparts, part, sh, &bc) * inv_w;
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) cm[0] = c;
    if (p < N) Y[p] = float(F[p] - c * wv[p]);
}

__global__ __launch_bounds__(kBlock) void k_deflate_out(int64_t N, const float* __restrict__ x,
                                                        const double* __restrict__ part, int nparts, double inv_w,
                                                        double* __restrict__ cm, const double* __restrict__ v,
                                                        double* __restrict__ y) {
    __shared__ double sh[kBlock / 64];
    __shared__ double bc;
    const double mu = reduce_parts_block(nparts, part, sh, &bc) * inv_w;
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const double c = cm[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) cm[1] = mu;
    if (n < N) y[n] = double(x[n]) - mu + c * v[n];
}

void launch_deflate_in(hipStream_t s, int64_t N, const double* F, const double* part, int nparts, double inv_w,
                       const double* wv, float* Y, double* cm) {
    hipLaunchKernelGGL(k_deflate_in, dim3((unsigned)cdiv(N, kBlock)), dim3(kBlock), 0, s, N, F, part, nparts, inv_w,
                       wv, Y, cm);
    H1W_LAUNCHED();
}

void launch_deflate_out(hipStream_t s, int64_t N, const float* x, const double* part, int nparts, double inv_w,
                        double* cm, const double* v, double* y) {
    hipLaunchKernelGGL(k_deflate_out, dim3((unsigned)cdiv(N, kBlock)), dim3(kBlock), 0, s, N, x, part, nparts, inv_w,
                       cm, v, y);
    H1W_LAUNCHED();
}

void launch_fill(hipStream_t s, int64_t N, double v, double* y) {
    hipLaunchKernelGGL(k_fill, dim3((unsigned)cdiv(N, kBlock)), dim3(kBlock), 0, s, N, v, y);
    H1W_LAUNCHED();
}

void launch_scale(hipStream_t s, int m, double a, const double* x, double* y) {
    hipLaunchKernelGGL(k_scale, dim3((unsigned)cdiv(m, kBlock)), dim3(kBlock), 0, s, m, a, x, y);
    H1W_LAUNCHED();
}

template <typename TZ>
void launch_p_stored(hipStream_t s, int m, int64_t N, const TZ* Z, int64_t ldz, const double* w,
                     const double* J, int64_t ldj, const double* jp, const double* y, double inv_alpha,
                     double beta, double* p, double* t) {
    hipLaunchKernelGGL((k_p_stored<TZ>), dim3((unsigned)cdiv(N, kBlock)), dim3(kBlock), 0, s, m, N, Z,
                       ldz, w, J, ldj, jp, y, inv_alpha, beta, p, t);
    H1W_LAUNCHED();
}

void launch_axpby(hipStream_t s, int64_t N, double a, const double* x, double b, double* y) {
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)cdiv(N, kBlock)), dim3(kBlock), 0, s, N, a, x, b, (const double*)nullptr,
                       y);
    H1W_LAUNCHED();
}

void launch_axpby_dev(hipStream_t s, int64_t N, double a, const double* x, const double* bdev, double* y) {
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)cdiv(N, kBlock)), dim3(kBlock), 0, s, N, a, x, 0.0, bdev, y);
    H1W_LAUNCHED();
}

// Scalars of the Gauss-Newton CG kept on the device (dsc = scal + kGnScal):
// dsc[0] = r.z, [1] = step length a, [2] = direction coefficient beta,
// [3] = p.q, [4] = r.r, [5] = 1 if r.z <= 0 at the last preconditioner step,
// [6] = 1 if p.q <= 0, [7] = 1 if p.q is not finite.
// beta from the dot products s[0], s[1] of the preconditioner step:
// mode 0 (recompute form) r.z = (s0 - s1) / alpha; mode 1 (stored Z)
// r.z = s0, z.q = s1; mode 2 (no Woodbury correction) r.z = s0 / alpha,
// z.q = s1 / alpha. beta = 0 on a first step, else z.(r_new - r_old)/r.z
// (flexible, with r_new - r_old = -a q) or r.z_new / r.z.
// Partial sums reduced in the order of k_reduce_parts: out[v] = sum over b
// of partial[v * nparts + b] (block-strided, then the waves in order).
__device__ void reduce_rows_block(const double* __restrict__ partial, int nvec, int nparts, double* out, double* sh) {
    for (int v = 0; v < nvec; ++v) {
        const double* p = partial + (int64_t)v * nparts;
        double acc = 0.0;
        for (int b = threadIdx.x; b < nparts; b += kBlock) acc += p[b];
        const double s = block_sum<kBlock>(acc, sh);
        if (threadIdx.x == 0) out[v] = s;
    }
}

// The dot products of a CG step, reduced here from their partial sums (na
// vectors of nba parts in pa, then nb vectors of nbb parts in pb) into
// sdot[0 .. na + nb - 1], then beta and r.z:
//   mode 0 (recompute form): r.z = (r.y - w.Jy) / alpha;
//   mode 1 (stored Z, flexible): r.z = sdot[0], z.q = sdot[1] (Polak-Ribiere);
//   mode 2 (B / alpha only):    r.z = r.y / alpha, z.q = y.q / alpha.
// dsc: [0] r.z, [2] beta, [5] 1 when r.z <= 0 (converged to rounding).
__global__ __launch_bounds__(kBlock) void k_gn_beta(const double* __restrict__ pa, int na, int nba,
                                                    const double* __restrict__ pb, int nb, int nbb, double ia,
                                                    int mode, int first, int flexible, double* __restrict__ sdot,
                                                    double* __restrict__ dsc) {
    __shared__ double sh[kBlock / 64];
    __shared__ double sd[4];
    reduce_rows_block(pa, na, nba, sd, sh);
    reduce_rows_block(pb, nb, nbb, sd + na, sh);
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int v = 0; v < na + nb; ++v) sdot[v] = sd[v];
    double rzn, zq = 0.0;
    if (mode == 0) {
        rzn = (sd[0] - sd[1]) * ia;
    } else if (mode == 1) {
        rzn = sd[0];
        zq = sd[1];
    } else {
        rzn = sd[0] * ia;
        zq = sd[1] * ia;
    }
    const bool ok = rzn > 0.0;
    double beta = 0.0;
    if (ok && !first) beta = flexible ? -dsc[1] * zq / dsc[0] : rzn / dsc[0];
    dsc[2] = beta;
    if (ok) dsc[0] = rzn;
    dsc[5] = ok ? 0.0 : 1.0;
}

// p.q reduced here from its nparts partial sums into dsc[3]; then the step
// a = r.z / p.q in dsc[1], or 0 when the step must not be taken
__global__ __launch_bounds__(kBlock) void k_gn_alpha(const double* __restrict__ partial, int nparts,
                                                     double* __restrict__ dsc) {
    __shared__ double sh[kBlock / 64];
    __shared__ double spq;
    reduce_rows_block(partial, 1, nparts, &spq, sh);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double pq = spq;
    dsc[3] = pq;
    const bool finite = pq >= -1.79e308 && pq <= 1.79e308;
    dsc[7] = finite ? 0.0 : 1.0;
    dsc[6] = (finite && !(pq > 0.0)) ? 1.0 : 0.0;
    dsc[1] = (dsc[5] == 0.0 && finite && pq > 0.0) ? dsc[0] / pq : 0.0;
}

// r.r reduced from its partial sums into dsc[4] (order of k_reduce_parts);
// then the eight scalars dsc[0..7] written to host-visible memory, so the
// host reads them after a stream synchronisation without a copy.
__global__ __launch_bounds__(kBlock) void k_gn_report(const double* __restrict__ partial, int nparts,
                                                      double* __restrict__ dsc, double* __restrict__ host) {
    __shared__ double sh[kBlock / 64];
    __shared__ double srr;
    reduce_rows_block(partial, 1, nparts, &srr, sh);
    __syncthreads();
    const int t = threadIdx.x;
    if (t == 4) dsc[4] = srr;
    if (t < 8) host[t] = t == 4 ? srr : dsc[t];
}

// out[v] = sum_b partial[v * nparts + b] (order of k_reduce_parts), written
// to host-visible memory; one block.
__global__ __launch_bounds__(kBlock) void k_reduce_host(int nvec, int nparts, const double* __restrict__ partial,
                                                        double* __restrict__ host) {
    __shared__ double sh[kBlock / 64];
    __shared__ double sv[4];
    reduce_rows_block(partial, nvec, nparts, sv, sh);
    __syncthreads();
    if ((int)threadIdx.x < nvec) host[threadIdx.x] = sv[threadIdx.x];
}

// Start of CG from x = 0: x = 0, r = b, p = q = 0, Jp = 0 (m values), and
// the partial sums of b.b with the grid and order of k_dots_partial<1>.
__global__ __launch_bounds__(kBlock) void k_cg_init(int64_t N, const double* __restrict__ b, double* __restrict__ x,
                                                    double* __restrict__ r, double* __restrict__ p,
                                                    double* __restrict__ q, int m, double* __restrict__ Jp,
                                                    double* __restrict__ partial) {
    __shared__ double sh[kBlock / 64];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += stride) {
        const double v = b[i];
        acc += v * v;
        x[i] = 0.0;
        r[i] = v;
        p[i] = 0.0;
        q[i] = 0.0;
    }
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) Jp[i] = 0.0;
    const double s = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

void launch_gn_report(hipStream_t s, const double* partial, int nparts, double* dsc, double* host) {
    hipLaunchKernelGGL(k_gn_report, dim3(1), dim3(kBlock), 0, s, partial, nparts, dsc, host);
    H1W_LAUNCHED();
}

void launch_reduce_host(hipStream_t s, int nvec, int nparts, const double* partial, double* host) {
    if (nvec < 1 || nvec > 4) throw Error{H1W_EINVAL, "internal: 1 to 4 reductions"};
    hipLaunchKernelGGL(k_reduce_host, dim3(1), dim3(kBlock), 0, s, nvec, nparts, partial, host);
    H1W_LAUNCHED();
}

int launch_cg_init(hipStream_t s, int64_t N, const double* b, double* x, double* r, double* p, double* q, int m,
                   double* Jp, double* partial) {
    const int nb = dot_blocks(N);
    hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(kBlock), 0, s, N, b, x, r, p, q, m, Jp, partial);
    H1W_LAUNCHED();
    return nb;
}

void launch_gn_beta(hipStream_t s, const double* pa, int na, int nba, const double* pb, int nb, int nbb, double ia,
                    int mode, bool first, bool flexible, double* sdot, double* dsc) {
    if (na + nb > 4) throw Error{H1W_EINVAL, "internal: at most 4 dot products"};
    hipLaunchKernelGGL(k_gn_beta, dim3(1), dim3(kBlock), 0, s, pa, na, nba, pb, nb, nbb, ia, mode, (int)first,
                       (int)flexible, sdot, dsc);
    H1W_LAUNCHED();
}

void launch_gn_alpha(hipStream_t s, const double* partial, int nparts, double* dsc) {
    hipLaunchKernelGGL(k_gn_alpha, dim3(1), dim3(kBlock), 0, s, partial, nparts, dsc);
    H1W_LAUNCHED();
}

void launch_sub(hipStream_t s, int64_t N, const double* b, const double* v, double* out) {
    hipLaunchKernelGGL(k_sub, dim3((unsigned)cdiv(N, kBlock)), dim3(kBlock), 0, s, N, b, v, out);
    H1W_LAUNCHED();
}

void launch_cg_update_dev(hipStream_t s, int64_t N, const double* adev, const double* p, const double* q,
                          double* x, double* r, double* partial, int* nparts, double* psum) {
    const int nb = dot_blocks(N);
    hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(kBlock), 0, s, N, adev, p, q, x, r, partial, psum);
    H1W_LAUNCHED();
    *nparts = nb;
}

void launch_batched_dots(hipStream_t s, int k, int64_t N, const double* X, int64_t ldx, const double* Y,
                         int64_t ldy, double* partial, double* out) {
    const int nb = (int)std::min<int64_t>(64, cdiv(N, kBlock * 4));
    hipLaunchKernelGGL(k_batched_dots, dim3(nb, k), dim3(kBlock), 0, s, N, X, ldx, Y, ldy, partial);
    H1W_LAUNCHED();
    launch_reduce_parts(s, k, nb, partial, out);
}

void launch_batched_cg_xr(hipStream_t s, int k, int64_t N, const double* a, const double* P, int64_t ldp,
                          const double* Q, int64_t ldq, double* X, int64_t ldx, double* R, int64_t ldr,
                          const int* active) {
    hipLaunchKernelGGL(k_batched_cg_xr, dim3((unsigned)cdiv(N, kBlock), k), dim3(kBlock), 0, s, N, a, P,
                       ldp, Q, ldq, X, ldx, R, ldr, active);
    H1W_LAUNCHED();
}

void launch_pcg_alpha(hipStream_t s, int k, const double* rz, const double* pq, const int* active, double* a,
                      int* flag) {
    hipLaunchKernelGGL(k_pcg_alpha, dim3((unsigned)cdiv(k, 64)), dim3(64), 0, s, k, rz, pq, active, a, flag);
    H1W_LAUNCHED();
}

void launch_pcg_beta(hipStream_t s, int k, const double* rzn, double* rz, const double* zq, const double* a,
                     const int* active, double* b) {
    hipLaunchKernelGGL(k_pcg_beta, dim3((unsigned)cdiv(k, 64)), dim3(64), 0, s, k, rzn, rz, zq, a, active, b);
    H1W_LAUNCHED();
}

void launch_batched_p(hipStream_t s, int k, int64_t N, const double* b, const double* Z, int64_t ldz,
                      double* P, int64_t ldp, const int* active) {
    hipLaunchKernelGGL(k_batched_p, dim3((unsigned)cdiv(N, kBlock), k), dim3(kBlock), 0, s, N, b, Z, ldz,
                       P, ldp, active);
    H1W_LAUNCHED();
}

template void launch_z_stored<double>(hipStream_t, int, int64_t, const double*, int64_t, const double*,
                                      const double*, double, const double*, const double*, double*, const double*,
                                      const double*);
template void launch_z_stored<float>(hipStream_t, int, int64_t, const float*, int64_t, const double*,
                                     const double*, double, const double*, const double*, double*, const double*,
                                     const double*);
template void launch_p_stored<double>(hipStream_t, int, int64_t, const double*, int64_t, const double*,
                                      const double*, int64_t, const double*, const double*, double,
                                      double, double*, double*);
template void launch_p_stored<float>(hipStream_t, int, int64_t, const float*, int64_t, const double*,
                                     const double*, int64_t, const double*, const double*, double,
                                     double, double*, double*);

}  // namespace h1w
