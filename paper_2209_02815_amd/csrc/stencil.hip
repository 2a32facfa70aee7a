// Multi-right-hand-side stencil kernels on one grid level: the H^1 Gram
// operator A = K + beta*W (5-/7-point with Neumann half weights), its
// Chebyshev-Jacobi smoothing steps, residual, full-weighting restriction
// R = 2^-d P^T, multilinear interpolation P, and the dense coarsest solve.
//
// Layout: a batch of k grid vectors, row r at base + r*ld, x fastest.
// blockIdx.x tiles the nodes of one vector, blockIdx.y walks the rows.
//
// Stencil at node (i, j, l) with boundary weights w = 1/2 on the first and
// last node of an axis, 1 elsewhere:
//   (A u)_p = beta wx wy wz u_p + sum_axes c_axis * sum_nbrs (u_p - u_nbr),
//   c_x = wy wz / hx^2, c_y = wx wz / hy^2, c_z = wx wy / hz^2
// (2D: drop z). The diagonal is D_p = beta wx wy wz + sum_axes c_axis * #nbrs.
#include "devutil.h"
#include "internal.h"

namespace h1w {

namespace {

template <typename T, int DIM>
struct NodeCoef {
    T cx, cy, cz, mass, diag;
    bool xm, xp, ym, yp, zm, zp;
};

template <typename T, int DIM>
__device__ __forceinline__ NodeCoef<T, DIM> node_coef(const Geom& g, int i, int j, int l) {
    NodeCoef<T, DIM> c;
    const T half = T(0.5), one = T(1);
    const T wx = (i == 0 || i == g.nx - 1) ? half : one;
    const T wy = (j == 0 || j == g.ny - 1) ? half : one;
    const T wz = (DIM == 3 && (l == 0 || l == g.nz - 1)) ? half : one;
    c.xm = i > 0; c.xp = i < g.nx - 1;
    c.ym = j > 0; c.yp = j < g.ny - 1;
    c.zm = DIM == 3 && l > 0; c.zp = DIM == 3 && l < g.nz - 1;
    c.cx = T(g.ihx2) * wy * wz;
    c.cy = T(g.ihy2) * wx * wz;
    c.cz = DIM == 3 ? T(g.ihz2) * wx * wy : T(0);
    c.mass = T(g.beta) * wx * wy * wz;
    c.diag = c.mass + c.cx * T(int(c.xm) + int(c.xp)) + c.cy * T(int(c.ym) + int(c.yp)) +
             c.cz * T(int(c.zm) + int(c.zp));
    return c;
}

template <typename T, int DIM>
__device__ __forceinline__ T apply_at(const Geom& g, const T* __restrict__ u, int p,
                                      const NodeCoef<T, DIM>& c) {
    const T u0 = u[p];
    T sx = T(0), sy = T(0), sz = T(0);
    if (c.xm) sx += u0 - u[p - 1];
    if (c.xp) sx += u0 - u[p + 1];
    if (c.ym) sy += u0 - u[p - g.nx];
    if (c.yp) sy += u0 - u[p + g.nx];
    if (DIM == 3) {
        const int pl = g.nx * g.ny;
        if (c.zm) sz += u0 - u[p - pl];
        if (c.zp) sz += u0 - u[p + pl];
    }
    T acc = c.mass * u0;
    acc += c.cx * sx;
    acc += c.cy * sy;
    if (DIM == 3) acc += c.cz * sz;
    return acc;
}

__device__ __forceinline__ void decompose(const Geom& g, int p, int& i, int& j, int& l) {
    i = p % g.nx;
    const int q = p / g.nx;
    j = q % g.ny;
    l = q / g.ny;
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_apply(Geom g, int k, const T* __restrict__ X,
                                                  int64_t ldx, T* __restrict__ Y, int64_t ldy,
                                                  T scale) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= g.N) return;
    int i, j, l;
    decompose(g, p, i, j, l);
    const auto c = node_coef<T, DIM>(g, i, j, l);
    for (int r = blockIdx.y; r < k; r += gridDim.y)
        Y[r * ldy + p] = scale * apply_at<T, DIM>(g, X + r * ldx, p, c);
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_smooth_first(Geom g, int k, const T* __restrict__ F,
                                                         int64_t ldf, T* __restrict__ X,
                                                         int64_t ldx, T w) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= g.N) return;
    int i, j, l;
    decompose(g, p, i, j, l);
    const auto c = node_coef<T, DIM>(g, i, j, l);
    for (int r = blockIdx.y; r < k; r += gridDim.y) X[r * ldx + p] = w * F[r * ldf + p] / c.diag;
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_smooth(Geom g, int k, const T* __restrict__ F,
                                                   int64_t ldf, const T* __restrict__ Xi,
                                                   int64_t ldi, T* __restrict__ Xo, int64_t ldo,
                                                   T w) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= g.N) return;
    int i, j, l;
    decompose(g, p, i, j, l);
    const auto c = node_coef<T, DIM>(g, i, j, l);
    for (int r = blockIdx.y; r < k; r += gridDim.y) {
        const T* x = Xi + r * ldi;
        const T res = F[r * ldf + p] - apply_at<T, DIM>(g, x, p, c);
        Xo[r * ldo + p] = x[p] + w * res / c.diag;
    }
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_residual(Geom g, int k, const T* __restrict__ F,
                                                     int64_t ldf, const T* __restrict__ X,
                                                     int64_t ldx, T* __restrict__ R,
                                                     int64_t ldr) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= g.N) return;
    int i, j, l;
    decompose(g, p, i, j, l);
    const auto c = node_coef<T, DIM>(g, i, j, l);
    for (int r = blockIdx.y; r < k; r += gridDim.y)
        R[r * ldr + p] = F[r * ldf + p] - apply_at<T, DIM>(g, X + r * ldx, p, c);
}

// Fc = 2^-d P^T R: coarse node (I,J,L) gathers the fine nodes 2I+{-1,0,1} (per
// axis) with weights 1 (centre) and 1/2 (neighbours). Loops run z, y, x in
// ascending fine index.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_restrict(Geom gf, Geom gc, int k,
                                                     const T* __restrict__ R, int64_t ldr,
                                                     T* __restrict__ Fc, int64_t ldc) {
    const int pc = blockIdx.x * kBlock + threadIdx.x;
    if (pc >= gc.N) return;
    int I, J, L;
    decompose(gc, pc, I, J, L);
    const int fi = 2 * I, fj = 2 * J, fl = DIM == 3 ? 2 * L : 0;
    const int pl = gf.nx * gf.ny;
    const T scale = DIM == 3 ? T(0.125) : T(0.25);
    for (int r = blockIdx.y; r < k; r += gridDim.y) {
        const T* rr = R + r * ldr;
        T acc = T(0);
        const int zlo = DIM == 3 ? -1 : 0, zhi = DIM == 3 ? 1 : 0;
        for (int dz = zlo; dz <= zhi; ++dz) {
            const int z = fl + dz;
            if (z < 0 || z >= gf.nz) continue;
            const T wz = dz ? T(0.5) : T(1);
            for (int dy = -1; dy <= 1; ++dy) {
                const int y = fj + dy;
                if (y < 0 || y >= gf.ny) continue;
                const T wy = dy ? T(0.5) : T(1);
                for (int dx = -1; dx <= 1; ++dx) {
                    const int x = fi + dx;
                    if (x < 0 || x >= gf.nx) continue;
                    const T wx = dx ? T(0.5) : T(1);
                    acc += (wz * wy * wx) * rr[z * pl + y * gf.nx + x];
                }
            }
        }
        Fc[r * ldc + pc] = scale * acc;
    }
}

// X += P Ec: fine node (i,j,l) interpolates from the coarse nodes floor(i/2)
// and, for odd i, floor(i/2)+1 (weights 1/2), per axis.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_prolong_add(Geom gf, Geom gc, int k,
                                                        const T* __restrict__ Ec, int64_t ldc,
                                                        T* __restrict__ X, int64_t ldx) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= gf.N) return;
    int i, j, l;
    decompose(gf, p, i, j, l);
    const int ci = i >> 1, cj = j >> 1, cl = l >> 1;
    const int ni = 1 + (i & 1), nj = 1 + (j & 1), nl = DIM == 3 ? 1 + (l & 1) : 1;
    const T wi = (i & 1) ? T(0.5) : T(1), wj = (j & 1) ? T(0.5) : T(1);
    const T wl = (DIM == 3 && (l & 1)) ? T(0.5) : T(1);
    const int pl = gc.nx * gc.ny;
    for (int r = blockIdx.y; r < k; r += gridDim.y) {
        const T* e = Ec + r * ldc;
        T acc = T(0);
        for (int a = 0; a < nl; ++a)
            for (int b = 0; b < nj; ++b)
                for (int c = 0; c < ni; ++c)
                    acc += (wl * wj * wi) * e[(cl + a) * pl + (cj + b) * gc.nx + (ci + c)];
        X[r * ldx + p] += acc;
    }
}

// X_r = Cinv F_r on the coarsest level. Cinv is the symmetric dense inverse
// (row-major Nc x Nc), so Cinv[j][i] = Cinv[i][j]: lane i of a wave reads
// Cinv[j*Nc + i], coalesced across the wave. Block = 64 rows x 4 waves, each
// wave summing a quarter of j; F_r is staged in LDS.
constexpr int kCoarseMax = 4096;
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_solve(int Nc, const T* __restrict__ Cinv,
                                                         int k, const T* __restrict__ F,
                                                         int64_t ldf, T* __restrict__ X,
                                                         int64_t ldx) {
    __shared__ T sf[kCoarseMax];
    __shared__ T part[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int q = (Nc + 3) / 4;
    const int j0 = wv * q, j1 = min(Nc, j0 + q);
    for (int r = blockIdx.y; r < k; r += gridDim.y) {
        __syncthreads();
        for (int j = threadIdx.x; j < Nc; j += kBlock) sf[j] = F[r * ldf + j];
        __syncthreads();
        T acc = T(0);
        if (i < Nc)
            for (int j = j0; j < j1; ++j) acc += Cinv[(int64_t)j * Nc + i] * sf[j];
        part[wv][lane] = acc;
        __syncthreads();
        if (wv == 0 && i < Nc) X[r * ldx + i] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    }
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_convert(int64_t N, int k, const TI* __restrict__ X,
                                                    int64_t ldx, TO* __restrict__ Y,
                                                    int64_t ldy, TI scale) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= N) return;
    for (int r = blockIdx.y; r < k; r += gridDim.y) Y[r * ldy + p] = TO(scale * X[r * ldx + p]);
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_apply_plus_dot(Geom g, double a,
                                                           const double* __restrict__ P,
                                                           const double* __restrict__ Tv,
                                                           double* __restrict__ Q,
                                                           double* __restrict__ partial) {
    __shared__ double sh[kBlock / 64];
    const int p = blockIdx.x * kBlock + threadIdx.x;
    double pq = 0.0;
    if (p < g.N) {
        int i, j, l;
        decompose(g, p, i, j, l);
        const auto c = node_coef<double, DIM>(g, i, j, l);
        const double q = a * apply_at<double, DIM>(g, P, p, c) + Tv[p];
        Q[p] = q;
        pq = P[p] * q;
    }
    const double s = block_sum<kBlock>(pq, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

dim3 grid_for(int64_t N, int k) { return dim3((unsigned)cdiv(N, kBlock), (unsigned)std::min(k, 65535)); }

}  // namespace

#define H1W_DIMCALL(KERNEL, T, grid, ...)                                               \
    do {                                                                                \
        if (dim == 3)                                                                   \
            hipLaunchKernelGGL((KERNEL<T, 3>), grid, dim3(kBlock), 0, s, __VA_ARGS__);  \
        else                                                                            \
            hipLaunchKernelGGL((KERNEL<T, 2>), grid, dim3(kBlock), 0, s, __VA_ARGS__);  \
        H1W_LAUNCHED();                                                                 \
    } while (0)

template <typename T>
void launch_apply(hipStream_t s, int dim, const Geom& g, int k, const T* X, int64_t ldx, T* Y,
                  int64_t ldy, double scale) {
    if (k <= 0) return;
    H1W_DIMCALL(k_apply, T, grid_for(g.N, k), g, k, X, ldx, Y, ldy, T(scale));
}

template <typename T>
void launch_smooth_first(hipStream_t s, int dim, const Geom& g, int k, const T* F, int64_t ldf,
                         T* X, int64_t ldx, double w) {
    if (k <= 0) return;
    H1W_DIMCALL(k_smooth_first, T, grid_for(g.N, k), g, k, F, ldf, X, ldx, T(w));
}

template <typename T>
void launch_smooth(hipStream_t s, int dim, const Geom& g, int k, const T* F, int64_t ldf,
                   const T* Xin, int64_t ldi, T* Xout, int64_t ldo, double w) {
    if (k <= 0) return;
    H1W_DIMCALL(k_smooth, T, grid_for(g.N, k), g, k, F, ldf, Xin, ldi, Xout, ldo, T(w));
}

template <typename T>
void launch_residual(hipStream_t s, int dim, const Geom& g, int k, const T* F, int64_t ldf,
                     const T* X, int64_t ldx, T* R, int64_t ldr) {
    if (k <= 0) return;
    H1W_DIMCALL(k_residual, T, grid_for(g.N, k), g, k, F, ldf, X, ldx, R, ldr);
}

template <typename T>
void launch_restrict(hipStream_t s, int dim, const Geom& gf, const Geom& gc, int k, const T* R,
                     int64_t ldr, T* Fc, int64_t ldc) {
    if (k <= 0) return;
    H1W_DIMCALL(k_restrict, T, grid_for(gc.N, k), gf, gc, k, R, ldr, Fc, ldc);
}

template <typename T>
void launch_prolong_add(hipStream_t s, int dim, const Geom& gf, const Geom& gc, int k,
                        const T* Ec, int64_t ldc, T* X, int64_t ldx) {
    if (k <= 0) return;
    H1W_DIMCALL(k_prolong_add, T, grid_for(gf.N, k), gf, gc, k, Ec, ldc, X, ldx);
}

template <typename T>
void launch_coarse_solve(hipStream_t s, int64_t Nc, const T* Cinv, int k, const T* F,
                         int64_t ldf, T* X, int64_t ldx) {
    if (k <= 0) return;
    if (Nc > kCoarseMax) throw Error{H1W_EINVAL, "coarsest level too large"};
    const dim3 grid((unsigned)cdiv(Nc, 64), (unsigned)std::min(k, 65535));
    hipLaunchKernelGGL((k_coarse_solve<T>), grid, dim3(kBlock), 0, s, (int)Nc, Cinv, k, F, ldf, X, ldx);
    H1W_LAUNCHED();
}

template <typename TI, typename TO>
void launch_convert(hipStream_t s, int64_t N, int k, const TI* X, int64_t ldx, TO* Y,
                    int64_t ldy, double scale) {
    if (k <= 0) return;
    hipLaunchKernelGGL((k_convert<TI, TO>), grid_for(N, k), dim3(kBlock), 0, s, N, k, X, ldx, Y,
                       ldy, TI(scale));
    H1W_LAUNCHED();
}

void launch_apply_plus_dot(hipStream_t s, int dim, const Geom& g, double a, const double* P,
                           const double* Tv, double* Q, double* partial, int* nparts) {
    const dim3 grid((unsigned)cdiv(g.N, kBlock));
    if (dim == 3)
        hipLaunchKernelGGL((k_apply_plus_dot<3>), grid, dim3(kBlock), 0, s, g, a, P, Tv, Q, partial);
    else
        hipLaunchKernelGGL((k_apply_plus_dot<2>), grid, dim3(kBlock), 0, s, g, a, P, Tv, Q, partial);
    H1W_LAUNCHED();
    *nparts = (int)grid.x;
}

#define H1W_INST(T)                                                                              \
    template void launch_apply<T>(hipStream_t, int, const Geom&, int, const T*, int64_t, T*,     \
                                  int64_t, double);                                              \
    template void launch_smooth_first<T>(hipStream_t, int, const Geom&, int, const T*, int64_t,  \
                                         T*, int64_t, double);                                   \
    template void launch_smooth<T>(hipStream_t, int, const Geom&, int, const T*, int64_t,        \
                                   const T*, int64_t, T*, int64_t, double);                      \
    template void launch_residual<T>(hipStream_t, int, const Geom&, int, const T*, int64_t,      \
                                     const T*, int64_t, T*, int64_t);                            \
    template void launch_restrict<T>(hipStream_t, int, const Geom&, const Geom&, int, const T*,  \
                                     int64_t, T*, int64_t);                                      \
    template void launch_prolong_add<T>(hipStream_t, int, const Geom&, const Geom&, int,         \
                                        const T*, int64_t, T*, int64_t);                         \
    template void launch_coarse_solve<T>(hipStream_t, int64_t, const T*, int, const T*, int64_t, \
                                         T*, int64_t);
H1W_INST(double)
H1W_INST(float)
template void launch_convert<double, float>(hipStream_t, int64_t, int, const double*, int64_t,
                                            float*, int64_t, double);
template void launch_convert<float, double>(hipStream_t, int64_t, int, const float*, int64_t,
                                            double*, int64_t, double);
template void launch_convert<double, double>(hipStream_t, int64_t, int, const double*, int64_t,
                                             double*, int64_t, double);

}  // namespace h1w
