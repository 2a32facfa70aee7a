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
#include <algorithm>

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

// ---------------------------------------------------------------- launch shape
// Work item = (plane tile of kBlock consecutive in-plane indices q = j*nx + i,
// run of zc consecutive z-planes, batch row r), tile index fastest. Each
// thread owns one q and marches up its z-run, keeping the z-neighbours in
// registers. Work-group ids are dealt round-robin to the 8 XCDs, so item w is
// given to XCD w / per (contiguous ranges): work-groups that touch the same
// planes share one L2.
struct Sweep {
    int PL;     // nodes per z-plane
    int nqt;    // plane tiles
    int zc;     // planes per run
    int nzc;    // runs
    int k;      // batch rows
    int total;  // work items
};

Sweep make_sweep(const Geom& g, int k, int target_items = 4096) {
    Sweep s;
    s.PL = g.nx * g.ny;
    s.nqt = (int)cdiv(s.PL, kBlock);
    s.k = k;
    const int64_t base = (int64_t)s.nqt * k;
    int nzc = (int)std::clamp<int64_t>(cdiv(target_items, base), 1, g.nz);
    s.zc = (int)cdiv(g.nz, nzc);
    s.nzc = (int)cdiv(g.nz, s.zc);
    s.total = (int)((int64_t)s.nqt * s.nzc * k);
    return s;
}

unsigned sweep_grid(const Sweep& s) { return 8u * (unsigned)cdiv(s.total, 8); }

__device__ __forceinline__ bool sweep_item(const Sweep& s, int& q, int& z0, int& z1, int& r, int nz) {
    const int bid = blockIdx.x;
    const int per = (s.total + 7) >> 3;
    const int w = (bid & 7) * per + (bid >> 3);
    if (w >= s.total) return false;
    const int qt = w % s.nqt;
    const int t = w / s.nqt;
    const int zi = t % s.nzc;
    r = t / s.nzc;
    q = qt * kBlock + threadIdx.x;
    z0 = zi * s.zc;
    z1 = min(nz, z0 + s.zc);
    return q < s.PL;
}

// In-plane part of the stencil at (i, j) and the z-dependent part at plane l.
template <typename T, int DIM>
struct Column {
    T wx, wy;
    bool xm, xp, ym, yp;
    __device__ Column(const Geom& g, int i, int j) {
        wx = (i == 0 || i == g.nx - 1) ? T(0.5) : T(1);
        wy = (j == 0 || j == g.ny - 1) ? T(0.5) : T(1);
        xm = i > 0; xp = i < g.nx - 1;
        ym = j > 0; yp = j < g.ny - 1;
    }
    // A x at node p of plane l; xb/xc/xa = x at planes l-1, l, l+1
    __device__ __forceinline__ T apply(const Geom& g, const T* __restrict__ x, int64_t p, int l, T xb, T xc,
                                       T xa, T& diag) const {
        const bool zm = DIM == 3 && l > 0, zp = DIM == 3 && l < g.nz - 1;
        const T wz = (DIM == 3 && (l == 0 || l == g.nz - 1)) ? T(0.5) : T(1);
        const T cx = T(g.ihx2) * wy * wz, cy = T(g.ihy2) * wx * wz;
        const T cz = DIM == 3 ? T(g.ihz2) * wx * wy : T(0);
        const T mass = T(g.beta) * wx * wy * wz;
        diag = mass + cx * T(int(xm) + int(xp)) + cy * T(int(ym) + int(yp)) + cz * T(int(zm) + int(zp));
        T sx = T(0), sy = T(0), sz = T(0);
        if (xm) sx += xc - x[p - 1];
        if (xp) sx += xc - x[p + 1];
        if (ym) sy += xc - x[p - g.nx];
        if (yp) sy += xc - x[p + g.nx];
        if (zm) sz += xc - xb;
        if (zp) sz += xc - xa;
        T acc = mass * xc;
        acc += cx * sx;
        acc += cy * sy;
        if (DIM == 3) acc += cz * sz;
        return acc;
    }
    __device__ __forceinline__ T diag_at(const Geom& g, int l) const {
        const bool zm = DIM == 3 && l > 0, zp = DIM == 3 && l < g.nz - 1;
        const T wz = (DIM == 3 && (l == 0 || l == g.nz - 1)) ? T(0.5) : T(1);
        const T cx = T(g.ihx2) * wy * wz, cy = T(g.ihy2) * wx * wz;
        const T cz = DIM == 3 ? T(g.ihz2) * wx * wy : T(0);
        return T(g.beta) * wx * wy * wz + cx * T(int(xm) + int(xp)) + cy * T(int(ym) + int(yp)) +
               cz * T(int(zm) + int(zp));
    }
};

// MODE 0: Y = scale * A X          (F unused)
// MODE 1: Y = F - A X              (residual)
// MODE 2: Y = X + w D^-1 (F - A X) (smoothing step; scale = w)
// The march is unrolled by kU planes: all loads of kU planes (z-neighbour,
// in-plane neighbours, right-hand side) are issued before the arithmetic, so
// each thread keeps several independent HBM requests in flight.
constexpr int kU = 4;
template <typename T, int DIM, int MODE>
__global__ __launch_bounds__(kBlock) void k_march(Geom g, Sweep s, const T* __restrict__ F, int64_t ldf,
                                                  const T* __restrict__ X, int64_t ldx, T* __restrict__ Y,
                                                  int64_t ldy, T scale) {
    int q, z0, z1, r;
    if (!sweep_item(s, q, z0, z1, r, g.nz)) return;
    const Column<T, DIM> col(g, q % g.nx, q / g.nx);
    const T* x = X + r * ldx;
    const T* f = F + r * ldf;
    T* y = Y + r * ldy;
    const int64_t PL = s.PL;
    const int nx = g.nx;
    T xb = (DIM == 3 && z0 > 0) ? x[(z0 - 1) * PL + q] : T(0);
    T xc = x[z0 * PL + q];
    for (int l0 = z0; l0 < z1; l0 += kU) {
        T xa[kU], fv[kU], nxm[kU], nxp[kU], nym[kU], nyp[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int l = l0 + u;
            const int64_t p = l * PL + q;
            const bool in = l < z1;
            xa[u] = (in && DIM == 3 && l + 1 < g.nz) ? x[p + PL] : T(0);
            fv[u] = (in && MODE != 0) ? f[p] : T(0);
            nxm[u] = (in && col.xm) ? x[p - 1] : T(0);
            nxp[u] = (in && col.xp) ? x[p + 1] : T(0);
            nym[u] = (in && col.ym) ? x[p - nx] : T(0);
            nyp[u] = (in && col.yp) ? x[p + nx] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int l = l0 + u;
            if (l >= z1) break;
            const int64_t p = l * PL + q;
            const bool zm = DIM == 3 && l > 0, zp = DIM == 3 && l < g.nz - 1;
            const T wz = (DIM == 3 && (l == 0 || l == g.nz - 1)) ? T(0.5) : T(1);
            const T cx = T(g.ihx2) * col.wy * wz, cy = T(g.ihy2) * col.wx * wz;
            const T cz = DIM == 3 ? T(g.ihz2) * col.wx * col.wy : T(0);
            const T mass = T(g.beta) * col.wx * col.wy * wz;
            T sx = T(0), sy = T(0), sz = T(0);
            if (col.xm) sx += xc - nxm[u];
            if (col.xp) sx += xc - nxp[u];
            if (col.ym) sy += xc - nym[u];
            if (col.yp) sy += xc - nyp[u];
            if (zm) sz += xc - xb;
            if (zp) sz += xc - xa[u];
            T acc = mass * xc;
            acc += cx * sx;
            acc += cy * sy;
            if (DIM == 3) acc += cz * sz;
            if (MODE == 0) y[p] = scale * acc;
            if (MODE == 1) y[p] = fv[u] - acc;
            if (MODE == 2) {
                const T diag = mass + cx * T(int(col.xm) + int(col.xp)) + cy * T(int(col.ym) + int(col.yp)) +
                               cz * T(int(zm) + int(zp));
                y[p] = xc + scale * (fv[u] - acc) / diag;
            }
            xb = xc;
            xc = xa[u];
        }
    }
}

// Diagonal of A at node (i, j, l) from its position alone.
template <typename T, int DIM>
__device__ __forceinline__ T diag_node(const Geom& g, int i, int j, int l) {
    const T wx = (i == 0 || i == g.nx - 1) ? T(0.5) : T(1);
    const T wy = (j == 0 || j == g.ny - 1) ? T(0.5) : T(1);
    const T wz = (DIM == 3 && (l == 0 || l == g.nz - 1)) ? T(0.5) : T(1);
    const int dx = int(i > 0) + int(i < g.nx - 1), dy = int(j > 0) + int(j < g.ny - 1);
    const int dz = DIM == 3 ? int(l > 0) + int(l < g.nz - 1) : 0;
    T d = T(g.beta) * wx * wy * wz + T(g.ihx2) * wy * wz * T(dx) + T(g.ihy2) * wx * wz * T(dy);
    if (DIM == 3) d += T(g.ihz2) * wx * wy * T(dz);
    return d;
}

// The first two smoothing steps from a zero initial guess in one pass:
//   x1 = w0 D^-1 f  (pointwise), x2 = x1 + w1 D^-1 (f - A x1).
// x1 at the stencil neighbours is rebuilt from f and the neighbours'
// diagonals, so only f is read and only x2 is written.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_pre2(Geom g, Sweep s, const T* __restrict__ F, int64_t ldf,
                                                 T* __restrict__ Y, int64_t ldy, T w0, T w1) {
    int q, z0, z1, r;
    if (!sweep_item(s, q, z0, z1, r, g.nz)) return;
    const int i = q % g.nx, j = q / g.nx;
    const Column<T, DIM> col(g, i, j);
    const T* f = F + r * ldf;
    T* y = Y + r * ldy;
    const int64_t PL = s.PL;
    const int nx = g.nx;
    // x1 below / at the current plane (carried along the march)
    T x1b = (DIM == 3 && z0 > 0) ? w0 * f[(z0 - 1) * PL + q] / diag_node<T, DIM>(g, i, j, z0 - 1) : T(0);
    T fc = f[z0 * PL + q];
    T x1c = w0 * fc / diag_node<T, DIM>(g, i, j, z0);
    for (int l0 = z0; l0 < z1; l0 += kU) {
        T fa[kU], nxm[kU], nxp[kU], nym[kU], nyp[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int l = l0 + u;
            const int64_t p = l * PL + q;
            const bool in = l < z1;
            fa[u] = (in && DIM == 3 && l + 1 < g.nz) ? f[p + PL] : T(0);
            nxm[u] = (in && col.xm) ? f[p - 1] : T(0);
            nxp[u] = (in && col.xp) ? f[p + 1] : T(0);
            nym[u] = (in && col.ym) ? f[p - nx] : T(0);
            nyp[u] = (in && col.yp) ? f[p + nx] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int l = l0 + u;
            if (l >= z1) break;
            const int64_t p = l * PL + q;
            const bool zm = DIM == 3 && l > 0, zp = DIM == 3 && l < g.nz - 1;
            const T wz = (DIM == 3 && (l == 0 || l == g.nz - 1)) ? T(0.5) : T(1);
            const T cx = T(g.ihx2) * col.wy * wz, cy = T(g.ihy2) * col.wx * wz;
            const T cz = DIM == 3 ? T(g.ihz2) * col.wx * col.wy : T(0);
            const T mass = T(g.beta) * col.wx * col.wy * wz;
            const T diag = mass + cx * T(int(col.xm) + int(col.xp)) + cy * T(int(col.ym) + int(col.yp)) +
                           cz * T(int(zm) + int(zp));
            const T x1a = zp ? w0 * fa[u] / diag_node<T, DIM>(g, i, j, l + 1) : T(0);
            T sx = T(0), sy = T(0), sz = T(0);
            if (col.xm) sx += x1c - w0 * nxm[u] / diag_node<T, DIM>(g, i - 1, j, l);
            if (col.xp) sx += x1c - w0 * nxp[u] / diag_node<T, DIM>(g, i + 1, j, l);
            if (col.ym) sy += x1c - w0 * nym[u] / diag_node<T, DIM>(g, i, j - 1, l);
            if (col.yp) sy += x1c - w0 * nyp[u] / diag_node<T, DIM>(g, i, j + 1, l);
            if (zm) sz += x1c - x1b;
            if (zp) sz += x1c - x1a;
            T acc = mass * x1c;
            acc += cx * sx;
            acc += cy * sy;
            if (DIM == 3) acc += cz * sz;
            y[p] = x1c + w1 * (fc - acc) / diag;
            x1b = x1c;
            x1c = x1a;
            fc = fa[u];
        }
    }
}

// X = w D^-1 F (first smoothing step from a zero initial guess)
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_smooth_first(Geom g, Sweep s, const T* __restrict__ F, int64_t ldf,
                                                         T* __restrict__ X, int64_t ldx, T w) {
    int q, z0, z1, r;
    if (!sweep_item(s, q, z0, z1, r, g.nz)) return;
    const Column<T, DIM> col(g, q % g.nx, q / g.nx);
    const T* f = F + r * ldf;
    T* x = X + r * ldx;
    for (int l = z0; l < z1; ++l) {
        const int64_t p = (int64_t)l * s.PL + q;
        x[p] = w * f[p] / col.diag_at(g, l);
    }
}

// Fc = 2^-d P^T R. One thread per coarse (I, J), marching over coarse planes L:
// fine plane z contributes the in-plane weighted sum
//   s(z) = sum_{dy,dx in {-1,0,1}} w(dy) w(dx) R[z][2J+dy][2I+dx],  w(0)=1, w(+-1)=1/2,
// and Fc[L] = 2^-d (s(2L-1)/2 + s(2L) + s(2L+1)/2); s(2L+1) is reused for L+1.
template <typename T, int DIM>
__device__ __forceinline__ T plane_sum(const Geom& gf, const T* __restrict__ rz, int fi, int fj) {
    T acc = T(0);
    for (int dy = -1; dy <= 1; ++dy) {
        const int y = fj + dy;
        if (y < 0 || y >= gf.ny) continue;
        const T wy = dy ? T(0.5) : T(1);
        T row = T(0);
        for (int dx = -1; dx <= 1; ++dx) {
            const int x = fi + dx;
            if (x < 0 || x >= gf.nx) continue;
            const T wx = dx ? T(0.5) : T(1);
            row += wx * rz[y * gf.nx + x];
        }
        acc += wy * row;
    }
    return acc;
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_restrict(Geom gf, Geom gc, Sweep s, const T* __restrict__ R,
                                                     int64_t ldr, T* __restrict__ Fc, int64_t ldc) {
    int q, z0, z1, r;
    if (!sweep_item(s, q, z0, z1, r, gc.nz)) return;
    const int I = q % gc.nx, J = q / gc.nx;
    const T* rr = R + r * ldr;
    T* fc = Fc + r * ldc;
    const int64_t PLf = (int64_t)gf.nx * gf.ny;
    const T scale = DIM == 3 ? T(0.125) : T(0.25);
    if (DIM == 2) {
        fc[q] = scale * plane_sum<T, DIM>(gf, rr, 2 * I, 2 * J);
        return;
    }
    T sb = (2 * z0 - 1 >= 0) ? plane_sum<T, DIM>(gf, rr + (2 * z0 - 1) * PLf, 2 * I, 2 * J) : T(0);
    for (int L = z0; L < z1; ++L) {
        const int z = 2 * L;
        const T sc = plane_sum<T, DIM>(gf, rr + z * PLf, 2 * I, 2 * J);
        const T sa = (z + 1 < gf.nz) ? plane_sum<T, DIM>(gf, rr + (z + 1) * PLf, 2 * I, 2 * J) : T(0);
        fc[(int64_t)L * s.PL + q] = scale * (T(0.5) * sb + sc + T(0.5) * sa);
        sb = sa;
    }
}

// X += P Ec: fine node (i,j,l) interpolates from the coarse nodes floor(i/2)
// and, for odd i, floor(i/2)+1 (weights 1/2), per axis.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_prolong_add(Geom gf, Geom gc, Sweep s, const T* __restrict__ Ec,
                                                        int64_t ldc, T* __restrict__ X, int64_t ldx) {
    int q, z0, z1, r;
    if (!sweep_item(s, q, z0, z1, r, gf.nz)) return;
    const int i = q % gf.nx, j = q / gf.nx;
    const int ci = i >> 1, cj = j >> 1;
    const int ni = 1 + (i & 1), nj = 1 + (j & 1);
    const T wi = (i & 1) ? T(0.5) : T(1), wj = (j & 1) ? T(0.5) : T(1);
    const int64_t PLc = (int64_t)gc.nx * gc.ny;
    const T* e = Ec + r * ldc;
    T* x = X + r * ldx;
    for (int l = z0; l < z1; ++l) {
        const int cl = l >> 1;
        const int nl = DIM == 3 ? 1 + (l & 1) : 1;
        const T wl = (DIM == 3 && (l & 1)) ? T(0.5) : T(1);
        T acc = T(0);
        for (int a = 0; a < nl; ++a)
            for (int b = 0; b < nj; ++b)
                for (int c = 0; c < ni; ++c)
                    acc += (wl * wj * wi) * e[(cl + a) * PLc + (cj + b) * gc.nx + (ci + c)];
        x[(int64_t)l * s.PL + q] += acc;
    }
}

// X_r = Cinv F_r on the coarsest level. Cinv is the symmetric dense inverse
// (row-major Nc x Nc), so Cinv[j][i] = Cinv[i][j]: lane i of a wave reads
// Cinv[j*Nc + i], coalesced across the wave. Work-group = 64 outputs i x
// (its share of j, split over 4 waves) x (every gridDim.z-th right-hand
// side). With few right-hand sides the j range is also split over
// gridDim.y work-groups whose partial sums go to part[split][r][i] and are
// added in a fixed order by k_coarse_reduce; with one split the sum is
// written to X directly.
constexpr int kCoarseMax = 4096;
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_solve(int Nc, const T* __restrict__ Cinv, int k,
                                                         const T* __restrict__ F, int64_t ldf, T* __restrict__ X,
                                                         int64_t ldx, T* __restrict__ part) {
    __shared__ T sf[kCoarseMax];
    __shared__ T red[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int splits = gridDim.y;
    const int js = (Nc + splits - 1) / splits;
    const int ja = blockIdx.y * js, jb = min(Nc, ja + js);
    const int q = (jb - ja + 3) / 4;
    const int j0 = ja + wv * q, j1 = min(jb, j0 + q);
    const int ic = min(i, Nc - 1);
    for (int r = blockIdx.z; r < k; r += gridDim.z) {
        __syncthreads();
        for (int j = ja + (int)threadIdx.x; j < jb; j += kBlock) sf[j] = F[r * ldf + j];
        __syncthreads();
        T acc = T(0);
#pragma unroll 8
        for (int j = j0; j < j1; ++j) acc += Cinv[(int64_t)j * Nc + ic] * sf[j];
        red[wv][lane] = acc;
        __syncthreads();
        if (wv == 0 && i < Nc) {
            const T v = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
            if (splits == 1)
                X[r * ldx + i] = v;
            else
                part[((int64_t)blockIdx.y * k + r) * Nc + i] = v;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_reduce(int Nc, int k, int splits, const T* __restrict__ part,
                                                          T* __restrict__ X, int64_t ldx) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)k * Nc) return;
    const int r = (int)(t / Nc), i = (int)(t % Nc);
    T acc = T(0);
    for (int s = 0; s < splits; ++s) acc += part[((int64_t)s * k + r) * Nc + i];
    X[r * ldx + i] = acc;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_convert(int64_t N, int k, const TI* __restrict__ X,
                                                    int64_t ldx, TO* __restrict__ Y,
                                                    int64_t ldy, TI scale) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= N) return;
    for (int r = blockIdx.y; r < k; r += gridDim.y) Y[r * ldy + p] = TO(scale * X[r * ldx + p]);
}

// W 1: trapezoid node weights wx wy wz (the lumped mass diagonal without beta)
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_node_weights(Geom g, double* __restrict__ out) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= g.N) return;
    int i, j, l;
    decompose(g, p, i, j, l);
    const double wx = (i == 0 || i == g.nx - 1) ? 0.5 : 1.0, wy = (j == 0 || j == g.ny - 1) ? 0.5 : 1.0;
    const double wz = (DIM == 3 && (l == 0 || l == g.nz - 1)) ? 0.5 : 1.0;
    out[p] = wx * wy * wz;
}

// Y_r = float(X_r - s_r W 1): FP32 right-hand sides with the constant mode removed
__global__ __launch_bounds__(kBlock) void k_convert_deflate(int64_t N, int k, const double* __restrict__ X, int64_t ldx,
                                                            const double* __restrict__ sv, const double* __restrict__ wv,
                                                            float* __restrict__ Y, int64_t ldy) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= N) return;
    const double w = wv[p];
    for (int r = blockIdx.y; r < k; r += gridDim.y) Y[r * ldy + p] = float(X[r * ldx + p] - sv[r] * w);
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

#define H1W_MARCH(MODE, T, ...)                                                                        \
    do {                                                                                               \
        const Sweep sw = make_sweep(g, k);                                                             \
        if (dim == 3)                                                                                  \
            hipLaunchKernelGGL((k_march<T, 3, MODE>), dim3(sweep_grid(sw)), dim3(kBlock), 0, s, g, sw, \
                               __VA_ARGS__);                                                           \
        else                                                                                           \
            hipLaunchKernelGGL((k_march<T, 2, MODE>), dim3(sweep_grid(sw)), dim3(kBlock), 0, s, g, sw, \
                               __VA_ARGS__);                                                           \
        H1W_LAUNCHED();                                                                                \
    } while (0)

template <typename T>
void launch_apply(hipStream_t s, int dim, const Geom& g, int k, const T* X, int64_t ldx, T* Y,
                  int64_t ldy, double scale) {
    if (k <= 0) return;
    H1W_MARCH(0, T, (const T*)nullptr, (int64_t)0, X, ldx, Y, ldy, T(scale));
}

template <typename T>
void launch_smooth_first(hipStream_t s, int dim, const Geom& g, int k, const T* F, int64_t ldf,
                         T* X, int64_t ldx, double w) {
    if (k <= 0) return;
    const Sweep sw = make_sweep(g, k);
    H1W_DIMCALL(k_smooth_first, T, dim3(sweep_grid(sw)), g, sw, F, ldf, X, ldx, T(w));
}

template <typename T>
void launch_pre2(hipStream_t s, int dim, const Geom& g, int k, const T* F, int64_t ldf, T* X, int64_t ldx,
                 double w0, double w1) {
    if (k <= 0) return;
    const Sweep sw = make_sweep(g, k);
    H1W_DIMCALL(k_pre2, T, dim3(sweep_grid(sw)), g, sw, F, ldf, X, ldx, T(w0), T(w1));
}

template <typename T>
void launch_smooth(hipStream_t s, int dim, const Geom& g, int k, const T* F, int64_t ldf,
                   const T* Xin, int64_t ldi, T* Xout, int64_t ldo, double w) {
    if (k <= 0) return;
    H1W_MARCH(2, T, F, ldf, Xin, ldi, Xout, ldo, T(w));
}

template <typename T>
void launch_residual(hipStream_t s, int dim, const Geom& g, int k, const T* F, int64_t ldf,
                     const T* X, int64_t ldx, T* R, int64_t ldr) {
    if (k <= 0) return;
    H1W_MARCH(1, T, F, ldf, X, ldx, R, ldr, T(1));
}

template <typename T>
void launch_restrict(hipStream_t s, int dim, const Geom& gf, const Geom& gc, int k, const T* R,
                     int64_t ldr, T* Fc, int64_t ldc) {
    if (k <= 0) return;
    const Sweep sw = make_sweep(gc, k);
    H1W_DIMCALL(k_restrict, T, dim3(sweep_grid(sw)), gf, gc, sw, R, ldr, Fc, ldc);
}

template <typename T>
void launch_prolong_add(hipStream_t s, int dim, const Geom& gf, const Geom& gc, int k,
                        const T* Ec, int64_t ldc, T* X, int64_t ldx) {
    if (k <= 0) return;
    const Sweep sw = make_sweep(gf, k);
    H1W_DIMCALL(k_prolong_add, T, dim3(sweep_grid(sw)), gf, gc, sw, Ec, ldc, X, ldx);
}

// Splits of the j range: enough work-groups to spread the read of Cinv over
// the chip when there are few right-hand sides, within the partial buffer.
int coarse_splits(int64_t Nc, int k, size_t part_elems) {
    const int64_t iblocks = cdiv(Nc, 64);
    int64_t sp = std::clamp<int64_t>(512 / std::max<int64_t>(1, iblocks * k), 1, cdiv(Nc, 32));
    while (sp > 1 && (size_t)(sp * k * Nc) > part_elems) --sp;
    return (int)sp;
}

size_t coarse_part_elems(int64_t Nc) {
    // the largest split count times k * Nc over k >= 1 (splits > 1 needs iblocks * k < 512)
    size_t best = 0;
    for (int k = 1; k <= 512; ++k) {
        const int64_t iblocks = cdiv(Nc, 64);
        const int64_t sp = std::clamp<int64_t>(512 / std::max<int64_t>(1, iblocks * k), 1, cdiv(Nc, 32));
        if (sp > 1) best = std::max(best, (size_t)(sp * k * Nc));
    }
    return best;
}

template <typename T>
void launch_coarse_solve(hipStream_t s, int64_t Nc, const T* Cinv, int k, const T* F, int64_t ldf, T* X,
                         int64_t ldx, T* part, size_t part_elems) {
    if (k <= 0) return;
    if (Nc > kCoarseMax) throw Error{H1W_EINVAL, "coarsest level too large"};
    const int splits = part ? coarse_splits(Nc, k, part_elems) : 1;
    const dim3 grid((unsigned)cdiv(Nc, 64), (unsigned)splits, (unsigned)std::min(k, 65535));
    hipLaunchKernelGGL((k_coarse_solve<T>), grid, dim3(kBlock), 0, s, (int)Nc, Cinv, k, F, ldf, X, ldx, part);
    H1W_LAUNCHED();
    if (splits > 1) {
        hipLaunchKernelGGL((k_coarse_reduce<T>), dim3((unsigned)cdiv((int64_t)k * Nc, kBlock)), dim3(kBlock), 0, s,
                           (int)Nc, k, splits, (const T*)part, X, ldx);
        H1W_LAUNCHED();
    }
}

template <typename TI, typename TO>
void launch_convert(hipStream_t s, int64_t N, int k, const TI* X, int64_t ldx, TO* Y,
                    int64_t ldy, double scale) {
    if (k <= 0) return;
    hipLaunchKernelGGL((k_convert<TI, TO>), grid_for(N, k), dim3(kBlock), 0, s, N, k, X, ldx, Y,
                       ldy, TI(scale));
    H1W_LAUNCHED();
}

void launch_node_weights(hipStream_t s, int dim, const Geom& g, double* out) {
    const dim3 grid((unsigned)cdiv(g.N, kBlock));
    if (dim == 3)
        hipLaunchKernelGGL((k_node_weights<3>), grid, dim3(kBlock), 0, s, g, out);
    else
        hipLaunchKernelGGL((k_node_weights<2>), grid, dim3(kBlock), 0, s, g, out);
    H1W_LAUNCHED();
}

void launch_convert_deflate(hipStream_t s, int64_t N, int k, const double* X, int64_t ldx, const double* sv,
                            const double* wv, float* Y, int64_t ldy) {
    if (k <= 0) return;
    // one thread per node walks the k rows: the weight w(p) is read once, not once per row
    hipLaunchKernelGGL(k_convert_deflate, dim3((unsigned)cdiv(N, kBlock), 1), dim3(kBlock), 0, s, N, k, X, ldx, sv,
                       wv, Y, ldy);
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
    template void launch_pre2<T>(hipStream_t, int, const Geom&, int, const T*, int64_t, T*, int64_t,  \
                                 double, double);                                                 \
    template void launch_smooth<T>(hipStream_t, int, const Geom&, int, const T*, int64_t,        \
                                   const T*, int64_t, T*, int64_t, double);                      \
    template void launch_residual<T>(hipStream_t, int, const Geom&, int, const T*, int64_t,      \
                                     const T*, int64_t, T*, int64_t);                            \
    template void launch_restrict<T>(hipStream_t, int, const Geom&, const Geom&, int, const T*,  \
                                     int64_t, T*, int64_t);                                      \
    template void launch_prolong_add<T>(hipStream_t, int, const Geom&, const Geom&, int,         \
                                        const T*, int64_t, T*, int64_t);                         \
    template void launch_coarse_solve<T>(hipStream_t, int64_t, const T*, int, const T*, int64_t, \
                                         T*, int64_t, T*, size_t);
H1W_INST(double)
H1W_INST(float)
template void launch_convert<double, float>(hipStream_t, int64_t, int, const double*, int64_t,
                                            float*, int64_t, double);
template void launch_convert<float, double>(hipStream_t, int64_t, int, const float*, int64_t,
                                            double*, int64_t, double);
template void launch_convert<double, double>(hipStream_t, int64_t, int, const double*, int64_t,
                                             double*, int64_t, double);

}  // namespace h1w
