// Fused passes of the 3D V-cycle with two smoothing steps on each side
// (the multigrid preconditioner B of Section 3: Chebyshev-Jacobi smoothing,
// full-weighting restriction, multilinear interpolation). The cycle is the
// one the unfused stencil kernels run step by step; only the passes over
// memory differ.
//
// down (one level, zero initial guess):
//     x1 = w0 D^-1 f,  x2 = x1 + w1 D^-1 (f - A x1)     pre-smoothing
//     r  = f - A x2,   fc = 2^-3 P^T r                  residual, restriction
//   reads f, writes x2 and the coarse right-hand side fc.
// up (one level):
//     y0 = x2 + P e,  y1 = y0 + w1 D^-1 (f - A y0),  y = y1 + w0 D^-1 (f - A y1)
//   reads x2, f and the coarse correction e, writes y.
// Fine-level HBM traffic per node: 2 words (down) + 3 words (up), against
// 14 for the unfused sequence.
//
// Work item = (in-plane tile, z-run, batch row); work-group ids are dealt to
// the 8 XCDs in contiguous ranges of items. A work-group owns a region of at
// most kReg in-plane columns: its tile plus a halo ring wide enough that
// every stage is computed from the group's own data (halo columns are
// recomputed by neighbouring tiles; their loads hit L2). Each of the 256
// threads owns kCPT columns and marches up z, stage s of the pipeline
// working on plane n - s at step n. Z-neighbours stay in registers; in-plane
// neighbours come from LDS planes that were written in step n - 1 (double
// buffered), so a single barrier per step orders every read after its write
// and every overwrite after its last read.
#include <algorithm>

#include "devutil.h"
#include "internal.h"

namespace h1w {

namespace {

constexpr int kFT = 256;           // threads per work-group
constexpr int kCPT = 2;            // region columns per thread
constexpr int kReg = kFT * kCPT;   // region columns per work-group (max)
constexpr int kCReg = 200;         // coarse columns staged by the up pass (max)

struct FTile {
    int TX, TY;     // tile size in nodes of the tiled level
    int ntx, nty;   // tiles per plane
    int zc, nzc;    // planes per z-run (tiled level), number of runs
    int k, total;   // batch rows, work items
    int RW, RH;     // region width, height (fine nodes)
    int CRW, CRH;   // staged coarse region (up pass)
};

__device__ __forceinline__ bool ftile_item(const FTile& s, int& tx, int& ty, int& zr, int& r) {
    const int bid = blockIdx.x;
    const int per = (s.total + 7) >> 3;
    const int w = (bid & 7) * per + (bid >> 3);
    if (w >= s.total) return false;
    const int nt = s.ntx * s.nty;
    const int t = w % nt;
    const int u = w / nt;
    tx = t % s.ntx;
    ty = t / s.ntx;
    zr = u % s.nzc;
    r = u / s.nzc;
    return true;
}

// One region column owned by a thread: position, ring membership and the
// stencil's in-plane weights. invd0/1/2 = 1/D on the first, an interior and
// the last z-plane (the only z-dependence of D).
template <typename T>
struct RCol {
    int p;          // region index (a + b * RW), -1 if beyond the region
    int64_t off;    // in-plane offset j * nx + i
    bool ing;       // inside the grid
    bool r1, r2;    // inside the grid and at least 1 / 2 columns from the region edge
    bool own;       // written by this work-group
    bool xm, xp, ym, yp;
    T wx, wy;
    T invd0, invd1, invd2;
};

template <typename T>
__device__ __forceinline__ T diag3(const Geom& g, const RCol<T>& c, T wz, int nzn) {
    const T cx = T(g.ihx2) * c.wy * wz, cy = T(g.ihy2) * c.wx * wz, cz = T(g.ihz2) * c.wx * c.wy;
    return T(g.beta) * c.wx * c.wy * wz + cx * T(int(c.xm) + int(c.xp)) + cy * T(int(c.ym) + int(c.yp)) +
           cz * T(nzn);
}

template <typename T>
__device__ __forceinline__ void rcol_init(RCol<T>& c, const Geom& g, int p, int RW, int RH, int i0, int j0,
                                          int own_lo) {
    const bool valid = p < RW * RH;
    const int a = valid ? p % RW : 0, b = valid ? p / RW : 0;
    const int i = i0 + a, j = j0 + b;
    c.p = valid ? p : -1;
    c.ing = valid && i >= 0 && i < g.nx && j >= 0 && j < g.ny;
    c.off = c.ing ? (int64_t)j * g.nx + i : 0;
    c.r1 = c.ing && a >= 1 && a <= RW - 2 && b >= 1 && b <= RH - 2;
    c.r2 = c.ing && a >= 2 && a <= RW - 3 && b >= 2 && b <= RH - 3;
    c.own = c.ing && a >= own_lo && a <= RW - 3 && b >= own_lo && b <= RH - 3;
    c.xm = i > 0;
    c.xp = i < g.nx - 1;
    c.ym = j > 0;
    c.yp = j < g.ny - 1;
    c.wx = (i == 0 || i == g.nx - 1) ? T(0.5) : T(1);
    c.wy = (j == 0 || j == g.ny - 1) ? T(0.5) : T(1);
    c.invd0 = T(1) / diag3(g, c, T(0.5), 1);
    c.invd1 = T(1) / diag3(g, c, T(1), 2);
    c.invd2 = T(1) / diag3(g, c, T(0.5), 1);
}

// (selects values, not fields: a select between field addresses would keep
// the column record in scratch memory)
template <typename T>
__device__ __forceinline__ T invd_at(const RCol<T>& c, int l, int nz) {
    const T v0 = c.invd0, v1 = c.invd1, v2 = c.invd2;
    T v = v1;
    if (l == 0) v = v0;
    if (l == nz - 1) v = v2;
    return v;
}

// (A x) at plane l of column c: xc centre, xb / xa below / above, xw xe xs xn
// the in-plane neighbours (-x, +x, -y, +y). Same arithmetic order as the
// unfused stencil kernels.
template <typename T>
__device__ __forceinline__ T stencil3(const Geom& g, const RCol<T>& c, int l, T xc, T xb, T xa, T xw, T xe, T xs,
                                      T xn) {
    const bool zm = l > 0, zp = l < g.nz - 1;
    const T wz = (l == 0 || l == g.nz - 1) ? T(0.5) : T(1);
    const T cx = T(g.ihx2) * c.wy * wz, cy = T(g.ihy2) * c.wx * wz, cz = T(g.ihz2) * c.wx * c.wy;
    const T mass = T(g.beta) * c.wx * c.wy * wz;
    T sx = T(0), sy = T(0), sz = T(0);
    if (c.xm) sx += xc - xw;
    if (c.xp) sx += xc - xe;
    if (c.ym) sy += xc - xs;
    if (c.yp) sy += xc - xn;
    if (zm) sz += xc - xb;
    if (zp) sz += xc - xa;
    T acc = mass * xc;
    acc += cx * sx;
    acc += cy * sy;
    acc += cz * sz;
    return acc;
}

// ---------------------------------------------------------------- down pass
// Tile = TX x TY coarse columns; the region is the fine columns
// [2 cX0 - 3, 2 (cX0 + TX) + 1] (width 2 TX + 5): x1 on all of it, x2 one
// column in, r two columns in (the 3 x 3 footprints of the tile's coarse
// nodes), owned fine columns 2 cX0 .. 2 cX0 + 2 TX - 1.
// Pipeline at step n: A f, x1 on plane n; B x2 on n-1; C r on n-2;
// D plane sum of r on n-3 into the coarse plane (n-3)/2.
template <typename T>
__global__ __launch_bounds__(kFT) void k_down(Geom gf, Geom gc, FTile s, const T* __restrict__ F, int64_t ldf,
                                              T* __restrict__ X, int64_t ldx, T* __restrict__ Fc, int64_t ldc,
                                              T w0, T w1) {
    __shared__ T s1[2][kReg];
    __shared__ T s2[2][kReg];
    __shared__ T sr[2][kReg];
    int tx, ty, zr, r;
    if (!ftile_item(s, tx, ty, zr, r)) return;
    const int RW = s.RW, RH = s.RH;
    const int cX0 = tx * s.TX, cY0 = ty * s.TY;
    const int cz0 = zr * s.zc, cz1 = min(gc.nz, cz0 + s.zc);
    const int nz = gf.nz;
    const int64_t PL = (int64_t)gf.nx * gf.ny, PLc = (int64_t)gc.nx * gc.ny;
    const T* f = F + r * ldf;
    T* x = X + r * ldx;
    T* fc = Fc + r * ldc;

    RCol<T> c[kCPT];
#pragma unroll
    for (int u = 0; u < kCPT; ++u) rcol_init(c[u], gf, threadIdx.x + u * kFT, RW, RH, 2 * cX0 - 3, 2 * cY0 - 3, 3);
    const int ci = threadIdx.x % s.TX, cj = threadIdx.x / s.TX;
    const bool cact = (int)threadIdx.x < s.TX * s.TY && cX0 + ci < gc.nx && cY0 + cj < gc.ny;
    const int pc = (2 * ci + 3) + (2 * cj + 3) * RW;
    const int64_t coff = cact ? (int64_t)(cY0 + cj) * gc.nx + (cX0 + ci) : 0;

    const int aLo = max(0, 2 * cz0 - 3), aHi = min(nz - 1, 2 * cz1 + 1);  // f, x1
    const int bLo = max(0, 2 * cz0 - 2), bHi = min(nz - 1, 2 * cz1);      // x2
    const int rLo = max(0, 2 * cz0 - 1), rHi = min(nz - 1, 2 * cz1 - 1);  // r and its plane sums
    const int oLo = 2 * cz0, oHi = min(nz - 1, 2 * cz1 - 1);              // x2 written

    T f0[kCPT], f1[kCPT], f2[kCPT];  // f  on planes n-2, n-1, n
    T a0[kCPT], a1[kCPT], a2[kCPT];  // x1 on planes n-2, n-1, n
    T b0[kCPT], b1[kCPT], b2[kCPT];  // x2 on planes n-3, n-2, n-1
#pragma unroll
    for (int u = 0; u < kCPT; ++u) {
        f0[u] = f1[u] = a0[u] = a1[u] = b0[u] = b1[u] = T(0);
    }
    T half = T(0), acc = T(0);
    const T scale = T(0.125);

    // f is loaded two steps ahead of its use (raw values; the validity test is
    // applied at use), with clamped addresses so that every load is issued
    // unconditionally and stays in flight across the barriers.
    auto fidx = [&](int u, int pl) -> int64_t { return (c[u].ing && pl <= aHi) ? pl * PL + c[u].off : 0; };
    T q0[kCPT], q1[kCPT];
#pragma unroll
    for (int u = 0; u < kCPT; ++u) {
        q0[u] = f[fidx(u, aLo)];
        q1[u] = f[fidx(u, aLo + 1)];
    }

    for (int n = aLo; n <= rHi + 3; ++n) {
        // A: f and x1 on plane n
#pragma unroll
        for (int u = 0; u < kCPT; ++u) {
            const T raw = q0[u];
            q0[u] = q1[u];
            q1[u] = f[fidx(u, n + 2)];
            const T fv = (n <= aHi && c[u].ing) ? raw : T(0);
            f2[u] = fv;
            a2[u] = w0 * fv * invd_at(c[u], n, nz);
            if (c[u].p >= 0) s1[n & 1][c[u].p] = a2[u];
        }
        // B: x2 on plane n - 1
        {
            const int m = n - 1;
            const bool in = m >= bLo && m <= bHi;
            const T* P = s1[m & 1];
#pragma unroll
            for (int u = 0; u < kCPT; ++u) {
                T v = T(0);
                if (in && c[u].r1) {
                    const int p = c[u].p;
                    const T ax = stencil3(gf, c[u], m, a1[u], a0[u], a2[u], P[p - 1], P[p + 1], P[p - RW], P[p + RW]);
                    v = a1[u] + w1 * (f1[u] - ax) * invd_at(c[u], m, nz);
                    if (c[u].own && m >= oLo && m <= oHi) x[m * PL + c[u].off] = v;
                }
                b2[u] = v;
                if (c[u].p >= 0) s2[m & 1][c[u].p] = v;
            }
        }
        // C: r on plane n - 2 (zero outside the grid)
        {
            const int m = n - 2;
            const bool in = m >= rLo && m <= rHi;
            const T* P = s2[m & 1];
#pragma unroll
            for (int u = 0; u < kCPT; ++u) {
                T v = T(0);
                if (in && c[u].r2) {
                    const int p = c[u].p;
                    v = f0[u] - stencil3(gf, c[u], m, b1[u], b0[u], b2[u], P[p - 1], P[p + 1], P[p - RW], P[p + RW]);
                }
                if (c[u].p >= 0) sr[m & 1][c[u].p] = v;
            }
        }
        // D: in-plane full-weighting sum of r on plane n - 3; coarse plane L
        // collects s(2L-1)/2 + s(2L) + s(2L+1)/2
        {
            const int m = n - 3;
            if (cact && m >= rLo && m <= rHi) {
                const T* R = sr[m & 1];
                T sum = T(0);
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy) {
                    const T wy = dy ? T(0.5) : T(1);
                    T row = T(0);
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx) row += (dx ? T(0.5) : T(1)) * R[pc + dy * RW + dx];
                    sum += wy * row;
                }
                const int L = m >> 1;
                if ((m & 1) == 0) {
                    acc = half + sum;
                    if (m + 1 >= nz && L >= cz0 && L < cz1) fc[L * PLc + coff] = scale * acc;
                } else {
                    if (L >= cz0 && L < cz1) fc[L * PLc + coff] = scale * (acc + T(0.5) * sum);
                    half = T(0.5) * sum;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kCPT; ++u) {
            f0[u] = f1[u];
            f1[u] = f2[u];
            a0[u] = a1[u];
            a1[u] = a2[u];
            b0[u] = b1[u];
            b1[u] = b2[u];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- up pass
// Tile = TX x TY fine columns; region = tile + 2 columns each side: y0 on all
// of it, y1 one column in, y on the tile. The coarse correction is staged per
// coarse plane in LDS (two planes: fine plane n interpolates from coarse
// planes n/2 and, for odd n, n/2 + 1).
// Pipeline at step n: A y0 on plane n; B y1 on n-1; C y on n-2.
// Thread t < CRW * CRH stages coarse column t of the region (CRW * CRH <=
// kCReg < kFT, one column per thread). cidx: its in-plane offset, -1 if the
// column is outside the coarse grid.
__device__ __forceinline__ int64_t coarse_idx(const Geom& gc, int64_t cidx, int L) {
    return (cidx >= 0 && L < gc.nz) ? L * ((int64_t)gc.nx * gc.ny) + cidx : 0;
}

template <typename T>
__global__ __launch_bounds__(kFT) void k_up(Geom gf, Geom gc, FTile s, const T* __restrict__ F, int64_t ldf,
                                            const T* __restrict__ X0, int64_t ldx0, const T* __restrict__ Ec,
                                            int64_t ldc, T* __restrict__ Y, int64_t ldy, T wa, T wb) {
    __shared__ T s0[2][kReg];
    __shared__ T s1[2][kReg];
    __shared__ T se[2][kCReg];
    int tx, ty, zr, r;
    if (!ftile_item(s, tx, ty, zr, r)) return;
    const int RW = s.RW, RH = s.RH;
    const int gx0 = tx * s.TX, gy0 = ty * s.TY;
    const int z0 = zr * s.zc, z1 = min(gf.nz, z0 + s.zc);
    const int nz = gf.nz;
    const int64_t PL = (int64_t)gf.nx * gf.ny;
    const int i0 = gx0 - 2, j0 = gy0 - 2;
    const int cI0 = i0 >> 1, cJ0 = j0 >> 1;  // floor
    const T* f = F + r * ldf;
    const T* x0 = X0 + r * ldx0;
    const T* e = Ec + r * ldc;
    T* y = Y + r * ldy;

    RCol<T> c[kCPT];
    int cb[kCPT];      // staged coarse index of the column's lower interpolation corner
    bool oi[kCPT], oj[kCPT];
#pragma unroll
    for (int u = 0; u < kCPT; ++u) {
        const int p = threadIdx.x + u * kFT;
        rcol_init(c[u], gf, p, RW, RH, i0, j0, 2);
        const int i = i0 + (p % RW), j = j0 + (p / RW);
        oi[u] = i & 1;
        oj[u] = j & 1;
        cb[u] = c[u].ing ? ((i >> 1) - cI0) + ((j >> 1) - cJ0) * s.CRW : 0;
    }

    const int aLo = max(0, z0 - 2), aHi = min(nz - 1, z1 + 1);  // y0
    const int bLo = max(0, z0 - 1), bHi = min(nz - 1, z1);      // y1
    const int cLo = z0, cHi = z1 - 1;                           // y

    // staged coarse column of this thread
    const int ct = threadIdx.x;
    const bool cst = ct < s.CRW * s.CRH;
    int64_t cidx = -1;
    if (cst) {
        const int I = cI0 + ct % s.CRW, J = cJ0 + ct / s.CRW;
        if (I >= 0 && I < gc.nx && J >= 0 && J < gc.ny) cidx = (int64_t)J * gc.nx + I;
    }
    auto stage_now = [&](int L) {
        if (cst) se[L & 1][ct] = (cidx >= 0 && L < gc.nz) ? e[coarse_idx(gc, cidx, L)] : T(0);
    };
    stage_now(aLo >> 1);
    if (aLo & 1) stage_now((aLo >> 1) + 1);
    // the coarse plane staged at the first even step, loaded now
    const int nEven = aLo + (aLo & 1);
    T cq = e[coarse_idx(gc, cidx, (nEven >> 1) + 1)];
    __syncthreads();

    // x0 and f are loaded two steps ahead of their use (see the down pass)
    auto xidx = [&](int u, int pl) -> int64_t { return (c[u].ing && pl <= aHi) ? pl * PL + c[u].off : 0; };
    auto fidx = [&](int u, int pl) -> int64_t { return (c[u].r1 && pl <= aHi) ? pl * PL + c[u].off : 0; };
    T xq0[kCPT], xq1[kCPT], fq0[kCPT], fq1[kCPT];
#pragma unroll
    for (int u = 0; u < kCPT; ++u) {
        xq0[u] = x0[xidx(u, aLo)];
        fq0[u] = f[fidx(u, aLo)];
        xq1[u] = x0[xidx(u, aLo + 1)];
        fq1[u] = f[fidx(u, aLo + 1)];
    }

    T p0[kCPT], p1[kCPT], p2[kCPT];  // y0 on planes n-2, n-1, n
    T f0[kCPT], f1[kCPT], f2[kCPT];  // f  on planes n-2, n-1, n
    T q0[kCPT], q1[kCPT], q2[kCPT];  // y1 on planes n-3, n-2, n-1
#pragma unroll
    for (int u = 0; u < kCPT; ++u) {
        p0[u] = p1[u] = f0[u] = f1[u] = q0[u] = q1[u] = T(0);
    }

    for (int n = aLo; n <= cHi + 2; ++n) {
        // the coarse plane that step n + 1 adds (odd n + 1 needs n/2 + 1), and
        // the load of the one the next even step adds
        if (!(n & 1)) {
            const int L = (n >> 1) + 1;
            if (n + 1 <= aHi && cst) se[L & 1][ct] = (cidx >= 0 && L < gc.nz) ? cq : T(0);
            cq = e[coarse_idx(gc, cidx, L + 1)];
        }
        // A: y0 = x2 + P e on plane n
        {
            const bool in = n <= aHi;
            const int L = n >> 1;
            const int nl = 1 + (n & 1);
            const T wl = (n & 1) ? T(0.5) : T(1);
#pragma unroll
            for (int u = 0; u < kCPT; ++u) {
                const T xr = xq0[u], fr = fq0[u];
                xq0[u] = xq1[u];
                fq0[u] = fq1[u];
                xq1[u] = x0[xidx(u, n + 2)];
                fq1[u] = f[fidx(u, n + 2)];
                T v = T(0), fv = T(0);
                if (in && c[u].ing) {
                    const int nj = 1 + int(oj[u]), ni = 1 + int(oi[u]);
                    const T wj = oj[u] ? T(0.5) : T(1), wi = oi[u] ? T(0.5) : T(1);
                    T pe = T(0);
                    for (int a = 0; a < nl; ++a) {
                        const T* E = se[(L + a) & 1];
                        for (int bb = 0; bb < nj; ++bb)
                            for (int cc = 0; cc < ni; ++cc) pe += (wl * wj * wi) * E[cb[u] + bb * s.CRW + cc];
                    }
                    v = xr;
                    v += pe;
                    if (c[u].r1) fv = fr;
                }
                p2[u] = v;
                f2[u] = fv;
                if (c[u].p >= 0) s0[n & 1][c[u].p] = v;
            }
        }
        // B: y1 on plane n - 1
        {
            const int m = n - 1;
            const bool in = m >= bLo && m <= bHi;
            const T* P = s0[m & 1];
#pragma unroll
            for (int u = 0; u < kCPT; ++u) {
                T v = T(0);
                if (in && c[u].r1) {
                    const int p = c[u].p;
                    const T ax = stencil3(gf, c[u], m, p1[u], p0[u], p2[u], P[p - 1], P[p + 1], P[p - RW], P[p + RW]);
                    v = p1[u] + wa * (f1[u] - ax) * invd_at(c[u], m, nz);
                }
                q2[u] = v;
                if (c[u].p >= 0) s1[m & 1][c[u].p] = v;
            }
        }
        // C: y on plane n - 2
        {
            const int m = n - 2;
            if (m >= cLo && m <= cHi) {
                const T* P = s1[m & 1];
#pragma unroll
                for (int u = 0; u < kCPT; ++u) {
                    if (c[u].own) {
                        const int p = c[u].p;
                        const T ax =
                            stencil3(gf, c[u], m, q1[u], q0[u], q2[u], P[p - 1], P[p + 1], P[p - RW], P[p + RW]);
                        y[m * PL + c[u].off] = q1[u] + wb * (f0[u] - ax) * invd_at(c[u], m, nz);
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kCPT; ++u) {
            p0[u] = p1[u];
            p1[u] = p2[u];
            f0[u] = f1[u];
            f1[u] = f2[u];
            q0[u] = q1[u];
            q1[u] = q2[u];
        }
        __syncthreads();
    }
}

// Tile shape: the region must fit kReg columns; the cost of a plane is
// (work-groups) x (fixed cost of one group + 128-byte lines its region rows
// touch), so wide rows (coalesced loads) and few groups both count.
FTile plan_tiles(int nx, int ny, int nzt, int k, bool down, int zmin, int es) {
    FTile best{};
    int64_t best_cost = -1, best_nt = 0;
    for (int TX = 1; TX <= nx; ++TX) {
        for (int TY = 1; TY <= ny; ++TY) {
            const int RW = down ? 2 * TX + 5 : TX + 4;
            const int RH = down ? 2 * TY + 5 : TY + 4;
            if (RW * RH > kReg) break;
            if (down && TX * TY > kFT) break;
            const int CRW = (RW + 1) / 2 + 2, CRH = (RH + 1) / 2 + 2;
            if (!down && CRW * CRH > kCReg) break;
            const int64_t nt = cdiv(nx, TX) * cdiv(ny, TY);
            const int64_t cost = nt * ((int64_t)kReg * 8 + (int64_t)RH * (cdiv(RW * es, 128) + 1) * 128);
            if (best_cost < 0 || cost < best_cost) {
                best_cost = cost;
                best_nt = nt;
                best.TX = TX;
                best.TY = TY;
                best.RW = RW;
                best.RH = RH;
                best.CRW = CRW;
                best.CRH = CRH;
            }
        }
    }
    best.ntx = (int)cdiv(nx, best.TX);
    best.nty = (int)cdiv(ny, best.TY);
    best.k = k;
    const int64_t base = best_nt * k;
    const int max_runs = std::max(1, nzt / zmin);
    int nzc = (int)std::clamp<int64_t>(cdiv(4096, base), 1, max_runs);
    best.zc = (int)cdiv(nzt, nzc);
    best.nzc = (int)cdiv(nzt, best.zc);
    best.total = (int)(base * best.nzc);
    return best;
}

unsigned ftile_grid(const FTile& s) { return 8u * (unsigned)cdiv(s.total, 8); }

}  // namespace

bool fused_levels_ok(const Geom& gf, const Geom& gc) {
    return gf.nz >= 3 && gf.nx == 2 * gc.nx - 1 && gf.ny == 2 * gc.ny - 1 && gf.nz == 2 * gc.nz - 1;
}

template <typename T>
void launch_vdown(hipStream_t st, const Geom& gf, const Geom& gc, int k, const T* F, int64_t ldf, T* X, int64_t ldx,
                  T* Fc, int64_t ldc, double w0, double w1) {
    if (k <= 0) return;
    require(fused_levels_ok(gf, gc), "internal: fused pass on non-nested levels");
    const FTile s = plan_tiles(gc.nx, gc.ny, gc.nz, k, true, 4, (int)sizeof(T));
    hipLaunchKernelGGL(k_down<T>, dim3(ftile_grid(s)), dim3(kFT), 0, st, gf, gc, s, F, ldf, X, ldx, Fc, ldc, T(w0),
                       T(w1));
    H1W_LAUNCHED();
}

template <typename T>
void launch_vup(hipStream_t st, const Geom& gf, const Geom& gc, int k, const T* F, int64_t ldf, const T* X0,
                int64_t ldx0, const T* Ec, int64_t ldc, T* Y, int64_t ldy, double wa, double wb) {
    if (k <= 0) return;
    require(fused_levels_ok(gf, gc), "internal: fused pass on non-nested levels");
    const FTile s = plan_tiles(gf.nx, gf.ny, gf.nz, k, false, 8, (int)sizeof(T));
    hipLaunchKernelGGL(k_up<T>, dim3(ftile_grid(s)), dim3(kFT), 0, st, gf, gc, s, F, ldf, X0, ldx0, Ec, ldc, Y, ldy,
                       T(wa), T(wb));
    H1W_LAUNCHED();
}

template void launch_vdown<double>(hipStream_t, const Geom&, const Geom&, int, const double*, int64_t, double*,
                                   int64_t, double*, int64_t, double, double);
template void launch_vdown<float>(hipStream_t, const Geom&, const Geom&, int, const float*, int64_t, float*,
                                  int64_t, float*, int64_t, double, double);
template void launch_vup<double>(hipStream_t, const Geom&, const Geom&, int, const double*, int64_t, const double*,
                                 int64_t, const double*, int64_t, double*, int64_t, double, double);
template void launch_vup<float>(hipStream_t, const Geom&, const Geom&, int, const float*, int64_t, const float*,
                                int64_t, const float*, int64_t, float*, int64_t, double, double);

}  // namespace h1w
