// Fused passes of the 2D V-cycle with two smoothing steps on each side (the
// multigrid preconditioner B of Section 3; the same cycle as the single-step
// 2D stencil kernels, with fewer passes over memory and fewer launches).
//
// down (one level, zero initial guess):
//     x1 = w0 D^-1 f,  x2 = x1 + w1 D^-1 (f - A x1),  r = f - A x2,  fc = 2^-2 P^T r
//   reads f, writes x2 and the coarse right-hand side fc.
// up (one level):
//     y0 = x2 + P e,  y1 = y0 + wa D^-1 (f - A y0),  y = y1 + wb D^-1 (f - A y1)
//   reads x2, f and the coarse correction e, writes y.
//
// A work-group takes one tile of one batch row and holds its whole region in
// LDS: the region is the tile plus a halo ring wide enough that every stage is
// computed from the group's own data (3 fine columns for the down pass, 2 for
// the up pass); the halo is recomputed by the neighbouring tiles. Stages are
// separated by barriers. The stencil is used in diagonal form,
//     (A x)_p = D_p x_p - S_p,  S_p = cx (x_w + x_e) + cy (x_s + x_n),
// with every value outside the grid held as 0, which drops exactly the
// couplings a Neumann boundary node lacks (D counts only its in-grid
// neighbours). Small grids run a few launches per level instead of six.
#include <algorithm>

#include "devutil.h"
#include "internal.h"

namespace h1w {

namespace {

constexpr int kF2Threads = 256;       // threads per work-group when the launch fills the GPU
constexpr int kF2ThreadsFew = 1024;   // ... and when it has fewer work-groups than 2 per CU
constexpr int kDownTC = 16;                   // coarse nodes per tile side (down pass)
constexpr int kDownRW = 2 * kDownTC + 5;      // region: fine columns 2 cX0 - 3 .. 2 (cX0 + TC) + 1
constexpr int kUpT = 32;                      // fine nodes per tile side (up pass)
constexpr int kUpRW = kUpT + 4;               // region: fine columns gx0 - 2 .. gx0 + T + 1
constexpr int kUpCW = kUpRW / 2 + 2;          // coarse columns staged by the up pass

template <typename T>
struct Coef2 {
    T cx, cy, dg, iv;
    bool ing;
};

// coefficients of the 2D H^1 Gram operator at fine node (i, j)
template <typename T>
__device__ __forceinline__ Coef2<T> coef2(const Geom& g, int i, int j) {
    Coef2<T> c;
    c.ing = i >= 0 && i < g.nx && j >= 0 && j < g.ny;
    const T wx = (i == 0 || i == g.nx - 1) ? T(0.5) : T(1);
    const T wy = (j == 0 || j == g.ny - 1) ? T(0.5) : T(1);
    const int nxn = int(i > 0) + int(i < g.nx - 1), nyn = int(j > 0) + int(j < g.ny - 1);
    c.cx = T(g.ihx2) * wy;
    c.cy = T(g.ihy2) * wx;
    c.dg = T(g.beta) * wx * wy + c.cx * T(nxn) + c.cy * T(nyn);
    c.iv = c.ing ? T(1) / c.dg : T(0);
    if (!c.ing) c.cx = c.cy = c.dg = T(0);
    return c;
}

template <typename T>
__device__ __forceinline__ T nsum2(const Coef2<T>& c, const T* P, int p, int RW) {
    return fma(c.cy, P[p - RW] + P[p + RW], c.cx * (P[p - 1] + P[p + 1]));
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_down2(Geom gf, Geom gc, int ntx, const T* __restrict__ F,
                                                      int64_t ldf, T* __restrict__ X, int64_t ldx,
                                                      T* __restrict__ Fc, int64_t ldc, T w0, T w1) {
    constexpr int RW = kDownRW, RN = RW * RW;
    __shared__ T sf[RN], s1[RN], s2[RN], sr[RN];
    const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
    const int64_t r = blockIdx.y;
    const int cX0 = tx * kDownTC, cY0 = ty * kDownTC;
    const int i0 = 2 * cX0 - 3, j0 = 2 * cY0 - 3;
    const T* f = F + r * ldf;
    T* x = X + r * ldx;
    // stage 1: f and x1 = w0 D^-1 f on the whole region (0 outside the grid)
    for (int p = threadIdx.x; p < RN; p += NT) {
        const int a = p % RW, b = p / RW;
        const int i = i0 + a, j = j0 + b;
        const Coef2<T> c = coef2<T>(gf, i, j);
        const T fv = c.ing ? f[(int64_t)j * gf.nx + i] : T(0);
        sf[p] = fv;
        s1[p] = w0 * c.iv * fv;
        s2[p] = T(0);
        sr[p] = T(0);
    }
    __syncthreads();
    // stage 2: x2 one ring in; written for the fine nodes this tile owns
    for (int p = threadIdx.x; p < RN; p += NT) {
        const int a = p % RW, b = p / RW;
        if (a < 1 || a > RW - 2 || b < 1 || b > RW - 2) continue;
        const int i = i0 + a, j = j0 + b;
        const Coef2<T> c = coef2<T>(gf, i, j);
        if (!c.ing) continue;
        const T x1 = s1[p];
        const T v = x1 + w1 * c.iv * (sf[p] - (c.dg * x1 - nsum2(c, s1, p, RW)));
        s2[p] = v;
        if (a >= 3 && a < 3 + 2 * kDownTC && b >= 3 && b < 3 + 2 * kDownTC) x[(int64_t)j * gf.nx + i] = v;
    }
    __syncthreads();
    // stage 3: r = f - A x2 two rings in
    for (int p = threadIdx.x; p < RN; p += NT) {
        const int a = p % RW, b = p / RW;
        if (a < 2 || a > RW - 3 || b < 2 || b > RW - 3) continue;
        const int i = i0 + a, j = j0 + b;
        const Coef2<T> c = coef2<T>(gf, i, j);
        if (!c.ing) continue;
        sr[p] = sf[p] - (c.dg * s2[p] - nsum2(c, s2, p, RW));
    }
    __syncthreads();
    // stage 4: fc = 2^-2 (full-weighting sum of r) on the tile's coarse nodes
    const int ci = threadIdx.x % kDownTC, cj = threadIdx.x / kDownTC;
    const int I = cX0 + ci, J = cY0 + cj;
    if (cj < kDownTC && I < gc.nx && J < gc.ny) {
        const int pc = (2 * ci + 3) + (2 * cj + 3) * RW;
        T sum = T(0);
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            T row = T(0);
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) row += (dx ? T(0.5) : T(1)) * sr[pc + dy * RW + dx];
            sum += (dy ? T(0.5) : T(1)) * row;
        }
        Fc[r * ldc + (int64_t)J * gc.nx + I] = T(0.25) * sum;
    }
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_up2(Geom gf, Geom gc, int ntx, const T* __restrict__ F, int64_t ldf,
                                                    const T* __restrict__ X0, int64_t ldx0,
                                                    const T* __restrict__ Ec, int64_t ldc, T* __restrict__ Y,
                                                    int64_t ldy, T wa, T wb) {
    constexpr int RW = kUpRW, RN = RW * RW, CW = kUpCW;
    __shared__ T sf[RN], s0[RN], s1[RN], se[CW * CW];
    const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
    const int64_t r = blockIdx.y;
    const int gx0 = tx * kUpT, gy0 = ty * kUpT;
    const int i0 = gx0 - 2, j0 = gy0 - 2;
    const int cI0 = (i0 >> 1), cJ0 = (j0 >> 1);  // floor
    const T* f = F + r * ldf;
    const T* x2 = X0 + r * ldx0;
    const T* e = Ec + r * ldc;
    T* y = Y + r * ldy;
    // the coarse correction under the region (0 outside the coarse grid)
    for (int q = threadIdx.x; q < CW * CW; q += NT) {
        const int I = cI0 + q % CW, J = cJ0 + q / CW;
        se[q] = (I >= 0 && I < gc.nx && J >= 0 && J < gc.ny) ? e[(int64_t)J * gc.nx + I] : T(0);
    }
    __syncthreads();
    // stage 1: f and y0 = x2 + P e on the whole region
    for (int p = threadIdx.x; p < RN; p += NT) {
        const int a = p % RW, b = p / RW;
        const int i = i0 + a, j = j0 + b;
        const bool ing = i >= 0 && i < gf.nx && j >= 0 && j < gf.ny;
        T fv = T(0), y0 = T(0);
        if (ing) {
            const int64_t o = (int64_t)j * gf.nx + i;
            fv = f[o];
            // multilinear interpolation from coarse nodes i/2 (and i/2 + 1 for odd i)
            const int ci = (i >> 1) - cI0, cj = (j >> 1) - cJ0;
            const T hx = (i & 1) ? T(0.5) : T(0), hy = (j & 1) ? T(0.5) : T(0);
            const T* s = se + cj * CW + ci;
            const T lo = s[0] + hx * (s[1] - s[0]);
            const T hi = s[CW] + hx * (s[CW + 1] - s[CW]);
            y0 = x2[o] + (lo + hy * (hi - lo));
        }
        sf[p] = fv;
        s0[p] = y0;
        s1[p] = T(0);
    }
    __syncthreads();
    // stage 2: y1 one ring in
    for (int p = threadIdx.x; p < RN; p += NT) {
        const int a = p % RW, b = p / RW;
        if (a < 1 || a > RW - 2 || b < 1 || b > RW - 2) continue;
        const Coef2<T> c = coef2<T>(gf, i0 + a, j0 + b);
        if (!c.ing) continue;
        const T v0 = s0[p];
        s1[p] = v0 + wa * c.iv * (sf[p] - (c.dg * v0 - nsum2(c, s0, p, RW)));
    }
    __syncthreads();
    // stage 3: y on the tile
    for (int q = threadIdx.x; q < kUpT * kUpT; q += NT) {
        const int a = 2 + q % kUpT, b = 2 + q / kUpT;
        const int i = i0 + a, j = j0 + b;
        const Coef2<T> c = coef2<T>(gf, i, j);
        if (!c.ing) continue;
        const int p = a + b * RW;
        const T v1 = s1[p];
        y[(int64_t)j * gf.nx + i] = v1 + wb * c.iv * (sf[p] - (c.dg * v1 - nsum2(c, s1, p, RW)));
    }
}

// ------------------------------------------------------------ coarse tail
// The levels from l0 (the first whose three arrays, and those of every
// coarser level, fit one work-group's LDS) down to the coarsest and back in
// one launch: one work-group per right-hand side runs the same cycle as the
// down and up passes above (same expressions, stage by stage, with barriers
// between stages) and the dense coarsest solve, so that small grids and the
// coarse end of large ones cost one launch instead of two per level plus the
// coarse solve. Level l holds f, x and t (g[l].N values each) at off[l]:
//   down: t = x1, x = x2, t = r, then f of level l + 1 = 2^-2 P^T r;
//   coarsest: x = Cinv f (the j range split over up to four thread groups,
//             their partial sums added in a fixed order);
//   up:   t = y0 = x2 + P e, x = y1, t = y; e of level l - 1 is t (x on the
//         coarsest level).
// Values outside the grid enter as 0 (the neighbour is dropped), as in the
// passes above.
constexpr int kTailThreads = 1024;

// The coefficients of coef2 depend on (i, j) only through the boundary class
// of each coordinate (first, interior, last node), so each level needs nine
// sets; they are computed once per launch by coef2 itself.
template <typename T>
struct TailCoef {
    T cx, cy, dg, iv;
};
__device__ __forceinline__ int tail_cls(int i, int n) { return i == 0 ? 0 : (i == n - 1 ? 2 : 1); }

// Node loop of one level: thread t owns column i = t % nx and rows
// t / nx, t / nx + rows, ... (rows = kTailThreads / nx), so no division per
// node. body(p, i, j, coefficient set).
template <typename T, typename B>
__device__ __forceinline__ void tail_nodes(const Geom& g, const TailCoef<T>* cf, B&& body) {
    const int nx = g.nx, ny = g.ny, rows = kTailThreads / nx;
    const int t = threadIdx.x;
    const int i = t % nx, j0 = t / nx;
    if (j0 >= rows) return;
    const int cxl = tail_cls(i, nx);
    for (int j = j0; j < ny; j += rows) {
        const TailCoef<T>& c = cf[cxl + 3 * tail_cls(j, ny)];
        body(j * nx + i, i, j, c);
    }
}

template <typename T>
__device__ __forceinline__ T nsum_lvl(const TailCoef<T>& c, const T* P, int p, int i, int j, int nx, int ny) {
    const T w = i > 0 ? P[p - (i > 0)] : T(0);
    const T e = i < nx - 1 ? P[p + (i < nx - 1)] : T(0);
    const T so = j > 0 ? P[p - (j > 0 ? nx : 0)] : T(0);
    const T no = j < ny - 1 ? P[p + (j < ny - 1 ? nx : 0)] : T(0);
    return fma(c.cy, so + no, c.cx * (w + e));
}

template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_vtail2(TailGeo tg, const T* __restrict__ Cinv, int k,
                                                         const T* __restrict__ F, int64_t ldf, T* __restrict__ X,
                                                         int64_t ldx, T w0, T w1) {
    __shared__ T sm[kTailElems];
    __shared__ TailCoef<T> scf[kTailLevels][9];
    const int L = tg.L, Nc = (int)tg.g[L - 1].N;
    const int tid = threadIdx.x;
    if (tid < 9 * L) {
        const int l = tid / 9, q = tid % 9, cxl = q % 3, cyl = q / 3;
        const Geom& g = tg.g[l];
        const int i = cxl == 0 ? 0 : (cxl == 1 ? 1 : g.nx - 1), j = cyl == 0 ? 0 : (cyl == 1 ? 1 : g.ny - 1);
        const Coef2<T> c = coef2<T>(g, i, j);
        scf[l][q] = TailCoef<T>{c.cx, c.cy, c.dg, c.iv};
    }
    for (int r = blockIdx.x; r < k; r += gridDim.x) {
        {
            T* f = sm + tg.off[0];
            const T* src = F + (int64_t)r * ldf;
            for (int p = tid; p < (int)tg.g[0].N; p += kTailThreads) f[p] = src[p];
        }
        __syncthreads();
        for (int l = 0; l + 1 < L; ++l) {
            const Geom& g = tg.g[l];
            const Geom& gc = tg.g[l + 1];
            const int nx = g.nx, ny = g.ny, N = (int)g.N;
            const TailCoef<T>* cf = scf[l];
            T* f = sm + tg.off[l];
            T* x = f + N;
            T* t = x + N;
            tail_nodes<T>(g, cf, [&](int p, int, int, const TailCoef<T>& c) { t[p] = w0 * c.iv * f[p]; });
            __syncthreads();
            tail_nodes<T>(g, cf, [&](int p, int i, int j, const TailCoef<T>& c) {
                const T x1 = t[p];
                x[p] = x1 + w1 * c.iv * (f[p] - (c.dg * x1 - nsum_lvl(c, t, p, i, j, nx, ny)));
            });
            __syncthreads();
            tail_nodes<T>(g, cf, [&](int p, int i, int j, const TailCoef<T>& c) {
                t[p] = f[p] - (c.dg * x[p] - nsum_lvl(c, x, p, i, j, nx, ny));
            });
            __syncthreads();
            T* fc = sm + tg.off[l + 1];
            tail_nodes<T>(gc, scf[l + 1], [&](int q, int I, int J, const TailCoef<T>&) {
                T sum = T(0);
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy) {
                    const int jj = 2 * J + dy;
                    T row = T(0);
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int ii = 2 * I + dx;
                        const bool in = ii >= 0 && ii < nx && jj >= 0 && jj < ny;
                        row += (dx ? T(0.5) : T(1)) * (in ? t[in ? jj * nx + ii : 0] : T(0));
                    }
                    sum += (dy ? T(0.5) : T(1)) * row;
                }
                fc[q] = T(0.25) * sum;
            });
            __syncthreads();
        }
        // coarsest: x = Cinv f with the decomposition of the separate coarse
        // solve for the same k, so the result is the same bit for bit: the j
        // range in csplit parts, each part in four consecutive chains added
        // as (c0 + c1) + (c2 + c3), the parts then added in order. Cinv is
        // symmetric, so output i reads column i (coalesced across threads).
        {
            T* f = sm + tg.off[L - 1];
            T* x = f + Nc;
            T* red = sm + tg.red;
            const int S = tg.csplit;
            const int js = (Nc + S - 1) / S;
            for (int job = tid; job < S * Nc; job += kTailThreads) {
                const int i = job % Nc, sp = job / Nc;
                const int ja = sp * js, jb = min(Nc, ja + js);
                const int q = (jb - ja + 3) / 4;
                T c4[4];
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const int j0 = ja + w * q, j1 = min(jb, j0 + q);
                    T acc = T(0);
#pragma unroll 8
                    for (int j = j0; j < j1; ++j) acc += Cinv[(int64_t)j * Nc + i] * f[j];
                    c4[w] = acc;
                }
                red[sp * Nc + i] = (c4[0] + c4[1]) + (c4[2] + c4[3]);
            }
            __syncthreads();
            for (int i = tid; i < Nc; i += kTailThreads) {
                T v = red[i];
                if (S > 1) {
                    v = T(0);
                    for (int sp = 0; sp < S; ++sp) v += red[sp * Nc + i];
                }
                x[i] = v;
            }
            __syncthreads();
        }
        for (int l = L - 2; l >= 0; --l) {
            const Geom& g = tg.g[l];
            const Geom& gc = tg.g[l + 1];
            const int nx = g.nx, ny = g.ny, N = (int)g.N, ncx = gc.nx;
            const TailCoef<T>* cf = scf[l];
            T* f = sm + tg.off[l];
            T* x = f + N;
            T* t = x + N;
            const T* e = sm + tg.off[l + 1] + (l + 1 == L - 1 ? 1 : 2) * gc.N;
            tail_nodes<T>(g, cf, [&](int p, int i, int j, const TailCoef<T>&) {
                const T* s0 = e + (j >> 1) * ncx + (i >> 1);
                const T a0 = s0[0];
                const T lo = (i & 1) ? a0 + T(0.5) * (s0[1] - a0) : a0;
                T pe = lo;
                if (j & 1) {
                    const T b0 = s0[ncx];
                    const T hi = (i & 1) ? b0 + T(0.5) * (s0[ncx + 1] - b0) : b0;
                    pe = lo + T(0.5) * (hi - lo);
                }
                t[p] = x[p] + pe;
            });
            __syncthreads();
            tail_nodes<T>(g, cf, [&](int p, int i, int j, const TailCoef<T>& c) {
                const T v0 = t[p];
                x[p] = v0 + w1 * c.iv * (f[p] - (c.dg * v0 - nsum_lvl(c, t, p, i, j, nx, ny)));
            });
            __syncthreads();
            tail_nodes<T>(g, cf, [&](int p, int i, int j, const TailCoef<T>& c) {
                const T v1 = x[p];
                t[p] = v1 + w0 * c.iv * (f[p] - (c.dg * v1 - nsum_lvl(c, x, p, i, j, nx, ny)));
            });
            __syncthreads();
        }
        {
            const T* t = sm + tg.off[0] + 2 * tg.g[0].N;
            T* dst = X + (int64_t)r * ldx;
            for (int p = tid; p < (int)tg.g[0].N; p += kTailThreads) dst[p] = t[p];
        }
        __syncthreads();
    }
}

}  // namespace

bool tail2_plan(const Geom* lv, int L, int& l0, TailGeo& tg) {
    l0 = L;
    if (L < 2 || lv[L - 1].N > kTailMaxNc) return false;
    for (int l = L - 2; l >= 0 && L - l <= kTailLevels; --l) {
        if (!fused2_levels_ok(lv[l], lv[l + 1]) || lv[l].nx > kTailThreads) break;
        int64_t need = cdiv(lv[L - 1].N, 32) * lv[L - 1].N;  // the most coarse-solve splits
        for (int q = l; q < L; ++q) need += 3 * lv[q].N;
        if (need > kTailElems) break;
        l0 = l;
    }
    if (l0 > L - 2) return false;
    tg.L = L - l0;
    int off = 0;
    for (int q = 0; q < tg.L; ++q) {
        tg.g[q] = lv[l0 + q];
        tg.off[q] = off;
        off += 3 * (int)lv[l0 + q].N;
    }
    tg.red = off;
    return true;
}

template <typename T>
void launch_vtail2(hipStream_t st, const TailGeo& tg, const T* Cinv, int k, const T* F, int64_t ldf, T* X,
                   int64_t ldx, double w0, double w1) {
    if (k <= 0) return;
    require(tg.L >= 2 && tg.L <= kTailLevels && tg.g[tg.L - 1].N <= kTailMaxNc && tg.csplit >= 1 &&
                tg.red + tg.csplit * tg.g[tg.L - 1].N <= kTailElems,
            "internal: coarse tail does not fit");
    hipLaunchKernelGGL((k_vtail2<T>), dim3((unsigned)std::min(k, 65535)), dim3(kTailThreads), 0, st, tg, Cinv, k, F,
                       ldf, X, ldx, T(w0), T(w1));
    H1W_LAUNCHED();
}

bool fused2_levels_ok(const Geom& gf, const Geom& gc) {
    return gf.nz == 1 && gc.nz == 1 && gf.nx >= 3 && gf.ny >= 3 && gf.nx == 2 * gc.nx - 1 && gf.ny == 2 * gc.ny - 1;
}

template <typename T>
void launch_vdown2(hipStream_t st, const Geom& gf, const Geom& gc, int k, const T* F, int64_t ldf, T* X, int64_t ldx,
                   T* Fc, int64_t ldc, double w0, double w1) {
    if (k <= 0) return;
    require(fused2_levels_ok(gf, gc), "internal: fused 2D pass on non-nested levels");
    require(k <= 65535, "internal: too many rows in one fused 2D launch");
    const int ntx = (int)cdiv(gc.nx, kDownTC), nty = (int)cdiv(gc.ny, kDownTC);
    const dim3 grid((unsigned)(ntx * nty), (unsigned)k);
    if ((int64_t)ntx * nty * k < 512)  // few groups: more threads each, shorter stages
        hipLaunchKernelGGL((k_down2<T, kF2ThreadsFew>), grid, dim3(kF2ThreadsFew), 0, st, gf, gc, ntx, F, ldf, X, ldx,
                           Fc, ldc, T(w0), T(w1));
    else
        hipLaunchKernelGGL((k_down2<T, kF2Threads>), grid, dim3(kF2Threads), 0, st, gf, gc, ntx, F, ldf, X, ldx, Fc,
                           ldc, T(w0), T(w1));
    H1W_LAUNCHED();
}

template <typename T>
void launch_vup2(hipStream_t st, const Geom& gf, const Geom& gc, int k, const T* F, int64_t ldf, const T* X0,
                 int64_t ldx0, const T* Ec, int64_t ldc, T* Y, int64_t ldy, double wa, double wb) {
    if (k <= 0) return;
    require(fused2_levels_ok(gf, gc), "internal: fused 2D pass on non-nested levels");
    require(k <= 65535, "internal: too many rows in one fused 2D launch");
    const int ntx = (int)cdiv(gf.nx, kUpT), nty = (int)cdiv(gf.ny, kUpT);
    const dim3 grid((unsigned)(ntx * nty), (unsigned)k);
    if ((int64_t)ntx * nty * k < 512)
        hipLaunchKernelGGL((k_up2<T, kF2ThreadsFew>), grid, dim3(kF2ThreadsFew), 0, st, gf, gc, ntx, F, ldf, X0, ldx0,
                           Ec, ldc, Y, ldy, T(wa), T(wb));
    else
        hipLaunchKernelGGL((k_up2<T, kF2Threads>), grid, dim3(kF2Threads), 0, st, gf, gc, ntx, F, ldf, X0, ldx0, Ec,
                           ldc, Y, ldy, T(wa), T(wb));
    H1W_LAUNCHED();
}

#define H1W_INST_F2(T)                                                                                         \
    template void launch_vdown2<T>(hipStream_t, const Geom&, const Geom&, int, const T*, int64_t, T*, int64_t, \
                                   T*, int64_t, double, double);                                              \
    template void launch_vup2<T>(hipStream_t, const Geom&, const Geom&, int, const T*, int64_t, const T*,     \
                                 int64_t, const T*, int64_t, T*, int64_t, double, double);
H1W_INST_F2(double)
H1W_INST_F2(float)
template void launch_vtail2<double>(hipStream_t, const TailGeo&, const double*, int, const double*, int64_t, double*,
                                    int64_t, double, double);
template void launch_vtail2<float>(hipStream_t, const TailGeo&, const float*, int, const float*, int64_t, float*,
                                   int64_t, double, double);

}  // namespace h1w
