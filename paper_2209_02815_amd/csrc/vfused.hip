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
// the 8 XCDs in contiguous ranges of items. A work-group of NT threads owns a
// region of at most 2 NT in-plane columns: its tile plus a halo ring wide
// enough that every stage is computed from the group's own data (halo
// columns are recomputed by neighbouring tiles; their loads hit L2). Each
// thread owns 2 columns and marches up z, stage s of the pipeline working on
// plane n - s at step n. Z-neighbours stay in registers (three rotating sets;
// the march is unrolled by three so that the rotation is static); in-plane
// neighbours come from LDS planes that were written in step n - 1 (double
// buffered), so a single barrier per step orders every read after its write
// and every overwrite after its last read. Global loads are issued three
// steps ahead of their use.
#include <algorithm>
#include <type_traits>

#include "devutil.h"
#include "internal.h"

namespace h1w {

namespace {

constexpr int kCPT = 2;             // region columns per thread
constexpr int kPad = 64;            // LDS margin around each plane (>= region width)
constexpr int kCReg = 200;          // coarse columns staged by the up pass (max, < its thread count)
constexpr int kDownThreads = 512;   // down pass: the 3-column halo favours large regions
constexpr int kUpThreads = 256;

// LDS array of two planes of NT * kCPT region columns laid out as
// [margin | plane 0 | margin | plane 1 | margin]: region index p and its
// neighbours p +- 1, p +- RW are inside the array for every p < NT * kCPT, so
// stages read them without bounds tests (values read for columns whose
// result is discarded are never used).
template <int NT>
struct Lds {
    static constexpr int REG = NT * kCPT;
    static constexpr int SLOT = REG + kPad;
    static constexpr int SIZE = 2 * SLOT + kPad;
    template <typename T>
    static __device__ __forceinline__ T* plane(T* arr, int slot) {
        return arr + kPad + slot * SLOT;
    }
};

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

// One region column owned by a thread. The stencil is used in diagonal form,
//   (A x)_p = D_p x_p - S_p,  S_p = wz (cx (x_w + x_e) + cy (x_s + x_n)) + cz (x_b + x_a),
// with every neighbour outside the grid held as 0 (LDS planes and z registers
// are zero there), which drops exactly the couplings a Neumann boundary node
// lacks. cx, cy, cz are the couplings on interior planes (wz = 1). On the
// first and last plane wz = 1/2, which halves every in-plane term of D while
// the single z-coupling cz replaces the interior 2 cz: D there is exactly
// D/2 of the interior, so one per-plane factor (uniform across the group)
// covers both plane classes. Offsets are 32-bit (a grid vector has fewer
// than 2^31 nodes).
template <typename T>
struct RCol {
    int p;          // region index (a + b * RW); >= RW * RH: idle column
    int off;        // in-plane offset j * nx + i (0 outside the grid)
    bool ing;       // inside the grid
    bool r1, r2;    // inside the grid and at least 1 / 2 columns from the region edge
    bool own;       // written by this work-group
    T cx, cy, cz;
    T dg;           // D on interior planes
    T iv;           // 1/D on interior planes (0 outside the grid)
};

template <typename T>
__device__ __forceinline__ void rcol_init(RCol<T>& c, const Geom& g, int p, int RW, int RH, int i0, int j0,
                                          int own_lo) {
    const bool valid = p < RW * RH;
    const int a = p % RW, b = p / RW;
    const int i = i0 + a, j = j0 + b;
    c.p = p;
    c.ing = valid && i >= 0 && i < g.nx && j >= 0 && j < g.ny;
    c.off = c.ing ? j * g.nx + i : 0;
    c.r1 = c.ing && a >= 1 && a <= RW - 2 && b >= 1 && b <= RH - 2;
    c.r2 = c.ing && a >= 2 && a <= RW - 3 && b >= 2 && b <= RH - 3;
    c.own = c.ing && a >= own_lo && a <= RW - 3 && b >= own_lo && b <= RH - 3;
    const T wx = (i == 0 || i == g.nx - 1) ? T(0.5) : T(1);
    const T wy = (j == 0 || j == g.ny - 1) ? T(0.5) : T(1);
    const int nxn = int(i > 0) + int(i < g.nx - 1), nyn = int(j > 0) + int(j < g.ny - 1);
    c.cx = T(g.ihx2) * wy;
    c.cy = T(g.ihy2) * wx;
    c.cz = T(g.ihz2) * wx * wy;
    c.dg = T(g.beta) * wx * wy + c.cx * T(nxn) + c.cy * T(nyn) + c.cz * T(2);
    c.iv = c.ing ? T(1) / c.dg : T(0);
    if (!c.ing) c.cx = c.cy = c.cz = T(0);
}

// S_p at plane class (wz) from the LDS plane P and the z-neighbours xb, xa
template <typename T>
__device__ __forceinline__ T nbr_sum(const RCol<T>& c, T wz, const T* P, int RW, T xb, T xa) {
    const int p = c.p;
    T s = c.cx * (P[p - 1] + P[p + 1]);
    s = fma(c.cy, P[p - RW] + P[p + RW], s);
    s *= wz;
    return fma(c.cz, xb + xa, s);
}

// Runs step(n, integral_constant<R>) for n = n0 .. n1 with R = (n - n0) % 3.
template <typename F>
__device__ __forceinline__ void march3(int n0, int n1, F&& step) {
    for (int n = n0;;) {
        if (n > n1) break;
        step(n, std::integral_constant<int, 0>{});
        if (++n > n1) break;
        step(n, std::integral_constant<int, 1>{});
        if (++n > n1) break;
        step(n, std::integral_constant<int, 2>{});
        ++n;
    }
}

// ---------------------------------------------------------------- down pass
// Tile = TX x TY coarse columns; the region is the fine columns
// [2 cX0 - 3, 2 (cX0 + TX) + 1] (width 2 TX + 5): x1 on all of it, x2 one
// column in, r two columns in (the 3 x 3 footprints of the tile's coarse
// nodes), owned fine columns 2 cX0 .. 2 cX0 + 2 TX - 1.
// Pipeline at step n: A f, x1 on plane n; B x2 on n-1; C r on n-2;
// D plane sum of r on n-3 into the coarse plane (n-3)/2.
// Smoothing step in diagonal form: x + w D^-1 (f - A x) = (1 - w) x + w D^-1 (f + S).
// Columns outside the grid carry zero coefficients and zero f, so their x1,
// x2 and r come out exactly 0 (the LDS starts zeroed, so every value read is
// finite); halo columns whose stencil reaches beyond the region compute
// values that no later stage reads. x2 on the planes -1 and nz (the absent
// z-neighbours of the first and last plane) is held at zero explicitly.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_down(Geom gf, Geom gc, FTile s, const T* __restrict__ F, int64_t ldf,
                                             T* __restrict__ X, int64_t ldx, T* __restrict__ Fc, int64_t ldc,
                                             T w0, T w1) {
    using L = Lds<NT>;
    __shared__ T s1[L::SIZE];
    __shared__ T s2[L::SIZE];
    __shared__ T sr[L::SIZE];
    int tx, ty, zr, r;
    if (!ftile_item(s, tx, ty, zr, r)) return;
    const int RW = s.RW, RH = s.RH;
    const int cX0 = tx * s.TX, cY0 = ty * s.TY;
    const int cz0 = zr * s.zc, cz1 = min(gc.nz, cz0 + s.zc);
    const int nz = gf.nz;
    const int PL = gf.nx * gf.ny, PLc = gc.nx * gc.ny;
    const T* f = F + r * ldf;
    T* x = X + r * ldx;
    T* fc = Fc + r * ldc;
    for (int t = threadIdx.x; t < L::SIZE; t += NT) s1[t] = s2[t] = sr[t] = T(0);

    RCol<T> c[kCPT];
#pragma unroll
    for (int u = 0; u < kCPT; ++u) rcol_init(c[u], gf, threadIdx.x + u * NT, RW, RH, 2 * cX0 - 3, 2 * cY0 - 3, 3);
    const int ci = threadIdx.x % s.TX, cj = threadIdx.x / s.TX;
    const bool cact = (int)threadIdx.x < s.TX * s.TY && cX0 + ci < gc.nx && cY0 + cj < gc.ny;
    const int pc = (2 * ci + 3) + (2 * cj + 3) * RW;
    const int coff = cact ? (cY0 + cj) * gc.nx + (cX0 + ci) : 0;

    const int aLo = max(0, 2 * cz0 - 3), aHi = min(nz - 1, 2 * cz1 + 1);  // f, x1
    // x2 is needed on planes max(0, 2 cz0 - 2) .. min(nz - 1, 2 cz1)
    const int rLo = max(0, 2 * cz0 - 1), rHi = min(nz - 1, 2 * cz1 - 1);  // r and its plane sums
    const int oLo = 2 * cz0, oHi = min(nz - 1, 2 * cz1 - 1);              // x2 written
    const T om1 = T(1) - w1;
    const T scale = T(0.125);

    // register sets: plane n of f / x1 in set (n - aLo) % 3, x2 of plane n - 1
    // likewise; Qr: raw f loads of planes n .. n+2 (validity applied at use;
    // clamped addresses keep every load unconditional)
    T Fr[3][kCPT], Ar[3][kCPT], Br[3][kCPT], Qr[3][kCPT];
#pragma unroll
    for (int k3 = 0; k3 < 3; ++k3) {
        const T* fp = f + min(aLo + k3, aHi) * PL;
#pragma unroll
        for (int u = 0; u < kCPT; ++u) {
            Fr[k3][u] = Ar[k3][u] = Br[k3][u] = T(0);
            Qr[k3][u] = fp[c[u].off];
        }
    }
    T half = T(0), acc = T(0);
    __syncthreads();

    march3(aLo, rHi + 3, [&](int n, auto Rc) {
        constexpr int R = decltype(Rc)::value, R1 = (R + 2) % 3, R2 = (R + 1) % 3;
        // A: f and x1 = w0 D^-1 f on plane n
        {
            const T w0s = (n == 0 || n == nz - 1) ? T(2) * w0 : w0;
            T* P = L::plane(s1, n & 1);
            const T* fp = f + min(n + 3, aHi) * PL;
#pragma unroll
            for (int u = 0; u < kCPT; ++u) {
                const T raw = Qr[R][u];
                Qr[R][u] = fp[c[u].off];
                const T fv = (n <= aHi && c[u].ing) ? raw : T(0);
                Fr[R][u] = fv;
                Ar[R][u] = (w0s * c[u].iv) * fv;
                P[c[u].p] = Ar[R][u];
            }
        }
        // B: x2 on plane n - 1 (x1 of n-2, n-1, n in Ar[R2], Ar[R1], Ar[R])
        {
            const int m = n - 1;
            const bool wr = m >= oLo && m <= oHi;
            const bool bnd = m == 0 || m == nz - 1;
            const T wz = bnd ? T(0.5) : T(1);
            const T w1s = bnd ? T(2) * w1 : w1;
            const T keep = (m >= 0 && m < nz) ? T(1) : T(0);
            const T* P = L::plane(s1, m & 1);
            T* Q = L::plane(s2, m & 1);
            T* xp = x + max(m, 0) * PL;
#pragma unroll
            for (int u = 0; u < kCPT; ++u) {
                const T sn = nbr_sum(c[u], wz, P, RW, Ar[R2][u], Ar[R][u]);
                const T v = keep * fma(w1s * c[u].iv, Fr[R1][u] + sn, om1 * Ar[R1][u]);
                if (wr && c[u].own) xp[c[u].off] = v;
                Br[R][u] = v;
                Q[c[u].p] = v;
            }
        }
        // C: r = f - D x2 + S on plane n - 2 (x2 of n-3, n-2, n-1 in Br[R2],
        // Br[R1], Br[R])
        {
            const int m = n - 2;
            const bool bnd = m == 0 || m == nz - 1;
            const T wz = bnd ? T(0.5) : T(1);
            const T* P = L::plane(s2, m & 1);
            T* Rp = L::plane(sr, m & 1);
#pragma unroll
            for (int u = 0; u < kCPT; ++u) {
                const T sn = nbr_sum(c[u], wz, P, RW, Br[R2][u], Br[R][u]);
                Rp[c[u].p] = fma(-wz * c[u].dg, Br[R1][u], Fr[R2][u]) + sn;
            }
        }
        // D: in-plane full-weighting sum of r on plane n - 3; coarse plane L
        // collects s(2L-1)/2 + s(2L) + s(2L+1)/2
        {
            const int m = n - 3;
            if (cact && m >= rLo && m <= rHi) {
                const T* Rp = L::plane(sr, m & 1);
                T sum = T(0);
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy) {
                    const T wy = dy ? T(0.5) : T(1);
                    T row = T(0);
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx) row += (dx ? T(0.5) : T(1)) * Rp[pc + dy * RW + dx];
                    sum += wy * row;
                }
                const int Lc = m >> 1;
                if ((m & 1) == 0) {
                    acc = half + sum;
                    if (m + 1 >= nz && Lc >= cz0 && Lc < cz1) fc[Lc * PLc + coff] = scale * acc;
                } else {
                    if (Lc >= cz0 && Lc < cz1) fc[Lc * PLc + coff] = scale * (acc + T(0.5) * sum);
                    half = T(0.5) * sum;
                }
            }
        }
        __syncthreads();
    });
}

// ---------------------------------------------------------------- up pass
// Tile = TX x TY fine columns; region = tile + 2 columns each side: y0 on all
// of it, y1 one column in, y on the tile. The coarse correction is staged per
// coarse plane in LDS (two planes: fine plane n interpolates from coarse
// planes n/2 and, for odd n, n/2 + 1); thread t < CRW * CRH stages coarse
// column t of the region (zero outside the coarse grid).
// Pipeline at step n: A y0 on plane n; B y1 on n-1; C y on n-2.
// Columns outside the grid carry zero coefficients and zero x2, so their y0
// and y1 come out exactly 0; y1 on the planes -1 and nz is held at zero
// explicitly (see the down pass).
__device__ __forceinline__ int coarse_idx(const Geom& gc, int cidx, int L) {
    return (cidx >= 0 && L < gc.nz) ? L * (gc.nx * gc.ny) + cidx : 0;
}

template <typename T, int NT>
__global__ __launch_bounds__(NT, 4) void k_up(Geom gf, Geom gc, FTile s, const T* __restrict__ F, int64_t ldf,
                                           const T* __restrict__ X0, int64_t ldx0, const T* __restrict__ Ec,
                                           int64_t ldc, T* __restrict__ Y, int64_t ldy, T wa, T wb) {
    static_assert(kCReg <= NT, "one staged coarse column per thread");
    using L = Lds<NT>;
    __shared__ T s0[L::SIZE];
    __shared__ T s1[L::SIZE];
    __shared__ T se[2][kCReg];
    int tx, ty, zr, r;
    if (!ftile_item(s, tx, ty, zr, r)) return;
    const int RW = s.RW, RH = s.RH;
    const int gx0 = tx * s.TX, gy0 = ty * s.TY;
    const int z0 = zr * s.zc, z1 = min(gf.nz, z0 + s.zc);
    const int nz = gf.nz;
    const int PL = gf.nx * gf.ny;
    const int i0 = gx0 - 2, j0 = gy0 - 2;
    const int cI0 = i0 >> 1, cJ0 = j0 >> 1;  // floor
    const T* f = F + r * ldf;
    const T* x0 = X0 + r * ldx0;
    const T* e = Ec + r * ldc;
    T* y = Y + r * ldy;
    for (int t = threadIdx.x; t < L::SIZE; t += NT) s0[t] = s1[t] = T(0);

    // per column: staged coarse index of the lower interpolation corner and
    // the x / y weight h of the upper corner (0 on even, 1/2 on odd nodes:
    // value = lo + h (hi - lo)); fo: the f offset, 0 (a harmless address)
    // where f is not needed
    RCol<T> c[kCPT];
    int cb[kCPT], fo[kCPT];
    T hx[kCPT], hy[kCPT];
#pragma unroll
    for (int u = 0; u < kCPT; ++u) {
        const int p = threadIdx.x + u * NT;
        rcol_init(c[u], gf, p, RW, RH, i0, j0, 2);
        const int i = i0 + (p % RW), j = j0 + (p / RW);
        cb[u] = c[u].ing ? ((i >> 1) - cI0) + ((j >> 1) - cJ0) * s.CRW : 0;
        fo[u] = c[u].r1 ? c[u].off : 0;
        hx[u] = (i & 1) ? T(0.5) : T(0);
        hy[u] = (j & 1) ? T(0.5) : T(0);
    }

    const int aLo = max(0, z0 - 2), aHi = min(nz - 1, z1 + 1);  // y0
    // y1 is needed on planes max(0, z0 - 1) .. min(nz - 1, z1)
    const int cLo = z0, cHi = z1 - 1;                           // y
    const T oma = T(1) - wa, omb = T(1) - wb;

    // staged coarse column of this thread
    const int ct = threadIdx.x;
    const bool cst = ct < s.CRW * s.CRH;
    int cidx = -1;
    if (cst) {
        const int I = cI0 + ct % s.CRW, J = cJ0 + ct / s.CRW;
        if (I >= 0 && I < gc.nx && J >= 0 && J < gc.ny) cidx = J * gc.nx + I;
    }
    auto stage_now = [&](int Lc) {
        if (cst) se[Lc & 1][ct] = (cidx >= 0 && Lc < gc.nz) ? e[coarse_idx(gc, cidx, Lc)] : T(0);
    };
    stage_now(aLo >> 1);
    stage_now((aLo >> 1) + 1);
    // the coarse plane staged at the first even step, loaded now
    const int nEven = aLo + (aLo & 1);
    T cq = e[coarse_idx(gc, cidx, (nEven >> 1) + 1)];
    __syncthreads();

    // register sets as in the down pass: y0, f of plane n and y1 of plane
    // n - 1 in set (n - aLo) % 3; XQ, FQ: raw loads of planes n .. n+2
    T Pr[3][kCPT], Fr[3][kCPT], Yr[3][kCPT], XQ[3][kCPT], FQ[3][kCPT];
#pragma unroll
    for (int k3 = 0; k3 < 3; ++k3) {
        const T* xp = x0 + min(aLo + k3, aHi) * PL;
        const T* fp = f + min(aLo + k3, aHi) * PL;
#pragma unroll
        for (int u = 0; u < kCPT; ++u) {
            Pr[k3][u] = Fr[k3][u] = Yr[k3][u] = T(0);
            XQ[k3][u] = xp[c[u].off];
            FQ[k3][u] = fp[fo[u]];
        }
    }

    march3(aLo, cHi + 2, [&](int n, auto Rc) {
        constexpr int R = decltype(Rc)::value, R1 = (R + 2) % 3, R2 = (R + 1) % 3;
        // the coarse plane that step n + 1 adds (odd n + 1 needs n/2 + 1), and
        // the load of the one the next even step adds
        if (!(n & 1)) {
            const int Lc = (n >> 1) + 1;
            if (n + 1 <= aHi && cst) se[Lc & 1][ct] = (cidx >= 0 && Lc < gc.nz) ? cq : T(0);
            cq = e[coarse_idx(gc, cidx, Lc + 1)];
        }
        // A: y0 = x2 + P e on plane n
        {
            const bool in = n <= aHi;
            const int Lc = n >> 1;
            const T* E0 = se[Lc & 1];
            const T* E1 = se[(Lc + 1) & 1];
            T* P = L::plane(s0, n & 1);
            const int CW = s.CRW;
            const T* xp = x0 + min(n + 3, aHi) * PL;
            const T* fp = f + min(n + 3, aHi) * PL;
#pragma unroll
            for (int u = 0; u < kCPT; ++u) {
                const T xr = XQ[R][u], fr = FQ[R][u];
                XQ[R][u] = xp[c[u].off];
                FQ[R][u] = fp[fo[u]];
                const int b = cb[u];
                auto bilin = [&](const T* E) {
                    const T lo = fma(hx[u], E[b + 1] - E[b], E[b]);
                    const T hi = fma(hx[u], E[b + CW + 1] - E[b + CW], E[b + CW]);
                    return fma(hy[u], hi - lo, lo);
                };
                T pe = bilin(E0);
                if (n & 1) pe = T(0.5) * (pe + bilin(E1));
                const T v = (in && c[u].ing) ? xr + pe : T(0);
                Pr[R][u] = v;
                Fr[R][u] = fr;
                P[c[u].p] = v;
            }
        }
        // B: y1 on plane n - 1 (y0 of n-2, n-1, n in Pr[R2], Pr[R1], Pr[R])
        {
            const int m = n - 1;
            const bool bnd = m == 0 || m == nz - 1;
            const T wz = bnd ? T(0.5) : T(1);
            const T was = bnd ? T(2) * wa : wa;
            const T keep = (m >= 0 && m < nz) ? T(1) : T(0);
            const T* P = L::plane(s0, m & 1);
            T* Q = L::plane(s1, m & 1);
#pragma unroll
            for (int u = 0; u < kCPT; ++u) {
                const T sn = nbr_sum(c[u], wz, P, RW, Pr[R2][u], Pr[R][u]);
                const T v = keep * fma(was * c[u].iv, Fr[R1][u] + sn, oma * Pr[R1][u]);
                Yr[R][u] = v;
                Q[c[u].p] = v;
            }
        }
        // C: y on plane n - 2 (y1 of n-3, n-2, n-1 in Yr[R2], Yr[R1], Yr[R])
        {
            const int m = n - 2;
            const bool in = m >= cLo && m <= cHi;
            const bool bnd = m == 0 || m == nz - 1;
            const T wz = bnd ? T(0.5) : T(1);
            const T wbs = bnd ? T(2) * wb : wb;
            const T* P = L::plane(s1, m & 1);
            T* yp = y + max(m, 0) * PL;
#pragma unroll
            for (int u = 0; u < kCPT; ++u) {
                const T sn = nbr_sum(c[u], wz, P, RW, Yr[R2][u], Yr[R][u]);
                const T v = fma(wbs * c[u].iv, Fr[R2][u] + sn, omb * Yr[R1][u]);
                if (in && c[u].own) yp[c[u].off] = v;
            }
        }
        __syncthreads();
    });
}

// Tile shape: the region must fit 2 NT columns; the cost of a plane is
// (work-groups) x (fixed cost of one group + 128-byte lines its region rows
// touch), so wide rows (coalesced loads) and few groups both count.
FTile plan_tiles(int nx, int ny, int nzt, int k, bool down, int zmin, int es, int nt_threads) {
    const int reg = nt_threads * kCPT;
    FTile best{};
    int64_t best_cost = -1, best_nt = 0;
    for (int TX = 1; TX <= nx; ++TX) {
        for (int TY = 1; TY <= ny; ++TY) {
            const int RW = down ? 2 * TX + 5 : TX + 4;
            const int RH = down ? 2 * TY + 5 : TY + 4;
            if (RW * RH > reg) break;
            if (RW > kPad) break;
            if (down && TX * TY > nt_threads) break;
            const int CRW = (RW + 1) / 2 + 2, CRH = (RH + 1) / 2 + 2;
            if (!down && CRW * CRH > kCReg) break;
            const int64_t nt = cdiv(nx, TX) * cdiv(ny, TY);
            const int64_t cost = nt * ((int64_t)reg * 8 + (int64_t)RH * (cdiv(RW * es, 128) + 1) * 128);
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
    const FTile s = plan_tiles(gc.nx, gc.ny, gc.nz, k, true, 4, (int)sizeof(T), kDownThreads);
    hipLaunchKernelGGL((k_down<T, kDownThreads>), dim3(ftile_grid(s)), dim3(kDownThreads), 0, st, gf, gc, s, F, ldf,
                       X, ldx, Fc, ldc, T(w0), T(w1));
    H1W_LAUNCHED();
}

template <typename T>
void launch_vup(hipStream_t st, const Geom& gf, const Geom& gc, int k, const T* F, int64_t ldf, const T* X0,
                int64_t ldx0, const T* Ec, int64_t ldc, T* Y, int64_t ldy, double wa, double wb) {
    if (k <= 0) return;
    require(fused_levels_ok(gf, gc), "internal: fused pass on non-nested levels");
    const FTile s = plan_tiles(gf.nx, gf.ny, gf.nz, k, false, 8, (int)sizeof(T), kUpThreads);
    hipLaunchKernelGGL((k_up<T, kUpThreads>), dim3(ftile_grid(s)), dim3(kUpThreads), 0, st, gf, gc, s, F, ldf, X0,
                       ldx0, Ec, ldc, Y, ldy, T(wa), T(wb));
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
