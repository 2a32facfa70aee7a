// ERT forward operator, its multigrid hierarchy and the pole-pole
// sensitivities (Section 4: eq. (model), eqs. (ert_qoi2), (ert_qoi_scaling)
// and (ert_qoi_derivative) with m = log sigma) on a structured 3D grid.
//
// Operator: vertex-centred finite volumes. Edge (p, q) along axis d carries
// c_pq = (sigma_p + sigma_q)/2 * g_pq with g_pq = (dual-face area)/h_d, the
// area being the product of the other two spacings, each halved when the edge
// lies in a boundary face normal to that axis. Per level we store, for every
// node p, the diagonal D_p = sum of the conductances of all its edges (1 on
// a Dirichlet node) and the couplings cx_p, cy_p, cz_p of its edges to p+x,
// p+y, p+z (0 when either end is a Dirichlet node or the edge leaves the
// grid), so that (A u)_p = D_p u_p - sum_q c_pq u_q is symmetric and u stays
// exactly 0 on the Dirichlet nodes.
//
// Multigrid: coarse conductivities are full-weighting averages of the finer
// level's, recomputed at every conductivity update; each level is
// rediscretised; restriction is P^T (the finite-volume scaling of the
// operator is h^(d-2), so no 2^-d factor) with coarse Dirichlet nodes set to
// zero; the coarsest level (at most kErtCoarseMax nodes) is inverted densely
// by Gauss-Jordan elimination in LDS by one work-group.
//
// Sensitivities: for node j and the six edges (j, q) around it,
// J[i, j] = -k_i sum_e w_e (u_a(j) - u_a(q)) (u_b(j) - u_b(q)),
// w_e = sigma_j g_e / 2 (the derivative of c_jq with respect to m_j), for
// measurement i = (a, b). A work-group stages the edge differences of every
// source field for TN consecutive nodes in LDS and then writes TN consecutive
// entries of each row of J (coalesced), or accumulates sum_i gbar_i J[i, j];
// the weighted differences of the first electrode stay in registers across
// consecutive pairs that share it (pairs listed with a fixed first electrode).
#include <algorithm>
#include <cmath>

#include "context.h"

namespace h1w {

namespace {

struct EG {  // level geometry for the ERT kernels
    int nx, ny, nz;
    int64_t N;
    double hx, hy, hz;
    unsigned mask;
};

EG make_eg(const Geom& g, unsigned mask) {
    return EG{g.nx, g.ny, g.nz, g.N, 1.0 / (g.nx - 1), 1.0 / (g.ny - 1), 1.0 / (g.nz - 1), mask};
}

__device__ __forceinline__ bool on_dirichlet(const EG& g, int i, int j, int l) {
    return ((g.mask & 1u) && i == 0) || ((g.mask & 2u) && i == g.nx - 1) || ((g.mask & 4u) && j == 0) ||
           ((g.mask & 8u) && j == g.ny - 1) || ((g.mask & 16u) && l == 0) || ((g.mask & 32u) && l == g.nz - 1);
}

__device__ __forceinline__ double endw(int i, int n) { return (i == 0 || i == n - 1) ? 0.5 : 1.0; }

// (dual-face area)/h of the x, y and z edges at node (i, j, l)
__device__ __forceinline__ double geom_x(const EG& g, int j, int l) {
    return g.hy * g.hz / g.hx * endw(j, g.ny) * endw(l, g.nz);
}
__device__ __forceinline__ double geom_y(const EG& g, int i, int l) {
    return g.hx * g.hz / g.hy * endw(i, g.nx) * endw(l, g.nz);
}
__device__ __forceinline__ double geom_z(const EG& g, int i, int j) {
    return g.hx * g.hy / g.hz * endw(i, g.nx) * endw(j, g.ny);
}

// node index -> (i, j, l) with two 32-bit divisions (N < 2^31)
__device__ __forceinline__ void split(const EG& g, int64_t p, int& i, int& j, int& l) {
    const unsigned q = (unsigned)p;
    const unsigned t = q / (unsigned)g.nx;
    i = (int)(q - t * (unsigned)g.nx);
    const unsigned z = t / (unsigned)g.ny;
    j = (int)(t - z * (unsigned)g.ny);
    l = (int)z;
}

__global__ __launch_bounds__(kBlock) void k_ert_sigma(int64_t N, const double* __restrict__ logsig,
                                                      double* __restrict__ sig, int* __restrict__ flag) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= N) return;
    const double s = exp(logsig[p]);
    sig[p] = s;
    if (!(s > 0.0 && s <= 1.79e308)) flag[0] = 1;
}

// coarse node (I, J, L) <- weighted mean of the fine nodes around (2I, 2J, 2L)
// with weights prod_d (1 or 1/2), normalised by the weights inside the grid
__global__ __launch_bounds__(kBlock) void k_ert_coarsen(EG gf, EG gc, const double* __restrict__ sf,
                                                        double* __restrict__ sc) {
    const int64_t P = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (P >= gc.N) return;
    int I, J, L;
    split(gc, P, I, J, L);
    double acc = 0.0, ws = 0.0;
    for (int c = -1; c <= 1; ++c) {
        const int l = 2 * L + c;
        if (l < 0 || l >= gf.nz) continue;
        for (int b = -1; b <= 1; ++b) {
            const int j = 2 * J + b;
            if (j < 0 || j >= gf.ny) continue;
            for (int a = -1; a <= 1; ++a) {
                const int i = 2 * I + a;
                if (i < 0 || i >= gf.nx) continue;
                const double w = (a ? 0.5 : 1.0) * (b ? 0.5 : 1.0) * (c ? 0.5 : 1.0);
                acc += w * sf[i + (int64_t)gf.nx * (j + (int64_t)gf.ny * l)];
                ws += w;
            }
        }
    }
    sc[P] = acc / ws;
}

__global__ __launch_bounds__(kBlock) void k_ert_coeffs(EG g, const double* __restrict__ sig, double* __restrict__ D,
                                                       double* __restrict__ cx, double* __restrict__ cy,
                                                       double* __restrict__ cz) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= g.N) return;
    int i, j, l;
    split(g, p, i, j, l);
    const int64_t PX = 1, PY = g.nx, PZ = (int64_t)g.nx * g.ny;
    const bool dp = on_dirichlet(g, i, j, l);
    const double s0 = sig[p];
    double dsum = 0.0, vx = 0.0, vy = 0.0, vz = 0.0;
    const double gx = geom_x(g, j, l), gy = geom_y(g, i, l), gz = geom_z(g, i, j);
    if (i < g.nx - 1) {
        const double c = 0.5 * (s0 + sig[p + PX]) * gx;
        dsum += c;
        vx = (dp || on_dirichlet(g, i + 1, j, l)) ? 0.0 : c;
    }
    if (i > 0) dsum += 0.5 * (s0 + sig[p - PX]) * gx;
    if (j < g.ny - 1) {
        const double c = 0.5 * (s0 + sig[p + PY]) * gy;
        dsum += c;
        vy = (dp || on_dirichlet(g, i, j + 1, l)) ? 0.0 : c;
    }
    if (j > 0) dsum += 0.5 * (s0 + sig[p - PY]) * gy;
    if (l < g.nz - 1) {
        const double c = 0.5 * (s0 + sig[p + PZ]) * gz;
        dsum += c;
        vz = (dp || on_dirichlet(g, i, j, l + 1)) ? 0.0 : c;
    }
    if (l > 0) dsum += 0.5 * (s0 + sig[p - PZ]) * gz;
    D[p] = dp ? 1.0 : dsum;
    cx[p] = vx;
    cy[p] = vy;
    cz[p] = vz;
}

enum { kErtApply = 0, kErtResidual = 1, kErtSmooth = 2, kErtFirst = 3 };

// One pass over a batch: APPLY Y = A X; RESIDUAL Y = F - A X;
// SMOOTH Y = X + w D^-1 (F - A X); FIRST Y = w D^-1 F.
// A thread owns one in-plane position and R right-hand sides and marches up a
// chunk of zc planes, keeping x on the planes below and at the current one in
// registers (each x is loaded once per chunk, plus one plane below it); the
// in-plane neighbours come from cache. Work items (in-plane tile of kBlock
// positions, z-chunk, group of R right-hand sides) are numbered with the
// right-hand-side group fastest and dealt to the 8 XCDs in contiguous
// ranges, so that the groups sharing a tile's coefficients, and neighbouring
// tiles, run behind the same L2. All loads are unconditional so that they
// issue together: a neighbour outside the grid is replaced by a clamped
// in-range index whose coupling is zero (the coupling of an edge that leaves
// the grid is stored as 0, and so is that of the node before the first node
// of a row or plane), and right-hand sides beyond k read row k - 1 and store
// nothing.
constexpr int kErtZChunk = 16;
constexpr int kErtRhs = 4;
struct MarchGrid {
    int ntile, nzc, ngrp, zc, total;
};
template <int MODE, int R>
__global__ __launch_bounds__(kBlock) void k_ert_march(EG g, ErtLevel c, int k, MarchGrid mg,
                                                      const double* __restrict__ F, int64_t ldf,
                                                      const double* __restrict__ X, int64_t ldx,
                                                      double* __restrict__ Y, int64_t ldy, double w) {
    const int bid = blockIdx.x;
    const int per = (mg.total + 7) >> 3;
    const int wi = (bid & 7) * per + (bid >> 3);
    if (wi >= mg.total) return;
    const int grp = wi % mg.ngrp;
    const int rest = wi / mg.ngrp;
    const int tile = rest % mg.ntile;
    const int zr = rest / mg.ntile;
    const int PL = g.nx * g.ny;
    const int q = tile * kBlock + threadIdx.x;
    if (q >= PL) return;
    const int r0 = grp * R;
    const int nr = min(R, k - r0);
    const int z0 = zr * mg.zc, z1 = min(g.nz, z0 + mg.zc);
    const int64_t last = g.N - 1;
    const double* xr[R];
    const double* fr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t row = min(r0 + r, k - 1);
        xr[r] = X + row * ldx;
        fr[r] = F + row * ldf;
    }
    double xb[R], x0[R];
    if (MODE != kErtFirst) {
        const int64_t p0 = (int64_t)z0 * PL + q;
        const int64_t pb = max(p0 - PL, (int64_t)0);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            xb[r] = xr[r][pb];
            x0[r] = xr[r][p0];
        }
    }
    for (int l = z0; l < z1; ++l) {
        const int64_t p = (int64_t)l * PL + q;
        const double d = c.D[p];
        if (MODE == kErtFirst) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r < nr) Y[(int64_t)(r0 + r) * ldy + p] = w * fr[r][p] / d;
            continue;
        }
        const int64_t pxm = max(p - 1, (int64_t)0), pym = max(p - g.nx, (int64_t)0);
        const int64_t pzm = max(p - PL, (int64_t)0);
        const int64_t pxp = min(p + 1, last), pyp = min(p + g.nx, last), pzp = min(p + PL, last);
        const double cxp = c.cx[p], cxm = c.cx[pxm] * (p > 0);
        const double cyp = c.cy[p], cym = c.cy[pym] * (p >= g.nx);
        const double czp = c.cz[p], czm = c.cz[pzm] * (p >= PL);
        double v[R], xa[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double* x = xr[r];
            xa[r] = x[pzp];
            const double s = ((cxp * x[pxp] + cxm * x[pxm]) + (cyp * x[pyp] + cym * x[pym])) +
                             (czp * xa[r] + czm * xb[r]);
            const double ax = d * x0[r] - s;
            if (MODE == kErtApply)
                v[r] = ax;
            else if (MODE == kErtResidual)
                v[r] = fr[r][p] - ax;
            else
                v[r] = x0[r] + w * (fr[r][p] - ax) / d;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r < nr) Y[(int64_t)(r0 + r) * ldy + p] = v[r];
            xb[r] = x0[r];
            x0[r] = xa[r];
        }
    }
}

// Fc = P^T R on the coarse nodes that are not on a Dirichlet face (0 there).
// Work items (block of coarse nodes, row of R) go to the 8 XCDs in
// contiguous ranges (block ids go round-robin over the XCDs): the fine plane
// that two neighbouring coarse planes share is then read into one L2.
__global__ __launch_bounds__(kBlock) void k_ert_restrict(EG gf, EG gc, int nblk, int total,
                                                         const double* __restrict__ R, int64_t ldr,
                                                         double* __restrict__ Fc, int64_t ldc) {
    const int per = (total + 7) / 8;
    const int u = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (u >= total) return;
    const int64_t r = u / nblk;
    const int64_t P = (u - r * nblk) * (int64_t)kBlock + threadIdx.x;
    if (P >= gc.N) return;
    int I, J, L;
    split(gc, P, I, J, L);
    double acc = 0.0;
    if (!on_dirichlet(gc, I, J, L)) {
        const double* rr = R + r * ldr;
        for (int c = -1; c <= 1; ++c) {
            const int l = 2 * L + c;
            if (l < 0 || l >= gf.nz) continue;
            for (int b = -1; b <= 1; ++b) {
                const int j = 2 * J + b;
                if (j < 0 || j >= gf.ny) continue;
                double row = 0.0;
                for (int a = -1; a <= 1; ++a) {
                    const int i = 2 * I + a;
                    if (i < 0 || i >= gf.nx) continue;
                    row += (a ? 0.5 : 1.0) * rr[i + (int64_t)gf.nx * (j + (int64_t)gf.ny * l)];
                }
                acc += ((b ? 0.5 : 1.0) * (c ? 0.5 : 1.0)) * row;
            }
        }
    }
    Fc[r * ldc + P] = acc;
}

// Dense inverse of the coarsest operator by Gauss-Jordan elimination without
// pivoting (the operator is symmetric positive definite), in LDS, one
// work-group. Writes the symmetrised inverse; flag[0] = 1 on a non-positive
// or non-finite pivot.
constexpr int kErtCoarseMax = 128;
constexpr int kGJThreads = 1024;
__global__ __launch_bounds__(kGJThreads) void k_ert_coarse_inverse(EG g, ErtLevel c, double* __restrict__ Cinv,
                                                                   int* __restrict__ flag) {
    __shared__ double a[kErtCoarseMax * kErtCoarseMax];
    __shared__ double prow[kErtCoarseMax], pcol[kErtCoarseMax];
    const int n = (int)g.N;
    const int tid = threadIdx.x;
    for (int t = tid; t < n * n; t += kGJThreads) a[t] = 0.0;
    __syncthreads();
    const int PY = g.nx, PZ = g.nx * g.ny;
    for (int p = tid; p < n; p += kGJThreads) {
        int i, j, l;
        split(g, p, i, j, l);
        double* row = a + p * n;
        row[p] = c.D[p];
        if (i < g.nx - 1) row[p + 1] = -c.cx[p];
        if (i > 0) row[p - 1] = -c.cx[p - 1];
        if (j < g.ny - 1) row[p + PY] = -c.cy[p];
        if (j > 0) row[p - PY] = -c.cy[p - PY];
        if (l < g.nz - 1) row[p + PZ] = -c.cz[p];
        if (l > 0) row[p - PZ] = -c.cz[p - PZ];
    }
    __syncthreads();
    // rows go to the waves, columns to the lanes (no index division)
    const int lane = tid & 63, wv = tid >> 6;
    constexpr int kWaves = kGJThreads / 64;
    for (int k = 0; k < n; ++k) {
        double piv = a[k * n + k];
        if (!(piv > 0.0 && piv <= 1.79e308)) {
            if (tid == 0) flag[1] = 1;
            piv = 1.0;
        }
        const double inv = 1.0 / piv;
        for (int t = tid; t < n; t += kGJThreads) {
            prow[t] = a[k * n + t] * inv;
            pcol[t] = a[t * n + k];
        }
        __syncthreads();
        for (int i = wv; i < n; i += kWaves) {
            const double ci = pcol[i];
            double* row = a + i * n;
            for (int j = lane; j < n; j += 64) {
                if (i == k)
                    row[j] = (j == k) ? inv : prow[j];
                else
                    row[j] = (j == k) ? -ci * inv : row[j] - ci * prow[j];
            }
        }
        __syncthreads();
    }
    for (int i = wv; i < n; i += kWaves)
        for (int j = lane; j < n; j += 64) Cinv[i * n + j] = 0.5 * (a[i * n + j] + a[j * n + i]);
}

__global__ __launch_bounds__(kBlock) void k_ert_unit_loads(int64_t N, const int* __restrict__ src,
                                                           double* __restrict__ F, int64_t ldf) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= N) return;
    const int r = blockIdx.y;
    F[(int64_t)r * ldf + p] = (p == (int64_t)src[r]) ? 1.0 : 0.0;
}

// k_i = 2 pi |x_a - x_b| from the node coordinates of the two electrodes
__global__ __launch_bounds__(kBlock) void k_ert_kgeo(EG g, int n_meas, const int* __restrict__ pair,
                                                     const int* __restrict__ src, double* __restrict__ k) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n_meas) return;
    int ia, ja, la, ib, jb, lb;
    split(g, src[pair[2 * t]], ia, ja, la);
    split(g, src[pair[2 * t + 1]], ib, jb, lb);
    const double dx = (ia - ib) * g.hx, dy = (ja - jb) * g.hy, dz = (la - lb) * g.hz;
    k[t] = 2.0 * 3.14159265358979323846 * sqrt(dx * dx + dy * dy + dz * dz);
}

__global__ __launch_bounds__(kBlock) void k_ert_meas(int n_meas, const int* __restrict__ pair,
                                                     const int* __restrict__ src, const double* __restrict__ k,
                                                     const double* __restrict__ U, int64_t ldu,
                                                     double* __restrict__ gout) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n_meas) return;
    const int a = pair[2 * t], b = pair[2 * t + 1];
    gout[t] = k[t] * U[(int64_t)a * ldu + src[b]];
}

// Pairwise-gradient sensitivities, narrow form (33..64 sources). TN nodes per
// work-group, NS sources at most (NS * TN = 1024); the 6 x n_src x TN edge
// differences sit in LDS.
constexpr int kSensThreads = 256;
template <int TN, bool VJP>
__global__ __launch_bounds__(kSensThreads) void k_ert_sens(EG g, const double* __restrict__ sig, int n_src,
                                                           const double* __restrict__ U, int64_t ldu, int n_meas,
                                                           const int* __restrict__ pair,
                                                           const double* __restrict__ k, double* __restrict__ J,
                                                           int64_t ldj, const double* __restrict__ gbar,
                                                           double* __restrict__ grad) {
    constexpr int NS = 1024 / TN;
    constexpr int G = kSensThreads / TN;  // measurement groups
    __shared__ double dl[6 * NS * TN];
    __shared__ double we[6 * TN];
    __shared__ double red[VJP ? G * TN : 1];
    const int tid = threadIdx.x;
    // node tiles in contiguous ranges per XCD (block ids go round-robin over
    // the 8 XCDs), so the neighbour rows and planes a tile reads were mostly
    // brought into the same L2 by the tiles next to it
    const int ntile = (int)((g.N + TN - 1) / TN);
    const int per = (ntile + 7) >> 3;
    const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (tile >= ntile) return;
    const int64_t j0 = (int64_t)tile * TN;
    const int64_t PY = g.nx, PZ = (int64_t)g.nx * g.ny;

    // edge differences of every field at the TN nodes (the seven loads of an
    // item issued together, as in the wide form)
    for (int q = tid; q < n_src * TN; q += kSensThreads) {
        const int s = q / TN, t = q - s * TN;
        const int64_t p = j0 + t;
        const bool live = p < g.N;
        int i = 0, j = 0, l = 0;
        if (live) split(g, p, i, j, l);
        const bool has[6] = {live && i < g.nx - 1, live && i > 0, live && j < g.ny - 1,
                             live && j > 0,        live && l < g.nz - 1, live && l > 0};
        const int64_t pc = live ? p : 0;
        const int64_t nb[6] = {has[0] ? p + 1 : pc,  has[1] ? p - 1 : pc,  has[2] ? p + PY : pc,
                               has[3] ? p - PY : pc, has[4] ? p + PZ : pc, has[5] ? p - PZ : pc};
        const double* u = U + (int64_t)s * ldu;
        double un[6];
        const double u0 = u[pc];
#pragma unroll
        for (int e = 0; e < 6; ++e) un[e] = u[nb[e]];
#pragma unroll
        for (int e = 0; e < 6; ++e) dl[(e * NS + s) * TN + t] = has[e] ? u0 - un[e] : 0.0;
    }
    if (tid < TN) {
        const int64_t p = j0 + tid;
        double w[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (p < g.N) {
            int i, j, l;
            split(g, p, i, j, l);
            const double hs = 0.5 * sig[p];
            const double gx = hs * geom_x(g, j, l), gy = hs * geom_y(g, i, l), gz = hs * geom_z(g, i, j);
            if (i < g.nx - 1) w[0] = gx;
            if (i > 0) w[1] = gx;
            if (j < g.ny - 1) w[2] = gy;
            if (j > 0) w[3] = gy;
            if (l < g.nz - 1) w[4] = gz;
            if (l > 0) w[5] = gz;
        }
#pragma unroll
        for (int e = 0; e < 6; ++e) we[e * TN + tid] = w[e];
    }
    __syncthreads();

    const int t = tid % TN, grp = tid / TN;
    const int64_t p = j0 + t;
    double w[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) w[e] = we[e * TN + t];
    double acc_all = 0.0;
    // each group takes a contiguous range of measurements; w_e (u_a(j) - u_a(q))
    // is kept in registers while consecutive pairs share their first electrode
    const int mper = (n_meas + G - 1) / G;
    const int i0 = grp * mper, i1 = min(n_meas, i0 + mper);
    int a_cur = -1;
    double wa[6];
    // the pair and factor of the next measurement are loaded one iteration ahead
    int a_nx = 0, b_nx = 0;
    double k_nx = 0.0;
    if (i0 < i1) {
        a_nx = pair[2 * i0];
        b_nx = pair[2 * i0 + 1];
        k_nx = k[i0];
    }
    for (int i = i0; i < i1; ++i) {
        const int a = a_nx, b = b_nx;
        const double ki = k_nx;
        if (i + 1 < i1) {
            a_nx = pair[2 * i + 2];
            b_nx = pair[2 * i + 3];
            k_nx = k[i + 1];
        }
        if (a != a_cur) {
#pragma unroll
            for (int e = 0; e < 6; ++e) wa[e] = w[e] * dl[(e * NS + a) * TN + t];
            a_cur = a;
        }
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e < 6; ++e) acc += wa[e] * dl[(e * NS + b) * TN + t];
        if (VJP) {
            acc_all += gbar[i] * ki * acc;
        } else if (p < g.N) {
            J[(int64_t)i * ldj + p] = -ki * acc;
        }
    }
    if (VJP) {
        red[grp * TN + t] = acc_all;
        __syncthreads();
        if (tid < TN && p < g.N) {
            double s = 0.0;
            for (int q = 0; q < G; ++q) s += red[q * TN + tid];
            grad[p] = -s;
        }
    }
}

// Pairwise-gradient sensitivities, wide form (n_src <= NS, NS = 16 or 32):
// a work-group of kSensWaves waves owns 64 consecutive nodes, one per lane,
// and the 6 x NS x 64 edge differences of its nodes sit in LDS. Every wave
// takes a contiguous range of measurements, so the measurement index, the
// electrode pair and k_i are wave-uniform (scalar loads, no divergent
// branches), and each store of J writes one 512-byte run of a row.
constexpr int kSensWaves = 16;
constexpr int kSensBatch = 4;  // measurements whose sums are formed before their stores
template <int NS, bool VJP>
__global__ __launch_bounds__(64 * kSensWaves) void k_ert_sens_wide(EG g, const double* __restrict__ sig, int n_src,
                                                                   const double* __restrict__ U, int64_t ldu,
                                                                   int n_meas, const int* __restrict__ pair,
                                                                   const double* __restrict__ k,
                                                                   double* __restrict__ J, int64_t ldj,
                                                                   const double* __restrict__ gbar,
                                                                   double* __restrict__ grad) {
    __shared__ double dl[6 * NS * 64];
    __shared__ double red[VJP ? kSensWaves * 64 : 1];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // node tiles in contiguous ranges per XCD (block ids go round-robin over
    // the 8 XCDs): the neighbour rows and planes of a tile were mostly
    // brought into the same L2 by the tiles next to it
    const int ntile = (int)((g.N + 63) / 64);
    const int per = (ntile + 7) >> 3;
    const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (tile >= ntile) return;
    const int64_t p = (int64_t)tile * 64 + lane;
    const bool live = p < g.N;
    const int64_t PY = g.nx, PZ = (int64_t)g.nx * g.ny;
    int i = 0, j = 0, l = 0;
    if (live) split(g, p, i, j, l);

    // edge differences of the fields at the lane's node: wave w takes
    // sources w, w + kSensWaves, ... The seven loads of a source are issued
    // together (an absent neighbour's address falls back to the node itself,
    // and its difference is set to 0), not one conditional load at a time.
    const bool has[6] = {live && i < g.nx - 1, live && i > 0, live && j < g.ny - 1,
                         live && j > 0,        live && l < g.nz - 1, live && l > 0};
    const int64_t pc = live ? p : 0;
    const int64_t nb[6] = {has[0] ? p + 1 : pc,  has[1] ? p - 1 : pc,  has[2] ? p + PY : pc,
                           has[3] ? p - PY : pc, has[4] ? p + PZ : pc, has[5] ? p - PZ : pc};
    for (int s = wave; s < n_src; s += kSensWaves) {
        const double* u = U + (int64_t)s * ldu;
        double un[6];
        const double u0 = u[pc];
#pragma unroll
        for (int e = 0; e < 6; ++e) un[e] = u[nb[e]];
#pragma unroll
        for (int e = 0; e < 6; ++e) dl[(e * NS + s) * 64 + lane] = has[e] ? u0 - un[e] : 0.0;
    }
    // edge weights of the lane's node (half its conductivity times the
    // face-over-length factor of each incident edge)
    double w[6];
    {
        const double hs = 0.5 * sig[pc];
        const double gx = hs * geom_x(g, j, l), gy = hs * geom_y(g, i, l), gz = hs * geom_z(g, i, j);
#pragma unroll
        for (int e = 0; e < 6; ++e) w[e] = has[e] ? (e < 2 ? gx : (e < 4 ? gy : gz)) : 0.0;
    }
    __syncthreads();

    const int mper = (n_meas + kSensWaves - 1) / kSensWaves;
    const int i0 = wave * mper, i1 = min(n_meas, i0 + mper);
    int a_cur = -1;
    double wa[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double acc_all = 0.0;
    // sum over the edges of w_e (u_a(p) - u_a(q)) (u_b(p) - u_b(q)) for
    // measurement (a, b); w_e (u_a(p) - u_a(q)) is kept while a repeats
    auto meas = [&](int a, int b) {
        if (a != a_cur) {  // wave-uniform
#pragma unroll
            for (int e = 0; e < 6; ++e) wa[e] = w[e] * dl[(e * NS + a) * 64 + lane];
            a_cur = a;
        }
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e < 6; ++e) acc += wa[e] * dl[(e * NS + b) * 64 + lane];
        return acc;
    };
    int ib = i0;
    // whole batches: the sums first, then their stores back to back, so that
    // several 512-byte runs of J are in flight per wave
    for (; ib + kSensBatch <= i1; ib += kSensBatch) {
        int qa[kSensBatch], qb[kSensBatch];
        double qk[kSensBatch], acc[kSensBatch];
#pragma unroll
        for (int u = 0; u < kSensBatch; ++u) {
            qa[u] = pair[2 * (ib + u)];
            qb[u] = pair[2 * (ib + u) + 1];
            qk[u] = k[ib + u];
        }
#pragma unroll
        for (int u = 0; u < kSensBatch; ++u) acc[u] = meas(qa[u], qb[u]);
        if (VJP) {
#pragma unroll
            for (int u = 0; u < kSensBatch; ++u) acc_all += gbar[ib + u] * qk[u] * acc[u];
        } else if (live) {
#pragma unroll
            for (int u = 0; u < kSensBatch; ++u) J[(int64_t)(ib + u) * ldj + p] = -qk[u] * acc[u];
        }
    }
    for (; ib < i1; ++ib) {
        const double acc = meas(pair[2 * ib], pair[2 * ib + 1]);
        if (VJP)
            acc_all += gbar[ib] * k[ib] * acc;
        else if (live)
            J[(int64_t)ib * ldj + p] = -k[ib] * acc;
    }
    if (VJP) {
        red[wave * 64 + lane] = acc_all;
        __syncthreads();
        if (wave == 0 && live) {
            double s = 0.0;
            for (int q = 0; q < kSensWaves; ++q) s += red[q * 64 + lane];
            grad[p] = -s;
        }
    }
}

void launch_step(hipStream_t s, int mode, const EG& g, const ErtLevel& c, int k, const double* F, int64_t ldf,
                 const double* X, int64_t ldx, double* Y, int64_t ldy, double w) {
    if (k <= 0) return;
    MarchGrid mg{};
    mg.ntile = (int)cdiv((int64_t)g.nx * g.ny, kBlock);
    mg.ngrp = (int)cdiv(k, kErtRhs);
    // planes per work item: as many as keep >= ~2048 work-groups in the launch
    const int64_t base = (int64_t)mg.ntile * mg.ngrp;
    mg.zc = (int)std::clamp<int64_t>(base * g.nz / 2048, 1, kErtZChunk);
    mg.nzc = (int)cdiv(g.nz, mg.zc);
    require(base * mg.nzc < (int64_t(1) << 31), "ERT launch too large");
    mg.total = (int)(base * mg.nzc);
    // 8 equal ranges of items, one per XCD (block ids go round-robin over the XCDs)
    const dim3 grid((unsigned)(8 * cdiv(mg.total, 8)));
    switch (mode) {
        case kErtApply:
            hipLaunchKernelGGL((k_ert_march<kErtApply, kErtRhs>), grid, dim3(kBlock), 0, s, g, c, k, mg, F, ldf, X,
                               ldx, Y, ldy, w);
            break;
        case kErtResidual:
            hipLaunchKernelGGL((k_ert_march<kErtResidual, kErtRhs>), grid, dim3(kBlock), 0, s, g, c, k, mg, F, ldf,
                               X, ldx, Y, ldy, w);
            break;
        case kErtSmooth:
            hipLaunchKernelGGL((k_ert_march<kErtSmooth, kErtRhs>), grid, dim3(kBlock), 0, s, g, c, k, mg, F, ldf, X,
                               ldx, Y, ldy, w);
            break;
        default:
            hipLaunchKernelGGL((k_ert_march<kErtFirst, kErtRhs>), grid, dim3(kBlock), 0, s, g, c, k, mg, F, ldf, X,
                               ldx, Y, ldy, w);
    }
    H1W_LAUNCHED();
}

}  // namespace

// ============================================================ context side

ErtLevel Ctx::ert_level(int l) const {
    double* b = ecoef.as<double>() + eoff[l];
    const int64_t P = pitch[l];
    return ErtLevel{b, b + P, b + 2 * P, b + 3 * P, b + 4 * P};
}

// host-only checks of an ERT description (before any device call)
void Ctx::ert_validate() {
    require(dim == 3, "ERT contexts are 3D");
    require(d.precision == H1W_FP64, "ERT contexts are FP64");
    require(d.flags == 0, "flags must be 0 for an ERT context");
    require(std::isfinite(d.beta), "beta must be finite (it is ignored by ERT contexts)");
    dmask = d.dirichlet_mask ? d.dirichlet_mask : 0x1Fu;
    require((dmask & ~0x3Fu) == 0, "dirichlet_mask has bits above bit 5");
    require(Nc <= kErtCoarseMax, "ERT coarsest level has " + std::to_string(Nc) + " nodes (> " +
                                     std::to_string(kErtCoarseMax) +
                                     "): use n_d = 2^k*c + 1 so the grid can be halved, or lower coarse_max");
}

void Ctx::ert_init() {
    eoff.resize(lv.size());
    int64_t tot = 0;
    for (size_t l = 0; l < lv.size(); ++l) {
        eoff[l] = tot;
        tot += 5 * pitch[l];
    }
    ecoef.reserve((size_t)tot * sizeof(double));
    cinv64.reserve((size_t)Nc * Nc * sizeof(double));
}

void Ctx::ert_set_conductivity(const double* logsig) {
    const int L = (int)lv.size();
    ert_ready = false;
    H1W_HIP(hipMemsetAsync(iflag.p, 0, 2 * sizeof(int), stream));
    {
        const ErtLevel c0 = ert_level(0);
        hipLaunchKernelGGL(k_ert_sigma, dim3((unsigned)cdiv(N(), kBlock)), dim3(kBlock), 0, stream, N(), logsig,
                           c0.sig, iflag.as<int>());
        H1W_LAUNCHED();
    }
    for (int l = 1; l < L; ++l) {
        const EG gf = make_eg(lv[l - 1], dmask), gc = make_eg(lv[l], dmask);
        hipLaunchKernelGGL(k_ert_coarsen, dim3((unsigned)cdiv(gc.N, kBlock)), dim3(kBlock), 0, stream, gf, gc,
                           ert_level(l - 1).sig, ert_level(l).sig);
        H1W_LAUNCHED();
    }
    for (int l = 0; l < L; ++l) {
        const EG g = make_eg(lv[l], dmask);
        const ErtLevel c = ert_level(l);
        hipLaunchKernelGGL(k_ert_coeffs, dim3((unsigned)cdiv(g.N, kBlock)), dim3(kBlock), 0, stream, g, c.sig, c.D,
                           c.cx, c.cy, c.cz);
        H1W_LAUNCHED();
    }
    hipLaunchKernelGGL(k_ert_coarse_inverse, dim3(1), dim3(kGJThreads), 0, stream, make_eg(lv[L - 1], dmask),
                       ert_level(L - 1), cinv64.as<double>(), iflag.as<int>());
    H1W_LAUNCHED();
    int hf[2] = {0, 0};
    H1W_HIP(hipMemcpyAsync(hf, iflag.p, sizeof(hf), hipMemcpyDeviceToHost, stream));
    sync();
    if (hf[0]) throw Error{H1W_ENUMERIC, "conductivity exp(logsig) is not finite and positive at some node"};
    if (hf[1]) throw Error{H1W_ENUMERIC, "coarsest ERT operator has a non-positive pivot"};
    ert_ready = true;
}

void Ctx::ert_apply(int k, const double* X, int64_t ldx, double* Y, int64_t ldy) {
    const EG g = make_eg(lv[0], dmask);
    timed(H1W_K_ERT_STENCIL, 8.0 * (2.0 * k + 4.0) * g.N, 0.0,
          [&] { launch_step(stream, kErtApply, g, ert_level(0), k, nullptr, 0, X, ldx, Y, ldy, 0.0); });
}

// One symmetric V(nu, nu) cycle from zero, like the unfused H1 cycle, on the
// ERT levels.
void Ctx::ert_vcycle_chunk(int k, const double* F, int64_t ldf, double* X, int64_t ldx) {
    const int L = (int)lv.size();
    const double ces = 8.0 * k;
    auto coarse = [&](const double* f, int64_t lf, double* x, int64_t lx) {
        timed(H1W_K_COARSE, ces * 2 * Nc + 8.0 * Nc * Nc, 2.0 * k * Nc * Nc, [&] {
            launch_coarse_solve<double>(stream, Nc, cinv64.as<double>(), k, f, lf, x, lx, cpart.as<double>(),
                                        cpart_elems);
        });
    };
    if (L == 1) {
        coarse(F, ldf, X, ldx);
        return;
    }
    size_t need = (size_t)k * pitch[0];
    for (int l = 1; l < L; ++l) need += (size_t)3 * k * pitch[l];
    vws.reserve(need * sizeof(double));
    double* base = vws.as<double>();
    std::vector<double*> tb(L), fb(L), xb(L);
    size_t off = 0;
    tb[0] = base;
    off += (size_t)k * pitch[0];
    for (int l = 1; l < L; ++l) {
        fb[l] = base + off;
        off += (size_t)k * pitch[l];
        xb[l] = base + off;
        off += (size_t)k * pitch[l];
        tb[l] = base + off;
        off += (size_t)k * pitch[l];
    }
    auto fptr = [&](int l) { return l == 0 ? F : (const double*)fb[l]; };
    auto fld = [&](int l) { return l == 0 ? ldf : pitch[l]; };
    auto xptr = [&](int l) { return l == 0 ? X : xb[l]; };
    auto xld = [&](int l) { return l == 0 ? ldx : pitch[l]; };
    const int nu = d.nu;
    std::vector<double*> cur(L), oth(L);
    std::vector<int64_t> ldcur(L), ldoth(L);
    auto step = [&](int mode, int l, const double* Xin, int64_t li, double* Y, int64_t ly, double wt) {
        const EG g = make_eg(lv[l], dmask);
        const double nl = (double)g.N;
        const double bytes = mode == kErtFirst ? 8.0 * (2.0 * k + 1.0) * nl : 8.0 * (3.0 * k + 4.0) * nl;
        timed(H1W_K_ERT_STENCIL, bytes, 0.0,
              [&] { launch_step(stream, mode, g, ert_level(l), k, fptr(l), fld(l), Xin, li, Y, ly, wt); });
    };
    for (int l = 0; l < L - 1; ++l) {
        // pre-smoothing from zero into t; with the residual written to the
        // other buffer and the post-smoothing alternating between the two,
        // the last post-smoothing step lands in x for every nu
        double* a = tb[l];
        int64_t la = pitch[l];
        double* b = xptr(l);
        int64_t lb = xld(l);
        step(kErtFirst, l, nullptr, 0, a, la, w[0]);
        for (int s = 1; s < nu; ++s) {
            step(kErtSmooth, l, a, la, b, lb, w[s]);
            std::swap(a, b);
            std::swap(la, lb);
        }
        step(kErtResidual, l, a, la, b, lb, 0.0);
        {
            const EG gf = make_eg(lv[l], dmask), gc = make_eg(lv[l + 1], dmask);
            timed(H1W_K_ERT_STENCIL, ces * (gf.N + gc.N), 0.0, [&] {
                const int nblk = (int)cdiv(gc.N, kBlock);
                require((int64_t)nblk * k < (int64_t(1) << 31), "ERT restriction launch too large");
                const int total = nblk * k;
                hipLaunchKernelGGL(k_ert_restrict, dim3((unsigned)(8 * cdiv(total, 8))), dim3(kBlock), 0, stream, gf,
                                   gc, nblk, total, (const double*)b, lb, fb[l + 1], pitch[l + 1]);
                H1W_LAUNCHED();
            });
        }
        cur[l] = a;
        ldcur[l] = la;
        oth[l] = b;
        ldoth[l] = lb;
    }
    coarse(fb[L - 1], pitch[L - 1], xb[L - 1], pitch[L - 1]);
    for (int l = L - 2; l >= 0; --l) {
        const Geom& g = lv[l];
        timed(H1W_K_PROLONG, ces * (2.0 * g.N + (double)lv[l + 1].N), 0.0, [&] {
            launch_prolong_add<double>(stream, dim, g, lv[l + 1], k, xb[l + 1], pitch[l + 1], cur[l], ldcur[l]);
        });
        double* a = cur[l];
        int64_t la = ldcur[l];
        double* b = oth[l];
        int64_t lb = ldoth[l];
        for (int s = nu - 1; s >= 0; --s) {
            step(kErtSmooth, l, a, la, b, lb, w[s]);
            std::swap(a, b);
            std::swap(la, lb);
        }
        if (a != xptr(l)) throw Error{H1W_EINVAL, "internal: ERT V-cycle buffer parity"};
    }
}

void Ctx::ert_fields(int n_src, const int* src, double* U, int64_t ldu, double rtol, int maxit, h1w_info* info) {
    const int64_t n = N();
    efs.reserve((size_t)n_src * pitch[0] * sizeof(double));
    hipLaunchKernelGGL(k_ert_unit_loads, dim3((unsigned)cdiv(n, kBlock), (unsigned)n_src), dim3(kBlock), 0, stream,
                       n, src, efs.as<double>(), pitch[0]);
    H1W_LAUNCHED();
    mg_solve(n_src, efs.as<double>(), pitch[0], U, ldu, rtol, maxit, info);
}

const double* Ctx::ert_kgeo(int n_meas, const int* pair, const int* src, const double* kgeo) {
    if (kgeo) return kgeo;
    ekg.reserve((size_t)std::max(1, n_meas) * sizeof(double));
    hipLaunchKernelGGL(k_ert_kgeo, dim3((unsigned)cdiv(n_meas, kBlock)), dim3(kBlock), 0, stream,
                       make_eg(lv[0], dmask), n_meas, pair, src, ekg.as<double>());
    H1W_LAUNCHED();
    return ekg.as<double>();
}

void Ctx::ert_measure(int n_meas, const int* pair, const int* src, const double* k, const double* U, int64_t ldu,
                      double* g) {
    hipLaunchKernelGGL(k_ert_meas, dim3((unsigned)cdiv(n_meas, kBlock)), dim3(kBlock), 0, stream, n_meas, pair, src,
                       k, U, ldu, g);
    H1W_LAUNCHED();
}

void Ctx::ert_sens(int n_src, const double* U, int64_t ldu, int n_meas, const int* pair, const double* k, double* J,
                   int64_t ldj, const double* gbar, double* grad) {
    const EG g = make_eg(lv[0], dmask);
    const double* sig = ert_level(0).sig;
    const bool vjp = gbar != nullptr;
    const double nn = (double)g.N;
    const double bytes = vjp ? 8.0 * nn * (n_src + 2.0) : 8.0 * nn * (n_src + 1.0 + n_meas);
    timed(H1W_K_ERT_SENS, bytes, 12.0 * n_meas * nn, [&] {
        if (n_src <= 32) {
            const unsigned blocks = (unsigned)(8 * cdiv(cdiv(g.N, 64), 8));
            const dim3 block(64 * kSensWaves);
#define H1W_SENS_WIDE(NS, V)                                                                                      \
    hipLaunchKernelGGL((k_ert_sens_wide<NS, V>), dim3(blocks), block, 0, stream, g, sig, n_src, U, ldu, n_meas, pair, \
                       k, J, ldj, gbar, grad)
            if (n_src <= 16) {
                if (vjp)
                    H1W_SENS_WIDE(16, true);
                else
                    H1W_SENS_WIDE(16, false);
            } else {
                if (vjp)
                    H1W_SENS_WIDE(32, true);
                else
                    H1W_SENS_WIDE(32, false);
            }
#undef H1W_SENS_WIDE
        } else {
            const unsigned blocks = (unsigned)(8 * cdiv(cdiv(g.N, 16), 8));
            if (vjp)
                hipLaunchKernelGGL((k_ert_sens<16, true>), dim3(blocks), dim3(kSensThreads), 0, stream, g, sig, n_src,
                                   U, ldu, n_meas, pair, k, J, ldj, gbar, grad);
            else
                hipLaunchKernelGGL((k_ert_sens<16, false>), dim3(blocks), dim3(kSensThreads), 0, stream, g, sig, n_src,
                                   U, ldu, n_meas, pair, k, J, ldj, gbar, grad);
        }
        H1W_LAUNCHED();
    });
}

bool ert_on_dirichlet_host(const Geom& g, unsigned mask, int64_t p) {
    const int i = (int)(p % g.nx);
    const int64_t t = p / g.nx;
    const int j = (int)(t % g.ny), l = (int)(t / g.ny);
    return ((mask & 1u) && i == 0) || ((mask & 2u) && i == g.nx - 1) || ((mask & 4u) && j == 0) ||
           ((mask & 8u) && j == g.ny - 1) || ((mask & 16u) && l == 0) || ((mask & 32u) && l == g.nz - 1);
}

}  // namespace h1w
