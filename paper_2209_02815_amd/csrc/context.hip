// Host runtime of the h1w library: context and multigrid hierarchy, the
// batched V-cycle B, MG-preconditioned CG for Poisson solves, the capacitance
// build, the Woodbury preconditioner apply and the preconditioned CG driver
// for the Gauss-Newton system G x = b, G = alpha*A + J^T J.
#include "context.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

namespace h1w {

// ============================================================ setup

static Geom make_geom(int dim, const int n[3], double beta) {
    Geom g{};
    g.nx = n[0];
    g.ny = n[1];
    g.nz = dim == 3 ? n[2] : 1;
    g.N = (int64_t)g.nx * g.ny * g.nz;
    auto ih2 = [](int nn) { return double(nn - 1) * double(nn - 1); };
    g.ihx2 = ih2(g.nx);
    g.ihy2 = ih2(g.ny);
    g.ihz2 = dim == 3 ? ih2(g.nz) : 0.0;
    g.beta = beta;
    return g;
}

// Dense A on one (small) level, row-major, same stencil as the device kernels.
static std::vector<double> dense_operator(int dim, const Geom& g) {
    const int64_t N = g.N;
    std::vector<double> A((size_t)(N * N), 0.0);
    auto w = [](int i, int n) { return (i == 0 || i == n - 1) ? 0.5 : 1.0; };
    for (int l = 0; l < g.nz; ++l)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i < g.nx; ++i) {
                const int64_t p = i + (int64_t)g.nx * (j + (int64_t)g.ny * l);
                const double wx = w(i, g.nx), wy = w(j, g.ny), wz = dim == 3 ? w(l, g.nz) : 1.0;
                const double cx = g.ihx2 * wy * wz, cy = g.ihy2 * wx * wz, cz = dim == 3 ? g.ihz2 * wx * wy : 0.0;
                double diag = g.beta * wx * wy * wz;
                auto couple = [&](int64_t q, double c) {
                    A[(size_t)(p * N + q)] -= c;
                    diag += c;
                };
                if (i > 0) couple(p - 1, cx);
                if (i < g.nx - 1) couple(p + 1, cx);
                if (j > 0) couple(p - g.nx, cy);
                if (j < g.ny - 1) couple(p + g.nx, cy);
                if (dim == 3) {
                    const int64_t pl = (int64_t)g.nx * g.ny;
                    if (l > 0) couple(p - pl, cz);
                    if (l < g.nz - 1) couple(p + pl, cz);
                }
                A[(size_t)(p * N + p)] = diag;
            }
    return A;
}

// Inverse of an SPD matrix through its Cholesky factor (host, FP64).
static std::vector<double> spd_inverse(std::vector<double> A, int64_t n) {
    for (int64_t k = 0; k < n; ++k) {  // lower Cholesky in place
        double d = A[(size_t)(k * n + k)];
        for (int64_t q = 0; q < k; ++q) d -= A[(size_t)(k * n + q)] * A[(size_t)(k * n + q)];
        if (!(d > 0.0)) throw Error{H1W_ENUMERIC, "coarsest operator is not positive definite"};
        d = std::sqrt(d);
        A[(size_t)(k * n + k)] = d;
        for (int64_t i = k + 1; i < n; ++i) {
            double s = A[(size_t)(i * n + k)];
            const double* ri = &A[(size_t)(i * n)];
            const double* rk = &A[(size_t)(k * n)];
            for (int64_t q = 0; q < k; ++q) s -= ri[q] * rk[q];
            A[(size_t)(i * n + k)] = s / d;
        }
    }
    // X = L^{-T} L^{-1} column by column
    std::vector<double> X((size_t)(n * n), 0.0), y((size_t)n);
    for (int64_t c = 0; c < n; ++c) {
        for (int64_t i = 0; i < n; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            const double* ri = &A[(size_t)(i * n)];
            for (int64_t q = c; q < i; ++q) s -= ri[q] * y[(size_t)q];
            y[(size_t)i] = (i < c) ? 0.0 : s / ri[i];
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = y[(size_t)i];
            for (int64_t q = i + 1; q < n; ++q) s -= A[(size_t)(q * n + i)] * X[(size_t)(q * n + c)];
            X[(size_t)(i * n + c)] = s / A[(size_t)(i * n + i)];
        }
    }
    return X;
}

// Symmetrised dense inverse of the coarsest operator of grid g. Coarsest
// levels of up to 1024 nodes are computed once per (dimension, grid, beta) in
// the process and shared (contexts of a batch mostly end on the same few).
static std::shared_ptr<const std::vector<double>> coarsest_inverse(int dim, const Geom& g) {
    auto compute = [&] {
        const int64_t n = g.N;
        auto v = std::make_shared<std::vector<double>>(spd_inverse(dense_operator(dim, g), n));
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) {
                const double a = 0.5 * ((*v)[(size_t)(i * n + j)] + (*v)[(size_t)(j * n + i)]);
                (*v)[(size_t)(i * n + j)] = (*v)[(size_t)(j * n + i)] = a;
            }
        return std::shared_ptr<const std::vector<double>>(v);
    };
    if (g.N > 1024) return compute();
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, double>, std::shared_ptr<const std::vector<double>>> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto& slot = cache[std::make_tuple(dim, g.nx, g.ny, g.nz, g.beta)];
    if (!slot) slot = compute();
    return slot;
}

void Ctx::init(const h1w_grid_desc& desc, hipStream_t s) {
    d = desc;
    stream = s;
    dim = d.dim;
    require(dim == 2 || dim == 3, "dim must be 2 or 3");
    int n[3] = {d.n[0], d.n[1], dim == 3 ? d.n[2] : 1};
    for (int a = 0; a < dim; ++a) require(n[a] >= 2, "every n[d] must be >= 2");
    require(d.op == H1W_OP_H1GRAM || d.op == H1W_OP_ERT, "op must be H1W_OP_H1GRAM or H1W_OP_ERT");
    ert = d.op == H1W_OP_ERT;
    require(ert || d.dirichlet_mask == 0, "dirichlet_mask is for ERT contexts only");
    if (!ert) require(std::isfinite(d.beta) && d.beta > 0.0, "beta must be finite and > 0");
    require(d.precision == H1W_FP64 || d.precision == H1W_MIXED, "precision must be H1W_FP64 or H1W_MIXED");
    require(d.nu >= 0 && d.nu <= 16, "nu must be in [0, 16]");
    require((d.flags & ~(H1W_FLAG_STREAM_Z | H1W_FLAG_UNFUSED_VCYCLE | H1W_FLAG_GRAPH_VCYCLE | H1W_FLAG_NO_VTAIL |
                         H1W_FLAG_CAP_FP32_GEMM)) == 0,
            "unknown bits in flags");
    require(!(d.flags & H1W_FLAG_CAP_FP32_GEMM) || d.precision == H1W_MIXED,
            "H1W_FLAG_CAP_FP32_GEMM needs a MIXED context");
    graphs = (d.flags & H1W_FLAG_GRAPH_VCYCLE) != 0;
    require(d.coarse_max >= 0, "coarse_max must be >= 0");
    require(d.rhs_chunk >= 0 && d.rhs_chunk <= 65535, "rhs_chunk must be in [0, 65535]");
    if (d.nu == 0) d.nu = 2;
    if (d.cheb_lo == 0.0 && d.cheb_hi == 0.0) {
        d.cheb_lo = kChebLoDefault;
        d.cheb_hi = kChebHiDefault;
    }
    require(d.cheb_lo > 0.0 && d.cheb_hi > d.cheb_lo && std::isfinite(d.cheb_hi), "need 0 < cheb_lo < cheb_hi");
    if (d.coarse_max == 0) d.coarse_max = ert ? 125 : (dim == 3 ? 729 : 81);
    fp32 = d.precision == H1W_MIXED;
    const int64_t N0 = (int64_t)n[0] * n[1] * n[2];
    require(N0 < (int64_t(1) << 31), "grid too large: N must be < 2^31");

    // hierarchy: halve while the level is above coarse_max and every n_d >= 5 is odd
    lv.clear();
    int cur[3] = {n[0], n[1], n[2]};
    for (;;) {
        lv.push_back(make_geom(dim, cur, ert ? 0.0 : d.beta));
        const Geom& g = lv.back();
        if (g.N <= d.coarse_max) break;
        bool ok = true;
        for (int a = 0; a < dim; ++a) ok = ok && cur[a] >= 5 && (cur[a] - 1) % 2 == 0;
        if (!ok) break;
        for (int a = 0; a < dim; ++a) cur[a] = (cur[a] - 1) / 2 + 1;
    }
    Nc = lv.back().N;
    if (ert) ert_validate();
    require(Nc <= 4096, "coarsest level has " + std::to_string(Nc) +
                            " nodes (> 4096): use n_d = 2^k*c + 1 so the grid can be halved, or lower coarse_max");

    // Chebyshev step weights: 1/theta_k, theta_k = (hi+lo)/2 + (hi-lo)/2 cos(pi (2k+1)/(2 nu))
    w.resize(d.nu);
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < d.nu; ++k)
        w[k] = 1.0 / (0.5 * (d.cheb_hi + d.cheb_lo) + 0.5 * (d.cheb_hi - d.cheb_lo) * std::cos(pi * (2 * k + 1) / (2.0 * d.nu)));

    pitch.resize(lv.size());
    for (size_t l = 0; l < lv.size(); ++l) pitch[l] = cdiv(lv[l].N, 64) * 64;
    // right-hand sides per batched V-cycle: about 2^28 values per fine-level
    // array (the workspace holds about 1.43 of them: 3 GB in FP64), so the
    // coarse levels of a large grid still launch enough work-groups
    chunk = d.rhs_chunk > 0 ? d.rhs_chunk : (int)std::clamp<int64_t>((int64_t(1) << 28) / N0, 1, 1024);
    {
        std::lock_guard<std::recursive_mutex> lk(capture_lock());
        H1W_HIP(hipHostMalloc((void**)&hscal, 64 * sizeof(double), hipHostMallocDefault));
        H1W_HIP(hipHostMalloc((void**)&hrep, 16 * sizeof(double), hipHostMallocCoherent));
        H1W_HIP(hipHostGetDevicePointer((void**)&drep, hrep, 0));
    }
    scal.reserve(64 * sizeof(double));
    iflag.reserve(16 * sizeof(int));
    cpart_elems = coarse_part_elems(Nc);
    if (cpart_elems) cpart.reserve(cpart_elems * sizeof(double));
    if (ert) {
        // the coarsest inverse depends on the conductivity: built on the device
        // by h1w_ert_set_conductivity
        ert_init();
        return;
    }

    // dense inverse of the coarsest operator, symmetrised so that the device
    // kernel may read it by columns; it depends only on the coarsest grid and
    // beta, so contexts share it through a process-wide cache
    const auto inv_ptr = coarsest_inverse(dim, lv.back());
    const std::vector<double>& inv = *inv_ptr;
    cinv64.reserve(inv.size() * sizeof(double));
    std::vector<float> inv32(inv.begin(), inv.end());
    cinv32.reserve(inv32.size() * sizeof(float));
    {
        std::lock_guard<std::recursive_mutex> lk(capture_lock());
        H1W_HIP(hipMemcpy(cinv64.p, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice));
        H1W_HIP(hipMemcpy(cinv32.p, inv32.data(), inv32.size() * sizeof(float), hipMemcpyHostToDevice));
    }

    fused = d.nu == 2 && lv.size() >= 2 && !(d.flags & H1W_FLAG_UNFUSED_VCYCLE);
    for (size_t l = 0; fused && l + 1 < lv.size(); ++l)
        fused = dim == 3 ? fused_levels_ok(lv[l], lv[l + 1]) : fused2_levels_ok(lv[l], lv[l + 1]);
    tail_l0 = (int)lv.size();
    if (fused && dim == 2 && !(d.flags & H1W_FLAG_NO_VTAIL)) tail2_plan(lv.data(), (int)lv.size(), tail_l0, tail);

    deflate = fp32;
    wsum = 1.0;
    for (int a = 0; a < dim; ++a) wsum *= double(n[a] - 1);  // sum of the trapezoid weights
}

Ctx::~Ctx() {
    std::lock_guard<std::recursive_mutex> lk(capture_lock());
    clear_graphs();
    if (cap_stream && own_cap_stream) (void)hipStreamDestroy(cap_stream);
    if (hscal) (void)hipHostFree(hscal);
    if (hrep) (void)hipHostFree(hrep);
    for (auto& p : pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto& e : evpool) (void)hipEventDestroy(e);
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
}

int64_t Ctx::N() const { return lv[0].N; }

void Ctx::sync() { H1W_HIP(hipStreamSynchronize(stream)); }

// read n device scalars (blocks the host)
void Ctx::read_scal(int n) {
    H1W_HIP(hipMemcpyAsync(hscal, scal.p, n * sizeof(double), hipMemcpyDeviceToHost, stream));
    sync();
}

// ============================================================ V-cycle

template <typename T>
void Ctx::vcycle_chunk(int k, const T* F, int64_t ldf, T* X, int64_t ldx) {
    const int L = (int)lv.size();
    const size_t es = sizeof(T);
    const double ces = (double)es * k;
    auto coarse = [&](const T* f, int64_t lf, T* x, int64_t lx) {
        timed(H1W_K_COARSE, ces * 2 * Nc + (double)es * Nc * Nc, 2.0 * k * Nc * Nc,
              [&] { launch_coarse_solve<T>(stream, Nc, fp_cinv<T>(), k, f, lf, x, lx, cpart.as<T>(), cpart_elems); });
    };
    if (L == 1) {
        coarse(F, ldf, X, ldx);
        return;
    }
    // workspace: level 0 scratch t; levels >= 1: f, x, t (k rows of pitch each)
    size_t need = (size_t)k * pitch[0];
    for (int l = 1; l < L; ++l) need += (size_t)3 * k * pitch[l];
    vws.reserve(need * es);
    T* base = vws.as<T>();
    std::vector<T*> tb(L), fb(L), xb(L);
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
    const int nu = d.nu;
    std::vector<T*> cur(L), oth(L);
    std::vector<int64_t> ldcur(L), ldoth(L);
    auto fptr = [&](int l) { return l == 0 ? F : (const T*)fb[l]; };
    auto fld = [&](int l) { return l == 0 ? ldf : pitch[l]; };
    auto xptr = [&](int l) { return l == 0 ? X : xb[l]; };
    auto xld = [&](int l) { return l == 0 ? ldx : pitch[l]; };

    if (fused) {
        // two smoothing steps per side: one pass down and one pass up per
        // level (3D z-march or 2D tiles in LDS); the pre-smoothed iterate of
        // level l is kept in tb[l]
        // 2D: the levels from tail_l0 on run in one launch
        const int lt = std::min(tail_l0, L - 1);
        for (int l = 0; l < lt; ++l) {
            const double nl = (double)lv[l].N, nc = (double)lv[l + 1].N;
            timed(H1W_K_VDOWN, ces * (2 * nl + nc), 0.0, [&] {
                if (dim == 3)
                    launch_vdown<T>(stream, lv[l], lv[l + 1], k, fptr(l), fld(l), tb[l], pitch[l], fb[l + 1],
                                    pitch[l + 1], w[0], w[1]);
                else
                    launch_vdown2<T>(stream, lv[l], lv[l + 1], k, fptr(l), fld(l), tb[l], pitch[l], fb[l + 1],
                                     pitch[l + 1], w[0], w[1]);
            });
        }
        if (lt < L - 1) {
            const double nt = (double)lv[lt].N;
            TailGeo tg = tail;
            tg.csplit = cpart_elems ? coarse_splits(Nc, k, cpart_elems) : 1;
            timed(H1W_K_VTAIL, ces * 2 * nt + (double)es * Nc * Nc, 2.0 * k * Nc * Nc, [&] {
                launch_vtail2<T>(stream, tg, fp_cinv<T>(), k, fptr(lt), fld(lt), xptr(lt), xld(lt), w[0], w[1]);
            });
        } else {
            coarse(fb[L - 1], pitch[L - 1], xb[L - 1], pitch[L - 1]);
        }
        for (int l = lt - 1; l >= 0; --l) {
            const double nl = (double)lv[l].N, nc = (double)lv[l + 1].N;
            timed(H1W_K_VUP, ces * (3 * nl + nc), 0.0, [&] {
                if (dim == 3)
                    launch_vup<T>(stream, lv[l], lv[l + 1], k, fptr(l), fld(l), tb[l], pitch[l], xb[l + 1],
                                  pitch[l + 1], xptr(l), xld(l), w[1], w[0]);
                else
                    launch_vup2<T>(stream, lv[l], lv[l + 1], k, fptr(l), fld(l), tb[l], pitch[l], xb[l + 1],
                                   pitch[l + 1], xptr(l), xld(l), w[1], w[0]);
            });
        }
        return;
    }

    for (int l = 0; l < L - 1; ++l) {
        const Geom& g = lv[l];
        // pre-smoothing from zero: first step writes t so that 2nu-1 flips end in x
        const double nl = (double)g.N;
        T* a = tb[l];
        int64_t la = pitch[l];
        T* b = xptr(l);
        int64_t lb = xld(l);
        int s = 1;
        if (nu >= 2) {  // steps 1 and 2 in one pass, written where step 2 would write
            timed(H1W_K_SMOOTH_FIRST, 2 * ces * nl, 0.0,
                  [&] { launch_pre2<T>(stream, dim, g, k, fptr(l), fld(l), b, lb, w[0], w[1]); });
            std::swap(a, b);
            std::swap(la, lb);
            s = 2;
        } else {
            timed(H1W_K_SMOOTH_FIRST, 2 * ces * nl, 0.0,
                  [&] { launch_smooth_first<T>(stream, dim, g, k, fptr(l), fld(l), tb[l], pitch[l], w[0]); });
        }
        for (; s < nu; ++s) {
            timed(H1W_K_SMOOTH, 3 * ces * nl, 0.0,
                  [&] { launch_smooth<T>(stream, dim, g, k, fptr(l), fld(l), a, la, b, lb, w[s]); });
            std::swap(a, b);
            std::swap(la, lb);
        }
        timed(H1W_K_RESIDUAL, 3 * ces * nl, 0.0,
              [&] { launch_residual<T>(stream, dim, g, k, fptr(l), fld(l), a, la, b, lb); });
        timed(H1W_K_RESTRICT, ces * (nl + (double)lv[l + 1].N), 0.0,
              [&] { launch_restrict<T>(stream, dim, g, lv[l + 1], k, b, lb, fb[l + 1], pitch[l + 1]); });
        cur[l] = a;
        ldcur[l] = la;
        oth[l] = b;
        ldoth[l] = lb;
    }
    coarse(fb[L - 1], pitch[L - 1], xb[L - 1], pitch[L - 1]);
    for (int l = L - 2; l >= 0; --l) {
        const Geom& g = lv[l];
        const double nl = (double)g.N;
        timed(H1W_K_PROLONG, ces * (2 * nl + (double)lv[l + 1].N), 0.0, [&] {
            launch_prolong_add<T>(stream, dim, g, lv[l + 1], k, xb[l + 1], pitch[l + 1], cur[l], ldcur[l]);
        });
        T* a = cur[l];
        int64_t la = ldcur[l];
        T* b = oth[l];
        int64_t lb = ldoth[l];
        for (int s = nu - 1; s >= 0; --s) {
            timed(H1W_K_SMOOTH, 3 * ces * nl, 0.0,
                  [&] { launch_smooth<T>(stream, dim, g, k, fptr(l), fld(l), a, la, b, lb, w[s]); });
            std::swap(a, b);
            std::swap(la, lb);
        }
        if (a != xptr(l)) throw Error{H1W_EINVAL, "internal: V-cycle buffer parity"};
    }
}

template <typename T>
void Ctx::vcycle(int k, const T* F, int64_t ldf, T* X, int64_t ldx) {
    for (int r0 = 0; r0 < k; r0 += chunk) {
        const int kk = std::min(chunk, k - r0);
        vcycle_chunk<T>(kk, F + (int64_t)r0 * ldf, ldf, X + (int64_t)r0 * ldx, ldx);
    }
}

void Ctx::apply_B(int k, const double* F, int64_t ldf, double* X, int64_t ldx) {
    if (exact_b) {
        mg_solve(k, F, ldf, X, ldx, exact_rtol, 200, nullptr);
        return;
    }
    vcycle_B(k, F, ldf, X, ldx);
}

// y = B r for FP64 vectors in the context's V-cycle precision.
void Ctx::vcycle_B(int k, const double* F, int64_t ldf, double* X, int64_t ldx) {
    if (graphs && !capturing && tmask == 0 && !ert) {
        vcycle_graph(k, F, ldf, X, ldx);
        return;
    }
    vcycle_B_eager(k, F, ldf, X, ldx);
}

std::vector<const void*> Ctx::workspace_signature() const {
    return {vws.p, stage.p, part.p, jpart.p, scal.p, cpart.p, wvec.p, vdef.p, ones.p, cinv64.p, cinv32.p};
}

void Ctx::clear_graphs() {
    for (auto& g : vgraphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    vgraphs.clear();
}

void Ctx::vcycle_graph(int k, const double* F, int64_t ldf, double* X, int64_t ldx) {
    auto sig = workspace_signature();
    if (sig != vg_sig) {
        clear_graphs();
        vg_sig = sig;
    }
    for (auto& g : vgraphs) {
        if (g.k != k || g.F != F || g.ldf != ldf || g.X != X || g.ldx != ldx) continue;
        if (!g.exec) {  // second use: capture the sequence, then replay it
            // captured on a private stream (the context's stream may be the
            // null stream, which cannot be captured); nothing runs during the
            // capture, the graph is then launched on the context's stream
            std::lock_guard<std::recursive_mutex> lk(capture_lock());
            if (!cap_stream) H1W_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
            hipGraph_t gr = nullptr;
            const hipStream_t own = stream;
            H1W_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
            capturing = true;
            stream = cap_stream;
            try {
                vcycle_B_eager(k, F, ldf, X, ldx);
            } catch (...) {
                stream = own;
                capturing = false;
                (void)hipStreamEndCapture(cap_stream, &gr);
                if (gr) (void)hipGraphDestroy(gr);
                throw;
            }
            stream = own;
            capturing = false;
            H1W_HIP(hipStreamEndCapture(cap_stream, &gr));
            hipGraphExec_t ex = nullptr;
            const hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            H1W_HIP(e);
            g.exec = ex;
            // the capture did not run the kernels
        }
        H1W_HIP(hipGraphLaunch(g.exec, stream));
        ++graph_launches;
        return;
    }
    // first use: run eagerly (this reserves the workspace) and remember the key
    vcycle_B_eager(k, F, ldf, X, ldx);
    sig = workspace_signature();
    if (sig != vg_sig) {
        clear_graphs();
        vg_sig = sig;
    }
    if (vgraphs.size() >= 8) clear_graphs();
    vgraphs.push_back(VGraph{k, F, ldf, X, ldx, nullptr});
}

void Ctx::vcycle_B_eager(int k, const double* F, int64_t ldf, double* X, int64_t ldx) {
    if (ert) {
        for (int r0 = 0; r0 < k; r0 += chunk) {
            const int kk = std::min(chunk, k - r0);
            ert_vcycle_chunk(kk, F + (int64_t)r0 * ldf, ldf, X + (int64_t)r0 * ldx, ldx);
        }
        return;
    }
    if (!fp32) {
        vcycle<double>(k, F, ldf, X, ldx);
        return;
    }
    const int64_t n = N();
    if (k == 1 && deflate) {
        // y = P B~(F - c W1) + c v: the constant mode (c = 1.F / sum W) is handled
        // exactly in FP64 and the W-mean mu of the FP32 cycle's output (rounding
        // error amplified by the coarse solve) is projected out
        ensure_deflation_vectors();
        ensure_cg_ws(m);
        stage.reserve((size_t)2 * pitch[0] * sizeof(float));
        float* fin = stage.as<float>();
        float* fout = fin + pitch[0];
        double* cm = scal.as<double>() + 12;  // cm[0] = c, cm[1] = mu
        if (F == rsum_of && rsum_part && !graphs) {
            // the GN-CG update left the partial sums of F = r (same order)
            launch_deflate_in(stream, n, F, rsum_part, rsum_nb, 1.0 / wsum, wvec.as<double>(), fin, cm);
        } else {
            const double* X1[1] = {ones.as<double>()};
            const double* Y1[1] = {F};
            const int nb = launch_dots_partial(stream, n, 1, X1, Y1, part.as<double>());
            launch_deflate_in(stream, n, F, part.as<double>(), nb, 1.0 / wsum, wvec.as<double>(), fin, cm);
        }
        rsum_of = nullptr;
        vcycle_chunk<float>(1, fin, pitch[0], fout, pitch[0]);
        const int nch = launch_rows_dot_partial_f32(stream, 1, n, fout, pitch[0], wvec.as<double>(), jpart.as<double>());
        launch_deflate_out(stream, n, fout, jpart.as<double>(), nch, 1.0 / wsum, cm, vdef.as<double>(), X);
        return;
    }
    for (int r0 = 0; r0 < k; r0 += chunk) {
        const int kk = std::min(chunk, k - r0);
        stage.reserve((size_t)2 * kk * pitch[0] * sizeof(float));
        float* fin = stage.as<float>();
        float* fout = fin + (size_t)kk * pitch[0];
        launch_convert<double, float>(stream, n, kk, F + (int64_t)r0 * ldf, ldf, fin, pitch[0], 1.0);
        vcycle_chunk<float>(kk, fin, pitch[0], fout, pitch[0]);
        launch_convert<float, double>(stream, n, kk, fout, pitch[0], X + (int64_t)r0 * ldx, ldx, 1.0);
    }
}

// ============================================================ MG-preconditioned CG (Poisson)

void Ctx::apply_A(int k, const double* X, int64_t ldx, double* Y, int64_t ldy) {
    if (ert)
        ert_apply(k, X, ldx, Y, ldy);
    else
        launch_apply<double>(stream, dim, lv[0], k, X, ldx, Y, ldy, 1.0);
}

void Ctx::mg_solve(int k, const double* F, int64_t ldf, double* X, int64_t ldx, double rtol, int maxit,
                   h1w_info* info) {
    const int64_t n = N();
    int max_iters = 0;
    for (int r0 = 0; r0 < k; r0 += chunk) {
        const int kk = std::min(chunk, k - r0);
        const double* Fc = F + (int64_t)r0 * ldf;
        double* Xc = X + (int64_t)r0 * ldx;
        const int64_t P = pitch[0];
        pcg.reserve((size_t)4 * kk * P * sizeof(double));
        double* R = pcg.as<double>();
        double* Zv = R + (size_t)kk * P;
        double* Pv = Zv + (size_t)kk * P;
        double* Q = Pv + (size_t)kk * P;
        // scratch of its own: vcycle_B may reserve (and so reallocate) the
        // GN-CG workspace (mvec, part) of a MIXED context, and an EXACT_B
        // solve runs inside the GN-CG, whose m-vectors live in mvec
        mgvec.reserve((size_t)8 * kk * sizeof(double) + 16 * kk * sizeof(int));
        double* dnrm = mgvec.as<double>();      // kk
        double* drz = dnrm + kk;                // kk: r.z of the current direction
        double* dpq = drz + kk;                 // kk
        double* da = dpq + kk;                  // kk
        double* db = da + kk;                   // kk
        double* dzq = db + kk;                  // kk
        double* drzn = dzq + kk;                // kk: r.z after the new preconditioner apply
        int* dact = (int*)(drzn + kk);          // kk
        mgpart.reserve((size_t)kk * 64 * sizeof(double));
        double* pp = mgpart.as<double>();
        std::vector<double> nb(kk), rr(kk);
        std::vector<int> act(kk, 1);
        int hflag = 0;
        // one host round trip per iteration: the residual norms (and the
        // breakdown flag); step lengths and direction coefficients stay on
        // the device
        auto fetch_norms = [&]() {
            H1W_HIP(hipMemcpyAsync(rr.data(), dnrm, kk * sizeof(double), hipMemcpyDeviceToHost, stream));
            H1W_HIP(hipMemcpyAsync(&hflag, iflag.as<int>() + 8, sizeof(int), hipMemcpyDeviceToHost, stream));
            sync();
        };
        auto put_act = [&]() {
            H1W_HIP(hipMemcpyAsync(dact, act.data(), kk * sizeof(int), hipMemcpyHostToDevice, stream));
        };
        H1W_HIP(hipMemsetAsync(iflag.as<int>() + 8, 0, sizeof(int), stream));  // slot 8: PCG breakdown
        H1W_HIP(hipMemset2DAsync(Xc, ldx * sizeof(double), 0, n * sizeof(double), kk, stream));
        H1W_HIP(hipMemcpy2DAsync(R, P * sizeof(double), Fc, ldf * sizeof(double), n * sizeof(double), kk,
                                 hipMemcpyDeviceToDevice, stream));
        launch_batched_dots(stream, kk, n, R, P, R, P, pp, dnrm);
        fetch_norms();
        for (int r = 0; r < kk; ++r) {
            if (!std::isfinite(rr[r])) throw Error{H1W_ENUMERIC, "non-finite right-hand side"};
            nb[r] = std::sqrt(rr[r]);
            if (nb[r] == 0.0) act[r] = 0;
        }
        put_act();
        vcycle_B(kk, R, P, Zv, P);
        H1W_HIP(hipMemcpy2DAsync(Pv, P * sizeof(double), Zv, P * sizeof(double), n * sizeof(double), kk,
                                 hipMemcpyDeviceToDevice, stream));
        launch_batched_dots(stream, kk, n, R, P, Zv, P, pp, drz);
        int it = 0;
        bool done = std::none_of(act.begin(), act.end(), [](int v) { return v; });
        while (!done) {
            if (it >= maxit) {
                if (info) info->iters = std::max(max_iters, it);
                throw Error{H1W_ENOCONV, "MG-PCG did not converge in maxit iterations"};
            }
            apply_A(kk, Pv, P, Q, P);
            launch_batched_dots(stream, kk, n, Pv, P, Q, P, pp, dpq);
            launch_pcg_alpha(stream, kk, drz, dpq, dact, da, iflag.as<int>() + 8);
            launch_batched_cg_xr(stream, kk, n, da, Pv, P, Q, P, Xc, ldx, R, P, dact);
            launch_batched_dots(stream, kk, n, R, P, R, P, pp, dnrm);
            fetch_norms();
            if (hflag) throw Error{H1W_ENUMERIC, "MG-PCG breakdown (p.Ap <= 0 or NaN)"};
            ++it;
            bool any = false;
            for (int r = 0; r < kk; ++r) {
                if (!act[r]) continue;
                if (!std::isfinite(rr[r])) throw Error{H1W_ENUMERIC, "non-finite residual in MG-PCG"};
                if (std::sqrt(rr[r]) <= rtol * nb[r]) act[r] = 0;
                any = any || act[r];
            }
            put_act();
            if (!any) break;
            vcycle_B(kk, R, P, Zv, P);
            launch_batched_dots(stream, kk, n, R, P, Zv, P, pp, drzn);
            // flexible (Polak-Ribiere) coefficient z.(r_new - r_old)/rz when B is an
            // FP32 cycle, with r_new - r_old = -a q
            if (fp32) launch_batched_dots(stream, kk, n, Zv, P, Q, P, pp, dzq);
            launch_pcg_beta(stream, kk, drzn, drz, fp32 ? dzq : nullptr, da, dact, db);
            launch_batched_p(stream, kk, n, db, Zv, P, Pv, P, dact);
        }
        // verify with the true residual
        apply_A(kk, Xc, ldx, Q, P);
        for (int r = 0; r < kk; ++r)
            launch_sub(stream, n, Fc + (int64_t)r * ldf, Q + (int64_t)r * P, R + (int64_t)r * P);
        launch_batched_dots(stream, kk, n, R, P, R, P, pp, dnrm);
        fetch_norms();
        double worst = 0.0;
        for (int r = 0; r < kk; ++r) worst = std::max(worst, nb[r] > 0 ? std::sqrt(rr[r]) / nb[r] : 0.0);
        if (info) info->relres_true = std::max(info->relres_true, worst);
        max_iters = std::max(max_iters, it);
    }
    if (info) {
        info->iters = max_iters;
        info->nlevels = (int)lv.size();
    }
}

// offset in `part` of a second set of dot-product partials (the first set
// holds at most 2 x 1024 of them; `part` holds at least 4 x 1024)
constexpr int kPartB = 2048;

// ============================================================ capacitance

void Ctx::capacitance_build(int m_, const double* J_, int64_t ldj_, double alpha_, int factor_, h1w_info* info) {
    const int64_t n = N();
    have_cap = false;
    m = m_;
    J = J_;
    ldj = ldj_;
    alpha = alpha_;
    ev_record(0);
    int fac = factor_;
    if (fac == H1W_FACTOR_AUTO) fac = fp32 ? H1W_FACTOR_LU : H1W_FACTOR_CHOL;
    const size_t zes = fp32 ? sizeof(float) : sizeof(double);
    Sbuf.reserve((size_t)m * m * sizeof(double));
    // Store Z = B J^T (row i = B J_i) unless it does not fit next to J: an FP64
    // Z larger than ~45% of the free device memory is streamed instead, in row
    // chunks that each meet the rows of J at and below them (S is symmetric).
    size_t freeb = 0, totalb = 0;
    H1W_HIP(hipMemGetInfo(&freeb, &totalb));
    const size_t zbytes = (size_t)m * n * zes;
    const size_t avail = freeb + Zbuf.bytes;
    z_streamed = !fp32 && ((d.flags & H1W_FLAG_STREAM_Z) || zbytes > avail / 100 * 45);
    if (fp32 && zbytes > avail / 100 * 90)
        throw Error{H1W_ENOMEM, "the FP32 Z of a MIXED context does not fit in device memory"};
    // S = alpha I + J Z^T. FP64 Z with a Cholesky factor (or a streamed Z):
    // lower triangle only, mirrored at the end; otherwise the full product.
    const bool lower = !fp32 && (z_streamed || fac == H1W_FACTOR_CHOL);
    // Z is built and multiplied in blocks of zb rows: one block when Z is
    // stored, row chunks (multiples of 128) when it is streamed. A lower block
    // S[r0:m, r0:r1] = J[r0:m] Z_b^T starts on the diagonal; a full block is
    // the column block S[0:m, r0:r1] = J Z_b^T.
    int zb = m;
    if (z_streamed) {
        Zbuf.release();
        // rows of Z per chunk: a multiple of 128 using at most ~30% of the free memory
        zb = (int)std::min<size_t>((size_t)m, (avail / 100 * 30) / ((size_t)n * sizeof(double)));
        zb = std::max(1, zb >= 128 ? zb / 128 * 128 : zb);
        if (d.flags & H1W_FLAG_STREAM_Z) zb = std::min(zb, 128);  // forced: 128-row chunks
        zchunk.reserve((size_t)zb * n * sizeof(double));
    } else {
        Zbuf.reserve(zbytes);
    }
    ldz = n;
    if (fp32) {
        // FP32 V-cycles on J_i - s_i W1; the constant mode s_i v stays exact in FP64
        ensure_deflation_vectors();
        sdef.reserve((size_t)m * sizeof(double));
        jvdef.reserve((size_t)m * sizeof(double));
        const size_t pe = rows_dot_partial_elems(m, n);
        dpart.reserve(2 * pe * sizeof(double));
        const int nch = launch_rows_dot2_partial(stream, m, n, J, ldj, ones.as<double>(), vdef.as<double>(),
                                                 dpart.as<double>(), dpart.as<double>() + pe);
        launch_reduce_parts(stream, m, nch, dpart.as<double>(), sdef.as<double>());
        launch_reduce_parts(stream, m, nch, dpart.as<double>() + pe, jvdef.as<double>());
        launch_scale(stream, m, 1.0 / wsum, sdef.as<double>(), sdef.as<double>());
    }
    size_t pe = 0;
    for (int r0 = 0; r0 < m; r0 += zb) {
        const int cc = std::min(zb, m - r0);
        pe = std::max(pe, lower ? gemm_partial_elems(m - r0, cc, n) : gemm_partial_elems(m, cc, n));
    }
    gpart.reserve(pe * sizeof(double));
    const bool one_block = zb >= m;
    for (int r0 = 0; r0 < m; r0 += zb) {
        const int cc = std::min(zb, m - r0);
        double* z64 = nullptr;
        float* z32 = nullptr;
        if (fp32) {
            z32 = Zbuf.as<float>() + (int64_t)r0 * ldz;
            for (int q0 = r0; q0 < r0 + cc; q0 += chunk) {
                const int kk = std::min(chunk, r0 + cc - q0);
                stage.reserve((size_t)kk * pitch[0] * sizeof(float));
                launch_convert_deflate(stream, n, kk, J + (int64_t)q0 * ldj, ldj, sdef.as<double>() + q0,
                                       wvec.as<double>(), stage.as<float>(), pitch[0]);
                vcycle_chunk<float>(kk, stage.as<float>(), pitch[0], Zbuf.as<float>() + (int64_t)q0 * ldz, ldz);
            }
        } else {
            z64 = z_streamed ? zchunk.as<double>() : Zbuf.as<double>() + (int64_t)r0 * ldz;
            apply_B(cc, J + (int64_t)r0 * ldj, ldj, z64, ldz);
        }
        if (one_block) ev_record(1);
        double* gp = gpart.as<double>();
        int splits = 0;
        if (lower) {
            const int rows = m - r0;
            const double useful = (double)cc * (cc + 1) * n + 2.0 * (rows - cc) * cc * n;
            timed(H1W_K_GEMM, (double)(rows + cc) * n * 8, useful, [&] {
                splits = launch_capacitance_partial<double>(stream, rows, cc, n, J + (int64_t)r0 * ldj, ldj, z64,
                                                            ldz, true, gp, pe);
            });
            launch_capacitance_reduce(stream, rows, cc, splits, gp, true, alpha, 0,
                                      Sbuf.as<double>() + (int64_t)r0 * m + r0, m);
        } else {
            const double fl = 2.0 * m * cc * n;
            timed(H1W_K_GEMM, (double)m * n * 8 + (double)cc * n * zes, fl, [&] {
                if (!fp32)
                    splits = launch_capacitance_partial<double>(stream, m, cc, n, J, ldj, z64, ldz, false, gp, pe);
                else if (d.flags & H1W_FLAG_CAP_FP32_GEMM)
                    splits = launch_capacitance_partial_f32acc(stream, m, cc, n, J, ldj, z32, ldz, gp, pe);
                else
                    splits = launch_capacitance_partial<float>(stream, m, cc, n, J, ldj, z32, ldz, false, gp, pe);
            });
            launch_capacitance_reduce(stream, m, cc, splits, gp, false, alpha, r0, Sbuf.as<double>() + r0, m);
        }
    }
    if (lower) launch_mirror_lower(stream, m, Sbuf.as<double>());
    if (fp32) {
        // Z = Z1 - 1 mu^T + v s^T with mu_i the W-mean of the stored row Z1_i:
        // S += (J v) s^T - (J 1) mu^T, J 1 = wsum * s
        mudef.reserve((size_t)m * sizeof(double));
        jneg.reserve((size_t)m * sizeof(double));
        const int nch = launch_rows_dot_partial_f32(stream, m, n, Zbuf.as<float>(), ldz, wvec.as<double>(),
                                                    dpart.as<double>());
        launch_reduce_parts(stream, m, nch, dpart.as<double>(), mudef.as<double>());
        launch_scale(stream, m, 1.0 / wsum, mudef.as<double>(), mudef.as<double>());
        launch_scale(stream, m, -wsum, sdef.as<double>(), jneg.as<double>());
        launch_rank2_add(stream, m, jvdef.as<double>(), sdef.as<double>(), jneg.as<double>(), mudef.as<double>(),
                         Sbuf.as<double>());
    }
    // with several blocks the V-cycles and the products interleave: their sum
    // is reported as the Z build and the GEMM time is 0
    if (!one_block) ev_record(1);
    ev_record(2);
    asym = 0.0;
    if (fp32 || fac != H1W_FACTOR_CHOL) {
        launch_asym(stream, m, Sbuf.as<double>(), scal.as<double>());
        read_scal(1);
        asym = hscal[0] / alpha;
    }
    // factorisation: blocked Cholesky, else blocked LU without pivoting, else
    // LU with partial pivoting
    F1.reserve((size_t)m * m * sizeof(double));
    F2.reserve((size_t)m * m * sizeof(double));
    Dfwd.reserve(blocked_inv_elems(m) * sizeof(double));
    Dbwd.reserve(blocked_inv_elems(m) * sizeof(double));
    pivb.reserve((size_t)m * sizeof(int));
    int* dinfo = iflag.as<int>();
    int hinfo = -1;
    failed_pivot = -1;
    factor = 0;
    lu_pivoted = false;
    auto blocked = [&](int mode) {
        H1W_HIP(hipMemcpyAsync(F1.p, Sbuf.p, (size_t)m * m * sizeof(double), hipMemcpyDeviceToDevice, stream));
        const double mm = m;
        timed(H1W_K_FACTOR, 16.0 * mm * mm, (mode == 0 ? 1.0 : 2.0) * mm * mm * mm / 3.0, [&] {
            launch_blocked_factor(stream, m, F1.as<double>(), mode, Dfwd.as<double>(), Dbwd.as<double>(), dinfo);
        });
        H1W_HIP(hipMemcpyAsync(&hinfo, dinfo, sizeof(int), hipMemcpyDeviceToHost, stream));
        sync();
        return hinfo;
    };
    if (fac == H1W_FACTOR_CHOL) {
        if (blocked(0) < 0) {
            launch_transpose(stream, m, F1.as<double>(), F2.as<double>());
            factor = H1W_FACTOR_CHOL;
        } else {
            failed_pivot = hinfo;
            if (factor_ == H1W_FACTOR_CHOL) {
                if (info) info->failed_pivot = hinfo;
                throw Error{H1W_ENOTSPD, "Cholesky of S failed at column " + std::to_string(hinfo)};
            }
            fac = H1W_FACTOR_LU;
        }
    }
    if (fac == H1W_FACTOR_LU) {
        if (blocked(1) < 0) {
            launch_transpose(stream, m, F1.as<double>(), F2.as<double>());
        } else {  // a zero pivot without pivoting: fall back to partial pivoting
            H1W_HIP(hipMemcpyAsync(F1.p, Sbuf.p, (size_t)m * m * sizeof(double), hipMemcpyDeviceToDevice, stream));
            launch_lu(stream, m, F1.as<double>(), pivb.as<int>(), dinfo);
            H1W_HIP(hipMemcpyAsync(&hinfo, dinfo, sizeof(int), hipMemcpyDeviceToHost, stream));
            sync();
            if (hinfo >= 0) throw Error{H1W_ENUMERIC, "LU of S met a zero pivot at column " + std::to_string(hinfo)};
            launch_transpose(stream, m, F1.as<double>(), F2.as<double>());
            lu_pivoted = true;
        }
        factor = H1W_FACTOR_LU;
    }
    ev_record(3);
    // diagonal statistics: a cheap estimate of cond(S) from the pivots (its
    // square for Cholesky, S = U^T U) and max S_ii / alpha
    launch_diag_stats(stream, m, Sbuf.as<double>(), F1.as<double>(), scal.as<double>());
    read_scal(4);
    {
        const double pr = hscal[3] > 0.0 ? hscal[2] / hscal[3] : INFINITY;
        kappa_est = factor == H1W_FACTOR_CHOL ? pr * pr : pr;
        s_over_alpha = hscal[0] / alpha;
    }
    have_cap = true;
    sync();
    flush_timing();
    if (info) {
        // with a streamed Z the V-cycles and the GEMM chunks interleave: their
        // sum is reported as the Z build and the GEMM time is 0
        info->t_zbuild_ms = ev_ms(0, 1);
        info->t_gemm_ms = ev_ms(1, 2);
        info->zmode_used = z_streamed ? H1W_Z_RECOMPUTE : H1W_Z_STORED;
        info->t_factor_ms = ev_ms(2, 3);
        info->factor_used = factor;
        info->failed_pivot = failed_pivot;
        info->asym_S_over_alpha = asym;
        info->kappa_S_est = kappa_est;
        info->s_max_over_alpha = s_over_alpha;
        info->nlevels = (int)lv.size();
    }
}

void Ctx::solve_S(const double* in, double* x) {
    const double tb = 2.0 * (4.0 * m * m + 8.0 * blocked_inv_elems(m)), tf = 2.0 * m * m;
    auto solve2 = [&](const double* C1, const double* C2) {
        timed(H1W_K_TRSV, tb, tf, [&] {
            launch_blocked_solve2(stream, m, C1, Dfwd.as<double>(), true, C2, Dbwd.as<double>(), false, in, x);
        });
    };
    if (factor == H1W_FACTOR_CHOL) {  // S = U^T U: U^T y = in, then U x = y
        solve2(F1.as<double>(), F2.as<double>());
    } else if (!lu_pivoted) {  // S = L U
        solve2(F2.as<double>(), F2.as<double>());
    } else {
        if (x != in) H1W_HIP(hipMemcpyAsync(x, in, (size_t)m * sizeof(double), hipMemcpyDeviceToDevice, stream));
        launch_lu_solve(stream, m, F2.as<double>(), F1.as<double>(), pivb.as<int>(), x);
    }
}

// ============================================================ workspace for the Krylov loop

void Ctx::ensure_cg_ws(int mneed) {
    const int64_t n = N();
    mstride = std::max({mstride, mneed, 1});
    nvec.reserve((size_t)kNVec * pitch[0] * sizeof(double));
    mvec.reserve((size_t)kMVec * mstride * sizeof(double));
    // dot partials: up to 4 x 1024 blocks, or one per block of the stencil+dot kernel
    part.reserve((size_t)std::max<int64_t>(4 * 1024, cdiv(n, kBlock)) * sizeof(double));
    jpart.reserve(rows_dot_partial_elems(mstride, n) * sizeof(double));
}

double* Ctx::nv(int i) { return nvec.as<double>() + (size_t)i * pitch[0]; }
double* Ctx::mv(int i) { return mvec.as<double>() + (size_t)i * mstride; }

// out[slot..] = dot products of the given pairs (device); returns after the
// values are in hscal[slot..] when fetch is true.
int Ctx::dots_parts(int64_t len, std::initializer_list<std::pair<const double*, const double*>> pairs,
                    double* dst) {
    const double* X[4];
    const double* Y[4];
    int q = 0;
    for (auto& pr : pairs) {
        X[q] = pr.first;
        Y[q] = pr.second;
        ++q;
    }
    return launch_dots_partial(stream, len, q, X, Y, dst);
}

void Ctx::dots(int64_t len, std::initializer_list<std::pair<const double*, const double*>> pairs, int slot) {
    const double* X[4];
    const double* Y[4];
    int q = 0;
    for (auto& pr : pairs) {
        X[q] = pr.first;
        Y[q] = pr.second;
        ++q;
    }
    const int nb = launch_dots_partial(stream, len, q, X, Y, part.as<double>());
    launch_reduce_parts(stream, q, nb, part.as<double>(), scal.as<double>() + slot);
}

// w = S^{-1} J y and the J-space update Jz, Jp (Jp = Jz + beta Jp)
void Ctx::woodbury_mspace(const double* y, double* Jy, double* w) {
    rows_dot(m, J, ldj, y, Jy);
    solve_S(Jy, w);
}

// z = (y - Z~^T w) / alpha with the deflated FP32 Z~ and its rank-one parts
// (s.w, mu.w reduced inside the kernel when m allows, else by two launches)
void Ctx::z_stored_fp32(const double* w, const double* y, double ia, double* z) {
    const int64_t n = N();
    if (m <= 1024) {
        launch_z_stored<float>(stream, m, n, Zbuf.as<float>(), ldz, w, y, ia, vdef.as<double>(), nullptr, z,
                               sdef.as<double>(), mudef.as<double>());
    } else {
        dots(m, {{sdef.as<double>(), w}, {mudef.as<double>(), w}}, 8);  // s.w, mu.w for the rank-1 parts of Z
        launch_z_stored<float>(stream, m, n, Zbuf.as<float>(), ldz, w, y, ia, vdef.as<double>(),
                               scal.as<double>() + 8, z);
    }
}

// one preconditioner apply z = P^{-1} r without CG bookkeeping (h1w_precond_apply)
void Ctx::precond_one(const double* r, double* z, int zm) {
    const int64_t n = N();
    double* y = nv(kY);
    double* u = nv(kU);
    double* Jy = mv(kJy);
    double* w = mv(kW);
    apply_B(1, r, n, y, n);
    woodbury_mspace(y, Jy, w);
    if (zm == H1W_Z_STORED) {
        if (fp32) {
            z_stored_fp32(w, y, 1.0 / alpha, z);
        } else {
            launch_z_stored<double>(stream, m, n, Zbuf.as<double>(), ldz, w, y, 1.0 / alpha, nullptr, nullptr, z);
        }
    } else {
        double* dummy = mv(kTmp);
        H1W_HIP(hipMemsetAsync(dummy, 0, (size_t)m * sizeof(double), stream));
        launch_jt_u_t(stream, m, n, J, ldj, w, dummy, r, 1.0 / alpha, u, nv(kT));
        apply_B(1, u, n, z, n);
    }
}

void Ctx::precond_apply(int k, const double* R, int64_t ldr, double* Zout, int64_t ldzo, int zm) {
    if (!have_cap) throw Error{H1W_ESTATE, "no capacitance matrix: call h1w_capacitance_build first"};
    if (zm == H1W_Z_AUTO) zm = fp32 ? H1W_Z_STORED : H1W_Z_RECOMPUTE;
    require(zm == H1W_Z_STORED || zm == H1W_Z_RECOMPUTE, "zmode must be AUTO, STORED or RECOMPUTE");
    require(!(fp32 && zm == H1W_Z_RECOMPUTE), "a MIXED context needs zmode STORED");
    require(!(z_streamed && zm == H1W_Z_STORED), "Z was streamed (not stored): use zmode RECOMPUTE");
    ensure_cg_ws(m);
    for (int i = 0; i < k; ++i) precond_one(R + (int64_t)i * ldr, Zout + (int64_t)i * ldzo, zm);
    sync();
}

// y = alpha*A x + J^T (J x)
void Ctx::gn_apply(int mm, const double* JJ, int64_t ldjj, double al, const double* x, double* y) {
    const int64_t n = N();
    double* tmp = nv(kTmpN);
    double* Jx = mv(kJx);
    timed(H1W_K_APPLY, 16.0 * n, 0.0, [&] { launch_apply<double>(stream, dim, lv[0], 1, x, n, tmp, n, al); });
    if (mm > 0) {
        rows_dot(mm, JJ, ldjj, x, Jx);
        timed(H1W_K_JTV, 8.0 * mm * n + 24.0 * n, 2.0 * mm * n,
              [&] { launch_jt_plain(stream, mm, n, JJ, ldjj, Jx, y, tmp, 1.0); });
    } else {
        H1W_HIP(hipMemcpyAsync(y, tmp, n * sizeof(double), hipMemcpyDeviceToDevice, stream));
    }
}

// ============================================================ GN solve

void Ctx::gn_solve(int m_, const double* J_, int64_t ldj_, double alpha_, const double* b_, const double* dvec,
                   const double* res, double* x, const h1w_solve_opts& o, h1w_info* info) {
    const int64_t n = N();
    const bool laplace = (o.flags & H1W_SOLVE_LAPLACE_ONLY) != 0;
    // EXACT_B: B = A^-1 (MG-PCG to exact_rtol) for the whole call; the
    // capacitance it builds is discarded at return
    struct ExactScope {
        Ctx& c;
        bool on;
        ExactScope(Ctx& cc, bool o) : c(cc), on(o) { c.exact_b = o; }
        ~ExactScope() {
            c.exact_b = false;
            if (on) c.have_cap = false;
        }
    } exact_scope(*this, (o.flags & H1W_SOLVE_EXACT_B) != 0);
    ev_reserve();
    rsum_of = nullptr;
    H1W_HIP(hipEventRecord(ev[5], stream));
    if (m_ > 0 && !laplace) {
        capacitance_build(m_, J_, ldj_, alpha_, o.factor, info);
    } else {
        have_cap = false;
        m = laplace ? m_ : 0;
        J = J_;
        ldj = ldj_;
        alpha = alpha_;
    }
    ensure_cg_ws(m);
    int zm = o.zmode;
    if (zm == H1W_Z_AUTO) zm = fp32 ? H1W_Z_STORED : H1W_Z_RECOMPUTE;
    require(laplace || !(fp32 && zm == H1W_Z_RECOMPUTE), "a MIXED context needs zmode STORED");
    if (m > 0 && !laplace && z_streamed) {
        require(zm != H1W_Z_STORED || o.zmode == H1W_Z_AUTO, "Z was streamed (not stored): use zmode RECOMPUTE");
        zm = H1W_Z_RECOMPUTE;
    }
    const bool flexible = fp32;
    const double rtol = o.rtol > 0 ? o.rtol : 1e-10;
    const int maxit = o.maxit > 0 ? o.maxit : 500;
    const double ia = 1.0 / alpha;
    ev_record(4);

    double *r = nv(kR), *p = nv(kP), *q = nv(kQ), *y = nv(kY), *u = nv(kU), *z = nv(kZ), *t = nv(kT),
           *bb = nv(kB), *tmp = nv(kTmpN);
    double *Jy = mv(kJy), *w = mv(kW), *Jz = mv(kJz), *Jp = mv(kJp);
    const double* b = b_;
    if (!b) {  // paper-form right-hand side b = -alpha*A d - J^T res
        launch_apply<double>(stream, dim, lv[0], 1, dvec, n, tmp, n, alpha);
        if (m > 0)
            launch_jt_plain(stream, m, n, J, ldj, res, bb, tmp, 1.0);
        else
            H1W_HIP(hipMemcpyAsync(bb, tmp, n * sizeof(double), hipMemcpyDeviceToDevice, stream));
        launch_axpby(stream, n, -1.0, bb, 0.0, bb);
        b = bb;
    }
    // x = 0, r = b, p = q = 0, Jp = 0 and b.b in two launches; the norm is
    // written to host-visible memory
    {
        const int nb = launch_cg_init(stream, n, b, x, r, p, q, m, Jp, part.as<double>());
        launch_reduce_host(stream, 1, nb, part.as<double>(), drep);
        sync();
    }
    const double bnorm = std::sqrt(hrep[0]);
    if (!std::isfinite(bnorm)) throw Error{H1W_ENUMERIC, "non-finite right-hand side"};

    int it = 0, restarts = 0;
    double relres_rec = 0.0, relres_true = 0.0;
    // Residual replacement. The Jz recurrence Jz = (Jy - (S - alpha I) w) / alpha
    // carries the rounding of S and of the J-space products amplified by
    // ||S|| / alpha, and in the recompute form also the difference between the
    // two V-cycles B (J^T w) and Z^T w; so the recursive residual drifts from
    // the true one by an amount that grows with the residual size during the
    // iteration (measured at 129^3: 4.5e-8 ||b|| in the recompute form, 5.5e-9
    // in the stored form, about 100 u max S_ii / alpha). Once the recursive
    // residual is below sqrt(rtol), r is replaced by the true residual, keeping
    // the search direction, which bounds the later drift far below rtol
    // (otherwise the final check can fail and force a late restart). Always in
    // the recompute form; in the stored form when the predicted drift reaches
    // a tenth of rtol.
    const bool drifts = 100.0 * 0.5 * DBL_EPSILON * s_over_alpha >= 0.1 * rtol;
    const double replace_tol =
        (m > 0 && !laplace && (zm == H1W_Z_RECOMPUTE || drifts)) ? std::sqrt(rtol) : 0.0;
    bool replaced = false;
    h1w_status status = H1W_OK;

    // z = P^{-1} r, p = z + beta p, t = J^T Jp. The scalars stay on the device
    // (dsc, see launch_gn_beta); r.z <= 0 (converged to rounding) is flagged
    // there and read with the residual norm after the next update.
    double* dsc = scal.as<double>() + kGnScal;
    auto precond_step = [&](bool first) {
        apply_B(1, r, n, y, n);
        if (m == 0 || laplace) {
            // z = B r / alpha (no Woodbury correction); t = J^T (J p) by two passes
            const int nb1 = dots_parts(n, {{r, y}, {y, q}}, part.as<double>());
            launch_gn_beta(stream, part.as<double>(), 2, nb1, nullptr, 0, 0, ia, 2, first, flexible,
                           scal.as<double>(), dsc);
            launch_axpby_dev(stream, n, ia, y, dsc + 2, p);
            if (m == 0) {
                H1W_HIP(hipMemsetAsync(t, 0, n * sizeof(double), stream));
            } else {
                rows_dot(m, J, ldj, p, Jp);
                timed(H1W_K_JTV, 8.0 * m * n + 8.0 * n, 2.0 * m * n,
                      [&] { launch_jt_plain(stream, m, n, J, ldj, Jp, t, nullptr, 0.0); });
            }
            return;
        }
        woodbury_mspace(y, Jy, w);
        if (zm == H1W_Z_RECOMPUTE) {
            // r.z = (r.y - w.Jy) / alpha with z = B(r - J^T w)/alpha
            const int nb1 = dots_parts(n, {{r, y}}, part.as<double>());
            const int nb2 = dots_parts(m, {{w, Jy}}, part.as<double>() + kPartB);
            launch_gn_beta(stream, part.as<double>(), 1, nb1, part.as<double>() + kPartB, 1, nb2, ia, 0, first,
                           false, scal.as<double>(), dsc);
            launch_jz_update_dev(stream, m, Sbuf.as<double>(), alpha, Jy, w, dsc + 2, Jz, Jp);
            timed(H1W_K_JTV, 8.0 * m * n + 24.0 * n, 4.0 * m * n,
                  [&] { launch_jt_u_t(stream, m, n, J, ldj, w, Jp, r, ia, u, t); });
            apply_B(1, u, n, z, n);
            launch_axpby_dev(stream, n, 1.0, z, dsc + 2, p);
        } else {
            timed(H1W_K_JTV, (fp32 ? 4.0 : 8.0) * m * n + 16.0 * n, 2.0 * m * n, [&] {
                if (fp32) {
                    z_stored_fp32(w, y, ia, z);
                } else {
                    launch_z_stored<double>(stream, m, n, Zbuf.as<double>(), ldz, w, y, ia, nullptr, nullptr, z);
                }
            });
            const int nb1 = dots_parts(n, {{z, r}, {z, q}}, part.as<double>());
            launch_gn_beta(stream, part.as<double>(), 2, nb1, nullptr, 0, 0, ia, 1, first, flexible,
                           scal.as<double>(), dsc);
            launch_jz_update_dev(stream, m, Sbuf.as<double>(), alpha, Jy, w, dsc + 2, Jz, Jp);
            launch_axpby_dev(stream, n, 1.0, z, dsc + 2, p);
            timed(H1W_K_JTV, 8.0 * m * n + 8.0 * n, 2.0 * m * n,
                  [&] { launch_jt_plain(stream, m, n, J, ldj, Jp, t, nullptr, 0.0); });
        }
    };
    auto true_relres = [&]() -> double {
        rsum_of = nullptr;  // r is replaced after a true-residual check
        gn_apply(m, J, ldj, alpha, x, z);  // z is free here; gn_apply uses tmp internally
        launch_sub(stream, n, b, z, u);
        const int nb = dots_parts(n, {{u, u}}, part.as<double>());
        launch_reduce_host(stream, 1, nb, part.as<double>(), drep);
        sync();
        return bnorm > 0 ? std::sqrt(hrep[0]) / bnorm : 0.0;
    };

    if (bnorm == 0.0) {
        relres_true = 0.0;
    } else {
        precond_step(true);
        for (;;) {
            // q = alpha A p + t, p.q, a = r.z / p.q (0 when r.z <= 0 or p.q <= 0
            // was flagged), x += a p, r -= a q, r.r: one host round trip
            int np = 0;
            timed(H1W_K_APPLY, 24.0 * n, 0.0,
                  [&] { launch_apply_plus_dot(stream, dim, lv[0], alpha, p, t, q, part.as<double>(), &np); });
            launch_gn_alpha(stream, part.as<double>(), np, dsc);
            // mixed: the update also leaves the partial sums of r for the
            // constant-mode deflation of the next preconditioner apply
            // (not with V-cycle graphs: a captured cycle must not depend on it)
            double* psum = (fp32 && deflate && !graphs) ? part.as<double>() + kPartB : nullptr;
            launch_cg_update_dev(stream, n, dsc + 1, p, q, x, r, part.as<double>(), &np, psum);
            if (psum) {
                rsum_of = r;
                rsum_part = psum;
                rsum_nb = np;
            }
            launch_gn_report(stream, part.as<double>(), np, dsc, drep);
            sync();
            const double* hs = hrep;
            if (hs[7] != 0.0) {
                status = H1W_ENUMERIC;
                break;
            }
            const bool ok = hs[5] == 0.0 && hs[6] == 0.0;
            if (ok) {
                if (!std::isfinite(hs[4])) {
                    status = H1W_ENUMERIC;
                    break;
                }
                relres_rec = std::sqrt(hs[4]) / bnorm;
                ++it;
            }
            if (!ok || relres_rec <= rtol) {
                relres_true = true_relres();
                if (!std::isfinite(relres_true)) {
                    status = H1W_ENUMERIC;
                    break;
                }
                if (relres_true <= rtol) break;
                if (++restarts > 8 || it >= maxit) {
                    status = H1W_ENOCONV;
                    break;
                }
                // restart from the true residual (a restart whose r.z <= 0 is
                // seen by the next check and ends in ENOCONV after 8 restarts)
                H1W_HIP(hipMemcpyAsync(r, u, n * sizeof(double), hipMemcpyDeviceToDevice, stream));
                precond_step(true);
                continue;
            }
            if (!replaced && relres_rec <= replace_tol && it < maxit) {
                replaced = true;
                relres_true = true_relres();
                if (!std::isfinite(relres_true)) {
                    status = H1W_ENUMERIC;
                    break;
                }
                if (relres_true <= rtol) break;
                ++restarts;
                H1W_HIP(hipMemcpyAsync(r, u, n * sizeof(double), hipMemcpyDeviceToDevice, stream));
                precond_step(false);  // the direction is kept
                continue;
            }
            if (it >= maxit) {
                relres_true = true_relres();
                status = relres_true <= rtol ? H1W_OK : H1W_ENOCONV;
                break;
            }
            precond_step(false);
        }
    }
    rsum_of = nullptr;
    ev_record(6);
    sync();
    flush_timing();
    if (info) {
        info->iters = it;
        info->restarts = restarts;
        info->relres_true = relres_true;
        info->relres_rec = relres_rec;
        info->zmode_used = (m > 0 && !laplace) ? zm : 0;
        info->t_cg_ms = ev_ms(4, 6);
        info->t_total_ms = ev_ms(5, 6);
        info->nlevels = (int)lv.size();
    }
    if (status == H1W_ENOCONV) throw Error{H1W_ENOCONV, "GN-CG did not reach rtol within maxit iterations"};
    if (status == H1W_ENUMERIC) throw Error{H1W_ENUMERIC, "NaN or Inf in the CG recurrences"};
}

// ============================================================ constant-mode deflation (mixed)

void Ctx::ensure_deflation_vectors() {
    if (vdef_ready) return;
    const int64_t n = N();
    wvec.reserve((size_t)n * sizeof(double));
    ones.reserve((size_t)n * sizeof(double));
    vdef.reserve((size_t)n * sizeof(double));
    launch_node_weights(stream, dim, lv[0], wvec.as<double>());
    launch_fill(stream, n, 1.0, ones.as<double>());
    vcycle<double>(1, wvec.as<double>(), n, vdef.as<double>(), n);  // v = B W1 in FP64
    vdef_ready = true;
}

// ============================================================ J v with timing

void Ctx::rows_dot(int mm, const double* M, int64_t ldm, const double* v, double* out) {
    const int64_t n = N();
    int nchunk = 0;
    timed(H1W_K_JV, 8.0 * mm * n + 8.0 * n, 2.0 * mm * n,
          [&] { nchunk = launch_rows_dot_partial(stream, mm, n, M, ldm, v, jpart.as<double>()); });
    if (mm > 0) launch_reduce_parts(stream, mm, nchunk, jpart.as<double>(), out);
}

// ============================================================ kernel timing

hipEvent_t Ctx::take_event() {
    if (!evpool.empty()) {
        hipEvent_t e = evpool.back();
        evpool.pop_back();
        return e;
    }
    hipEvent_t e;
    H1W_HIP(hipEventCreate(&e));
    return e;
}

void Ctx::flush_timing() {
    if (pending.empty()) return;
    sync();
    for (const auto& p : pending) {
        float ms = 0.f;
        H1W_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        h1w_kstat& s = kst[p.cls];
        s.launches += 1;
        s.ms += ms;
        s.bytes += p.bytes;
        s.flops += p.flops;
        evpool.push_back(p.a);
        evpool.push_back(p.b);
    }
    pending.clear();
}

// ============================================================ events

void Ctx::ev_reserve() {
    for (auto& e : ev)
        if (!e) H1W_HIP(hipEventCreate(&e));
}
void Ctx::ev_record(int i) {
    ev_reserve();
    H1W_HIP(hipEventRecord(ev[i], stream));
}
double Ctx::ev_ms(int a, int b) {
    float ms = 0.f;
    H1W_HIP(hipEventElapsedTime(&ms, ev[a], ev[b]));
    return ms;
}

template void Ctx::vcycle<double>(int, const double*, int64_t, double*, int64_t);
template void Ctx::vcycle<float>(int, const float*, int64_t, float*, int64_t);

}  // namespace h1w
