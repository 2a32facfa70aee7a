// C ABI entry points (include/h1w.h): argument validation on the host,
// translation of internal errors to status codes; no exception crosses the ABI.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "context.h"

struct h1w_ctx {
    h1w::Ctx c;
};

namespace {

thread_local std::string g_setup_error;

// H1W_TRACE=1 in the environment: one line per entry-point call on stderr
// (name, context, status, host wall time, and the error message on failure)
bool trace_on() {
    static const bool on = [] {
        const char* v = std::getenv("H1W_TRACE");
        return v && *v && std::strcmp(v, "0") != 0;
    }();
    return on;
}

h1w_status traced(const char* name, const h1w_ctx* ctx, h1w_status st,
                  std::chrono::steady_clock::time_point t0) {
    if (trace_on()) {
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        std::fprintf(stderr, "[h1w] %s ctx=%p status=%d %.3f ms%s%s\n", name, (const void*)ctx, (int)st, ms,
                     st != H1W_OK && ctx ? " : " : "", st != H1W_OK && ctx ? ctx->c.err.c_str() : "");
    }
    return st;
}

template <typename Fn>
h1w_status guarded(const char* name, h1w_ctx* ctx, Fn&& fn) {
    const auto t0 = std::chrono::steady_clock::now();
    try {
        fn();
        if (ctx) ctx->c.err.clear();
        return traced(name, ctx, H1W_OK, t0);
    } catch (const h1w::Error& e) {
        if (ctx) ctx->c.err = e.msg;
        return traced(name, ctx, e.st, t0);
    } catch (const std::bad_alloc&) {
        if (ctx) ctx->c.err = "host allocation failed";
        return traced(name, ctx, H1W_ENOMEM, t0);
    } catch (const std::exception& e) {
        if (ctx) ctx->c.err = e.what();
        return traced(name, ctx, H1W_EINVAL, t0);
    }
}

using h1w::require;

void need_ptr(const void* p, size_t align, const char* what) {
    require(p != nullptr, std::string(what) + " is NULL");
    require(reinterpret_cast<uintptr_t>(p) % align == 0, std::string(what) + " is not aligned");
}

// rows [0, k) of length n with leading dimension ld, element size es
bool overlap(const void* a, int64_t lda, const void* b, int64_t ldb, int k, int64_t n, size_t es) {
    if (k <= 0) return false;
    const char* a0 = static_cast<const char*>(a);
    const char* b0 = static_cast<const char*>(b);
    const char* a1 = a0 + ((int64_t)(k - 1) * lda + n) * es;
    const char* b1 = b0 + ((int64_t)(k - 1) * ldb + n) * es;
    return a0 < b1 && b0 < a1;
}

}  // namespace

namespace {

// copies a device int32 array of n entries to the host (synchronous)
std::vector<int> fetch_ints(h1w::Ctx& c, const int* d, size_t n) {
    std::vector<int> h(n);
    if (n) {
        H1W_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(int), hipMemcpyDeviceToHost, c.stream));
        c.sync();
    }
    return h;
}

void check_sources(h1w::Ctx& c, int n_src, const int* src_node) {
    require(n_src >= 1 && n_src <= 64, "n_src must be in [1, 64]");
    need_ptr(src_node, 4, "src_node");
    for (int v : fetch_ints(c, src_node, (size_t)n_src)) {
        require(v >= 0 && v < c.N(), "src_node entry out of range");
        require(!h1w::ert_on_dirichlet_host(c.lv[0], c.dmask, v), "a source node lies on a Dirichlet face");
    }
}

// validated options of a Gauss-Newton solve on context c
h1w_solve_opts gn_options(const h1w::Ctx& c, const h1w_solve_opts* opts) {
    h1w_solve_opts o{};
    if (opts) o = *opts;
    require(std::isfinite(o.rtol) && o.rtol >= 0.0, "rtol must be >= 0");
    require(o.maxit >= 0, "maxit must be >= 0");
    require(o.zmode >= H1W_Z_AUTO && o.zmode <= H1W_Z_RECOMPUTE, "zmode must be AUTO, STORED or RECOMPUTE");
    require(o.factor >= H1W_FACTOR_AUTO && o.factor <= H1W_FACTOR_LU, "factor must be AUTO, CHOL or LU");
    require(o.check_every == 0, "check_every must be 0");
    require((o.flags & ~(H1W_SOLVE_LAPLACE_ONLY | H1W_SOLVE_EXACT_B)) == 0, "unknown bits in flags");
    require(o.flags != (H1W_SOLVE_LAPLACE_ONLY | H1W_SOLVE_EXACT_B), "LAPLACE_ONLY and EXACT_B exclude each other");
    require(!(o.flags & H1W_SOLVE_EXACT_B) || !c.fp32, "EXACT_B needs an FP64 context");
    return o;
}

h1w_solve_opts ert_options(const h1w_solve_opts* opts) {
    h1w_solve_opts o{};
    if (opts) o = *opts;
    require(std::isfinite(o.rtol) && o.rtol >= 0.0, "rtol must be >= 0");
    require(o.maxit >= 0, "maxit must be >= 0");
    if (o.rtol == 0.0) o.rtol = 1e-12;
    if (o.maxit == 0) o.maxit = 500;
    return o;
}

void check_pairs(h1w::Ctx& c, int n_src, int n_meas, const int* pair) {
    require(n_meas >= 0, "n_meas must be >= 0");
    if (n_meas == 0) return;
    need_ptr(pair, 4, "pair");
    const std::vector<int> h = fetch_ints(c, pair, (size_t)2 * n_meas);
    for (int i = 0; i < n_meas; ++i) {
        const int a = h[2 * i], b = h[2 * i + 1];
        require(a >= 0 && a < n_src && b >= 0 && b < n_src, "pair index out of [0, n_src)");
        require(a != b, "a pair needs two different electrodes");
    }
}

}  // namespace

extern "C" {

const char* h1w_status_string(h1w_status s) {
    switch (s) {
        case H1W_OK: return "ok";
        case H1W_EINVAL: return "invalid argument";
        case H1W_ENOMEM: return "out of device memory";
        case H1W_EHIP: return "HIP runtime error";
        case H1W_ENOTSPD: return "capacitance matrix not positive definite";
        case H1W_ENOCONV: return "no convergence within maxit";
        case H1W_ENUMERIC: return "NaN or Inf encountered";
        case H1W_ENOTIMPL: return "not implemented";
        case H1W_ESTATE: return "call order violated";
    }
    return "unknown status";
}

h1w_status h1w_setup(const h1w_grid_desc* desc, void* hip_stream, h1w_ctx** out) {
    g_setup_error.clear();
    if (!desc || !out) {
        g_setup_error = "desc and out must not be NULL";
        return H1W_EINVAL;
    }
    *out = nullptr;
    h1w_ctx* ctx = nullptr;
    try {
        ctx = new h1w_ctx();
    } catch (...) {
        g_setup_error = "host allocation failed";
        return H1W_ENOMEM;
    }
    const h1w_status st = guarded(__func__, ctx, [&] { ctx->c.init(*desc, static_cast<hipStream_t>(hip_stream)); });
    if (st != H1W_OK) {
        g_setup_error = ctx->c.err;
        delete ctx;
        return st;
    }
    // the address of the static scratch of h1w_gn_apply_noalloc on this
    // device (a failure here is reported by that entry point's first call)
    h1w::noalloc_init_device();
    *out = ctx;
    return H1W_OK;
}

void h1w_destroy(h1w_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->c.stream);
    delete ctx;
}

const char* h1w_last_error(const h1w_ctx* ctx) { return ctx ? ctx->c.err.c_str() : g_setup_error.c_str(); }

h1w_status h1w_get_sizes(const h1w_ctx* ctx, int64_t* N, int* nlevels) {
    if (!ctx) return H1W_EINVAL;
    if (N) *N = ctx->c.N();
    if (nlevels) *nlevels = (int)ctx->c.lv.size();
    return H1W_OK;
}

h1w_status h1w_operator_apply(h1w_ctx* ctx, int k, const void* X, int64_t ldx, void* Y, int64_t ldy, int dtype) {
    if (!ctx) return H1W_EINVAL;
    return guarded(__func__, ctx, [&] {
        auto& c = ctx->c;
        const int64_t n = c.N();
        require(k >= 0, "k must be >= 0");
        require(dtype == H1W_DT_F64 || dtype == H1W_DT_F32, "dtype must be H1W_DT_F64 or H1W_DT_F32");
        if (k == 0) return;
        const size_t es = dtype == H1W_DT_F64 ? 8 : 4;
        need_ptr(X, es, "X");
        need_ptr(Y, es, "Y");
        require(ldx >= n && ldy >= n, "leading dimensions must be >= N");
        require(!overlap(X, ldx, Y, ldy, k, n, es), "X and Y overlap");
        if (c.ert) {
            require(dtype == H1W_DT_F64, "an ERT context is FP64: dtype must be H1W_DT_F64");
            if (!c.ert_ready) throw h1w::Error{H1W_ESTATE, "no conductivity set (h1w_ert_set_conductivity)"};
            for (int r0 = 0; r0 < k; r0 += 65535) {
                const int kk = std::min(65535, k - r0);
                c.apply_A(kk, (const double*)X + (int64_t)r0 * ldx, ldx, (double*)Y + (int64_t)r0 * ldy, ldy);
            }
            return;
        }
        for (int r0 = 0; r0 < k; r0 += 65535) {
            const int kk = std::min(65535, k - r0);
            if (dtype == H1W_DT_F64)
                h1w::launch_apply<double>(c.stream, c.dim, c.lv[0], kk, (const double*)X + (int64_t)r0 * ldx, ldx,
                                          (double*)Y + (int64_t)r0 * ldy, ldy, 1.0);
            else
                h1w::launch_apply<float>(c.stream, c.dim, c.lv[0], kk, (const float*)X + (int64_t)r0 * ldx, ldx,
                                         (float*)Y + (int64_t)r0 * ldy, ldy, 1.0);
        }
    });
}

h1w_status h1w_poisson_solve_batched(h1w_ctx* ctx, int k, const void* F, int64_t ldf, void* X, int64_t ldx,
                                     int dtype, int mode, double rtol, int maxit, h1w_info* info) {
    if (!ctx) return H1W_EINVAL;
    if (info) *info = h1w_info{};
    if (info) info->failed_pivot = -1;
    return guarded(__func__, ctx, [&] {
        auto& c = ctx->c;
        const int64_t n = c.N();
        require(k >= 0, "k must be >= 0");
        require(mode == H1W_VCYCLE_ONCE || mode == H1W_MG_SOLVE, "mode must be H1W_VCYCLE_ONCE or H1W_MG_SOLVE");
        if (mode == H1W_VCYCLE_ONCE)
            require(dtype == (c.fp32 ? H1W_DT_F32 : H1W_DT_F64),
                    "VCYCLE_ONCE needs dtype F64 for an FP64 context and F32 for a MIXED one");
        else
            require(dtype == H1W_DT_F64, "MG_SOLVE needs dtype F64");
        if (info) info->nlevels = (int)c.lv.size();
        if (k == 0) return;
        const size_t es = dtype == H1W_DT_F64 ? 8 : 4;
        need_ptr(F, es, "F");
        need_ptr(X, es, "X");
        require(ldf >= n && ldx >= n, "leading dimensions must be >= N");
        require(!overlap(F, ldf, X, ldx, k, n, es), "F and X overlap");
        if (c.ert && !c.ert_ready) throw h1w::Error{H1W_ESTATE, "no conductivity set (h1w_ert_set_conductivity)"};
        if (mode == H1W_VCYCLE_ONCE && c.ert) {
            c.vcycle_B(k, (const double*)F, ldf, (double*)X, ldx);
        } else if (mode == H1W_VCYCLE_ONCE) {
            if (c.fp32)
                c.vcycle<float>(k, (const float*)F, ldf, (float*)X, ldx);
            else
                c.vcycle<double>(k, (const double*)F, ldf, (double*)X, ldx);
        } else {
            require(std::isfinite(rtol) && rtol > 0.0, "rtol must be > 0");
            require(maxit >= 0, "maxit must be >= 0");
            c.mg_solve(k, (const double*)F, ldf, (double*)X, ldx, rtol, maxit > 0 ? maxit : 200, info);
        }
    });
}

h1w_status h1w_capacitance_build(h1w_ctx* ctx, int m, const double* J, int64_t ldj, double alpha, int factor,
                                 double* S_out, int64_t lds, void* Z_out, int64_t ldz, h1w_info* info) {
    if (!ctx) return H1W_EINVAL;
    if (info) {
        *info = h1w_info{};
        info->failed_pivot = -1;
    }
    return guarded(__func__, ctx, [&] {
        auto& c = ctx->c;
        require(!c.ert, "this entry point needs an H1 Gram context (op = H1W_OP_H1GRAM)");
        const int64_t n = c.N();
        c.have_cap = false;
        require(m >= 1 && m <= 4096, "m must be in [1, 4096]");
        need_ptr(J, 8, "J");
        require(ldj >= n, "ldj must be >= N");
        require(std::isfinite(alpha) && alpha > 0.0, "alpha must be finite and > 0");
        require(factor >= H1W_FACTOR_AUTO && factor <= H1W_FACTOR_LU, "factor must be AUTO, CHOL or LU");
        if (S_out) {
            need_ptr(S_out, 8, "S_out");
            require(lds >= m, "lds must be >= m");
        }
        if (Z_out) {
            need_ptr(Z_out, c.fp32 ? 4 : 8, "Z_out");
            require(ldz >= n, "ldz must be >= N");
        }
        c.capacitance_build(m, J, ldj, alpha, factor, info);
        require(!(Z_out && c.z_streamed), "Z was streamed (too large to keep): Z_out is not available");
        if (S_out)
            H1W_HIP(hipMemcpy2DAsync(S_out, lds * sizeof(double), c.Sbuf.p, m * sizeof(double), m * sizeof(double), m,
                                     hipMemcpyDeviceToDevice, c.stream));
        if (Z_out) {
            if (c.fp32) {  // full Z = Z1 + v s^T rounded to FP32
                h1w::launch_zout_deflated(c.stream, m, n, c.Zbuf.as<float>(), c.ldz, c.sdef.as<double>(),
                                          c.mudef.as<double>(), c.vdef.as<double>(), (float*)Z_out, ldz);
            } else {
                H1W_HIP(hipMemcpy2DAsync(Z_out, ldz * 8, c.Zbuf.p, c.ldz * 8, n * 8, m, hipMemcpyDeviceToDevice,
                                         c.stream));
            }
        }
        c.sync();
    });
}

h1w_status h1w_precond_apply(h1w_ctx* ctx, int k, const double* R, int64_t ldr, double* Zout, int64_t ldz,
                             int zmode) {
    if (!ctx) return H1W_EINVAL;
    return guarded(__func__, ctx, [&] {
        auto& c = ctx->c;
        require(!c.ert, "this entry point needs an H1 Gram context (op = H1W_OP_H1GRAM)");
        const int64_t n = c.N();
        require(k >= 0, "k must be >= 0");
        if (k == 0) return;
        need_ptr(R, 8, "R");
        need_ptr(Zout, 8, "Zout");
        require(ldr >= n && ldz >= n, "leading dimensions must be >= N");
        require(!overlap(R, ldr, Zout, ldz, k, n, 8), "R and Zout overlap");
        c.precond_apply(k, R, ldr, Zout, ldz, zmode);
    });
}

h1w_status h1w_gn_solve(h1w_ctx* ctx, int m, const double* J, int64_t ldj, double alpha, const double* b,
                        const double* d, const double* res, double* x, const h1w_solve_opts* opts, h1w_info* info) {
    if (!ctx) return H1W_EINVAL;
    if (info) {
        *info = h1w_info{};
        info->failed_pivot = -1;
    }
    return guarded(__func__, ctx, [&] {
        auto& c = ctx->c;
        require(!c.ert, "this entry point needs an H1 Gram context (op = H1W_OP_H1GRAM)");
        const int64_t n = c.N();
        require(m >= 0 && m <= 4096, "m must be in [0, 4096]");
        if (m > 0) {
            need_ptr(J, 8, "J");
            require(ldj >= n, "ldj must be >= N");
        }
        require(std::isfinite(alpha) && alpha > 0.0, "alpha must be finite and > 0");
        need_ptr(x, 8, "x");
        if (b) {
            need_ptr(b, 8, "b");
            require(!overlap(b, n, x, n, 1, n, 8), "b and x overlap");
        } else {
            need_ptr(d, 8, "d (b is NULL)");
            if (m > 0) need_ptr(res, 8, "res (b is NULL)");
            require(!overlap(d, n, x, n, 1, n, 8), "d and x overlap");
        }
        c.gn_solve(m, J, ldj, alpha, b, d, res, x, gn_options(c, opts), info);
    });
}

h1w_status h1w_gn_apply(h1w_ctx* ctx, int m, const double* J, int64_t ldj, double alpha, const double* x,
                        double* y) {
    if (!ctx) return H1W_EINVAL;
    return guarded(__func__, ctx, [&] {
        auto& c = ctx->c;
        require(!c.ert, "this entry point needs an H1 Gram context (op = H1W_OP_H1GRAM)");
        const int64_t n = c.N();
        require(m >= 0, "m must be >= 0");
        if (m > 0) {
            need_ptr(J, 8, "J");
            require(ldj >= n, "ldj must be >= N");
        }
        require(std::isfinite(alpha), "alpha must be finite");
        need_ptr(x, 8, "x");
        need_ptr(y, 8, "y");
        require(!overlap(x, n, y, n, 1, n, 8), "x and y overlap");
        c.ensure_cg_ws(m);
        c.gn_apply(m, J, ldj, alpha, x, y);
        c.sync();
    });
}

h1w_status h1w_gn_apply_noalloc(h1w_ctx* ctx, int m, const double* J, int64_t ldj, double alpha, const double* x,
                                double* y) {
    if (!ctx) return H1W_EINVAL;
    return guarded(__func__, ctx, [&] {
        auto& c = ctx->c;
        require(!c.ert, "this entry point needs an H1 Gram context (op = H1W_OP_H1GRAM)");
        const int64_t n = c.N();
        require(m >= 0, "m must be >= 0");
        h1w::noalloc_require_fits(m, n);
        if (m > 0) {
            need_ptr(J, 8, "J");
            require(ldj >= n, "ldj must be >= N");
        }
        require(std::isfinite(alpha), "alpha must be finite");
        need_ptr(x, 8, "x");
        need_ptr(y, 8, "y");
        require(!overlap(x, n, y, n, 1, n, 8), "x and y overlap");
        if (m > 0) {  // J (m rows of pitch ldj) against y (one row of N)
            const char* j0 = reinterpret_cast<const char*>(J);
            const char* j1 = j0 + ((int64_t)(m - 1) * ldj + n) * 8;
            const char* y0 = reinterpret_cast<const char*>(y);
            require(!(j0 < y0 + n * 8 && y0 < j1), "J and y overlap");
        }
        c.gn_apply_noalloc(m, J, ldj, alpha, x, y);
    });
}

h1w_status h1w_set_kernel_timing(h1w_ctx* ctx, unsigned mask) {
    if (!ctx) return H1W_EINVAL;
    return guarded(__func__, ctx, [&] {
        ctx->c.flush_timing();
        ctx->c.tmask = mask & ((1u << H1W_K_NCLASS) - 1);
    });
}

h1w_status h1w_get_kernel_timing(h1w_ctx* ctx, int kclass, h1w_kstat* out) {
    if (!ctx) return H1W_EINVAL;
    return guarded(__func__, ctx, [&] {
        require(kclass >= 0 && kclass < H1W_K_NCLASS, "kclass out of range");
        require(out != nullptr, "out is NULL");
        ctx->c.flush_timing();
        *out = ctx->c.kst[kclass];
    });
}

h1w_status h1w_reset_kernel_timing(h1w_ctx* ctx) {
    if (!ctx) return H1W_EINVAL;
    return guarded(__func__, ctx, [&] {
        ctx->c.flush_timing();
        for (auto& s : ctx->c.kst) s = h1w_kstat{};
    });
}

h1w_status h1w_batch_solve(int count, const h1w_batch_item* items, const h1w_batch_opts* opts,
                           h1w_info* infos, h1w_status* status, h1w_batch_report* report) {
    g_setup_error.clear();
    h1w_status st = H1W_OK;
    std::string item_msg;
    try {
        require(count >= 0, "count must be >= 0");
        require(count == 0 || items != nullptr, "items is NULL");
        require(opts != nullptr, "opts is NULL");
        require(opts->precision == H1W_FP64 || opts->precision == H1W_MIXED, "precision must be FP64 or MIXED");
        require(opts->nworkers >= 0 && opts->nu >= 0 && opts->nu <= 16 && opts->maxit >= 0,
                "nworkers, nu and maxit must be >= 0 (nu <= 16)");
        require(std::isfinite(opts->rtol) && opts->rtol >= 0.0, "rtol must be >= 0");
        require(opts->graphs == 0 || opts->graphs == 1, "graphs must be 0 or 1");
        require(opts->grouped == 0 || opts->grouped == 1, "grouped must be 0 or 1");
        require(opts->autotune >= 0 && opts->autotune <= 2, "autotune must be 0, 1 or 2");
        std::vector<h1w_status> own;
        h1w_status* stp = status;
        if (!stp) {
            own.assign((size_t)count, H1W_OK);
            stp = own.data();
        }
        h1w::batch_solve(count, items, *opts, infos, stp, report, &item_msg);
        for (int i = 0; i < count && st == H1W_OK; ++i) st = stp[i];
    } catch (const h1w::Error& e) {
        g_setup_error = e.msg;
        return e.st;
    } catch (const std::bad_alloc&) {
        g_setup_error = "host allocation failed";
        return H1W_ENOMEM;
    } catch (const std::exception& e) {
        g_setup_error = e.what();
        return H1W_EINVAL;
    }
    if (st != H1W_OK)
        g_setup_error = std::string("a batch item failed: ") + h1w_status_string(st) + " (" + item_msg + ")";
    return st;
}

h1w_status h1w_ert_set_conductivity(h1w_ctx* ctx, const double* logsig) {
    if (!ctx) return H1W_EINVAL;
    return guarded(__func__, ctx, [&] {
        auto& c = ctx->c;
        require(c.ert, "h1w_ert_set_conductivity needs an ERT context (op = H1W_OP_ERT)");
        need_ptr(logsig, 8, "logsig");
        c.ert_set_conductivity(logsig);
    });
}

h1w_status h1w_ert_sensitivities(h1w_ctx* ctx, const double* logsig, int n_src, const int* src_node, int n_meas,
                                 const int* pair, const double* kgeo, double* g_out, double* J_out, int64_t ldj,
                                 double* U_out, int64_t ldu, const h1w_solve_opts* opts, h1w_info* info) {
    if (!ctx) return H1W_EINVAL;
    if (info) {
        *info = h1w_info{};
        info->failed_pivot = -1;
    }
    return guarded(__func__, ctx, [&] {
        auto& c = ctx->c;
        require(c.ert, "h1w_ert_sensitivities needs an ERT context (op = H1W_OP_ERT)");
        const int64_t n = c.N();
        check_sources(c, n_src, src_node);
        check_pairs(c, n_src, n_meas, pair);
        if (kgeo && n_meas > 0) need_ptr(kgeo, 8, "kgeo");
        if (g_out && n_meas > 0) need_ptr(g_out, 8, "g_out");
        if (J_out && n_meas > 0) {
            need_ptr(J_out, 8, "J_out");
            require(ldj >= n, "ldj must be >= N");
        }
        if (U_out) {
            need_ptr(U_out, 8, "U_out");
            require(ldu >= n, "ldu must be >= N");
            require(!(J_out && n_meas > 0 && overlap(U_out, ldu, J_out, ldj, std::min(n_src, n_meas), n, 8)),
                    "U_out and J_out overlap");
        }
        const h1w_solve_opts o = ert_options(opts);
        if (logsig) need_ptr(logsig, 8, "logsig");
        c.ev_reserve();
        c.ev_record(0);
        if (logsig) c.ert_set_conductivity(logsig);
        if (!c.ert_ready) throw h1w::Error{H1W_ESTATE, "no conductivity set: pass logsig"};
        c.ev_record(1);
        double* U = U_out;
        int64_t lu = ldu;
        if (!U) {
            c.efield.reserve((size_t)n_src * c.pitch[0] * sizeof(double));
            U = c.efield.as<double>();
            lu = c.pitch[0];
        }
        c.efield_n = 0;
        c.ert_fields(n_src, src_node, U, lu, o.rtol, o.maxit, info);
        if (!U_out) c.efield_n = n_src;
        c.ev_record(2);
        if (n_meas > 0 && (g_out || J_out)) {
            const double* k = c.ert_kgeo(n_meas, pair, src_node, kgeo);
            if (g_out) c.ert_measure(n_meas, pair, src_node, k, U, lu, g_out);
            if (J_out) c.ert_sens(n_src, U, lu, n_meas, pair, k, J_out, ldj, nullptr, nullptr);
        }
        c.ev_record(3);
        c.sync();
        c.flush_timing();
        if (info) {
            info->t_zbuild_ms = c.ev_ms(0, 1);
            info->t_cg_ms = c.ev_ms(1, 2);
            info->t_gemm_ms = c.ev_ms(2, 3);
            info->t_total_ms = c.ev_ms(0, 3);
            info->nlevels = (int)c.lv.size();
        }
    });
}

h1w_status h1w_ert_vjp(h1w_ctx* ctx, int n_src, const int* src_node, const double* U, int64_t ldu, int n_meas,
                       const int* pair, const double* kgeo, const double* gbar, double* grad) {
    if (!ctx) return H1W_EINVAL;
    return guarded(__func__, ctx, [&] {
        auto& c = ctx->c;
        require(c.ert, "h1w_ert_vjp needs an ERT context (op = H1W_OP_ERT)");
        if (!c.ert_ready) throw h1w::Error{H1W_ESTATE, "no conductivity set"};
        const int64_t n = c.N();
        require(n_src >= 1 && n_src <= 64, "n_src must be in [1, 64]");
        check_pairs(c, n_src, n_meas, pair);
        need_ptr(grad, 8, "grad");
        if (!U) {
            if (c.efield_n != n_src)
                throw h1w::Error{H1W_ESTATE, "no kept pole fields with n_src rows (pass U)"};
            U = c.efield.as<double>();
            ldu = c.pitch[0];
        } else {
            need_ptr(U, 8, "U");
            require(ldu >= n, "ldu must be >= N");
        }
        if (n_meas == 0) {
            h1w::launch_fill(c.stream, n, 0.0, grad);
            return;
        }
        need_ptr(gbar, 8, "gbar");
        if (kgeo)
            need_ptr(kgeo, 8, "kgeo");
        else
            check_sources(c, n_src, src_node);
        const double* k = c.ert_kgeo(n_meas, pair, src_node, kgeo);
        c.ert_sens(n_src, U, ldu, n_meas, pair, k, nullptr, 0, gbar, grad);
        c.sync();
    });
}

h1w_status h1w_ert_gn_step(h1w_ctx* ert, h1w_ctx* h1, double* m, const double* m_ref, int n_src,
                           const int* src_node, int n_meas, const int* pair, const double* kgeo,
                           const double* g_obs, double alpha, double* J, int64_t ldj, double* dm, double* g_out,
                           const h1w_solve_opts* ert_opts, const h1w_solve_opts* gn_opts, h1w_info* info) {
    if (!ert || !h1) return H1W_EINVAL;
    if (info) {
        *info = h1w_info{};
        info->failed_pivot = -1;
    }
    return guarded(__func__, h1, [&] {
        auto& E = ert->c;
        auto& G = h1->c;
        require(E.ert, "the first context must be an ERT context");
        require(!G.ert, "the second context must be an H1 Gram context");
        const h1w::Geom& ge = E.lv[0];
        const h1w::Geom& gg = G.lv[0];
        require(ge.nx == gg.nx && ge.ny == gg.ny && ge.nz == gg.nz, "the two contexts must share the grid");
        const int64_t n = G.N();
        require(n_meas >= 1 && n_meas <= 4096, "n_meas must be in [1, 4096]");
        need_ptr(m, 8, "m");
        need_ptr(m_ref, 8, "m_ref");
        need_ptr(g_obs, 8, "g_obs");
        need_ptr(J, 8, "J");
        need_ptr(dm, 8, "dm");
        require(ldj >= n, "ldj must be >= N");
        require(std::isfinite(alpha) && alpha > 0.0, "alpha must be finite and > 0");
        require(!overlap(m, n, dm, n, 1, n, 8), "m and dm overlap");
        if (kgeo) need_ptr(kgeo, 8, "kgeo");
        if (g_out) need_ptr(g_out, 8, "g_out");
        check_sources(E, n_src, src_node);
        check_pairs(E, n_src, n_meas, pair);
        const h1w_solve_opts eo = ert_options(ert_opts);
        const h1w_solve_opts go = gn_options(G, gn_opts);
        // forward map and sensitivities at m (ERT context, its stream)
        h1w_info finfo{};
        E.ert_set_conductivity(m);
        E.efield.reserve((size_t)n_src * E.pitch[0] * sizeof(double));
        E.efield_n = 0;
        E.ert_fields(n_src, src_node, E.efield.as<double>(), E.pitch[0], eo.rtol, eo.maxit, &finfo);
        E.efield_n = n_src;
        E.egn.reserve((size_t)(n + 2 * n_meas) * sizeof(double));
        double* d = E.egn.as<double>();
        double* g = d + n;
        double* res = g + n_meas;
        const double* k = E.ert_kgeo(n_meas, pair, src_node, kgeo);
        E.ert_measure(n_meas, pair, src_node, k, E.efield.as<double>(), E.pitch[0], g);
        E.ert_sens(n_src, E.efield.as<double>(), E.pitch[0], n_meas, pair, k, J, ldj, nullptr, nullptr);
        E.sync();
        E.flush_timing();
        // GN step on the H1 context (its stream): d = m - m_ref, res = g - g_obs
        h1w::launch_sub(G.stream, n, m, m_ref, d);
        h1w::launch_sub(G.stream, n_meas, g, g_obs, res);
        G.gn_solve(n_meas, J, ldj, alpha, nullptr, d, res, dm, go, info);
        if (g_out) H1W_HIP(hipMemcpyAsync(g_out, g, n_meas * sizeof(double), hipMemcpyDeviceToDevice, G.stream));
        h1w::launch_axpby(G.stream, n, 1.0, dm, 1.0, m);
        G.sync();
    });
}

}  // extern "C"
