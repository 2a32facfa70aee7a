// Internal declarations of the h1w HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "h1w.h"

namespace h1w {

// Geometry of one grid level, passed by value to the stencil kernels.
// 2D grids use nz = 1 and the DIM = 2 kernels.
struct Geom {
    int nx, ny, nz;
    int64_t N;
    double ihx2, ihy2, ihz2;  // 1/h_d^2
    double beta;
};

constexpr int kBlock = 256;

// ---------------------------------------------------------------- errors
struct Error {
    h1w_status st;
    std::string msg;
};

#define H1W_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::h1w::Error{H1W_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define H1W_LAUNCHED() H1W_HIP(hipGetLastError())

inline void require(bool ok, const std::string& msg) {
    if (!ok) throw Error{H1W_EINVAL, msg};
}

// ---------------------------------------------------------------- graph capture
// Process-wide lock between stream captures (V-cycle graphs) and the runtime
// calls that synchronise with every stream (allocation, release, blocking
// copies): such a call made by another thread during a capture fails, so the
// two never overlap. Recursive, so that a capture that had to allocate would
// fail with the runtime's error instead of deadlocking.
inline std::recursive_mutex& capture_lock() {
    static std::recursive_mutex mu;
    return mu;
}

// ---------------------------------------------------------------- device memory
// Owning device buffer (the library's own workspace; caller arrays are raw pointers).
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        // work queued on any stream may still use the buffer
        if (p) {
            std::lock_guard<std::recursive_mutex> lk(capture_lock());
            (void)hipDeviceSynchronize();
            (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
    }
    // grow to at least `need` bytes (contents not preserved)
    void reserve(size_t need) {
        if (need <= bytes) return;
        release();
        std::lock_guard<std::recursive_mutex> lk(capture_lock());
        hipError_t e = hipMalloc(&p, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            throw Error{e == hipErrorOutOfMemory ? H1W_ENOMEM : H1W_EHIP,
                        "hipMalloc of " + std::to_string(need) + " bytes failed: " + hipGetErrorName(e) + " (" +
                            hipGetErrorString(e) + ")"};
        }
        bytes = need;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------- kernel launchers
// stencil.hip (T = double or float)
template <typename T>
void launch_apply(hipStream_t s, int dim, const Geom& g, int k, const T* X, int64_t ldx, T* Y,
                  int64_t ldy, double scale);
template <typename T>
void launch_smooth_first(hipStream_t s, int dim, const Geom& g, int k, const T* F, int64_t ldf,
                         T* X, int64_t ldx, double w);
template <typename T>
void launch_smooth(hipStream_t s, int dim, const Geom& g, int k, const T* F, int64_t ldf,
                   const T* Xin, int64_t ldi, T* Xout, int64_t ldo, double w);
// first two smoothing steps from zero fused: X = x1 + w1 D^-1 (F - A x1), x1 = w0 D^-1 F
template <typename T>
void launch_pre2(hipStream_t s, int dim, const Geom& g, int k, const T* F, int64_t ldf, T* X, int64_t ldx,
                 double w0, double w1);
template <typename T>
void launch_residual(hipStream_t s, int dim, const Geom& g, int k, const T* F, int64_t ldf,
                     const T* X, int64_t ldx, T* R, int64_t ldr);
template <typename T>
void launch_restrict(hipStream_t s, int dim, const Geom& gf, const Geom& gc, int k, const T* R,
                     int64_t ldr, T* Fc, int64_t ldc);
template <typename T>
void launch_prolong_add(hipStream_t s, int dim, const Geom& gf, const Geom& gc, int k,
                        const T* Ec, int64_t ldc, T* X, int64_t ldx);
// X = Cinv F (k rows); part: partial-sum workspace of part_elems elements
// (may be null: no j splitting), at most coarse_part_elems(Nc) are used
template <typename T>
void launch_coarse_solve(hipStream_t s, int64_t Nc, const T* Cinv, int k, const T* F,
                         int64_t ldf, T* X, int64_t ldx, T* part, size_t part_elems);
size_t coarse_part_elems(int64_t Nc);
// j-range splits of the coarsest solve for k right-hand sides (1 .. ceil(Nc / 32))
int coarse_splits(int64_t Nc, int k, size_t part_elems);
template <typename TI, typename TO>
void launch_convert(hipStream_t s, int64_t N, int k, const TI* X, int64_t ldx, TO* Y,
                    int64_t ldy, double scale);
// q = a*A p + t  and per-block partial sums of p.q  (double only)
void launch_apply_plus_dot(hipStream_t s, int dim, const Geom& g, double a, const double* P,
                           const double* Tv, double* Q, double* partial, int* nparts);

// vfused.hip: fused V-cycle passes on nested 3D levels (two smoothing steps per side)
bool fused_levels_ok(const Geom& gf, const Geom& gc);
// X = two pre-smoothing steps from zero on F (weights w0, w1), Fc = 2^-3 P^T (F - A X)
template <typename T>
void launch_vdown(hipStream_t s, const Geom& gf, const Geom& gc, int k, const T* F, int64_t ldf, T* X, int64_t ldx,
                  T* Fc, int64_t ldc, double w0, double w1);
// Y = two post-smoothing steps (weights wa, wb) on F from X0 + P Ec (Y must not alias X0)
template <typename T>
void launch_vup(hipStream_t s, const Geom& gf, const Geom& gc, int k, const T* F, int64_t ldf, const T* X0,
                int64_t ldx0, const T* Ec, int64_t ldc, T* Y, int64_t ldy, double wa, double wb);

// ert.hip: host check of a node against the Dirichlet faces of an ERT grid
bool ert_on_dirichlet_host(const Geom& g, unsigned mask, int64_t p);

// vfused2d.hip: fused passes of the 2D V-cycle (two smoothing steps per side)
bool fused2_levels_ok(const Geom& gf, const Geom& gc);
// The coarse end of a 2D fused V-cycle in one launch (one work-group per
// right-hand side, every level in LDS): levels l0 .. L-1 of the hierarchy.
constexpr int kTailLevels = 6;
constexpr int kTailElems = 19712;  // LDS values per work-group (FP64: 154 KiB)
constexpr int kTailMaxNc = 289;    // largest coarsest level it solves
struct TailGeo {
    int L;                    // levels in the tail; the last is the coarsest
    Geom g[kTailLevels];
    int off[kTailLevels];     // LDS offset of level q's f, x, t (g[q].N values each)
    int red;                  // LDS offset of the coarse solve's partial sums
    int csplit;               // j-range splits of the coarsest solve (those of the separate solve)
};
// l0 = first level of the tail and its layout; false (l0 = L) when no tail fits
bool tail2_plan(const Geom* lv, int L, int& l0, TailGeo& tg);
template <typename T>
void launch_vtail2(hipStream_t s, const TailGeo& tg, const T* Cinv, int k, const T* F, int64_t ldf, T* X,
                   int64_t ldx, double w0, double w1);
template <typename T>
void launch_vdown2(hipStream_t s, const Geom& gf, const Geom& gc, int k, const T* F, int64_t ldf, T* X, int64_t ldx,
                   T* Fc, int64_t ldc, double w0, double w1);
template <typename T>
void launch_vup2(hipStream_t s, const Geom& gf, const Geom& gc, int k, const T* F, int64_t ldf, const T* X0,
                 int64_t ldx0, const T* Ec, int64_t ldc, T* Y, int64_t ldy, double wa, double wb);

// batch.hip: the executor behind h1w_batch_solve (throws Error on setup failures;
// per-item failures go to status[])
void batch_solve(int count, const h1w_batch_item* items, const h1w_batch_opts& o, h1w_info* infos,
                 h1w_status* status, h1w_batch_report* report, std::string* first_err);

// blas.hip
// partial dot products of npair vector pairs over N entries; returns #parts
int launch_dots_partial(hipStream_t s, int64_t N, int npair, const double* const* X,
                        const double* const* Y, double* partial);
void launch_reduce_parts(hipStream_t s, int nvec, int nparts, const double* partial,
                         double* out);
// per-row dot products out[i] = sum_n M[i,n] v[n] for i < m (M double), deterministic
int launch_rows_dot_partial(hipStream_t s, int m, int64_t N, const double* M, int64_t ldm,
                            const double* v, double* partial);  // returns #chunks
size_t rows_dot_partial_elems(int m, int64_t N);
// noalloc.hip: the static device scratch of h1w_gn_apply_noalloc (its
// address taken once per device; elements it needs for m rows on N nodes)
void noalloc_init_device();
size_t noalloc_scratch_elems(int m, int64_t N);
void noalloc_require_fits(int m, int64_t N);  // EINVAL beyond the array's size
// transpose products, see blas.hip for the epilogue modes
void launch_jt_u_t(hipStream_t s, int m, int64_t N, const double* J, int64_t ldj,
                   const double* w, const double* jp, const double* r, double inv_alpha,
                   double* u, double* t);
void launch_jt_plain(hipStream_t s, int m, int64_t N, const double* J, int64_t ldj,
                     const double* v, double* out, const double* add, double add_coef);
template <typename TZ>
void launch_p_stored(hipStream_t s, int m, int64_t N, const TZ* Z, int64_t ldz, const double* w,
                     const double* J, int64_t ldj, const double* jp, const double* y,
                     double inv_alpha, double beta, double* p, double* t);
// z = (y - Z^T w - c0 v + c1) * inv_alpha with (c0, c1) = cptr[0..1] (v may be null: no extra terms);
// with sd and md given (m <= 1024), c0 = sd.w and c1 = md.w are computed in the kernel (cptr unused)
template <typename TZ>
void launch_z_stored(hipStream_t s, int m, int64_t N, const TZ* Z, int64_t ldz, const double* w,
                     const double* y, double inv_alpha, const double* v, const double* cptr, double* z,
                     const double* sd = nullptr, const double* md = nullptr);
int launch_rows_dot2_partial(hipStream_t s, int m, int64_t N, const double* M, int64_t ldm, const double* v1,
                             const double* v2, double* part1, double* part2);
void launch_rank2_add(hipStream_t s, int m, const double* a, const double* b, const double* c, const double* d,
                      double* S);
int launch_rows_dot_partial_f32(hipStream_t s, int m, int64_t N, const float* M, int64_t ldm, const double* v,
                                double* partial);
// deflation steps of the single-vector FP32 V-cycle, partial sums reduced in the kernel
void launch_deflate_in(hipStream_t s, int64_t N, const double* F, const double* part, int nparts, double inv_w,
                       const double* wv, float* Y, double* cm);
void launch_deflate_out(hipStream_t s, int64_t N, const float* x, const double* part, int nparts, double inv_w,
                        double* cm, const double* v, double* y);
void launch_scale(hipStream_t s, int m, double a, const double* x, double* y);
void launch_fill(hipStream_t s, int64_t N, double v, double* y);
void launch_zout_deflated(hipStream_t s, int m, int64_t N, const float* Z1, int64_t ldz, const double* sv,
                          const double* mu, const double* v, float* out, int64_t ldo);
void launch_node_weights(hipStream_t s, int dim, const Geom& g, double* out);
void launch_convert_deflate(hipStream_t s, int64_t N, int k, const double* X, int64_t ldx, const double* sv,
                            const double* wv, float* Y, int64_t ldy);
void launch_axpby(hipStream_t s, int64_t N, double a, const double* x, double b, double* y);
// y = a x + b y with b read from device memory
void launch_axpby_dev(hipStream_t s, int64_t N, double a, const double* x, const double* bdev, double* y);
// device-side scalars of the GN CG (see blas.hip): beta from the preconditioner
// step's dot products, then the step length
// CG scalars on the device from dot-product partial sums (reduced in the
// kernel, in the order of launch_reduce_parts): beta and r.z from na vectors
// of nba parts in pa and nb vectors of nbb parts in pb (sdot receives the
// na + nb dot products); the step length from the nparts partials of p.q
void launch_gn_beta(hipStream_t s, const double* pa, int na, int nba, const double* pb, int nb, int nbb, double ia,
                    int mode, bool first, bool flexible, double* sdot, double* dsc);
void launch_gn_alpha(hipStream_t s, const double* partial, int nparts, double* dsc);
// r.r from its partials into dsc[4], then dsc[0..7] to host-visible memory
void launch_gn_report(hipStream_t s, const double* partial, int nparts, double* dsc, double* host);
// nvec (<= 4) sums of nparts partials each, written to host-visible memory
void launch_reduce_host(hipStream_t s, int nvec, int nparts, const double* partial, double* host);
// x = 0, r = b, p = q = 0, Jp[0..m) = 0 and the partials of b.b (returns their count)
int launch_cg_init(hipStream_t s, int64_t N, const double* b, double* x, double* r, double* p, double* q, int m,
                   double* Jp, double* partial);
// x += a p, r -= a q, partials of r.r (and of sum(r) into psum when given)
void launch_cg_update_dev(hipStream_t s, int64_t N, const double* adev, const double* p, const double* q,
                          double* x, double* r, double* partial, int* nparts, double* psum = nullptr);
void launch_sub(hipStream_t s, int64_t N, const double* b, const double* v, double* out);
// batched (per-row coefficient) helpers for MG-PCG
void launch_batched_dots(hipStream_t s, int k, int64_t N, const double* X, int64_t ldx,
                         const double* Y, int64_t ldy, double* partial, double* out);
void launch_batched_cg_xr(hipStream_t s, int k, int64_t N, const double* a, const double* P,
                          int64_t ldp, const double* Q, int64_t ldq, double* X, int64_t ldx,
                          double* R, int64_t ldr, const int* active);
// device-side step lengths and direction coefficients of the batched PCG
void launch_pcg_alpha(hipStream_t s, int k, const double* rz, const double* pq, const int* active, double* a,
                      int* flag);
void launch_pcg_beta(hipStream_t s, int k, const double* rzn, double* rz, const double* zq, const double* a,
                     const int* active, double* b);
void launch_batched_p(hipStream_t s, int k, int64_t N, const double* b, const double* Z,
                      int64_t ldz, double* P, int64_t ldp, const int* active);

// gemm.hip: S = alpha*I + J Z^T with FP64 accumulation on MFMA
// (partial: the MFMA kernel writing per-split partial sums; reduce: the
// fixed-order sum over splits plus alpha on the diagonal)
// C (m x m2) = J (m rows) Z^T (m2 rows); lower_only requires m == m2 and Z
// symmetric-compatible (S mirrored from its lower triangle)
template <typename TZ>
int launch_capacitance_partial(hipStream_t s, int m, int m2, int64_t N, const double* J, int64_t ldj,
                               const TZ* Z, int64_t ldz, bool lower_only, double* partial,
                               size_t partial_elems);
// the same product with FP32 operands (J rounded on load) on the FP32 matrix
// cores, FP32 accumulation within each K split, splits summed in FP64 by the
// reduce kernel (opt-in H1W_FLAG_CAP_FP32_GEMM)
int launch_capacitance_partial_f32acc(hipStream_t s, int m, int m2, int64_t N, const double* J, int64_t ldj,
                                      const float* Z, int64_t ldz, double* partial, size_t partial_elems);
void launch_capacitance_reduce(hipStream_t s, int m, int m2, int splits, const double* partial, bool lower_only,
                               double alpha, int diag_off, double* S, int64_t lds);
void launch_mirror_lower(hipStream_t s, int m, double* S);
size_t gemm_partial_elems(int m, int m2, int64_t N);
// grouped products of a lock-step batch: instance g has m[g] <= 128 rows at
// row ro[g] of the stacked J and Z (leading dimensions ldj, ldz); its K range
// is cut into the work items io[g] .. io[g+1]-1 of kper[g] values each, whose
// partial m x m products go to partial + poff[g] + (item - io[g]) m^2;
// reduce: S_g (at soff[g], m x m row-major) = alpha[g] I + the sum of the
// partials in item order
struct GrpGemm {
    int G, total;
    const int* m;
    const int* ro;
    const int* io;
    const int64_t* kper;
    const int64_t* poff;
    const int64_t* soff;
    const double* alpha;
};
void launch_grp_gemm_partial(hipStream_t s, const GrpGemm& t, int64_t N, const double* J, int64_t ldj,
                             const double* Z, int64_t ldz, double* partial);
void launch_grp_gemm_reduce(hipStream_t s, const GrpGemm& t, const double* partial, double* S);

// dense.hip (single-workgroup factorisations for m <= a few thousand)
void launch_lu(hipStream_t s, int m, double* A, int* piv, int* info);
void launch_transpose(hipStream_t s, int m, const double* A, double* At);
void launch_lu_solve(hipStream_t s, int m, const double* LUt, const double* LU, const int* piv,
                     double* x);
void launch_jz_update_dev(hipStream_t s, int m, const double* S, double alpha, const double* Jy, const double* w,
                          const double* bdev, double* Jz, double* Jp);
void launch_asym(hipStream_t s, int m, const double* S, double* out);
// out[0..3] = max S_ii, min S_ii, max |F_ii|, min |F_ii| of S and its factor F
void launch_diag_stats(hipStream_t s, int m, const double* S, const double* F, double* out);
// blocked.hip: right-looking blocked Cholesky (mode 0, upper) or LU without
// pivoting (mode 1) in place, with diagonal-block inverses; triangular solves
size_t blocked_inv_elems(int m);
void launch_blocked_factor(hipStream_t s, int m, double* A, int mode, double* Dfwd, double* Dbwd, int* info);
// out = T2^{-1} T1^{-1} in with T1, T2 block-triangular (given as C[j][i] =
// T[i][j] and the diagonal-block inverses D); one launch, out may equal in
void launch_blocked_solve2(hipStream_t s, int m, const double* C1, const double* D1, bool lower1, const double* C2,
                           const double* D2, bool lower2, const double* in, double* out);

}  // namespace h1w
