/*
 * h1w.h -- C ABI of the MI355X library for the Gauss-Newton linear systems of
 * H^1-regularised parameter identification (Blechta & Ernst, arXiv 2209.02815).
 *
 * Problem (Section 2.2, eq. (block_primal), multiplied by the regularisation
 * parameter, which is called alpha here):
 *
 *     G x = b,    G = alpha*A + J^T J,
 *
 * where A = K + beta*W is the discrete H^1 Gram operator on a structured
 * vertex-centred grid of the unit square/cube with natural (Neumann) boundary
 * conditions, and J is the dense m x N sensitivity matrix (Section 2.3, the
 * matrix J_m). On an n_x x n_y (x n_z) grid with h_d = 1/(n_d - 1):
 *
 *     A = sum_d W1 (x) .. K1^(d) .. (x) W1 + beta * (W1 (x) .. (x) W1),
 *     K1 = h^-2 tridiag(-1, 2, -1) with first/last diagonal entries 1,
 *     W1 = diag(1/2, 1, .., 1, 1/2);
 * interior rows are the 5-/7-point -Laplacian + beta.
 *
 * Method (Section 3.2, Algorithm 3, rebuilt for the symmetric positive
 * definite primal system): conjugate gradients preconditioned by the Woodbury
 * formula around B ~ A^{-1}, one symmetric geometric-multigrid V-cycle:
 *     Z = B J^T (m batched Poisson solves), S = alpha*I + J Z (capacitance),
 *     P^{-1} r = (1/alpha) (B r - Z S^{-1} J B r)  = (alpha B^{-1} + J^T J)^{-1} r.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers owned by the caller, 8-byte aligned,
 *    stored row-major: a batch of k grid vectors is k rows of N = n_x n_y n_z
 *    values each (x fastest), row i starting at ptr + i*ld with ld >= N.
 *    J is m x N row-major with leading dimension ldj >= N.
 *  - All work is enqueued on the stream given to h1w_setup. Calls that read
 *    convergence scalars (h1w_gn_solve, H1W_MG_SOLVE) block the host until
 *    they return; the others return once their work is enqueued, except where
 *    stated.
 *  - Every call returns an h1w_status and never aborts; on failure
 *    h1w_last_error(ctx) describes the cause. Arguments are validated on the
 *    host before any kernel is launched.
 *  - One host thread per context. Contexts are independent.
 *  - The library owns the context, its workspace (allocated in h1w_setup and
 *    grown in h1w_capacitance_build / h1w_gn_solve) and the current
 *    capacitance factor. Nothing is allocated inside the CG iteration.
 */
#ifndef H1W_H
#define H1W_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct h1w_ctx h1w_ctx;

typedef enum {
    H1W_OK = 0,
    H1W_EINVAL = -1,   /* invalid argument (null pointer, bad size, ld < N, ...) */
    H1W_ENOMEM = -2,   /* device allocation failed */
    H1W_EHIP = -3,     /* HIP runtime error (message in h1w_last_error) */
    H1W_ENOTSPD = -4,  /* Cholesky met a non-positive pivot (info->failed_pivot) */
    H1W_ENOCONV = -5,  /* maxit reached; outputs hold the last iterate */
    H1W_ENUMERIC = -6, /* NaN or Inf in a residual or pivot */
    H1W_ENOTIMPL = -7, /* entry point not built in this version */
    H1W_ESTATE = -8    /* call order violated (e.g. precond before capacitance) */
} h1w_status;

typedef enum { H1W_FP64 = 0, H1W_MIXED = 1 } h1w_precision;
typedef enum { H1W_DT_F64 = 0, H1W_DT_F32 = 1 } h1w_dtype;
typedef enum { H1W_VCYCLE_ONCE = 0, H1W_MG_SOLVE = 1 } h1w_poisson_mode;
typedef enum { H1W_Z_AUTO = 0, H1W_Z_STORED = 1, H1W_Z_RECOMPUTE = 2 } h1w_zmode;
typedef enum { H1W_FACTOR_AUTO = 0, H1W_FACTOR_CHOL = 1, H1W_FACTOR_LU = 2 } h1w_factor;
typedef enum { H1W_OP_H1GRAM = 0, H1W_OP_ERT = 1 } h1w_opkind;

/* Grid and multigrid description (h1w_setup). Zero fields take defaults. */
typedef struct {
    int dim;             /* 2 or 3 */
    int n[3];            /* nodes per axis (x, y, z), each >= 2; n[2] ignored for dim 2 */
    double beta;         /* mass weight in A = K + beta*W, > 0 */
    int precision;       /* h1w_precision: V-cycles and stored Z in FP64 (H1W_FP64)
                            or FP32 (H1W_MIXED); J, S, its factor and CG are FP64 */
    int nu;              /* smoothing steps per side = Chebyshev degree (0 -> 2) */
    double cheb_lo;      /* Chebyshev interval for eig(D^-1 A): [lo, hi] */
    double cheb_hi;      /* (0, 0) -> [0.3, 2.0] */
    int64_t coarse_max;  /* coarsest level: first level with <= coarse_max nodes
                            (or that cannot be halved); 0 -> 729 (3D) / 81 (2D) */
    int rhs_chunk;       /* right-hand sides per batched V-cycle launch (0 -> auto:
                            2^28 / N, clamped to [1, 1024]) */
    unsigned flags;      /* H1W_FLAG_* bits, other bits must be 0 */
    int op;              /* h1w_opkind: H1W_OP_H1GRAM (the regularisation operator A
                            above) or H1W_OP_ERT (the conductivity operator of the
                            ERT forward problem, see the ERT section below) */
    unsigned dirichlet_mask; /* ERT only: bit f set = u = 0 on face f, faces ordered
                            x=0, x=1, y=0, y=1, z=0, z=1 (bits 0..5), at least one
                            bit; 0 -> 0x1f (every face but the top z = 1) */
} h1w_grid_desc;

/* grid_desc.flags: always stream Z in FP64 capacitance builds (Z is built in
 * row chunks and multiplied against J chunk by chunk instead of being kept;
 * the preconditioner then recomputes Z w as B (J^T w)). Without the flag this
 * happens only when an FP64 Z would not fit next to J. */
#define H1W_FLAG_STREAM_Z 1u
/* grid_desc.flags: run 3D V-cycles with two smoothing steps per side as the
 * sequence of single-step stencil kernels instead of the fused down/up passes
 * (same cycle, same result up to rounding; more memory traffic). */
#define H1W_FLAG_UNFUSED_VCYCLE 2u
/* grid_desc.flags: replay V-cycles from HIP graphs. The kernel sequence of a
 * V-cycle applied to the same (k, F, X) buffers is captured into a graph on
 * its second use and replayed afterwards (the CG's preconditioner applies
 * reuse the same context buffers at every iteration and across solves), which
 * removes the per-kernel launch cost for small grids. Same results, bit for
 * bit. Ignored while kernel timing is on. H1 contexts only. */
#define H1W_FLAG_GRAPH_VCYCLE 4u
/* grid_desc.flags: in 2D fused V-cycles (two smoothing steps per side), run
 * every level as its own down and up pass. Without the flag the levels from
 * the first one that fits one work-group's LDS (with every coarser level)
 * down to the coarsest, and back, run in one launch per V-cycle: the same
 * cycle with the same arithmetic, so the result is the same bit for bit. */
#define H1W_FLAG_NO_VTAIL 8u
/* grid_desc.flags, MIXED contexts only (EINVAL otherwise): form the product
 * J Z^T of the capacitance (Algorithm 3, second step) on the FP32 matrix cores
 * with FP32 operands (J rounded to FP32 as it is read) and FP32 accumulation
 * over each K split of the GEMM, the splits then summed in FP64; the
 * constant-mode terms and alpha*I stay FP64. Its error, about
 * eps32 * sqrt(K / splits) * |J| |Z| per entry, breaks the consistency
 * J (I - Z S^{-1} J) = alpha S^{-1} J that the Woodbury correction needs once
 * ||S|| / alpha is large, so flexible CG slows down or stops converging as
 * alpha falls. Off by default: S is accumulated in FP64. */
#define H1W_FLAG_CAP_FP32_GEMM 16u

/* Krylov options (h1w_gn_solve). A zeroed struct selects the defaults. */
typedef struct {
    double rtol;         /* stop when ||b - G x||_2 <= rtol ||b||_2, recomputed
                            in FP64 from x (0 -> 1e-10) */
    int maxit;           /* 0 -> 500 */
    int zmode;           /* h1w_zmode: how the preconditioner applies Z w:
                            STORED reads Z, RECOMPUTE runs a second V-cycle
                            B (J^T w); AUTO = RECOMPUTE for FP64, STORED for MIXED
                            (MIXED requires STORED) */
    int factor;          /* h1w_factor: AUTO = Cholesky for FP64 (LU if it fails),
                            LU for MIXED */
    int check_every;     /* reserved (0) */
    unsigned flags;      /* H1W_SOLVE_* bits (at most one), other bits must be 0 */
} h1w_solve_opts;

/* h1w_solve_opts.flags: comparison modes of the Gauss-Newton solve.
 * LAPLACE_ONLY (the Laplace preconditioner of Algorithm 4, without the
 *   Woodbury correction): CG on G x = b preconditioned by B / alpha; no
 *   capacitance is built and each iteration passes over J twice (J p, then
 *   J^T (J p)). Its iteration count grows with m and 1/alpha.
 * EXACT_B (the exact Woodbury inverse of Algorithm 1, with the Poisson solve
 *   done by multigrid instead of a sparse factorisation): every application of
 *   B, in the capacitance and in the preconditioner, is an MG-preconditioned
 *   CG solve of A to a relative residual of 1e-12, so the preconditioner is
 *   G^-1 up to that tolerance and CG stops after one or two iterations.
 *   Needs an FP64 context. The capacitance it leaves in the context belongs
 *   to this B and is discarded at return (h1w_precond_apply then needs a new
 *   h1w_capacitance_build). */
#define H1W_SOLVE_LAPLACE_ONLY 1u
#define H1W_SOLVE_EXACT_B 2u

/* Diagnostics filled by the calls that take an h1w_info* (may be NULL). */
typedef struct {
    int iters;               /* Krylov iterations */
    int factor_used;         /* h1w_factor actually used */
    int zmode_used;          /* h1w_zmode actually used */
    int failed_pivot;        /* first non-positive Cholesky pivot, -1 if none */
    int nlevels;             /* multigrid levels */
    int restarts;            /* CG restarts from the true residual: after a failed final check, and
                                (recompute form) the one replacement made once the recursive
                                residual is below sqrt(rtol) */
    double relres_true;      /* ||b - G x|| / ||b|| recomputed from x in FP64 */
    double relres_rec;       /* recursive residual estimate at exit */
    double t_zbuild_ms;      /* batched V-cycles for Z */
    double t_gemm_ms;        /* capacitance GEMM */
    double t_factor_ms;      /* factorisation and inverse of S */
    double t_cg_ms;          /* Krylov loop including the final true residual */
    double t_total_ms;       /* whole call */
    double asym_S_over_alpha;/* max |S - S^T| / alpha (full GEMM only, else 0) */
    double kappa_S_est;      /* estimate of cond(S) from the pivots u_ii of its factor:
                                (max u_ii / min u_ii)^2 for Cholesky, max |u_ii| / min |u_ii|
                                for LU (a lower estimate) */
    double s_max_over_alpha; /* max_i S_ii / alpha: the factor by which rounding errors in S
                                are amplified in the Woodbury correction */
} h1w_info;

/* Create a context for one grid: builds the multigrid hierarchy, the dense
 * inverse of the coarsest operator and the V-cycle workspace.
 * hip_stream: a hipStream_t (NULL = default stream). */
h1w_status h1w_setup(const h1w_grid_desc* desc, void* hip_stream, h1w_ctx** out);

/* Free the context and all device memory it owns. NULL is ignored. */
void h1w_destroy(h1w_ctx* ctx);

/* Message for the last failed call on ctx (valid until the next call); with
 * ctx == NULL, of the calling thread's last failed h1w_setup or
 * h1w_batch_solve. */
const char* h1w_last_error(const h1w_ctx* ctx);

/* Static description of a status code. */
const char* h1w_status_string(h1w_status s);

/* Number of grid nodes N and multigrid levels of a context. */
h1w_status h1w_get_sizes(const h1w_ctx* ctx, int64_t* N, int* nlevels);

/* Y = A X for k grid vectors (the regularisation operator of eq.
 * (block_primal) with the mass term). dtype selects double or float arrays.
 * X and Y must not overlap. */
h1w_status h1w_operator_apply(h1w_ctx* ctx, int k, const void* X, int64_t ldx,
                              void* Y, int64_t ldy, int dtype);

/* Batched Poisson solves with A (the Laplace solve inside the preconditioner,
 * Section 3.2 and Algorithm 3, first step).
 * mode H1W_VCYCLE_ONCE: X = B F, one symmetric V-cycle from a zero initial
 *   guess in the context's V-cycle precision; dtype must be H1W_DT_F64 for an
 *   FP64 context and H1W_DT_F32 for a MIXED one. rtol and maxit are ignored.
 * mode H1W_MG_SOLVE: X ~ A^{-1} F by FP64 conjugate gradients preconditioned
 *   by B (flexible when B is FP32) until ||F_i - A X_i|| <= rtol ||F_i|| for
 *   every row i, at most maxit iterations (ENOCONV otherwise); dtype must be
 *   H1W_DT_F64. Blocks the host.
 * F and X must not overlap. info->iters = the largest iteration count. */
h1w_status h1w_poisson_solve_batched(h1w_ctx* ctx, int k, const void* F, int64_t ldf,
                                     void* X, int64_t ldx, int dtype, int mode,
                                     double rtol, int maxit, h1w_info* info);

/* Capacitance build (Algorithm 3, first three steps): Z = B J^T (kept in the
 * context, FP64 or FP32 by the context precision), S = alpha*I + J Z^T
 * (FP64 accumulation) and its factorisation (Cholesky, or LU with partial
 * pivoting for a MIXED context or when Cholesky fails; factor selects it).
 * J (m x N, FP64) is NOT copied: it must stay valid and unchanged until the
 * next h1w_capacitance_build or h1w_gn_solve on this context.
 * S_out (optional, m x m row-major FP64, leading dimension lds >= m) receives S.
 * Z_out (optional, m x N, leading dimension ldz >= N, dtype of the context's
 * V-cycle precision) receives Z; EINVAL if Z was streamed (H1W_FLAG_STREAM_Z,
 * or an FP64 Z too large to keep), info->zmode_used tells which.
 * MIXED contexts keep the constant mode of Z exactly: with the trapezoid node
 * weights W1 and s_i = (J_i . 1) / sum(W1), the FP32 V-cycle is applied to
 * J_i - s_i W1 and its W-weighted mean mu_i is projected out, so
 * Z = Z1 - 1 mu^T + (B W1) s^T with Z1 stored in FP32 and B W1 (an FP64
 * V-cycle) and mu, s in FP64; the preconditioner's own V-cycle on r is
 * deflated the same way. S is formed consistently with that representation
 * (FP64 accumulation), which keeps the Woodbury correction accurate when
 * ||S||/alpha is large. Z_out then receives Z rounded to FP32.
 * Returns ENOTSPD if factor = CHOL was forced and a pivot is not positive. */
h1w_status h1w_capacitance_build(h1w_ctx* ctx, int m, const double* J, int64_t ldj,
                                 double alpha, int factor, double* S_out, int64_t lds,
                                 void* Z_out, int64_t ldz, h1w_info* info);

/* Woodbury preconditioner apply for k vectors using the context's current
 * capacitance (Algorithm 3, preconditioner formula):
 *   Zout_i = (1/alpha)(B R_i - Z S^{-1} J B R_i)   (zmode STORED), or
 *   Zout_i = (1/alpha) B (R_i - J^T S^{-1} J B R_i) (zmode RECOMPUTE).
 * FP64 arrays. ESTATE if no capacitance has been built. */
h1w_status h1w_precond_apply(h1w_ctx* ctx, int k, const double* R, int64_t ldr,
                             double* Zout, int64_t ldz, int zmode);

/* Full Gauss-Newton linear solve: capacitance build + preconditioned CG
 * from x0 = 0 (Algorithm 3 with MINRES replaced by CG on the SPD primal form).
 * b (N, FP64) is the right-hand side; if b is NULL, the paper's right-hand
 * side b = -alpha*A d - J^T res is formed from d = m - m_ref (N) and
 * res = g - g_obs (m) (eq. (block_primal) times alpha); then dm = x.
 * x (N, FP64) receives the solution. J must stay valid during the call.
 * Returns ENOCONV (x = last iterate, info->relres_true filled) when maxit is
 * reached, ENUMERIC on NaN/Inf. Blocks the host. */
h1w_status h1w_gn_solve(h1w_ctx* ctx, int m, const double* J, int64_t ldj, double alpha,
                        const double* b, const double* d, const double* res, double* x,
                        const h1w_solve_opts* opts, h1w_info* info);

/* y = G x = alpha*A x + J^T (J x) for one vector (FP64); used for true
 * residuals. J is m x N. */
h1w_status h1w_gn_apply(h1w_ctx* ctx, int m, const double* J, int64_t ldj, double alpha,
                        const double* x, double* y);

/* y = G x as h1w_gn_apply, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no allocation, no memset and no host synchronisation happen in
 * the call. Its scratch (the m-vector J x and the partial sums of the J x
 * pass) lives in a static device array of 32 MiB that the library holds on
 * every GPU it runs on until the process ends; sizes that need more,
 * m * ceil(N / 2048) + (m rounded up to 32) > 4194304 doubles, return EINVAL
 * (m <= 3994 at 129^3, m <= 505 at 257^3). Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU race. The work is enqueued on the
 * context's stream and y is valid once that stream has synchronised. Arguments
 * and errors as h1w_gn_apply; J and y must not overlap. */
h1w_status h1w_gn_apply_noalloc(h1w_ctx* ctx, int m, const double* J, int64_t ldj, double alpha,
                                const double* x, double* y);

/* ---------------------------------------------------------------- kernel timing
 * Optional per-kernel-class timing with HIP events recorded on the context's
 * stream around every launch of the selected classes (bit (1 << class) in
 * mask; 0 switches timing off). Each launch also adds the algorithmic bytes
 * it must move (its inputs read once, its outputs written once) and the
 * algorithmic flops of its contraction, so achieved GB/s or TFLOP/s of a
 * class = bytes / ms or flops / ms. Statistics accumulate until reset.
 * Timing adds two event records per timed launch; it is off by default. */
typedef enum {
    H1W_K_SMOOTH = 0,      /* Chebyshev-Jacobi smoothing step (all levels) */
    H1W_K_SMOOTH_FIRST = 1,/* first smoothing step from a zero guess */
    H1W_K_RESIDUAL = 2,    /* r = f - A x */
    H1W_K_RESTRICT = 3,    /* f_c = 2^-d P^T r */
    H1W_K_PROLONG = 4,     /* x += P e_c */
    H1W_K_COARSE = 5,      /* dense coarsest solve */
    H1W_K_GEMM = 6,        /* capacitance GEMM J Z^T (MFMA) */
    H1W_K_JV = 7,          /* J v pass */
    H1W_K_JTV = 8,         /* J^T (and Z^T) passes with CG epilogues */
    H1W_K_FACTOR = 9,      /* blocked factorisation of S */
    H1W_K_TRSV = 10,       /* triangular solves with the factors of S */
    H1W_K_APPLY = 11,      /* operator apply A x (incl. the CG q = alpha A p + t) */
    H1W_K_VDOWN = 12,      /* fused 3D pass: two pre-smoothing steps, residual, restriction */
    H1W_K_VUP = 13,        /* fused 3D pass: interpolation, two post-smoothing steps */
    H1W_K_ERT_STENCIL = 14,/* ERT operator: apply, residual, smoothing steps, restriction */
    H1W_K_ERT_SENS = 15,   /* ERT pairwise-gradient sensitivities (J) and their transpose product */
    H1W_K_VTAIL = 16,      /* 2D coarse levels and coarsest solve of a V-cycle in one launch */
    H1W_K_NCLASS = 17
} h1w_kclass;

typedef struct {
    int64_t launches;
    double ms;       /* sum of event-measured launch durations */
    double bytes;    /* sum of algorithmic bytes */
    double flops;    /* sum of algorithmic flops */
} h1w_kstat;

h1w_status h1w_set_kernel_timing(h1w_ctx* ctx, unsigned mask);
h1w_status h1w_get_kernel_timing(h1w_ctx* ctx, int kclass, h1w_kstat* out);
h1w_status h1w_reset_kernel_timing(h1w_ctx* ctx);

/* ------------------------------------------------------------------------
 * Batched solves of many independent Gauss-Newton systems of uneven size
 * (each one the system of h1w_gn_solve on its own grid, Algorithm 3 with the
 * multigrid Poisson solver): a native executor overlaps them on one GPU.
 *
 * The items are ordered by decreasing work N * (m + 1) and pulled from one
 * queue by opts.nworkers host threads; each thread drives a worker that owns
 * a HIP stream (default priority) and one context per (grid, precision,
 * smoother schedule, beta, graph replay) it meets, reused by later items of
 * that key. Workers are kept for the process and reused by later batches
 * (at most 24 contexts each, the least recently used dropped beyond that; a
 * context whose item failed is dropped), so their device memory stays
 * allocated until the process ends; a batch on grids met before allocates
 * no device memory. With opts.autotune, the smoother schedule is tuned per
 * (grid, precision) key: the first item of a key is solved by one worker,
 * back to back, with the Chebyshev intervals [0.4, 2] and [0.5, 2] for
 * eig(D^-1 A) and then the default [0.3, 2] (opts.nu smoothing steps per side
 * in each; the same kernels per iteration), and the later items of the key
 * use the interval with the fewest CG iterations, the default on a tie (the
 * default solve is the item's result; until a key is tuned its items use the
 * default).
 * Items of one grid must share beta. All pointers are device
 * pointers owned by the caller; J, b, x follow h1w_gn_solve (J m x N with
 * leading dimension ldj, x receives the solution). infos and status (count
 * entries each, may be NULL) receive each item's diagnostics and status;
 * the call returns H1W_OK when every item succeeded, else the status of the
 * failing item with the lowest index, and blocks until all items are done.
 * ------------------------------------------------------------------------ */
typedef struct {
    int dim;             /* 2 or 3 */
    int n[3];            /* nodes per axis (n[2] ignored in 2D) */
    double beta;         /* mass weight of A */
    double alpha;        /* regularisation weight (> 0) */
    int m;               /* rows of J (>= 0) */
    const double* J;     /* m x N, leading dimension ldj (may be NULL if m == 0) */
    int64_t ldj;
    const double* b;     /* right-hand side (N) */
    double* x;           /* solution (N) */
} h1w_batch_item;

typedef struct {
    int precision;       /* H1W_FP64 or H1W_MIXED, for every item */
    int nworkers;        /* host threads / streams (0 -> 8, at most 16) */
    int autotune;        /* 1: choose the smoother schedule per grid as described above,
                            reusing the keys tuned by earlier batches of the process;
                            2: tune every key again (and keep the new choice); 0: off */
    int nu;              /* smoothing steps when not tuned (0 -> 2) */
    double rtol;         /* as h1w_solve_opts.rtol (0 -> 1e-10) */
    int maxit;           /* as h1w_solve_opts.maxit (0 -> 500) */
    int graphs;          /* 1: contexts replay their V-cycles from HIP graphs
                            (H1W_FLAG_GRAPH_VCYCLE) */
    int grouped;         /* 1: lock-step mode. The items of one grid (same dim, n,
                            beta) are solved together by one worker: their vectors
                            stacked, so that each step of the iteration is one launch
                            for the whole group (V-cycles, operator, J and J^T passes
                            over the stacked rows, dot products, updates with
                            per-item step lengths and activity masks); each item's
                            S = alpha I + J Z^T is one tile of a grouped MFMA product
                            and is inverted in one work-group. Items with m > 128 are
                            solved after the groups, one solve per item as with
                            grouped = 0 (same options); graphs is ignored by the
                            groups. With
                            autotune, a group whose key is untuned is solved whole with
                            each interval and then the default, and keeps the interval
                            with the least work (its items' CG iterations weighted by
                            m + 1; the default on a tie), solving once more with it
                            unless that is the default. Grouped keys are kept apart
                            from those of the per-item mode, which choose on one
                            item's iterations. The preconditioned CG (stored-Z Woodbury apply,
                            flexible direction coefficient) stops each item on its
                            recursive residual and checks its true residual (up to two
                            restarts; maxit counts the group's iterations). Each item
                            gets its own status: ENOCONV if it misses rtol, ENUMERIC
                            if its values turn non-finite or its CG breaks down, the
                            other items unaffected; a failure of the whole group (its
                            set-up, a zero capacitance pivot) gives its status to all
                            of its items. 0: one solve per item (above). */
} h1w_batch_opts;

#define H1W_BATCH_MAX_KEYS 64
typedef struct {
    int dim;
    int n[3];
    int m_bucket;        /* ceil(log2 m) of the item the key was tuned on (grouped:
                            of the group's first item) */
    int nu;              /* smoothing steps per side (opts.nu) */
    double ms_per_unit;  /* the chosen schedule's wall time per N * (m + 1), in ms
                            (grouped: per the group's sum of N * (m + 1)) */
    int reused;          /* 1: the choice of an earlier batch */
    double cheb_lo;      /* chosen lower end of the Chebyshev interval (upper end 2) */
    int iters;           /* CG iterations of the tuning item with the chosen schedule
                            (grouped: summed over the tuning group's items) */
    int iters_default;   /* ... and with the default one (-1: the default failed) */
    int grouped;         /* 1: a key of the grouped mode */
} h1w_batch_tuned;

typedef struct {
    double t_total_ms;   /* wall time of the whole batch */
    int nworkers;
    int ntuned;          /* entries of tuned[] (autotune) */
    h1w_batch_tuned tuned[H1W_BATCH_MAX_KEYS];
} h1w_batch_report;

h1w_status h1w_batch_solve(int count, const h1w_batch_item* items, const h1w_batch_opts* opts,
                           h1w_info* infos, h1w_status* status, h1w_batch_report* report);

/* ------------------------------------------------------------------------
 * ERT forward map and sensitivities (Section 4: eq. (model), the pole-pole
 * voltages of eqs. (ert_qoi2)/(ert_qoi_scaling) and their derivative,
 * eq. (ert_qoi_derivative), in the log parametrisation m = log sigma).
 *
 * A context created with desc.op = H1W_OP_ERT (3D, FP64, beta ignored) holds
 * the operator -div(sigma grad u) on the grid of the unit cube in its
 * vertex-centred finite-volume form: the edge (p, q) along axis d carries the
 * conductance (sigma_p + sigma_q)/2 * (dual-face area)/h_d, the dual-face area
 * being the product of the other axes' h, halved for each of them on which
 * the edge lies in a boundary face; nodes on the faces of dirichlet_mask have
 * u = 0 (their rows are the identity, their couplings are removed), the other
 * faces have zero normal flux. A unit pole source at node a is the nodal load
 * e_a, so u_a = A_sigma^{-1} e_a. The pole-pole voltage of pair i = (a, b)
 * (return electrodes at infinity, as the paper's B electrode) is
 *     g_i = k_i u_a(x_b),   k_i = 2 pi |x_a - x_b|   (default geometric factor),
 * and its sensitivity to m_j, the adjoint field of b being u_b (A symmetric):
 *     J[i, j] = -k_i sum_{edges (j, q)} (sigma_j/2) (area/h) (u_a(j) - u_a(q)) (u_b(j) - u_b(q)).
 * Multigrid: the same geometric V-cycle as the H1 context (Chebyshev-Jacobi
 * smoothing, R = P^T with the Dirichlet nodes masked, multilinear P), with
 * the coarse conductivities recomputed from the fine ones by full-weighting
 * averages at every h1w_ert_set_conductivity, rediscretised coarse operators
 * and a dense coarsest inverse (at most 128 nodes) computed on the device.
 * h1w_operator_apply (F64) and h1w_poisson_solve_batched (F64) work on an
 * ERT context once a conductivity is set (ESTATE before); the Gauss-Newton
 * entry points need an H1 context (EINVAL on an ERT one).
 * Index arrays (src_node, pair) are device int32 arrays; they are copied to
 * the host and validated before any kernel runs, so these calls synchronise.
 * ------------------------------------------------------------------------ */

/* sigma = exp(logsig) at the N nodes (device FP64); builds every level's
 * coefficients and the coarsest inverse on the device. ENUMERIC if some
 * sigma is not finite and positive. */
h1w_status h1w_ert_set_conductivity(h1w_ctx* ctx, const double* logsig);

/* Pole fields, voltages and (optionally) the sensitivity matrix.
 * logsig      N log-conductivities, or NULL to keep the current conductivity
 * src_node    n_src node indices of the pole sources (1 <= n_src <= 64; not on
 *             a Dirichlet face)
 * pair        n_meas x 2 indices into src_node: (a, b), a != b
 * kgeo        n_meas geometric factors, or NULL for 2 pi |x_a - x_b|
 * g_out       n_meas voltages g_i (may be NULL)
 * J_out       n_meas x N sensitivities, row-major with leading dimension
 *             ldj >= N (may be NULL). The kernel writes each row in runs of
 *             64 values; with ldj a multiple of 16 (rows on 128-byte
 *             boundaries) those runs do not straddle cache lines and J is
 *             written about twice as fast as with an odd ldj
 * U_out       n_src x N pole fields u_a, leading dimension ldu >= N (may be
 *             NULL: the context keeps them for h1w_ert_vjp with U = NULL)
 * opts        rtol (0 -> 1e-12) and maxit (0 -> 500) of the batched
 *             MG-preconditioned CG for the n_src fields (all in one batch)
 * info        iters (largest over the fields), relres_true (worst field
 *             residual), t_zbuild_ms (conductivity setup), t_cg_ms (field
 *             solves), t_gemm_ms (voltages and sensitivities), t_total_ms.
 * Returns ENOCONV if a field does not reach rtol in maxit iterations. Blocks
 * the host. */
h1w_status h1w_ert_sensitivities(h1w_ctx* ctx, const double* logsig, int n_src,
                                 const int* src_node, int n_meas, const int* pair,
                                 const double* kgeo, double* g_out, double* J_out,
                                 int64_t ldj, double* U_out, int64_t ldu,
                                 const h1w_solve_opts* opts, h1w_info* info);

/* grad = J^T gbar (N, FP64) without forming J, for the current conductivity
 * and the pole fields U (n_src x N, leading dimension ldu; NULL = the fields
 * of the last h1w_ert_sensitivities call on this context). src_node is
 * needed only when kgeo is NULL. */
h1w_status h1w_ert_vjp(h1w_ctx* ctx, int n_src, const int* src_node, const double* U,
                       int64_t ldu, int n_meas, const int* pair, const double* kgeo,
                       const double* gbar, double* grad);

/* One Gauss-Newton step of Algorithm 2 on an ERT survey: the voltages g(m)
 * and the sensitivities J(m) on the ERT context (as h1w_ert_sensitivities),
 * the step dm from the Woodbury-preconditioned GN system on the H1 context
 * (as h1w_gn_solve with the paper-form right-hand side, d = m - m_ref and
 * res = g(m) - g_obs, eq. (block_primal)), then m := m + dm.
 * ert         ERT context; h1: H1 Gram context with the same n[3]
 * m           N log-conductivities (in/out); m_ref: N reference values
 * g_obs       n_meas observed voltages (1 <= n_meas <= 4096)
 * J, ldj      n_meas x N workspace; holds J(m) of the old m on return
 * dm          N workspace; holds the step on return
 * g_out       n_meas, optional: g of the old m
 * ert_opts    field solves (rtol 0 -> 1e-12); gn_opts: as for h1w_gn_solve
 * info        the GN solve's diagnostics.
 * m is updated only when every part succeeded. Errors are reported on h1
 * (h1w_last_error(h1)). Blocks the host. */
h1w_status h1w_ert_gn_step(h1w_ctx* ert, h1w_ctx* h1, double* m, const double* m_ref, int n_src,
                           const int* src_node, int n_meas, const int* pair, const double* kgeo,
                           const double* g_obs, double alpha, double* J, int64_t ldj, double* dm,
                           double* g_out, const h1w_solve_opts* ert_opts,
                           const h1w_solve_opts* gn_opts, h1w_info* info);

#ifdef __cplusplus
}
#endif
#endif /* H1W_H */
