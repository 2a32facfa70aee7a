// The h1w context: one structured grid, its multigrid hierarchy and the
// device workspace of the batched V-cycle, the capacitance system and the
// Krylov loop.
#pragma once

#include <initializer_list>
#include <utility>

#include "devutil.h"
#include "internal.h"

namespace h1w {

// default Chebyshev interval for the eigenvalues of D^-1 A (grid_desc cheb_lo,
// cheb_hi both 0): 2 bounds that spectrum for the 5- and 7-point operators
constexpr double kChebLoDefault = 0.3, kChebHiDefault = 2.0;

// coefficient arrays of one ERT level (each N_l long, pitch-aligned)
struct ErtLevel {
    double *sig, *D, *cx, *cy, *cz;
};

struct Ctx {
    h1w_grid_desc d{};
    int dim = 0;
    hipStream_t stream = nullptr;
    std::string err;
    bool fp32 = false;               // V-cycles and stored Z in FP32 (mixed precision)
    std::vector<Geom> lv;            // levels, fine to coarsest
    std::vector<int64_t> pitch;      // workspace row pitch per level (elements)
    std::vector<double> w;           // Chebyshev step weights
    bool fused = false;              // V-cycles as fused down/up passes (3D, nu = 2)
    int tail_l0 = 0;                 // 2D fused: first level of the one-launch coarse tail (L: none)
    TailGeo tail{};                  // its levels and LDS layout
    int64_t Nc = 0;                  // nodes on the coarsest level
    DevBuf cinv64, cinv32;           // dense inverse of the coarsest operator
    DevBuf cpart;                    // partial sums of the coarsest solve (split over j)
    size_t cpart_elems = 0;
    int chunk = 1;                   // right-hand sides per V-cycle launch
    DevBuf vws;                      // V-cycle level workspace
    DevBuf stage;                    // FP32 staging (mixed precision)
    DevBuf pcg;                      // MG-PCG batch vectors
    DevBuf mgvec, mgpart;            // MG-PCG per-RHS scalars and dot partials (its own: the
                                     // V-cycle of a MIXED context may grow the GN-CG buffers)

    // capacitance state (valid when have_cap)
    bool have_cap = false;
    int m = 0;
    const double* J = nullptr;
    int64_t ldj = 0;
    double alpha = 0.0;
    DevBuf Zbuf;                     // Z = B J^T, m x N (double or float), ld = ldz
    DevBuf zchunk;                   // rows of Z when Z is streamed
    bool z_streamed = false;         // Z not kept (FP64, too large next to J)
    // mixed precision: the constant mode of Z is kept exactly in FP64,
    // Z = Z1 - 1 mu^T + v s^T with v = B W1 (FP64 V-cycle), s_i = (J_i . 1) / sum(W),
    // Z1 the FP32 cycle applied to J_i - s_i W1 and mu_i the W-mean of Z1_i
    bool deflate = false;
    double wsum = 0.0;
    DevBuf wvec, ones, vdef, sdef, jvdef, dpart, mudef, jneg;
    bool vdef_ready = false;
    void ensure_deflation_vectors();
    int64_t ldz = 0;
    DevBuf Sbuf;                     // S = alpha I + J Z^T (m x m)
    DevBuf F1, F2, pivb;             // factors: Cholesky U / L=U^T, or LU / (LU)^T (+ pivots)
    DevBuf Dfwd, Dbwd;               // inverses of the 64x64 diagonal blocks of the factors
    int factor = 0;
    bool lu_pivoted = false;         // fallback LU with partial pivoting in use
    int failed_pivot = -1;
    double asym = 0.0;
    double kappa_est = 0.0;   // pivot-ratio estimate of cond(S) from its factor
    double s_over_alpha = 0.0;  // max S_ii / alpha: the amplification of rounding in S by 1/alpha

    // Krylov workspace
    enum { kR, kP, kQ, kY, kU, kZ, kT, kB, kTmpN, kNVec };
    enum { kJy, kW, kJz, kJp, kJx, kTmp, kMVec };
    DevBuf nvec, mvec, part, jpart, gpart, scal, iflag;
    int mstride = 1;                 // m-vector slot stride (grows only)
    double* hscal = nullptr;         // pinned host copy of device scalars
    double* hrep = nullptr;          // coherent pinned host memory written by kernels (CG scalars, norms)
    const double* rsum_of = nullptr; // vector whose sum(.) partials are at rsum_part (mixed GN-CG residual)
    const double* rsum_part = nullptr;
    int rsum_nb = 0;
    double* drep = nullptr;          // hrep as seen by the device
    static constexpr int kGnScal = 32;  // slots of the GN CG's device scalars in scal
    hipEvent_t ev[8] = {};

    ~Ctx();
    void init(const h1w_grid_desc& desc, hipStream_t s);
    int64_t N() const;
    void sync();
    void read_scal(int n);

    template <typename T> const T* fp_cinv() const {
        if constexpr (sizeof(T) == 8) return cinv64.as<double>();
        else return cinv32.as<float>();
    }
    template <typename T> void vcycle_chunk(int k, const T* F, int64_t ldf, T* X, int64_t ldx);
    template <typename T> void vcycle(int k, const T* F, int64_t ldf, T* X, int64_t ldx);
    // y = B r: one V-cycle in the context precision (vcycle_B), or an MG-PCG
    // solve to exact_rtol while exact_b is set (the EXACT_B solve mode)
    void apply_B(int k, const double* F, int64_t ldf, double* X, int64_t ldx);
    void vcycle_B(int k, const double* F, int64_t ldf, double* X, int64_t ldx);
    void vcycle_B_eager(int k, const double* F, int64_t ldf, double* X, int64_t ldx);

    // hipGraph replay of the V-cycle (H1W_FLAG_GRAPH_VCYCLE): the kernel
    // sequence of vcycle_B for one (k, F, X) is captured on its second use
    // and replayed afterwards; the graphs refer to the workspace buffers, so
    // they are dropped whenever one of those is reallocated
    struct VGraph {
        int k;
        const double* F;
        int64_t ldf;
        double* X;
        int64_t ldx;
        hipGraphExec_t exec;
    };
    bool graphs = false;
    bool capturing = false;
    hipStream_t cap_stream = nullptr;  // private stream the V-cycle graphs are captured on
    bool own_cap_stream = true;        // destroyed with the context (false: lent by a batch worker,
                                       // which keeps it for the process)
    std::vector<VGraph> vgraphs;
    std::vector<const void*> vg_sig;
    int64_t graph_launches = 0;
    std::vector<const void*> workspace_signature() const;
    void clear_graphs();
    void vcycle_graph(int k, const double* F, int64_t ldf, double* X, int64_t ldx);
    bool exact_b = false;
    double exact_rtol = 1e-12;
    void mg_solve(int k, const double* F, int64_t ldf, double* X, int64_t ldx, double rtol, int maxit,
                  h1w_info* info);
    // Y = A X with the context's operator (FP64; the H1 Gram operator or the ERT one)
    void apply_A(int k, const double* X, int64_t ldx, double* Y, int64_t ldy);

    // lock-step solve of G GN systems on this grid (grouped.hip): item g has
    // m_g <= 128 rows J_g (leading dimension ldj_g), weight alpha_g, b_g, x_g
    struct GroupItem {
        int m;
        const double* J;
        int64_t ldj;
        double alpha;
        const double* b;
        double* x;
    };
    static constexpr int kGroupMaxRows = 128;
    DevBuf grpJ, grpZ, grpVec, grpS, grpSinv, grpPart, grpTab, grpScal, grpDefl;
    void vcycle_group(int k, const double* F, int64_t ldf, double* X, int64_t ldx);
    // status[g]: H1W_OK, or ENOCONV / ENUMERIC for an instance that failed
    // alone; failures of the whole group (set-up, a capacitance pivot) throw
    void gn_group_solve(int G, const GroupItem* items, const h1w_solve_opts& so, h1w_info* infos,
                        h1w_status* status);

    // ERT context (op = H1W_OP_ERT): conductivity operator, see ert.hip
    bool ert = false;
    unsigned dmask = 0;              // Dirichlet faces
    bool ert_ready = false;          // a conductivity has been set
    std::vector<int64_t> eoff;       // offset of each level's coefficient block in ecoef
    DevBuf ecoef;                    // per level: sigma, D, cx, cy, cz
    DevBuf efs, ekg, efield;         // unit loads, geometric factors, kept pole fields
    DevBuf egn;                      // GN step: d = m - m_ref, g, res = g - g_obs
    int efield_n = 0;                // rows held by efield
    ErtLevel ert_level(int l) const;
    void ert_validate();
    void ert_init();
    void ert_set_conductivity(const double* logsig);
    void ert_apply(int k, const double* X, int64_t ldx, double* Y, int64_t ldy);
    void ert_vcycle_chunk(int k, const double* F, int64_t ldf, double* X, int64_t ldx);
    void ert_fields(int n_src, const int* src, double* U, int64_t ldu, double rtol, int maxit, h1w_info* info);
    const double* ert_kgeo(int n_meas, const int* pair, const int* src, const double* kgeo);
    void ert_measure(int n_meas, const int* pair, const int* src, const double* k, const double* U, int64_t ldu,
                     double* g);
    void ert_sens(int n_src, const double* U, int64_t ldu, int n_meas, const int* pair, const double* k, double* J,
                  int64_t ldj, const double* gbar, double* grad);

    void capacitance_build(int m, const double* J, int64_t ldj, double alpha, int factor, h1w_info* info);
    void solve_S(const double* in, double* x);  // x = S^{-1} in (x may equal in)
    void ensure_cg_ws(int mneed);
    double* nv(int i);
    double* mv(int i);
    void dots(int64_t len, std::initializer_list<std::pair<const double*, const double*>> pairs, int slot);
    // partial sums only (launch_dots_partial layout) into dst; returns the parts per pair
    int dots_parts(int64_t len, std::initializer_list<std::pair<const double*, const double*>> pairs, double* dst);
    void woodbury_mspace(const double* y, double* Jy, double* w);
    void rows_dot(int mm, const double* M, int64_t ldm, const double* v, double* out);
    void z_stored_fp32(const double* w, const double* y, double ia, double* z);
    void precond_one(const double* r, double* z, int zmode);
    void precond_apply(int k, const double* R, int64_t ldr, double* Zout, int64_t ldz, int zmode);
    void gn_apply(int m, const double* J, int64_t ldj, double alpha, const double* x, double* y);
    // the same product with its scratch in the library's static device array
    // (no allocation; noalloc.hip)
    void gn_apply_noalloc(int m, const double* J, int64_t ldj, double alpha, const double* x, double* y);
    void gn_solve(int m, const double* J, int64_t ldj, double alpha, const double* b, const double* d,
                  const double* res, double* x, const h1w_solve_opts& o, h1w_info* info);

    void ev_reserve();
    void ev_record(int i);
    double ev_ms(int a, int b);

    // optional per-kernel-class timing (h1w_set_kernel_timing)
    unsigned tmask = 0;
    struct Pending {
        int cls;
        hipEvent_t a, b;
        double bytes, flops;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> evpool;
    h1w_kstat kst[H1W_K_NCLASS] = {};
    hipEvent_t take_event();
    void flush_timing();  // after the stream has been synchronised
    template <typename Fn>
    void timed(int cls, double bytes, double flops, Fn&& fn) {
        if (!(tmask & (1u << cls))) {
            fn();
            return;
        }
        Pending p{cls, take_event(), take_event(), bytes, flops};
        H1W_HIP(hipEventRecord(p.a, stream));
        fn();
        H1W_HIP(hipEventRecord(p.b, stream));
        pending.push_back(p);
    }
};

}  // namespace h1w
