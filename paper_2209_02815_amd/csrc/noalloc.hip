// h1w_gn_apply_noalloc: y = G x = alpha A x + J^T (J x) (the product whose
// residual is the stopping quantity of the Table 1 caption) for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc). It runs the kernels of
// h1w_gn_apply, with the two scratch arrays of that product (the m-vector
// J x and the per-chunk partial sums of the J x pass) placed in one static
// device array instead of the context's workspace:
//   - y itself takes alpha A x first, then J^T (J x) is added in place, so no
//     N-vector scratch is needed;
//   - the array is `scratch` below, kScratchBytes per device, held by every
//     GPU the library runs on until the process ends;
//   - its device address is taken once per device with hipGetSymbolAddress
//     (at h1w_setup, else at the first call on that device) and kept; host
//     code uses that address, never the array's name (which on the host is a
//     stand-in, not a device address).
// Every call on one GPU uses that GPU's array: calls that overlap in time on
// one GPU (two streams, two contexts, two threads) race. No memset is issued:
// every scratch value read is written by an earlier kernel of the same call.
#include <map>
#include <mutex>

#include "context.h"

namespace h1w {

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB per device
constexpr size_t kScratchElems = kScratchBytes / sizeof(double);

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, double*> g_addr;  // device -> device address of `scratch`

// the current device's address of `scratch` (taken once per device)
double* scratch_addr(std::string* err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        if (err) *err = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_addr.find(dev);
    if (it != g_addr.end()) return it->second;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        if (err) *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return nullptr;
    }
    g_addr.emplace(dev, static_cast<double*>(p));
    return static_cast<double*>(p);
}

}  // namespace

void noalloc_init_device() { (void)scratch_addr(nullptr); }

size_t noalloc_scratch_elems(int m, int64_t N) {
    const size_t jx = (size_t)cdiv(std::max(m, 0), 32) * 32;
    return jx + rows_dot_partial_elems(m, N);
}

void noalloc_require_fits(int m, int64_t N) {
    const size_t need = noalloc_scratch_elems(m, N);
    if (need > kScratchElems)
        throw Error{H1W_EINVAL, "h1w_gn_apply_noalloc: m = " + std::to_string(m) + " on " + std::to_string(N) +
                                    " nodes needs " + std::to_string(need * sizeof(double)) +
                                    " bytes of scratch, above the static " + std::to_string(kScratchBytes)};
}

void Ctx::gn_apply_noalloc(int mm, const double* JJ, int64_t ldjj, double al, const double* x, double* y) {
    const int64_t n = N();
    noalloc_require_fits(mm, n);
    std::string err;
    double* s = scratch_addr(&err);
    if (!s) throw Error{H1W_EHIP, err};
    double* Jx = s;
    double* part = s + cdiv(std::max(mm, 0), 32) * 32;
    launch_apply<double>(stream, dim, lv[0], 1, x, n, y, n, al);  // y = alpha A x
    if (mm > 0) {
        const int nchunk = launch_rows_dot_partial(stream, mm, n, JJ, ldjj, x, part);
        launch_reduce_parts(stream, mm, nchunk, part, Jx);
        launch_jt_plain(stream, mm, n, JJ, ldjj, Jx, y, y, 1.0);  // y += J^T (J x), in place
    }
}

}  // namespace h1w
