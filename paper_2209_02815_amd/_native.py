"""ctypes binding of libh1w.so (include/h1w.h): argument marshalling only.

Every function here has the name of the C entry point it calls and takes torch
tensors already resident on the GPU; all arithmetic happens in the HIP
library. Import fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libh1w.so")

H1W_OK, H1W_EINVAL, H1W_ENOMEM, H1W_EHIP, H1W_ENOTSPD, H1W_ENOCONV, H1W_ENUMERIC, H1W_ENOTIMPL, H1W_ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
H1W_FP64, H1W_MIXED = 0, 1
H1W_DT_F64, H1W_DT_F32 = 0, 1
H1W_VCYCLE_ONCE, H1W_MG_SOLVE = 0, 1
H1W_Z_AUTO, H1W_Z_STORED, H1W_Z_RECOMPUTE = 0, 1, 2
H1W_FACTOR_AUTO, H1W_FACTOR_CHOL, H1W_FACTOR_LU = 0, 1, 2

KCLASS = ["smooth", "smooth_first", "residual", "restrict", "prolong", "coarse", "gemm", "jv", "jtv",
          "factor", "trsv", "apply", "vdown", "vup", "ert_stencil", "ert_sens", "vtail"]

EXPORTED = [
    "h1w_setup", "h1w_destroy", "h1w_last_error", "h1w_status_string", "h1w_get_sizes",
    "h1w_operator_apply", "h1w_poisson_solve_batched", "h1w_capacitance_build",
    "h1w_precond_apply", "h1w_gn_solve", "h1w_gn_apply", "h1w_ert_sensitivities",
    "h1w_set_kernel_timing", "h1w_get_kernel_timing", "h1w_reset_kernel_timing", "h1w_batch_solve",
    "h1w_ert_set_conductivity", "h1w_ert_vjp", "h1w_ert_gn_step", "h1w_gn_apply_noalloc",
]


class h1w_grid_desc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("beta", C.c_double), ("precision", C.c_int),
                ("nu", C.c_int), ("cheb_lo", C.c_double), ("cheb_hi", C.c_double),
                ("coarse_max", C.c_int64), ("rhs_chunk", C.c_int), ("flags", C.c_uint),
                ("op", C.c_int), ("dirichlet_mask", C.c_uint)]


class h1w_solve_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int), ("zmode", C.c_int), ("factor", C.c_int),
                ("check_every", C.c_int), ("flags", C.c_uint)]


class h1w_info(C.Structure):
    _fields_ = [("iters", C.c_int), ("factor_used", C.c_int), ("zmode_used", C.c_int),
                ("failed_pivot", C.c_int), ("nlevels", C.c_int), ("restarts", C.c_int),
                ("relres_true", C.c_double), ("relres_rec", C.c_double),
                ("t_zbuild_ms", C.c_double), ("t_gemm_ms", C.c_double), ("t_factor_ms", C.c_double),
                ("t_cg_ms", C.c_double), ("t_total_ms", C.c_double), ("asym_S_over_alpha", C.c_double),
                ("kappa_S_est", C.c_double), ("s_max_over_alpha", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class h1w_batch_item(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("beta", C.c_double), ("alpha", C.c_double),
                ("m", C.c_int), ("J", C.c_void_p), ("ldj", C.c_int64), ("b", C.c_void_p), ("x", C.c_void_p)]


class h1w_batch_opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("nworkers", C.c_int), ("autotune", C.c_int), ("nu", C.c_int),
                ("rtol", C.c_double), ("maxit", C.c_int), ("graphs", C.c_int), ("grouped", C.c_int)]


H1W_BATCH_MAX_KEYS = 64


class h1w_batch_tuned(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("m_bucket", C.c_int), ("nu", C.c_int),
                ("ms_per_unit", C.c_double), ("reused", C.c_int), ("cheb_lo", C.c_double),
                ("iters", C.c_int), ("iters_default", C.c_int), ("grouped", C.c_int)]


class h1w_batch_report(C.Structure):
    _fields_ = [("t_total_ms", C.c_double), ("nworkers", C.c_int), ("ntuned", C.c_int),
                ("tuned", h1w_batch_tuned * H1W_BATCH_MAX_KEYS)]


class h1w_kstat(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("bytes", C.c_double), ("flops", C.c_double)]


class H1WError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


def _load():
    # torch's HIP libraries need the unversioned libamdhip64.so; loading torch
    # first makes libh1w.so (which needs libamdhip64.so.7) bind to that same
    # runtime instead of pulling a second HIP runtime into the process.
    import torch  # noqa: F401
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with paper_2209_02815_amd.build.build()")
    lib = C.CDLL(_LIB_PATH)
    P, I, I64, D = C.c_void_p, C.c_int, C.c_int64, C.c_double
    sig = {
        "h1w_setup": (I, [C.POINTER(h1w_grid_desc), P, C.POINTER(P)]),
        "h1w_destroy": (None, [P]),
        "h1w_last_error": (C.c_char_p, [P]),
        "h1w_status_string": (C.c_char_p, [I]),
        "h1w_get_sizes": (I, [P, C.POINTER(I64), C.POINTER(I)]),
        "h1w_operator_apply": (I, [P, I, P, I64, P, I64, I]),
        "h1w_poisson_solve_batched": (I, [P, I, P, I64, P, I64, I, I, D, I, C.POINTER(h1w_info)]),
        "h1w_capacitance_build": (I, [P, I, P, I64, D, I, P, I64, P, I64, C.POINTER(h1w_info)]),
        "h1w_precond_apply": (I, [P, I, P, I64, P, I64, I]),
        "h1w_gn_solve": (I, [P, I, P, I64, D, P, P, P, P, C.POINTER(h1w_solve_opts), C.POINTER(h1w_info)]),
        "h1w_gn_apply": (I, [P, I, P, I64, D, P, P]),
        "h1w_gn_apply_noalloc": (I, [P, I, P, I64, D, P, P]),
        "h1w_ert_sensitivities": (I, [P, P, I, P, I, P, P, P, P, I64, P, I64, C.POINTER(h1w_solve_opts),
                                      C.POINTER(h1w_info)]),
        "h1w_ert_set_conductivity": (I, [P, P]),
        "h1w_ert_vjp": (I, [P, I, P, P, I64, I, P, P, P, P]),
        "h1w_ert_gn_step": (I, [P, P, P, P, I, P, I, P, P, P, D, P, I64, P, P, C.POINTER(h1w_solve_opts),
                                C.POINTER(h1w_solve_opts), C.POINTER(h1w_info)]),
        "h1w_set_kernel_timing": (I, [P, C.c_uint]),
        "h1w_get_kernel_timing": (I, [P, I, C.POINTER(h1w_kstat)]),
        "h1w_reset_kernel_timing": (I, [P]),
        "h1w_batch_solve": (I, [I, C.POINTER(h1w_batch_item), C.POINTER(h1w_batch_opts), C.POINTER(h1w_info),
                                C.POINTER(C.c_int), C.POINTER(h1w_batch_report)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def _check(ctx, st: int):
    if st != H1W_OK:
        msg = lib.h1w_last_error(ctx)
        raise H1WError(st, (msg or b"").decode() or lib.h1w_status_string(st).decode())


# ------------------------------------------------------------------ tensor helpers
def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _rows(t, N: int, what: str):
    """(k, ld) of a 1-D (one row) or 2-D row-major CUDA tensor with N columns."""
    if t is None:
        return 0, N
    if not t.is_cuda:
        raise ValueError(f"{what} must be a CUDA tensor")
    if t.dim() == 1:
        if t.shape[0] != N or t.stride(0) != 1:
            raise ValueError(f"{what} must have {N} contiguous entries")
        return 1, N
    if t.dim() != 2 or t.shape[1] != N or t.stride(1) != 1:
        raise ValueError(f"{what} must be (k, {N}) with unit stride along rows")
    return t.shape[0], max(t.stride(0), N)


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return H1W_DT_F64
    if t.dtype == torch.float32:
        return H1W_DT_F32
    raise ValueError("tensors must be float64 or float32")


# ------------------------------------------------------------------ entry points
H1W_FLAG_STREAM_Z = 1
H1W_FLAG_UNFUSED_VCYCLE = 2
H1W_FLAG_GRAPH_VCYCLE = 4
H1W_FLAG_NO_VTAIL = 8
H1W_FLAG_CAP_FP32_GEMM = 16
H1W_SOLVE_LAPLACE_ONLY = 1
H1W_SOLVE_EXACT_B = 2
H1W_OP_H1GRAM, H1W_OP_ERT = 0, 1


def h1w_setup(shape, beta: float, precision: int = H1W_FP64, nu: int = 0, cheb=(0.0, 0.0),
              coarse_max: int = 0, rhs_chunk: int = 0, stream=None, flags: int = 0, op: int = H1W_OP_H1GRAM,
              dirichlet_mask: int = 0):
    """Create a context; returns the opaque handle (c_void_p)."""
    d = h1w_grid_desc()
    d.dim = len(shape)
    for i, n in enumerate(shape):
        d.n[i] = int(n)
    d.beta, d.precision, d.nu = float(beta), int(precision), int(nu)
    d.cheb_lo, d.cheb_hi = float(cheb[0]), float(cheb[1])
    d.coarse_max, d.rhs_chunk, d.flags = int(coarse_max), int(rhs_chunk), int(flags)
    d.op, d.dirichlet_mask = int(op), int(dirichlet_mask)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    h = C.c_void_p()
    st = lib.h1w_setup(C.byref(d), C.c_void_p(stream), C.byref(h))
    if st != H1W_OK:
        raise H1WError(st, lib.h1w_last_error(None).decode())
    return h


def h1w_destroy(ctx):
    lib.h1w_destroy(ctx)


def h1w_get_sizes(ctx):
    N, L = C.c_int64(), C.c_int()
    _check(ctx, lib.h1w_get_sizes(ctx, C.byref(N), C.byref(L)))
    return N.value, L.value


def h1w_operator_apply(ctx, X, Y):
    N, _ = h1w_get_sizes(ctx)
    k, ldx = _rows(X, N, "X")
    k2, ldy = _rows(Y, N, "Y")
    if k != k2 or X.dtype != Y.dtype:
        raise ValueError("X and Y must have the same rows and dtype")
    _check(ctx, lib.h1w_operator_apply(ctx, k, _ptr(X), ldx, _ptr(Y), ldy, _dtype_code(X)))
    return Y


def h1w_poisson_solve_batched(ctx, F, X, mode: int = H1W_VCYCLE_ONCE, rtol: float = 1e-10, maxit: int = 0):
    N, _ = h1w_get_sizes(ctx)
    k, ldf = _rows(F, N, "F")
    k2, ldx = _rows(X, N, "X")
    if k != k2 or F.dtype != X.dtype:
        raise ValueError("F and X must have the same rows and dtype")
    info = h1w_info()
    _check(ctx, lib.h1w_poisson_solve_batched(ctx, k, _ptr(F), ldf, _ptr(X), ldx, _dtype_code(F), mode,
                                              float(rtol), int(maxit), C.byref(info)))
    return info


def h1w_capacitance_build(ctx, J, alpha: float, factor: int = H1W_FACTOR_AUTO, S_out=None, Z_out=None):
    N, _ = h1w_get_sizes(ctx)
    m, ldj = _rows(J, N, "J")
    lds = 0 if S_out is None else S_out.stride(0)
    _, ldz = _rows(Z_out, N, "Z_out")
    info = h1w_info()
    _check(ctx, lib.h1w_capacitance_build(ctx, m, _ptr(J), ldj, float(alpha), int(factor), _ptr(S_out), lds,
                                          _ptr(Z_out), ldz, C.byref(info)))
    return info


def h1w_precond_apply(ctx, R, Zout, zmode: int = H1W_Z_AUTO):
    N, _ = h1w_get_sizes(ctx)
    k, ldr = _rows(R, N, "R")
    k2, ldz = _rows(Zout, N, "Zout")
    if k != k2:
        raise ValueError("R and Zout must have the same rows")
    _check(ctx, lib.h1w_precond_apply(ctx, k, _ptr(R), ldr, _ptr(Zout), ldz, int(zmode)))
    return Zout


def h1w_gn_solve(ctx, J, alpha: float, x, b=None, d=None, res=None, rtol: float = 0.0, maxit: int = 0,
                 zmode: int = H1W_Z_AUTO, factor: int = H1W_FACTOR_AUTO, raise_on_error: bool = True,
                 flags: int = 0):
    N, _ = h1w_get_sizes(ctx)
    m, ldj = (0, N) if J is None else _rows(J, N, "J")
    o = h1w_solve_opts(float(rtol), int(maxit), int(zmode), int(factor), 0, int(flags))
    info = h1w_info()
    st = lib.h1w_gn_solve(ctx, m, _ptr(J), ldj, float(alpha), _ptr(b), _ptr(d), _ptr(res), _ptr(x),
                          C.byref(o), C.byref(info))
    if raise_on_error:
        _check(ctx, st)
    return (info, st) if not raise_on_error else info


def h1w_gn_apply(ctx, J, alpha: float, x, y):
    N, _ = h1w_get_sizes(ctx)
    m, ldj = (0, N) if J is None else _rows(J, N, "J")
    _check(ctx, lib.h1w_gn_apply(ctx, m, _ptr(J), ldj, float(alpha), _ptr(x), _ptr(y)))
    return y


def h1w_gn_apply_noalloc(ctx, J, alpha: float, x, y):
    """y = G x with the library's static device scratch (no allocation, no
    synchronisation: y is valid once the context's stream has synchronised)."""
    N, _ = h1w_get_sizes(ctx)
    m, ldj = (0, N) if J is None else _rows(J, N, "J")
    _check(ctx, lib.h1w_gn_apply_noalloc(ctx, m, _ptr(J), ldj, float(alpha), _ptr(x), _ptr(y)))
    return y


def _ints(t, what: str, cols: int = 1):
    import torch
    if t is None:
        return 0
    if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous int32 CUDA tensor")
    if cols > 1 and (t.dim() != 2 or t.shape[1] != cols):
        raise ValueError(f"{what} must have shape (n, {cols})")
    return t.shape[0]


def h1w_ert_set_conductivity(ctx, logsig):
    N, _ = h1w_get_sizes(ctx)
    _rows(logsig, N, "logsig")
    _check(ctx, lib.h1w_ert_set_conductivity(ctx, _ptr(logsig)))


def h1w_ert_sensitivities(ctx, src_node, pair, logsig=None, kgeo=None, g_out=None, J_out=None, U_out=None,
                          rtol: float = 0.0, maxit: int = 0, raise_on_error: bool = True):
    """Pole fields, voltages and sensitivities of an ERT context (see the
    header); src_node: int32 (n_src,), pair: int32 (n_meas, 2) CUDA tensors."""
    N, _ = h1w_get_sizes(ctx)
    n_src = _ints(src_node, "src_node")
    n_meas = _ints(pair, "pair", 2)
    if logsig is not None:
        _rows(logsig, N, "logsig")
    _, ldj = _rows(J_out, N, "J_out")
    _, ldu = _rows(U_out, N, "U_out")
    o = h1w_solve_opts(float(rtol), int(maxit), 0, 0, 0, 0)
    info = h1w_info()
    st = lib.h1w_ert_sensitivities(ctx, _ptr(logsig), n_src, _ptr(src_node), n_meas, _ptr(pair), _ptr(kgeo),
                                   _ptr(g_out), _ptr(J_out), ldj, _ptr(U_out), ldu, C.byref(o), C.byref(info))
    if raise_on_error:
        _check(ctx, st)
        return info
    return info, st


def h1w_ert_vjp(ctx, pair, gbar, grad, U=None, n_src: int | None = None, src_node=None, kgeo=None):
    """grad = J^T gbar for the current conductivity and the fields U (None:
    the fields kept by the last h1w_ert_sensitivities call)."""
    N, _ = h1w_get_sizes(ctx)
    n_meas = _ints(pair, "pair", 2)
    k, ldu = _rows(U, N, "U")
    if U is None:
        k = int(n_src if n_src is not None else _ints(src_node, "src_node"))
    _rows(grad, N, "grad")
    _check(ctx, lib.h1w_ert_vjp(ctx, k, _ptr(src_node), _ptr(U), ldu, n_meas, _ptr(pair), _ptr(kgeo),
                                _ptr(gbar), _ptr(grad)))
    return grad


def h1w_set_kernel_timing(ctx, mask: int):
    _check(ctx, lib.h1w_set_kernel_timing(ctx, int(mask)))


def h1w_get_kernel_timing(ctx, kclass: int) -> dict:
    st = h1w_kstat()
    _check(ctx, lib.h1w_get_kernel_timing(ctx, int(kclass), C.byref(st)))
    return {"launches": st.launches, "ms": st.ms, "bytes": st.bytes, "flops": st.flops}


def h1w_reset_kernel_timing(ctx):
    _check(ctx, lib.h1w_reset_kernel_timing(ctx))


def h1w_batch_solve(items, precision: int = H1W_FP64, nworkers: int = 0, autotune: int = 0, nu: int = 0,
                    rtol: float = 0.0, maxit: int = 0, raise_on_error: bool = True, graphs: bool = False,
                    grouped: bool = False):
    """items: list of dicts with shape, beta, alpha, J (CUDA (m, N) float64 or None), b, x.
    grouped: solve the items of one grid in lock step (items with more than 128
    rows one at a time after the groups); otherwise one solve per item on
    nworkers streams. Returns (infos, statuses, report); raises for the failing
    item with the lowest index unless raise_on_error is False."""
    arr = (h1w_batch_item * max(1, len(items)))()
    for i, it in enumerate(items):
        shape = tuple(it["shape"])
        N = 1
        for nn in shape:
            N *= int(nn)
        e = arr[i]
        e.dim = len(shape)
        for a, nn in enumerate(shape):
            e.n[a] = int(nn)
        e.beta, e.alpha = float(it["beta"]), float(it["alpha"])
        J = it.get("J")
        m, ldj = _rows(J, N, "J") if J is not None else (0, N)
        e.m, e.ldj = m, ldj
        e.J = None if J is None else J.data_ptr()
        for name in ("b", "x"):
            t = it[name]
            if not t.is_cuda or t.dtype != __import__("torch").float64 or t.numel() != N or not t.is_contiguous():
                raise ValueError(f"item {i}: {name} must be a contiguous float64 CUDA vector of N entries")
        e.b, e.x = it["b"].data_ptr(), it["x"].data_ptr()
    opts = h1w_batch_opts(int(precision), int(nworkers), int(autotune), int(nu), float(rtol), int(maxit),
                          int(bool(graphs)), int(bool(grouped)))
    infos = (h1w_info * max(1, len(items)))()
    stats = (C.c_int * max(1, len(items)))()
    rep = h1w_batch_report()
    st = lib.h1w_batch_solve(len(items), arr, C.byref(opts), infos, stats, C.byref(rep))
    out = ([infos[i] for i in range(len(items))], [stats[i] for i in range(len(items))], rep)
    if raise_on_error and st != H1W_OK:
        raise H1WError(st, lib.h1w_last_error(None).decode())
    return out


def h1w_ert_gn_step(ert, h1, m, m_ref, src_node, pair, g_obs, alpha: float, J, dm, g_out=None, kgeo=None,
                    ert_rtol: float = 0.0, gn_rtol: float = 0.0, gn_maxit: int = 0):
    """One Gauss-Newton step (see the header); m is updated in place. Errors are
    reported on the H1 context h1."""
    N, _ = h1w_get_sizes(h1)
    n_src = _ints(src_node, "src_node")
    n_meas = _ints(pair, "pair", 2)
    _, ldj = _rows(J, N, "J")
    for t, what in ((m, "m"), (m_ref, "m_ref"), (dm, "dm")):
        _rows(t, N, what)
    eo = h1w_solve_opts(float(ert_rtol), 0, 0, 0, 0, 0)
    go = h1w_solve_opts(float(gn_rtol), int(gn_maxit), 0, 0, 0, 0)
    info = h1w_info()
    _check(h1, lib.h1w_ert_gn_step(ert, h1, _ptr(m), _ptr(m_ref), n_src, _ptr(src_node), n_meas, _ptr(pair),
                                   _ptr(kgeo), _ptr(g_obs), float(alpha), _ptr(J), ldj, _ptr(dm), _ptr(g_out),
                                   C.byref(eo), C.byref(go), C.byref(info)))
    return info
