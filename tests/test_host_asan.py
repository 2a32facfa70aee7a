"""The library's host code under AddressSanitizer (libh1w_asan.so, built by
build() with host-only instrumentation): argument validation and error
reporting of every entry point that can run without a GPU, in a child
process with the ASan runtime preloaded. A memory error on these paths (an
overflow in a message buffer, a use after free of a context) aborts the child
with an AddressSanitizer report."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2209_02815_amd", "libh1w_asan.so")

CHILD = r'''
import ctypes as C, sys
assert "libclang_rt.asan" in open("/proc/self/maps").read()   # the ASan runtime is live
lib = C.CDLL(sys.argv[1])
P, I, D, I64 = C.c_void_p, C.c_int, C.c_double, C.c_int64

class Desc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("beta", C.c_double), ("precision", C.c_int),
                ("nu", C.c_int), ("cheb_lo", C.c_double), ("cheb_hi", C.c_double),
                ("coarse_max", C.c_int64), ("rhs_chunk", C.c_int), ("flags", C.c_uint), ("op", C.c_int),
                ("dirichlet_mask", C.c_uint)]

lib.h1w_setup.argtypes = [C.POINTER(Desc), P, C.POINTER(P)]
lib.h1w_last_error.restype = C.c_char_p
lib.h1w_last_error.argtypes = [P]
lib.h1w_status_string.restype = C.c_char_p
lib.h1w_destroy.argtypes = [P]
bad = [dict(dim=4), dict(n=(1, 9, 9)), dict(beta=0.0), dict(beta=float("nan")), dict(precision=7),
       dict(nu=-1), dict(cheb=(2.0, 1.0)), dict(flags=64), dict(flags=16), dict(rhs_chunk=-3),
       dict(op=5), dict(dirichlet_mask=3)]
for b in bad:
    d = Desc()
    d.dim = b.get("dim", 3)
    for i, n in enumerate(b.get("n", (9, 9, 9))):
        d.n[i] = n
    d.beta = b.get("beta", 1e-2)
    d.precision = b.get("precision", 0)
    d.nu = b.get("nu", 0)
    d.cheb_lo, d.cheb_hi = b.get("cheb", (0.0, 0.0))
    d.flags = b.get("flags", 0)
    d.rhs_chunk = b.get("rhs_chunk", 0)
    d.op = b.get("op", 0)
    d.dirichlet_mask = b.get("dirichlet_mask", 0)
    out = P()
    st = lib.h1w_setup(C.byref(d), None, C.byref(out))
    msg = lib.h1w_last_error(None)
    assert st == -1 and out.value is None and msg, (b, st, msg)
assert lib.h1w_setup(None, None, None) == -1
for s in range(-9, 2):
    assert lib.h1w_status_string(s)
lib.h1w_destroy(None)
# NULL contexts are EINVAL at every entry point that takes one
for name, nargs in [("h1w_gn_solve", 11), ("h1w_gn_apply", 7), ("h1w_gn_apply_noalloc", 7),
                    ("h1w_precond_apply", 7), ("h1w_capacitance_build", 11), ("h1w_operator_apply", 7),
                    ("h1w_poisson_solve_batched", 11), ("h1w_set_kernel_timing", 2),
                    ("h1w_reset_kernel_timing", 1), ("h1w_ert_set_conductivity", 2)]:
    f = getattr(lib, name)
    f.argtypes = [P] * nargs
    assert f(*([None] * nargs)) == -1, name
# batch options are validated before any device work
class BatchOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("nworkers", C.c_int), ("autotune", C.c_int), ("nu", C.c_int),
                ("rtol", C.c_double), ("maxit", C.c_int), ("graphs", C.c_int), ("grouped", C.c_int)]

lib.h1w_batch_solve.argtypes = [I, P, P, P, P, P]
item = (C.c_char * 256)()
for b in [dict(grouped=2), dict(graphs=3), dict(precision=7), dict(autotune=5), dict(rtol=float("nan")),
          dict(nworkers=-1), dict(nu=17), dict(maxit=-2)]:
    o = BatchOpts()
    o.precision = b.get("precision", 0)
    o.nworkers = b.get("nworkers", 0)
    o.autotune = b.get("autotune", 0)
    o.nu = b.get("nu", 0)
    o.rtol = b.get("rtol", 1e-8)
    o.maxit = b.get("maxit", 0)
    o.graphs = b.get("graphs", 0)
    o.grouped = b.get("grouped", 0)
    st = lib.h1w_batch_solve(1, C.cast(item, P), C.cast(C.byref(o), P), None, None, None)
    assert st == -1 and lib.h1w_last_error(None), (b, st)
o = BatchOpts()
assert lib.h1w_batch_solve(-1, None, C.cast(C.byref(o), P), None, None, None) == -1
assert lib.h1w_batch_solve(1, None, C.cast(C.byref(o), P), None, None, None) == -1
assert lib.h1w_batch_solve(1, C.cast(item, P), None, None, None, None) == -1
print("ASAN-CHILD-OK")
'''


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_paths_under_address_sanitizer():
    rt = _asan_runtime()
    if not os.path.exists(LIB) or rt is None:
        pytest.skip("libh1w_asan.so (build()) or the ASan runtime is missing")
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=77")
    r = subprocess.run([sys.executable, "-c", CHILD, LIB], env=env, capture_output=True, text=True, timeout=120)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.returncode == 0 and "ASAN-CHILD-OK" in r.stdout, (r.returncode, r.stdout[-500:], r.stderr[-2000:])
