"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/h1w.h, and rejects invalid setup arguments on the
host before any device call."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "h1w.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(h1w_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ["h1w_setup", "h1w_poisson_solve_batched", "h1w_capacitance_build", "h1w_precond_apply",
              "h1w_gn_solve", "h1w_ert_sensitivities", "h1w_operator_apply", "h1w_gn_apply"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2209_02815_amd import _native
    lib = C.CDLL(_native._LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(_native.EXPORTED) == _declared()


def test_status_strings_and_notimpl():
    from paper_2209_02815_amd import _native as nat
    assert nat.lib.h1w_status_string(nat.H1W_OK) == b"ok"
    assert nat.lib.h1w_status_string(nat.H1W_ENOTSPD).startswith(b"capacitance")
    assert nat.lib.h1w_status_string(nat.H1W_ENOTIMPL) == b"not implemented"
    assert nat.lib.h1w_ert_sensitivities(None, None, 0, None, 0, None, None, None, None, 0, None, 0, None,
                                         None) == nat.H1W_EINVAL
    assert nat.lib.h1w_ert_set_conductivity(None, None) == nat.H1W_EINVAL
    assert nat.lib.h1w_ert_vjp(None, 0, None, None, 0, 0, None, None, None, None) == nat.H1W_EINVAL


@pytest.mark.parametrize("bad", [
    dict(dim=4), dict(n=(1, 9, 9)), dict(beta=0.0), dict(beta=float("nan")), dict(precision=7),
    dict(nu=-1), dict(cheb=(2.0, 1.0)), dict(flags=64), dict(flags=16), dict(rhs_chunk=-3),
])
def test_setup_rejects_invalid_arguments_on_host(bad):
    from paper_2209_02815_amd import _native as nat
    d = nat.h1w_grid_desc()
    d.dim = bad.get("dim", 3)
    for i, n in enumerate(bad.get("n", (9, 9, 9))):
        d.n[i] = n
    d.beta = bad.get("beta", 1e-2)
    d.precision = bad.get("precision", 0)
    d.nu = bad.get("nu", 0)
    d.cheb_lo, d.cheb_hi = bad.get("cheb", (0.0, 0.0))
    d.flags = bad.get("flags", 0)
    d.rhs_chunk = bad.get("rhs_chunk", 0)
    h = C.c_void_p()
    st = nat.lib.h1w_setup(C.byref(d), None, C.byref(h))
    assert st == nat.H1W_EINVAL
    assert h.value is None
    assert len(nat.lib.h1w_last_error(None)) > 0


@pytest.mark.parametrize("bad", [
    dict(op=2), dict(dim=2, n=(17, 17, 1)), dict(precision=1), dict(flags=1), dict(mask=0x40),
    dict(n=(11, 11, 11)),  # coarsest level 6^3 = 216 nodes > 128 (the dense in-LDS inverse)
    dict(op=0, mask=0x1F),  # a Dirichlet mask on an H1 Gram context
])
def test_ert_setup_rejects_invalid_arguments_on_host(bad):
    from paper_2209_02815_amd import _native as nat
    d = nat.h1w_grid_desc()
    d.dim = bad.get("dim", 3)
    for i, n in enumerate(bad.get("n", (17, 17, 17))):
        d.n[i] = n
    d.beta = 1e-2
    d.precision = bad.get("precision", 0)
    d.flags = bad.get("flags", 0)
    d.op = bad.get("op", nat.H1W_OP_ERT)
    d.dirichlet_mask = bad.get("mask", 0)
    h = C.c_void_p()
    st = nat.lib.h1w_setup(C.byref(d), None, C.byref(h))
    assert st == nat.H1W_EINVAL, nat.lib.h1w_last_error(None)
    assert h.value is None
    assert len(nat.lib.h1w_last_error(None)) > 0


def test_null_context_is_rejected():
    from paper_2209_02815_amd import _native as nat
    assert nat.lib.h1w_operator_apply(None, 1, None, 1, None, 1, 0) == nat.H1W_EINVAL
    assert nat.lib.h1w_gn_solve(None, 0, None, 1, 1.0, None, None, None, None, None, None) == nat.H1W_EINVAL
