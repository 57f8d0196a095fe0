"""Host-side checks of the C ABI: the library loads, exports every function
declared in include/p3t.h, and validates parameters without touching a GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "p3t.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(p3t_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1506_04553_amd import load_library
    return load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    so = os.path.join(ROOT, "paper_1506_04553_amd", "libp3t.so")
    out = subprocess.run(["nm", "-D", "--defined-only", so], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (p3t_[a-z_]+)", out))
    assert set(names) <= exported, set(names) - exported


def test_library_has_gfx950_code():
    so = os.path.join(ROOT, "paper_1506_04553_amd", "libp3t.so")
    data = open(so, "rb").read()
    assert b"gfx950" in data


def _p(**kw):
    from paper_1506_04553_amd import make_params
    d = dict(eps=1e-3, r_in=1e-3, r_out=1e-2, theta=0.5, r_search=1.1e-2, n_crit=64, n_leaf=16)
    d.update(kw)
    return make_params(**d)


@pytest.mark.parametrize("bad", [dict(eps=-1.0), dict(r_out=0.0), dict(r_in=0.01), dict(r_in=-1e-4),
                                 dict(theta=-0.1), dict(r_search=0.0), dict(n_leaf=0),
                                 dict(n_crit=8), dict(use_quadrupole=2), dict(precision=3),
                                 dict(eps=float("nan")), dict(theta=float("inf"))])
def test_invalid_params_rejected(lib, bad):
    p = _p(**bad)
    assert lib.p3t_check_params(C.byref(p)) == -1


def test_valid_params_accepted(lib):
    for kw in (dict(), dict(r_in=0.0), dict(theta=0.0), dict(eps=0.0), dict(precision=1),
               dict(use_quadrupole=0), dict(n_crit=16, n_leaf=16)):
        p = _p(**kw)
        assert lib.p3t_check_params(C.byref(p)) == 0, kw
    assert lib.p3t_check_params(None) == -1


def test_null_context_and_status_strings(lib):
    assert lib.p3t_build_tree(None, 10, None, None, None) == -1
    assert lib.p3t_long_force(None, None, None) == -1
    nnz = C.c_int64(0)
    assert lib.p3t_neighbors(None, None, None, 0, C.byref(nnz)) == -1
    assert lib.p3t_long_force_vjp(None, None, None, None, None) == -1
    assert lib.p3t_get_stats(None, None) == -1
    assert lib.p3t_copy_array(None, 0, None, 0) == -1
    assert lib.p3t_kick_drift(None, 1, None, None, None, 0.0, 0.0) == -1
    assert lib.p3t_hard_force(None, 1, None, None, None, None, None, None, None, None, None,
                              None) == -1
    assert lib.p3t_hermite_hard(None, 1, None, None, None, None, None, None, None, None, None,
                                None) == -1
    assert lib.p3t_step(None, 1, None, None, None, None, None, None, None, None, None) == -1
    assert lib.p3t_kinds_soft(None, 1, None, None, None, None, None, None) == -1
    assert lib.p3t_kinds_neighbors(None, 1, None, None, None, None, None, None, 0, None) == -1
    assert lib.p3t_direct(None, 1, None, None, None, 0, None, None) == -1
    assert lib.p3t_release_lists(None) == -1
    lib.p3t_destroy(None)
    assert lib.p3t_status_string(0) == b"ok"
    assert lib.p3t_status_string(-3) == b"capacity exceeded"
    assert lib.p3t_status_string(-6) == b"iteration limit reached"
    assert lib.p3t_status_string(7) == b"unknown status"
    assert lib.p3t_last_error(None) == b"null context"


def test_create_rejects_bad_arguments(lib):
    from paper_1506_04553_amd.p3t import ALLOC_FN, FREE_FN
    h = C.c_void_p()
    # allocator and free must be given together
    rc = lib.p3t_create(C.byref(h), 0, None, ALLOC_FN(lambda n, u: None), FREE_FN(0), None)
    assert rc == -1 and not h.value
    rc = lib.p3t_create(C.byref(h), -1, None, ALLOC_FN(0), FREE_FN(0), None)
    assert rc == -1 and not h.value


def test_make_params_rejects_unknown_names():
    """A misspelt parameter name must not be dropped silently."""
    from paper_1506_04553_amd import make_params
    d = dict(eps=1e-3, r_in=1e-3, r_out=1e-2, theta=0.5, r_search=1.1e-2)
    make_params(**d)
    with pytest.raises(TypeError):
        make_params(**d, n_crti=64)
    with pytest.raises(TypeError):
        make_params(**d, quadrupole=1)
