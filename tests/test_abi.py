"""C-ABI checks that need no GPU: the library loads, exports every symbol
declared in include/acr.h, and validates arguments on the host before any
device work."""
import ctypes
import os
import re

import pytest

import paper_1712_08872_amd as acr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "acr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(acr_\w+|krylov_\w+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = acr.lib()
    names = _declared()
    assert "acr_setup" in names and "krylov_solve" in names and "acr_grad_kappa" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(acr.SYMBOLS) <= set(names)


def test_default_options_and_status_strings():
    o = acr.default_options()
    assert o.eps == 1e-4 and o.eta == 2.0 and o.leaf_size == 32 and o.precision == acr.FP64
    L = acr.lib()
    for s in range(9):
        assert L.acr_status_string(s)


def _setup(p, o):
    out = ctypes.c_void_p(1234)
    st = acr.lib().acr_setup(ctypes.byref(p) if p is not None else None,
                             ctypes.byref(o) if o is not None else None, None, ctypes.byref(out))
    return st, out


@pytest.mark.parametrize("field,value", [("nx", 0), ("ny", -1), ("nz", 0), ("kind", 7)])
def test_problem_validation(field, value):
    p = acr.Problem(8, 8, 8, acr.POISSON_HARMONIC, None, 0.0, 0.0, None, 0.0, None)
    setattr(p, field, value)
    st, out = _setup(p, acr.default_options())
    assert st == 1 and out.value is None
    assert acr.lib().acr_last_error()


@pytest.mark.parametrize("field,value", [("eps", 0.0), ("eps", -1e-3), ("eps", 1.5), ("eps", 9.9e-8),
                                         ("eps", 1e-10), ("eta", 0.0),
                                         ("eta", float("nan")), ("leaf_size", 2), ("leaf_size", 65),
                                         ("precision", 5), ("max_rank", -1), ("max_rank", 57),
                                         ("dense_work", 65), ("flags", 1)])
def test_option_validation(field, value):
    p = acr.Problem(8, 8, 8, acr.POISSON_HARMONIC, None, 0.0, 0.0, None, 0.0, None)
    o = acr.default_options()
    setattr(o, field, value)
    st, out = _setup(p, o)
    assert st == 1 and out.value is None


def test_missing_inputs_rejected():
    o = acr.default_options()
    assert _setup(None, o)[0] == 1
    p = acr.Problem(8, 8, 8, acr.HELMHOLTZ, None, 0.0, 0.0, None, 1.0, None)
    assert _setup(p, o)[0] == 1
    p = acr.Problem(8, 8, 8, acr.STENCIL7_RAW, None, 0.0, 0.0, None, 0.0, None)
    assert _setup(p, o)[0] == 1
    L = acr.lib()
    assert L.acr_apply(None, None, None, 1, None) == 1
    assert L.acr_apply_T(None, None, None, 1, None) == 1
    assert L.krylov_solve(None, 0, 30, 0, 1e-8, 10, None, None, None, None) == 1
    assert L.acr_grad_kappa(None, None, None, None, None) == 1
    assert L.acr_stats(None, None) == 1
    L.acr_destroy(None)


def test_valid_setup_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = acr.Problem(8, 8, 8, acr.POISSON_HARMONIC, None, 0.0, 0.0, None, 0.0, None)
    st, out = _setup(p, acr.default_options())
    assert st == 7 and out.value is None


def test_bf16_factors_need_loose_eps():
    p = acr.Problem(8, 8, 8, acr.POISSON_HARMONIC, None, 0.0, 0.0, None, 0.0, None)
    o = acr.default_options()
    o.precision = acr.MIXED_BF16
    o.eps = 1e-4
    st, out = _setup(p, o)
    assert st == 1 and out.value is None
    assert b"BF16" in acr.lib().acr_last_error()
    import torch
    if torch.cuda.is_available():
        return
    o.eps = 1e-2  # accepted by validation; without a device the setup then fails on the device
    st, out = _setup(p, o)
    assert st == 7 and out.value is None


def test_eps_floor_is_stated():
    """eps below the truncation's resolvable floor is refused with a message
    that says why (the Gram-matrix truncation resolves singular values only
    down to about 1e-8 of the largest)."""
    p = acr.Problem(8, 8, 8, acr.POISSON_HARMONIC, None, 0.0, 0.0, None, 0.0, None)
    o = acr.default_options()
    o.eps = 5e-8
    st, out = _setup(p, o)
    assert st == 1 and out.value is None
    assert b"1e-7" in acr.lib().acr_last_error()
