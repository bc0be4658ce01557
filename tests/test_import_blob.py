"""acr_import_factors without a device: the oracle's factors encoded in the
library's leaf order decode back to the same matrices (the encoding the GPU
test relies on), and malformed factor lists are refused on the host with
ACR_E_INVALID before any device work."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import assembly, hacr
from factor_blob import decode, oracle_factors

import paper_1712_08872_amd as acr


@pytest.fixture(scope="module")
def small():
    nx, ny, nz = 13, 9, 6
    kap = np.exp(synth.gaussian_field_exp((nz + 2, ny + 2, nx + 2), 1))
    S = assembly.stencil7("poisson", nx, ny, nz, kappa=kap)
    H = hacr.HACR(S, nx, ny, nz, eps=1e-5, eta=2.0, leaf=16)
    facs, leaves = oracle_factors(H, 2.0, 16)
    return H, facs, leaves


def test_encoding_round_trip(small):
    H, facs, leaves = small
    B = H.nx * H.ny
    assert len(facs) == len(H.factor_list())
    for f, (r, role, p, obj) in zip(facs, H.factor_list()):
        ref = np.diag(obj) if isinstance(obj, np.ndarray) else obj.to_dense()
        np.testing.assert_array_equal(decode(f, leaves, B), ref)


def _call(facs, nx=13, ny=9, nz=6, leaf=16, precision=acr.FP64, eps=1e-5):
    keep = []
    arr = (acr.Factor * max(len(facs), 1))()
    for i, f in enumerate(facs):
        data = np.ascontiguousarray(f["data"], dtype=np.float64)
        rk = None if f.get("diag") else np.ascontiguousarray(f["ranks"], dtype=np.int32)
        keep.append((data, rk))
        arr[i] = acr.Factor(f["level"], f["role"], f["plane"], int(bool(f.get("diag"))),
                            None if rk is None else rk.ctypes.data_as(ctypes.c_void_p),
                            data.ctypes.data_as(ctypes.c_void_p))
    blob = acr.FactorBlob(len(facs), arr)
    p = acr.Problem(nx, ny, nz, acr.POISSON_HARMONIC, None, 0.0, 0.0, None, 0.0, None)
    o = acr.default_options(eps=eps, leaf_size=leaf, precision=precision)
    out = ctypes.c_void_p(1234)
    st = acr.lib().acr_import_factors(ctypes.byref(p), ctypes.byref(o), ctypes.byref(blob), None, ctypes.byref(out))
    return st, out


def _expect_invalid(facs, text, **kw):
    st, out = _call(facs, **kw)
    assert st == 1 and out.value is None
    assert text.encode() in acr.lib().acr_last_error(), acr.lib().acr_last_error()


def test_invalid_blobs_are_refused_on_the_host(small):
    H, facs, leaves = small
    dinv = [i for i, f in enumerate(facs) if f["role"] == acr.FACTOR_DINV]
    _expect_invalid([f for i, f in enumerate(facs) if i != dinv[0]], "missing inverse")
    _expect_invalid(facs + [facs[0]], "duplicated")
    bad = dict(facs[0], level=9)
    _expect_invalid([bad] + facs[1:], "level out of range")
    k = next(i for i, f in enumerate(facs) if f["role"] == acr.FACTOR_A)
    _expect_invalid(facs + [dict(facs[k], level=len(H.levels), plane=H.top[0])], "top inverse only")
    j = next(i for i, f in enumerate(facs) if not f["diag"])
    rk = facs[j]["ranks"].copy()
    lr = int(np.flatnonzero(leaves[:, 5] == 1)[0])
    rk[lr] = min(leaves[lr, 2], leaves[lr, 3]) + 1
    _expect_invalid(facs[:j] + [dict(facs[j], ranks=rk)] + facs[j + 1:], "rank out of range")
    _expect_invalid([dict(facs[dinv[0]], plane=1)] + facs, "not eliminated")
    _expect_invalid(facs, "FP64 and FP32", precision=acr.MIXED_BF16, eps=1e-2)


def test_valid_blob_reaches_the_device_check(small):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    H, facs, leaves = small
    st, out = _call(facs)
    assert st == 7 and out.value is None
