"""BF16 stored factors (ACR_MIXED_BF16, eps >= 1e-2) through the C ABI.

The setup is the FP32 one; its stored factors are then rounded to BF16
(nearest even) and the apply streams them.  Checks:
  * the factor bytes are exactly half of the FP32 setup's (same ranks: the
    two setups run the same arithmetic);
  * apply and apply_T within 10 eps of the oracle's FP64 H-matrix cyclic
    reduction at the same eps (the apply tolerance of the parity tests), and apply within
    the BF16 rounding of the FP32 apply;
  * the exact-transpose dot test (the same BF16 values serve both maps);
  * the Krylov solution within 1e-8 of a sparse direct solve.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import assembly, hacr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1712_08872_amd as acr  # noqa: E402

CASES = {
    # name: (kind, nx, ny, nz, eps, leaf)
    "poisson15_e2": ("poisson", 15, 15, 15, 1e-2, 32),
    "convdiff_ragged_e2": ("convdiff", 14, 11, 9, 3e-2, 16),
}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


@pytest.mark.parametrize("name", list(CASES))
def test_bf16_factors(name):
    kind, nx, ny, nz, eps, leaf = CASES[name]
    print(f"\n[case {name}] {kind} {nx}x{ny}x{nz} eps={eps} leaf={leaf}", flush=True)
    kap = np.exp(synth.gaussian_field_exp((nz + 2, ny + 2, nx + 2), 7))
    if kind == "poisson":
        S = assembly.stencil7(kind, nx, ny, nz, kappa=kap)
        kw = dict(kappa=_dev(kap))
        k = acr.POISSON_HARMONIC
    else:
        S = assembly.stencil7(kind, nx, ny, nz, kappa=kap, beta_amp=40.0, beta_phase=0.3)
        kw = dict(kappa=_dev(kap), beta_amp=40.0, beta_phase=0.3)
        k = acr.CONVDIFF_UPWIND
    N = nx * ny * nz
    f = np.random.default_rng(8).uniform(-1, 1, N)
    fd = _dev(f)
    h32 = acr.acr_setup(nx, ny, nz, k, eps=eps, leaf_size=leaf, precision=acr.MIXED_FP32, **kw)
    h16 = acr.acr_setup(nx, ny, nz, k, eps=eps, leaf_size=leaf, precision=acr.MIXED_BF16, **kw)
    s32, s16 = acr.acr_stats(h32), acr.acr_stats(h16)
    assert s16["precision"] == acr.MIXED_BF16
    assert s16["max_rank"] == s32["max_rank"]
    assert 2 * s16["bytes_factors"] == s32["bytes_factors"]
    assert s16["bytes_per_apply"] < s32["bytes_per_apply"]

    H = hacr.HACR(S, nx, ny, nz, eps=eps, eta=2.0, leaf=leaf)
    z16 = acr.acr_apply(h16, fd).cpu().numpy()
    zt16 = acr.acr_apply_T(h16, fd).cpu().numpy()
    z32 = acr.acr_apply(h32, fd).cpu().numpy()
    for mine, ref in ((z16, H.apply(f)), (zt16, H.apply_T(f))):
        err = np.linalg.norm(mine - ref) / np.linalg.norm(ref)
        print(f"  BF16 vs oracle {err:.2e}", flush=True)
        assert err <= 10 * eps
    # per-entry rounding 2^-9 of the stored factors, through a few levels
    d = np.linalg.norm(z16 - z32) / np.linalg.norm(z32)
    print(f"  BF16 vs FP32 apply {d:.2e}", flush=True)
    assert 0 < d <= 2e-2

    rng = np.random.default_rng(9)
    r, s = _dev(rng.uniform(-1, 1, N)), _dev(rng.uniform(-1, 1, N))
    a = float(torch.dot(acr.acr_apply(h16, r), s))
    b = float(torch.dot(r, acr.acr_apply_T(h16, s)))
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))

    method = acr.CG if kind == "poisson" else acr.GMRES
    x, info = acr.krylov_solve(h16, fd, method=method, restart=30, rtol=1e-12, maxit=400)
    assert info["status"] == 0, info
    xs = spla.spsolve(assembly.to_sparse(S, nx, ny, nz).tocsc(), f)
    assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-8 * np.linalg.norm(xs)
    h16.close()
    h32.close()
