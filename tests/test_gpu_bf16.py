"""BF16 matrix-core products in the setup (ACR_MIXED_BF16, eps >= 1e-2)
through the C ABI: the setup of ACR_MIXED_FP32 with the operands of its
piece products rounded to BF16 and accumulated in FP32; FP32 factors.
Checks:
  * apply and apply_T within 10 eps of the oracle's FP64 H-matrix cyclic
    reduction at the same eps (the apply tolerance of the parity tests);
  * the application differs from the FP32-product setup's (the BF16 path
    ran) by less than 10 eps;
  * the exact-transpose dot test;
  * the Krylov solution within 1e-8 of a sparse direct solve;
  * at full size (127^3, six-decade sub-cube kappa, eps 1e-2) CG converges
    to 1e-8 with the residual recomputed by the oracle's operator.
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
    assert s16["precision"] == acr.MIXED_BF16 and s16["rank_overflow"] == 0
    assert abs(s16["max_rank_all"] - s32["max_rank_all"]) <= 2

    H = hacr.HACR(S, nx, ny, nz, eps=eps, eta=2.0, leaf=leaf)
    z16 = acr.acr_apply(h16, fd).cpu().numpy()
    zt16 = acr.acr_apply_T(h16, fd).cpu().numpy()
    z32 = acr.acr_apply(h32, fd).cpu().numpy()
    for mine, ref in ((z16, H.apply(f)), (zt16, H.apply_T(f))):
        err = np.linalg.norm(mine - ref) / np.linalg.norm(ref)
        print(f"  BF16 vs oracle {err:.2e}", flush=True)
        assert err <= 10 * eps
    # BF16 rounding (2^-9) of the product operands: a change below the truncation accuracy
    d = np.linalg.norm(z16 - z32) / np.linalg.norm(z32)
    print(f"  BF16-product vs FP32-product apply {d:.2e}", flush=True)
    assert 0 < d <= 10 * eps

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


def test_bf16_products_127_full_size():
    """127^3 sub-cube Poisson (six decades of contrast) at eps 1e-2: setup
    with BF16 and with FP32 piece products, CG to 1e-8 with the oracle's
    residual."""
    n, eps = 127, 1e-2
    inp = synth.config_inputs("poisson127")
    S = assembly.stencil7("poisson", n, n, n, kappa=inp["kappa"])
    f = inp["f"]
    times = {}
    for name, prec in (("fp32", acr.MIXED_FP32), ("bf16", acr.MIXED_BF16)):
        h = acr.acr_setup(n, n, n, acr.POISSON_HARMONIC, kappa=_dev(inp["kappa"]), eps=eps, precision=prec)
        x, info = acr.krylov_solve(h, _dev(f), method=acr.CG, rtol=1e-8, maxit=300)
        st = acr.acr_stats(h)
        times[name] = st["setup_seconds"]
        r = f - assembly.apply_stencil(S, x.cpu().numpy(), n, n, n)
        rel = float(np.linalg.norm(r) / np.linalg.norm(f))
        print(f"  127^3 eps 1e-2 {name} products: setup {st['setup_seconds']:.2f} s, CG {info['iters']} "
              f"iterations, oracle residual {rel:.1e}", flush=True)
        assert info["status"] == 0 and rel <= 1e-8
        h.close()
        torch.cuda.empty_cache()
