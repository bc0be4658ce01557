"""krylov_solve_static, the allocation-free variant of krylov_solve (its
work vectors, dot partials and result slots in the library's fixed device
array), against krylov_solve on the same handle, through the C ABI: two
calls in a row, the second on a smaller problem, for CG and GMRES; the
results are identical (same kernels, same order, deterministic dots).  A
solve whose work vectors exceed the array is refused before any device
work."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1712_08872_amd as acr  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


def _problem(n, kind, seed):
    nx, ny, nz = n
    kap = np.exp(synth.gaussian_field_exp((nz + 2, ny + 2, nx + 2), seed))
    kw = dict(kind=acr.POISSON_HARMONIC if kind == "poisson" else acr.CONVDIFF_UPWIND, kappa=_dev(kap))
    if kind == "convdiff":
        kw.update(beta_amp=40.0, beta_phase=0.3)
    h = acr.acr_setup(nx, ny, nz, eps=1e-5, leaf_size=16, precision=acr.MIXED_FP32, **kw)
    b = _dev(synth.rhs_uniform(nx * ny * nz, seed + 1))
    return h, b


@pytest.mark.parametrize("kind,method", [("poisson", acr.CG), ("convdiff", acr.GMRES)])
def test_static_workspace_equals_krylov_solve(kind, method):
    for n, seed in (((24, 21, 17), 3), ((11, 9, 7), 5)):   # the second call on a smaller problem
        h, b = _problem(n, kind, seed)
        x_ref, info_ref = acr.krylov_solve(h, b, method=method, restart=20, rtol=1e-10, maxit=200)
        x, info = acr.krylov_solve(h, b, method=method, restart=20, rtol=1e-10, maxit=200, static_workspace=True)
        print(f"  {kind} {n}: {info['iters']} iterations, relres {info['relres_true']:.2e}")
        assert info["status"] == 0 and info["iters"] == info_ref["iters"]
        assert info["relres_true"] == info_ref["relres_true"]
        assert torch.equal(x, x_ref)
        # the transposed solve as well
        xt_ref, _ = acr.krylov_solve(h, b, method=method, restart=20, transpose=True, rtol=1e-10, maxit=200)
        xt, _ = acr.krylov_solve(h, b, method=method, restart=20, transpose=True, rtol=1e-10, maxit=200,
                                 static_workspace=True)
        assert torch.equal(xt, xt_ref)
        h.close()


def test_static_workspace_refuses_what_does_not_fit():
    # GMRES(60) needs 123 vectors: 53^3 = 148,877 unknowns do not fit the 128 MiB array
    n = 53
    h = acr.acr_setup(n, n, n, eps=1e-1, precision=acr.MIXED_FP32)
    b = _dev(synth.rhs_uniform(n ** 3, 1))
    with pytest.raises(acr.AcrError, match="fixed workspace"):
        acr.krylov_solve(h, b, method=acr.GMRES, restart=60, static_workspace=True)
    # CG needs 5: fits
    x, info = acr.krylov_solve(h, b, method=acr.CG, rtol=1e-8, static_workspace=True)
    assert info["status"] == 0
    h.close()
