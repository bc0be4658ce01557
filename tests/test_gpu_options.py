"""Rank capacity semantics through the C ABI.

max_rank = 0: the capacity starts at 6 + 6 log10(1/eps) and is grown (the
setup redone) when a truncation needs more; the factors then carry their
eps-accurate ranks and no overflow is reported.
max_rank > 0: a fixed cap; stored ranks never exceed it, the overflow is
reported and not retried, and the (less accurate) preconditioner still
drives CG to the requested residual.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1712_08872_amd as acr  # noqa: E402


def _kappa(n, seed):
    return torch.from_numpy(synth.kappa_subcubes(n, seed).reshape(-1)).cuda()


def test_fixed_rank_cap_is_honoured_and_reported():
    n = 23
    kap = _kappa(n, 71)
    f = torch.from_numpy(synth.rhs_uniform(n ** 3, 72)).cuda()
    h_auto = acr.acr_setup(n, n, n, acr.POISSON_HARMONIC, kappa=kap, eps=1e-6, leaf_size=16)
    st_auto = acr.acr_stats(h_auto)
    assert st_auto["rank_overflow"] == 0
    assert st_auto["max_rank_all"] > 4
    cap = 4
    h_cap = acr.acr_setup(n, n, n, acr.POISSON_HARMONIC, kappa=kap, eps=1e-6, leaf_size=16, max_rank=cap)
    st_cap = acr.acr_stats(h_cap)
    assert st_cap["rank_overflow"] == 1 and st_cap["retries"] == 0
    assert max(st_cap["max_rank"][:st_cap["levels"]]) <= cap
    assert st_cap["bytes_factors"] < st_auto["bytes_factors"]
    x_auto, i_auto = acr.krylov_solve(h_auto, f, method=acr.CG, rtol=1e-10, maxit=300)
    x_cap, i_cap = acr.krylov_solve(h_cap, f, method=acr.CG, rtol=1e-10, maxit=300)
    assert i_auto["status"] == 0 and i_cap["status"] == 0
    assert i_cap["iters"] >= i_auto["iters"]
    rel = float(torch.linalg.norm(x_cap - x_auto) / torch.linalg.norm(x_auto))
    assert rel <= 1e-7
    h_auto.close()
    h_cap.close()


def test_peak_and_held_memory_reported():
    n = 15
    h = acr.acr_setup(n, n, n, acr.POISSON_HARMONIC, kappa=_kappa(n, 73), eps=1e-4,
                      precision=acr.MIXED_FP32)
    st = acr.acr_stats(h)
    # after setup the handle holds the packed factors (plus work vectors)
    assert st["bytes_factors"] <= st["bytes_allocated"] <= st["bytes_peak"]
    assert st["bytes_allocated"] < 4 * st["bytes_factors"] + (64 << 20)
    h.close()


def test_apply_schedule_autotuning_changes_no_result(monkeypatch):
    # the tuner picks the coefficient kernel's schedule per phase by timing;
    # the schedule moves leaves between wavefronts but not their arithmetic
    n = 23
    kap = _kappa(n, 74)
    f = torch.from_numpy(synth.rhs_uniform(n ** 3, 75)).cuda()
    monkeypatch.setenv("ACR_AUTOTUNE", "0")
    h0 = acr.acr_setup(n, n, n, acr.POISSON_HARMONIC, kappa=kap, eps=1e-5, leaf_size=16, precision=acr.MIXED_FP32)
    monkeypatch.setenv("ACR_AUTOTUNE", "1")
    h1 = acr.acr_setup(n, n, n, acr.POISSON_HARMONIC, kappa=kap, eps=1e-5, leaf_size=16, precision=acr.MIXED_FP32)
    assert torch.equal(acr.acr_apply(h0, f), acr.acr_apply(h1, f))
    assert torch.equal(acr.acr_apply_T(h0, f), acr.acr_apply_T(h1, f))
    h0.close()
    h1.close()
