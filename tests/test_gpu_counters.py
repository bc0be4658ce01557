"""The in-kernel counters of the H-arithmetic kernels (ACR_KERNEL_TIMING=1
at setup): launch counts, summed launch times, algorithmic flops by class
and algorithmic bytes.  They feed the benchmark's rooflines, so they must be
present, consistent with each other and the same on every run of the same
setup (the counts depend only on the operand sizes and the ranks, which a
deterministic setup reproduces bit for bit)."""
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1712_08872_amd as acr  # noqa: E402


def _setup(n, precision):
    kap = torch.from_numpy(synth.kappa_subcubes(n, 5).reshape(-1)).cuda()
    h = acr.acr_setup(n, n, n, acr.POISSON_HARMONIC, kappa=kap, eps=1e-4, leaf_size=16, precision=precision)
    st = acr.acr_stats(h)
    h.close()
    return st


@pytest.mark.parametrize("precision", [acr.FP64, acr.MIXED_FP32], ids=["fp64", "mixed"])
def test_kernel_counters(monkeypatch, precision):
    monkeypatch.setenv("ACR_KERNEL_TIMING", "1")
    a, b = _setup(23, precision), _setup(23, precision)
    for k in ("accum_launches", "dense_launches", "accum_seconds", "dense_seconds", "accum_flops", "dense_flops",
              "accum_bytes", "dense_bytes"):
        assert a[k] > 0, k
    for k in ("accum_launches", "dense_launches", "accum_flops", "dense_flops", "accum_bytes", "dense_bytes",
              "setup_flops"):
        assert a[k] == b[k], k
    cls = a["setup_flops_class"]
    assert sum(cls.values()) == pytest.approx(a["accum_flops"] + a["dense_flops"], rel=1e-12)
    assert a["setup_flops"] == pytest.approx(a["accum_flops"] + a["dense_flops"] + a["leaf_inverse_flops"],
                                             rel=1e-12)
    # every counted byte is an operand or a target entry at storage precision:
    # at least one 4- or 8-byte word per launch, and far below the factor bytes
    # times the number of products that read them
    esz = 8 if precision == acr.FP64 else 4
    assert a["accum_bytes"] % esz == 0 and a["dense_bytes"] % esz == 0
    assert a["dense_bytes"] >= a["dense_launches"] * esz


def test_counters_off_by_default(monkeypatch):
    monkeypatch.delenv("ACR_KERNEL_TIMING", raising=False)
    st = _setup(15, acr.MIXED_FP32)
    assert st["accum_launches"] > 0  # launches are always counted
    for k in ("accum_seconds", "dense_seconds", "accum_flops", "dense_flops", "accum_bytes", "dense_bytes"):
        assert st[k] == 0, k
