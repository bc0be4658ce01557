"""The seeded input recipes: the structure every workload is stated to
have (shapes, value ranges, contrast, piecewise constancy, covariance,
problem mix), and determinism in the seed.  Host only."""
import numpy as np

import synth
from synth import fields


def test_subcube_kappa_structure():
    """127^3 headline coefficient: 8^3 sub-cubes, values 10^U(-3,3)."""
    n = 127
    k = synth.kappa_subcubes(n, 11)
    assert k.shape == (n + 2,) * 3
    assert k.min() >= 1e-3 and k.max() <= 1e3
    assert k.max() / k.min() > 1e5  # six decades requested, more than five reached by the draw
    x = fields.node_coords(n)
    cube = np.minimum(np.floor(8 * x).astype(int), 7)
    for axis in range(3):  # constant inside a cube along every axis, different across most faces
        a = np.moveaxis(k, axis, 0)
        same = np.all(a[1:] == a[:-1], axis=(1, 2))
        inside = cube[1:] == cube[:-1]
        assert np.all(same[inside])
        assert not np.any(same[~inside])
    assert len(np.unique(k)) == 512
    np.testing.assert_array_equal(k, synth.kappa_subcubes(n, 11))
    assert not np.array_equal(k, synth.kappa_subcubes(n, 13))


def test_rhs_uniform():
    f = synth.rhs_uniform(127 ** 3, 12)
    assert f.shape == (127 ** 3,) and f.min() >= -1.0 and f.max() < 1.0
    assert abs(f.mean()) < 2e-3 and abs(f.std() - 1 / np.sqrt(3)) < 2e-3
    np.testing.assert_array_equal(f, synth.rhs_uniform(127 ** 3, 12))


def test_exponential_covariance_field():
    """Circulant embedding: unit variance and covariance exp(-r/lam) at lag
    lam along an axis, averaged over the grid and several seeds."""
    n, lam = 48, 0.2
    h = 1.0 / (n - 1)
    lag = int(round(lam / h))
    var, cov = [], []
    for seed in range(6):
        g, info = fields.gaussian_field_exp((n, n, n), seed, sigma=1.0, lam=lam, return_info=True)
        assert info["clipped_fraction"] < 1e-2
        var.append(np.mean(g * g))
        cov.append(np.mean(g[:, :, lag:] * g[:, :, :-lag]))
    assert abs(np.mean(var) - 1.0) < 0.15
    assert abs(np.mean(cov) - np.exp(-lag * h / lam)) < 0.1


def test_helmholtz_velocity_and_frequency():
    n = 31
    c = synth.helmholtz_velocity(n, 31)
    assert c.shape == (n + 2,) * 3
    assert abs(np.abs(c - 1.0).max() - 0.5) < 1e-12 and c.min() >= 0.5 and c.max() <= 1.5
    w = synth.helmholtz_omega(c, n, ppw=12.0)
    # 12 points per minimum wavelength: lambda_min = 2 pi c_min / omega = 12 h
    assert abs(2 * np.pi * c.min() / w - 12.0 / (n + 1)) < 1e-12


def test_batched_problem_mix():
    probs = synth.batched_problems()
    assert len(probs) == 48
    sizes = [p["n"] for p in probs]
    assert {31: sizes.count(31), 47: sizes.count(47), 63: sizes.count(63)} == {31: 16, 47: 21, 63: 11}
    for p in probs:
        assert p["kappa"].shape == (p["n"] + 2,) * 3 and p["f"].shape == (p["n"] ** 3,)
        assert 0.0 <= p["beta_phase"] < 2 * np.pi and p["beta_amp"] == 100.0
