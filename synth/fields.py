"""Seeded coefficient fields and right-hand sides (numpy PCG64 only).

Field recipes (the paper's DUNE fields and PetIGA meshes are not
available; these synthetic stand-ins keep the paper's shapes, contrast
and structure):

* ``gaussian_field_exp``: zero-mean Gaussian field with exponential
  covariance ``sigma^2 exp(-|r|/lam)`` (the covariance family of the
  variable-Poisson section), sampled exactly on the node grid by
  circulant embedding on a periodic grid of twice the size; negative
  embedding eigenvalues are clipped to zero and their mass reported.
* ``kappa_subcubes``: piecewise-constant coefficient on 8^3 sub-cubes with
  values ``10**U(-3,3)`` (six orders of magnitude of contrast, the hardest
  contrast of the Poisson comparison table).
* ``helmholtz_velocity``: ``1 + 0.5 g`` with ``g`` white noise smoothed
  by a Gaussian kernel of standard deviation 0.1 and scaled to
  ``max|g| = 1``.
"""
import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def node_coords(n):
    """Coordinates of the ``n+2`` nodes of one axis, boundary included."""
    return np.arange(n + 2, dtype=np.float64) / (n + 1)


def gaussian_field_exp(shape, seed, sigma=1.0, lam=0.2, return_info=False):
    """Exponential-covariance Gaussian field on a node grid of ``shape``
    (z, y, x) with spacing ``1/(shape-1)`` per axis, by circulant embedding."""
    shape = tuple(int(s) for s in shape)
    h = [1.0 / (s - 1) for s in shape]
    m = [2 * s for s in shape]
    axes = []
    for mi, hi in zip(m, h):
        k = np.arange(mi)
        k = np.minimum(k, mi - k)
        axes.append(k * hi)
    rz, ry, rx = np.meshgrid(*axes, indexing="ij")
    r = np.sqrt(rz ** 2 + ry ** 2 + rx ** 2)
    cov = sigma ** 2 * np.exp(-r / lam)
    lam_k = np.fft.fftn(cov).real
    neg = float(-lam_k[lam_k < 0].sum() / np.abs(lam_k).sum())
    lam_k = np.maximum(lam_k, 0.0)
    g = _rng(seed)
    xi = g.standard_normal(m) + 1j * g.standard_normal(m)
    field = np.fft.fftn(np.sqrt(lam_k / np.prod(m)) * xi)
    out = field.real[: shape[0], : shape[1], : shape[2]].copy()
    if return_info:
        return out, {"clipped_fraction": neg}
    return out


def kappa_lognormal(n, seed, sigma=1.0, lam=0.2, nz=None, ny=None):
    """``kappa = exp(g)`` on the node grid, ``g`` exponential-covariance field."""
    nz = n if nz is None else nz
    ny = n if ny is None else ny
    g = gaussian_field_exp((nz + 2, ny + 2, n + 2), seed, sigma, lam)
    return np.exp(g)


def kappa_subcubes(n, seed, cubes=8, lo=-3.0, hi=3.0):
    """Piecewise-constant kappa on ``cubes^3`` sub-cubes; cube index of a
    node is ``min(floor(cubes*x), cubes-1)`` per axis; values
    ``10**U(lo,hi)`` drawn in cube order, x fastest."""
    vals = 10.0 ** _rng(seed).uniform(lo, hi, size=cubes ** 3)
    x = node_coords(n)
    c = np.minimum(np.floor(cubes * x).astype(np.int64), cubes - 1)
    cz, cy, cx = np.meshgrid(c, c, c, indexing="ij")
    return vals[cx + cubes * (cy + cubes * cz)].reshape(n + 2, n + 2, n + 2)


def rhs_uniform(N, seed):
    """Right-hand side ``f ~ U(-1, 1)`` of length ``N``."""
    return _rng(seed).uniform(-1.0, 1.0, size=int(N))


def cd_phase(seed):
    """Random phase ``phi ~ U[0, 2 pi)`` of the convection field."""
    return float(_rng(seed).uniform(0.0, 2.0 * np.pi))


def helmholtz_velocity(n, seed, std=0.1):
    """``c = 1 + 0.5 g`` on the node grid; ``g`` smoothed white noise,
    ``max|g| = 1``; so ``c`` lies in ``[0.5, 1.5]``."""
    w = _rng(seed).standard_normal((n + 2,) * 3)
    h = 1.0 / (n + 1)
    m = 2 * (n + 2)
    k = np.fft.fftfreq(m, d=h) * 2.0 * np.pi
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    ker = np.exp(-0.5 * std ** 2 * (kx ** 2 + ky ** 2 + kz ** 2))
    pad = np.zeros((m,) * 3)
    pad[: n + 2, : n + 2, : n + 2] = w
    sm = np.fft.ifftn(np.fft.fftn(pad) * ker).real[: n + 2, : n + 2, : n + 2]
    sm /= np.abs(sm).max()
    return 1.0 + 0.5 * sm


def helmholtz_omega(c, n, ppw=12.0):
    """Angular frequency giving ``ppw`` points per minimum wavelength:
    ``lambda_min = c_min / f = ppw h``, ``omega = 2 pi f``."""
    h = 1.0 / (n + 1)
    return 2.0 * np.pi * float(c.min()) / (ppw * h)


def point_source(n):
    """Unit point source at the centre node, ``delta / h^3``."""
    h = 1.0 / (n + 1)
    f = np.zeros((n, n, n))
    m = n // 2
    f[m, m, m] = 1.0 / h ** 3
    return f.reshape(-1)


def batched_problems(count=48, sizes=(31, 47, 63)):
    """Independent convection-diffusion problems of uneven size: problem i
    draws n from ``sizes`` and its phase, ``kappa = exp(g)`` (lognormal
    field) and ``f ~ U(-1, 1)`` from seed ``100 + i``; ``beta_amp = 100``.
    Returns a list of dicts (n, kappa, beta_amp, beta_phase, f)."""
    out = []
    for i in range(count):
        rng = _rng(100 + i)
        n = int(sizes[int(rng.integers(len(sizes)))])
        out.append(dict(n=n, kappa=np.exp(gaussian_field_exp((n + 2,) * 3, 100 + i)),
                        beta_amp=100.0, beta_phase=float(rng.uniform(0.0, 2.0 * np.pi)),
                        f=rhs_uniform(n ** 3, 100 + i)))
    return out


def config_inputs(name, seed_offset=0):
    """Inputs of the named workload as a dict of numpy arrays/scalars.

    ``poisson31``: lognormal kappa, n=31, eps 1e-6.
    ``poisson127``: 8^3 sub-cube kappa with 6 decades, n=127, eps 1e-4.
    ``cd127``: upwind convection-diffusion, n=127.
    ``helmholtz127``: indefinite Helmholtz, n=127.
    ``adjoint63``: lognormal kappa, n=63, for the adjoint gradient.
    """
    s = seed_offset
    if name == "poisson31":
        n = 31
        return dict(n=n, kind="poisson", kappa=kappa_lognormal(n, 1 + s),
                    f=rhs_uniform(n ** 3, 2 + s), eps=1e-6, eta=2.0, leaf=32)
    if name == "poisson127":
        n = 127
        return dict(n=n, kind="poisson", kappa=kappa_subcubes(n, 11 + 2 * s),
                    f=rhs_uniform(n ** 3, 12 + 2 * s), eps=1e-4, eta=2.0, leaf=32)
    if name == "cd127":
        n = 127
        return dict(n=n, kind="convdiff", kappa=np.ones((n + 2,) * 3),
                    beta_amp=100.0, beta_phase=cd_phase(21 + s),
                    f=rhs_uniform(n ** 3, 22 + s), eps=1e-4, eta=2.0, leaf=32)
    if name == "helmholtz127":
        n = 127
        c = helmholtz_velocity(n, 31 + s)
        return dict(n=n, kind="helmholtz", c=c, omega=helmholtz_omega(c, n),
                    f=point_source(n), eps=1e-5, eta=1.0, leaf=32)
    if name == "adjoint63":
        n = 63
        return dict(n=n, kind="poisson", g=gaussian_field_exp((n + 2,) * 3, 41 + s),
                    g2=gaussian_field_exp((n + 2,) * 3, 42 + s),
                    xi=_rng(43 + s).standard_normal(n ** 3),
                    eps=1e-4, eta=2.0, leaf=32)
    raise KeyError(name)
