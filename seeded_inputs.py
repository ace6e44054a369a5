"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the operator or the solvers.  It only draws
random numbers and shapes them into the storage layouts:

  * gauge links: (8, 3, 3, Vh) complex128, slot = 2*mu + parity of the link's
    start site, then row, column, half-lattice site index;
  * fields: (nrhs, 3, Vh) complex128 on one parity;
  * per-site SU(3) matrices (for gauge transformations): (3, 3, Vh) complex128.

Random SU(3) recipe: two complex Gaussian rows g1, g2 (real and imaginary parts
i.i.d. N(0,1)); r1 = g1/|g1|; r2 = normalised (g2 - <r1,g2> r1); r3 = conj(r1 x
r2).  This is the Haar measure on SU(3) and det = 1 up to rounding.  Every link
of the 8*Vh slots is drawn independently, in slot order, so no lattice geometry
is needed here.  Links on such "random" (infinite-coupling) configurations
stand in for the thermalised physics ensembles the paper measures on.
"""
from __future__ import annotations

import numpy as np


def rng(*seed):
    return np.random.default_rng([int(s) for s in seed])


def half_volume(dims) -> int:
    n = 1
    for d in dims:
        n *= int(d)
    return n // 2


def _random_su3(gen, count):
    """(count, 3, 3) Haar-random SU(3) matrices by Gram-Schmidt of Gaussian rows."""
    g = gen.standard_normal((count, 2, 3, 2))
    g = g[..., 0] + 1j * g[..., 1]
    r1 = g[:, 0] / np.linalg.norm(g[:, 0], axis=1, keepdims=True)
    proj = np.sum(np.conj(r1) * g[:, 1], axis=1, keepdims=True)
    v2 = g[:, 1] - proj * r1
    r2 = v2 / np.linalg.norm(v2, axis=1, keepdims=True)
    r3 = np.conj(np.cross(r1, r2))
    return np.stack([r1, r2, r3], axis=1)


def su3_links(dims, *seed):
    """Random SU(3) gauge field, (8, 3, 3, Vh) complex128."""
    vh = half_volume(dims)
    m = _random_su3(rng(*seed), 8 * vh)                # (8*Vh, 3, 3)
    return np.ascontiguousarray(m.reshape(8, vh, 3, 3).transpose(0, 2, 3, 1))


def su3_site_field(dims, *seed):
    """One random SU(3) matrix per site of one parity, (3, 3, Vh)."""
    vh = half_volume(dims)
    m = _random_su3(rng(*seed), vh)
    return np.ascontiguousarray(m.transpose(1, 2, 0))


def gaussian_field(dims, nrhs, *seed):
    """Complex Gaussian colour-vector field(s), (nrhs, 3, Vh) complex128."""
    vh = half_volume(dims)
    z = rng(*seed).standard_normal((nrhs, 3, vh, 2))
    return np.ascontiguousarray(z[..., 0] + 1j * z[..., 1])


def real_link_field(dims, *seed, low=-1.0, high=1.0):
    """Arbitrary real per-link factors, (8, Vh) float64 (uniform in [low, high))."""
    vh = half_volume(dims)
    return rng(*seed).uniform(low, high, size=(8, vh))


def sign_link_field(dims, *seed):
    """Random +-1 per-link factors, (8, Vh) float64."""
    vh = half_volume(dims)
    return np.where(rng(*seed).random((8, vh)) < 0.5, -1.0, 1.0)


def log_shifts(n, lo=1e-4, hi=10.0):
    """n shifts log-spaced in [lo, hi] (the rational-approximation pole set)."""
    if n == 1:
        return np.array([lo])
    return lo * (hi / lo) ** (np.arange(n) / (n - 1))


def traceless_hermitian_field(dims, *seed):
    """Random traceless Hermitian 3x3 matrix per link, (8, 3, 3, Vh) complex128:
    a Gaussian complex matrix A, (A + A^dag)/2, its trace / 3 removed (the
    momenta of the molecular dynamics, up to normalisation)."""
    vh = half_volume(dims)
    z = rng(*seed).standard_normal((8, 3, 3, vh, 2))
    a = z[..., 0] + 1j * z[..., 1]
    h = 0.5 * (a + np.conj(np.transpose(a, (0, 2, 1, 3))))
    tr = np.einsum("saan->sn", h)
    for i in range(3):
        h[:, i, i, :] -= tr / 3.0
    return np.ascontiguousarray(h)
