"""Pins of the oracle's site indexing (Sec. 4.1, Eq. lexicographic_eo) and of the
seeded generators.  CPU only."""
import itertools

import numpy as np
import pytest

import seeded_inputs as si
from oracle import oracle_np as on

DIMS = [(2, 2, 2, 2), (4, 4, 4, 4), (2, 4, 6, 4), (6, 2, 4, 8), (8, 4, 2, 6)]


@pytest.mark.parametrize("dims", DIMS)
def test_half_index_is_bijection_per_parity(dims):
    """Every site of a parity gets a distinct h in [0, Vh), and coords() inverts it."""
    vh = on.half_volume(dims)
    for parity in (0, 1):
        x = on.coords(dims, parity)
        assert np.all(on.site_parity(x) == parity)
        h = on.half_index(dims, x)
        assert np.array_equal(h, np.arange(vh))
        for mu in range(4):
            assert x[mu].min() >= 0 and x[mu].max() < dims[mu]


@pytest.mark.parametrize("dims", DIMS)
def test_paper_formula_for_even_sites(dims):
    """Brute-force walk over all sites: idxh = (int)(lex/2) for even sites,
    the two parities together cover every site exactly once."""
    seen = {0: set(), 1: set()}
    for x3, x2, x1, x0 in itertools.product(*(range(n) for n in dims[::-1])):
        lex = x0 + dims[0] * (x1 + dims[1] * (x2 + dims[2] * x3))
        par = (x0 + x1 + x2 + x3) % 2
        h = int(lex) // 2
        assert h not in seen[par]
        seen[par].add(h)
        xc = on.coords(dims, par)[:, h]
        assert tuple(xc) == (x0, x1, x2, x3)
    assert len(seen[0]) == len(seen[1]) == on.half_volume(dims)


@pytest.mark.parametrize("dims", DIMS)
def test_neighbours_flip_parity_and_invert(dims):
    for parity in (0, 1):
        x = on.coords(dims, parity)
        for mu in range(4):
            xf = on.shifted(dims, x, mu, +1)
            xb = on.shifted(dims, x, mu, -1)
            assert np.all(on.site_parity(xf) == 1 - parity)
            assert np.all(on.site_parity(xb) == 1 - parity)
            assert np.array_equal(on.shifted(dims, xf, mu, -1), x)
            assert np.array_equal(on.shifted(dims, xb, mu, +1), x)


def test_odd_dims_rejected():
    with pytest.raises(ValueError):
        on.check_dims((3, 4, 4, 4))
    with pytest.raises(ValueError):
        on.check_dims((0, 4, 4, 4))


def test_standard_phases_values():
    """eta_mu(x) = (-1)^(x0+..+x_{mu-1}); the x3 links leaving x3 = N3-1 carry -1."""
    dims = (4, 2, 6, 4)
    ph = on.standard_phases(dims)
    for parity in (0, 1):
        x = on.coords(dims, parity)
        for h in range(x.shape[1]):
            xs = x[:, h]
            for mu in range(4):
                want = (-1) ** int(sum(xs[:mu]))
                if mu == 3 and xs[3] == dims[3] - 1:
                    want = -want
                assert ph[2 * mu + parity, h] == want


def test_c_and_numpy_phases_agree(corc):
    for dims in DIMS:
        assert np.array_equal(corc.standard_phases(dims), on.standard_phases(dims))


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 4)])
def test_su3_generator(dims):
    u = si.su3_links(dims, 1, 2, 3)
    vh = on.half_volume(dims)
    assert u.shape == (8, 3, 3, vh)
    m = u.transpose(0, 3, 1, 2).reshape(-1, 3, 3)
    eye = np.eye(3)
    uu = np.einsum("nab,ncb->nac", m, m.conj())
    assert np.max(np.abs(uu - eye)) < 1e-14
    assert np.max(np.abs(np.linalg.det(m) - 1.0)) < 1e-14
    # seeded: same seed same field, different seed different field
    assert np.array_equal(u, si.su3_links(dims, 1, 2, 3))
    assert not np.allclose(u, si.su3_links(dims, 1, 2, 4))


def test_su3_haar_moments():
    """Haar SU(3): E|U_ab|^2 = 1/3, E U_ab = 0, E tr U = 0."""
    m = si.su3_links((8, 8, 8, 8), 7).transpose(0, 3, 1, 2).reshape(-1, 3, 3)
    assert abs(np.mean(np.abs(m) ** 2) - 1 / 3) < 2e-3
    assert np.abs(np.mean(m)) < 5e-3
    assert np.abs(np.mean(np.trace(m, axis1=1, axis2=2))) < 1e-2


def test_gaussian_field():
    v = si.gaussian_field((4, 4, 4, 4), 2, 9, 9)
    assert v.shape == (2, 3, 128) and v.dtype == np.complex128
    assert np.array_equal(v, si.gaussian_field((4, 4, 4, 4), 2, 9, 9))


def test_log_shifts():
    s = si.log_shifts(16)
    assert abs(s[0] - 1e-4) < 1e-18 and abs(s[-1] - 10.0) < 1e-12
    assert np.allclose(np.diff(np.log10(s)), 5 / 15)
