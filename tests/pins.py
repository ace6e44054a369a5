"""Checks that pin an implementation of the staggered hop to what the theory fixes.

Each check takes the hop as a callable ``dslash(dims, links, phases, out_parity,
vin)`` (and, where the standard phases matter, ``phases_fn(dims)``) and returns
an error figure; the tests assert it is below a tolerance.  The same checks run
on the two oracles and on deliberately broken copies (planted mistakes), which
must fail at least one of them.

Paper anchors (arXiv:1701.00426): Sec. 2.2 Eq. diracblock (D_oe^dag = -D_eo,
blocks connect only even and odd sites), Eq. lineqeo (m^2 - D_eo D_oe is
Hermitian positive definite), Sec. 4.1 (layouts), Sec. 2.3 (SU(3) links).
The closed forms (free-field plane waves, gauge covariance, pure-gauge
eigenvectors) are textbook properties of the staggered operator.
"""
import math

import numpy as np

import seeded_inputs as si
from oracle import oracle_np as on


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def anti_hermiticity(dslash, dims, seed=1, phases=None):
    """|<chi_e, D_eo psi_o> + <D_oe chi_e, psi_o>| / (|chi||psi|)."""
    links = si.su3_links(dims, seed, 0)
    if phases is None:
        phases = si.real_link_field(dims, seed, 1)
    chi = si.gaussian_field(dims, 1, seed, 2)[0]
    psi = si.gaussian_field(dims, 1, seed, 3)[0]
    lhs = np.vdot(chi, dslash(dims, links, phases, 0, psi))
    rhs = np.vdot(dslash(dims, links, phases, 1, chi), psi)
    return abs(lhs + rhs) / (np.linalg.norm(chi) * np.linalg.norm(psi))


def free_plane_waves(dslash, phases_fn, dims, mass=0.1, nmom=6, seed=4):
    """Unit links: D_oe on a plane wave equals i c e^{ipx} sum_mu eta_mu sin p_mu, and
    the normal operator has eigenvalue m^2 + sum sin^2 p.  Returns max abs error."""
    g = si.rng(seed)
    links = on.unit_links(dims)
    phases = phases_fn(dims)
    err = 0.0
    for _ in range(nmom):
        n = [int(g.integers(0, d)) for d in dims]
        p = on.momenta(dims, n)
        c = g.standard_normal(3) + 1j * g.standard_normal(3)
        pw = on.plane_wave(dims, 0, p, c)
        t = dslash(dims, links, phases, 1, pw)
        err = max(err, float(np.max(np.abs(t - on.free_doe_plane_wave(dims, p, c)))))
        a = mass * mass * pw - dslash(dims, links, phases, 0, t)
        err = max(err, float(np.max(np.abs(a - on.free_eigenvalue(mass, p) * pw))))
    return err


def dense_normal(dslash, dims, links, phases, mass, sigma=0.0):
    """Dense (3Vh x 3Vh) matrix of m^2 + sigma - D_eo D_oe, column by column."""
    vh = on.half_volume(dims)
    n = 3 * vh
    eye = np.eye(n, dtype=np.complex128).reshape(n, 3, vh)
    t = dslash(dims, links, phases, 1, eye)
    cols = (mass * mass + sigma) * eye - dslash(dims, links, phases, 0, t)
    return cols.reshape(n, n).T


def free_spectrum(dslash, phases_fn, dims, mass=0.1):
    """Full eigenvalue list of the free normal operator vs the closed form."""
    a = dense_normal(dslash, dims, on.unit_links(dims), phases_fn(dims), mass)
    ev = np.linalg.eigvalsh(0.5 * (a + a.conj().T))
    return float(np.max(np.abs(np.sort(ev) - on.free_spectrum(dims, mass))))


def gauge_covariance(dslash, dims, seed=5):
    """D[U^g](g psi) = g D[U] psi for both output parities."""
    links = si.su3_links(dims, seed, 0)
    phases = si.real_link_field(dims, seed, 1)
    ge = si.su3_site_field(dims, seed, 2)
    go = si.su3_site_field(dims, seed, 3)
    lg = on.gauge_transform_links(dims, links, ge, go)
    err = 0.0
    for out_parity, g_in, g_out in ((0, go, ge), (1, ge, go)):
        psi = si.gaussian_field(dims, 1, seed, 4 + out_parity)[0]
        lhs = dslash(dims, lg, phases, out_parity, on.site_matrices_apply(g_in, psi))
        rhs = on.site_matrices_apply(g_out, dslash(dims, links, phases, out_parity, psi))
        err = max(err, _rel(lhs, rhs))
    return err


def pure_gauge_eigen(dslash, phases_fn, dims, mass=0.1, seed=6, nmom=3):
    """U = g(x) g(x+mu)^dag: g * plane wave is an eigenvector with the free eigenvalue."""
    ge = si.su3_site_field(dims, seed, 0)
    go = si.su3_site_field(dims, seed, 1)
    links = on.pure_gauge_links(dims, ge, go)
    phases = phases_fn(dims)
    g = si.rng(seed, 2)
    err = 0.0
    for _ in range(nmom):
        p = on.momenta(dims, [int(g.integers(0, d)) for d in dims])
        c = g.standard_normal(3) + 1j * g.standard_normal(3)
        v = on.site_matrices_apply(ge, on.plane_wave(dims, 0, p, c))
        t = dslash(dims, links, phases, 1, v)
        a = mass * mass * v - dslash(dims, links, phases, 0, t)
        err = max(err, float(np.max(np.abs(a - on.free_eigenvalue(mass, p) * v))))
    return err


def dense_brute_force(dslash, dims, seed=7):
    """Hop vs the blocks of the dense full-lattice matrix built entry by entry."""
    links = si.su3_links(dims, seed, 0)
    phases = si.real_link_field(dims, seed, 1)
    dee, deo, doe, doo = on.dense_blocks(dims, links, phases)
    vh = on.half_volume(dims)
    err = float(max(np.max(np.abs(dee)), np.max(np.abs(doo))))  # no same-parity hops
    psi_o = si.gaussian_field(dims, 1, seed, 2)[0]
    psi_e = si.gaussian_field(dims, 1, seed, 3)[0]
    want_e = (deo @ psi_o.reshape(-1)).reshape(3, vh)
    want_o = (doe @ psi_e.reshape(-1)).reshape(3, vh)
    err = max(err, _rel(dslash(dims, links, phases, 0, psi_o), want_e))
    err = max(err, _rel(dslash(dims, links, phases, 1, psi_e), want_o))
    return err


def translation(dslash, phases_fn, dims, seed=8):
    """Shifting links and field by two sites along x0, x1 or x2 commutes with D."""
    links = si.su3_links(dims, seed, 0)
    phases = phases_fn(dims)
    err = 0.0
    for s in ((2, 0, 0, 0), (0, 2, 0, 0), (0, 0, 2, 0), (2, 2, 2, 0)):
        lt = on.translate_links(dims, links, s)
        for out_parity in (0, 1):
            psi = si.gaussian_field(dims, 1, seed, 1 + out_parity)[0]
            lhs = dslash(dims, lt, phases, out_parity,
                         on.translate_field(dims, psi, 1 - out_parity, s))
            rhs = on.translate_field(dims, dslash(dims, links, phases, out_parity, psi),
                                     out_parity, s)
            err = max(err, _rel(lhs, rhs))
    return err


def hermitian_positive(dslash, dims, mass=0.1, seed=9):
    """Dense normal operator: Hermitian, smallest eigenvalue >= m^2.  Returns
    (hermiticity error, lambda_min - m^2)."""
    links = si.su3_links(dims, seed, 0)
    a = dense_normal(dslash, dims, links, on.standard_phases(dims), mass)
    herm = float(np.max(np.abs(a - a.conj().T)) / np.max(np.abs(a)))
    lam = float(np.min(np.linalg.eigvalsh(0.5 * (a + a.conj().T))))
    return herm, lam - mass * mass


ALL_OPERATOR_PINS = ("anti_hermiticity", "free_plane_waves", "free_spectrum", "gauge_covariance",
                     "pure_gauge_eigen", "dense_brute_force", "translation")


def run_operator_pins(dslash, phases_fn):
    """Runs every operator pin on small lattices; returns {name: (error, tolerance)}."""
    out = {}
    out["anti_hermiticity"] = (max(anti_hermiticity(dslash, (4, 4, 4, 4)),
                                   anti_hermiticity(dslash, (2, 4, 6, 4), seed=2,
                                                    phases=phases_fn((2, 4, 6, 4)))), 1e-14)
    out["free_plane_waves"] = (max(free_plane_waves(dslash, phases_fn, (4, 6, 4, 8)),
                                   free_plane_waves(dslash, phases_fn, (2, 2, 2, 2), nmom=3)), 1e-13)
    out["free_spectrum"] = (free_spectrum(dslash, phases_fn, (2, 4, 2, 4)), 1e-12)
    out["gauge_covariance"] = (gauge_covariance(dslash, (4, 2, 4, 6)), 1e-13)
    out["pure_gauge_eigen"] = (pure_gauge_eigen(dslash, phases_fn, (4, 4, 2, 6)), 1e-12)
    out["dense_brute_force"] = (max(dense_brute_force(dslash, (2, 2, 2, 2)),
                                    dense_brute_force(dslash, (2, 4, 2, 4), seed=3)), 1e-13)
    out["translation"] = (translation(dslash, phases_fn, (4, 6, 4, 2)), 1e-14)
    return out


def rel_err(a, b):
    return _rel(a, b)


def vec_rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sqrt(x):
    return math.sqrt(x)
