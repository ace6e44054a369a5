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


# --------------------------------------------------------------------------
# Staples of the tree-level Symanzik gauge force (Sec. 2.1 action, Sec. 4.3
# staples: products of 3 and 5 links on C-shaped paths).  Each check takes
# ``staples_fn(dims, links, c0, c1) -> (8, 3, 3, Vh)``.  The closed forms are
# textbook properties of closed Wilson loops: unit and pure-gauge fields make
# every loop the identity, gauge transformations act on a staple at its two
# ends, and a loop sum is linear in each link it contains once.
# --------------------------------------------------------------------------


def _mat_rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _site_gauge(dims, seed):
    return si.su3_site_field(dims, seed, 0), si.su3_site_field(dims, seed, 1)


def _g_at(dims, g, y):
    """g(y), (3, 3, n), for sites y of any parity."""
    par = on.site_parity(y)
    h = on.half_index(dims, y)
    return np.where(par[None, None, :] == 0, g[0][:, :, h], g[1][:, :, h])


def staple_unit_links(staples_fn, dims, c0=1.3, c1=-0.35):
    """Unit links: every loop is 1, so Sigma = (6 c0 + 18 c1) I exactly."""
    s = staples_fn(dims, on.unit_links(dims), c0, c1)
    want = np.zeros_like(s)
    for a in range(3):
        want[:, a, a, :] = 6 * c0 + 18 * c1
    return _mat_rel(s, want)


def staple_pure_gauge(staples_fn, dims, c0=0.7, c1=0.45, seed=21):
    """U_mu(x) = g(x) g(x+mu)^dag: a path from x+mu to x multiplies to
    g(x+mu) g(x)^dag, so Sigma_mu(x) = (6 c0 + 18 c1) g(x+mu) g(x)^dag."""
    g = _site_gauge(dims, seed)
    s = staples_fn(dims, on.pure_gauge_links(dims, *g), c0, c1)
    want = np.empty_like(s)
    for parity in (0, 1):
        x = on.coords(dims, parity)
        for mu in range(4):
            gf = _g_at(dims, g, on.shifted(dims, x, mu, +1))
            want[2 * mu + parity] = (6 * c0 + 18 * c1) * np.einsum(
                "abn,cbn->acn", gf, np.conj(g[parity]))
    return _mat_rel(s, want)


def staple_gauge_covariance(staples_fn, dims, c0=1.1, c1=-0.6, seed=22):
    """Sigma[U^g]_mu(x) = g(x+mu) Sigma[U]_mu(x) g(x)^dag."""
    links = si.su3_links(dims, seed, 0)
    g = _site_gauge(dims, seed + 100)
    s = staples_fn(dims, links, c0, c1)
    sg = staples_fn(dims, on.gauge_transform_links(dims, links, *g), c0, c1)
    want = np.empty_like(s)
    for parity in (0, 1):
        x = on.coords(dims, parity)
        for mu in range(4):
            gf = _g_at(dims, g, on.shifted(dims, x, mu, +1))
            want[2 * mu + parity] = np.einsum("abn,bcn,dcn->adn", gf, s[2 * mu + parity],
                                              np.conj(g[parity]))
    return _mat_rel(sg, want)


def staple_linear_response(staples_fn, dims, c0, c1, seed=23, nlinks=3):
    """Each 1x1 and 1x2 loop holds a given link at most once (extents >= 3), so
    replacing U by U + E changes c0 P + c1 R by exactly Re Tr(E Sigma).  With E
    the 18 real basis directions this reads every entry of Sigma off the loop
    sums; compared at nlinks links per slot."""
    links = si.su3_links(dims, seed, 0)
    s = staples_fn(dims, links, c0, c1)
    base = on.weighted_loop_sum(dims, links, c0, c1)
    vh = on.half_volume(dims)
    pick = si.rng(seed, 1).integers(0, vh, size=(8, nlinks))
    err = 0.0
    for slot in range(8):
        for h in pick[slot]:
            got = np.empty((3, 3), dtype=np.complex128)
            for a in range(3):
                for b in range(3):
                    d = []
                    for e in (1.0, 1j):
                        pert = links.copy()
                        pert[slot, a, b, h] += e
                        d.append(on.weighted_loop_sum(dims, pert, c0, c1) - base)
                    got[b, a] = d[0] - 1j * d[1]
            err = max(err, _mat_rel(s[slot, :, :, h], got))
    return err


def staple_loop_identity(staples_fn, dims, c0=1.0, c1=1.0, seed=24):
    """sum over links of Re Tr(U Sigma) = 4 c0 P + 6 c1 R: a 1x1 loop has 4 links
    and a 1x2 loop 6, and each loop appears once in the staple of each of them."""
    links = si.su3_links(dims, seed, 0)
    s = staples_fn(dims, links, c0, c1)
    lhs = float(np.sum(np.real(np.einsum("sabn,sban->sn", links, s))))
    plaq, rect = on.loop_sums(dims, links)
    rhs = 4 * c0 * plaq + 6 * c1 * rect
    return abs(lhs - rhs) / max(abs(rhs), 1.0)


def staple_translation(staples_fn, dims, c0=0.9, c1=0.2, seed=25, shift=(2, 1, 0, 3)):
    """Staples of a translated field are the translated staples (any shift whose
    components sum to an even number keeps each parity in place)."""
    links = si.su3_links(dims, seed, 0)
    s = staples_fn(dims, links, c0, c1)
    st = staples_fn(dims, on.translate_links(dims, links, shift), c0, c1)
    return _mat_rel(st, on.translate_links(dims, s, shift))


ALL_STAPLE_PINS = ("unit_links", "pure_gauge", "gauge_covariance", "linear_response_plaq",
                   "linear_response_rect", "loop_identity", "translation")


def run_staple_pins(staples_fn, first_failure=False):
    """Runs the staple pins on small lattices, cheapest first; returns {name: (error,
    tolerance)}.  With first_failure it stops after the first pin that fails."""
    checks = [
        ("unit_links", lambda: staple_unit_links(staples_fn, (4, 4, 4, 4)), 1e-14),
        ("pure_gauge", lambda: staple_pure_gauge(staples_fn, (4, 6, 4, 4)), 1e-13),
        ("gauge_covariance", lambda: staple_gauge_covariance(staples_fn, (4, 4, 6, 4)), 1e-13),
        ("translation", lambda: staple_translation(staples_fn, (4, 6, 4, 4)), 1e-15),
        ("loop_identity", lambda: staple_loop_identity(staples_fn, (6, 4, 4, 8)), 1e-13),
        ("linear_response_plaq",
         lambda: staple_linear_response(staples_fn, (4, 4, 4, 6), 1.0, 0.0, nlinks=1), 1e-10),
        ("linear_response_rect",
         lambda: staple_linear_response(staples_fn, (4, 6, 4, 4), 0.0, 1.0, seed=26, nlinks=1),
         1e-10),
    ]
    out = {}
    for name, fn, tol in checks:
        err = fn()
        out[name] = (err, tol)
        if first_failure and not err <= tol:
            break
    return out


# --------------------------------------------------------------------------
# Fermion force of the rational action (Sec. 2.2 Eq. shlineq, Eq. lineqeo).
# Each check takes ``force_fn(dims, phases, coeffs, x_even, y_odd) -> (8,3,3,Vh)``.
# --------------------------------------------------------------------------


def _entries_from_response(f, links, slot, h):
    """G[slot, :, :, h] read off f(U + E) - f(U) = Re Tr(E G) over the 18 real
    directions E (central differences when f is not linear)."""
    got = np.empty((3, 3), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            d = []
            for e in (1.0, 1j):
                plus = links.copy()
                plus[slot, a, b, h] += e
                minus = links.copy()
                minus[slot, a, b, h] -= e
                d.append(0.5 * (f(plus) - f(minus)))
            got[b, a] = d[0] - 1j * d[1]
    return got


def force_linear_response(force_fn, dims, seed=50, nlinks=2):
    """For any X_k (even), Y_k (odd): f(U) = sum_k a_k 2 Re(X_k^dag D_eo(U) Y_k) is
    linear in each link, and G must be its exact derivative."""
    links = si.su3_links(dims, seed, 0)
    ph = si.real_link_field(dims, seed, 1)
    coeffs = [0.7, -0.3, 1.1]
    xs = si.gaussian_field(dims, 3, seed, 2)
    ys = si.gaussian_field(dims, 3, seed, 3)
    g = force_fn(dims, ph, coeffs, xs, ys)

    def f(lk):
        return sum(a * 2 * float(np.real(np.vdot(x, on.d_eo(dims, lk, ph, y))))
                   for a, x, y in zip(coeffs, xs, ys))

    pick = si.rng(seed, 4).integers(0, on.half_volume(dims), size=(8, nlinks))
    err = 0.0
    for slot in range(8):
        for h in pick[slot]:
            err = max(err, _mat_rel(g[slot, :, :, h], _entries_from_response(f, links, slot, h)))
    return err


def force_action_derivative(force_fn, dims=(2, 2, 2, 4), seed=51, eps=1e-6):
    """With X_k = (A + sigma_k)^{-1} phi and Y_k = D_oe X_k from dense solves, G is
    the derivative of S = Re phi^dag sum_k a_k (A + sigma_k)^{-1} phi: central
    differences of S (dense solves) in all 18 directions of one link per slot."""
    links = si.su3_links(dims, seed, 0)
    ph = on.standard_phases(dims)
    mass, shifts, coeffs = 0.3, [0.0, 0.05, 0.5], [0.4, 0.8, -0.2]
    phi = si.gaussian_field(dims, 1, seed, 1)[0]

    def solver(lk):
        _, deo, doe, _ = on.dense_blocks(dims, lk, ph)
        a = mass * mass * np.eye(deo.shape[0]) - deo @ doe
        return lambda sig, b: np.linalg.solve(a + sig * np.eye(a.shape[0]),
                                              b.reshape(-1)).reshape(3, -1)

    sol = solver(links)
    xs = np.array([sol(s, phi) for s in shifts])
    ys = np.array([on.d_oe(dims, links, ph, x) for x in xs])
    g = force_fn(dims, ph, coeffs, xs, ys)

    def f(lk):
        return on.rational_action(dims, lk, ph, mass, shifts, coeffs, phi, solve=solver(lk))

    err = 0.0
    for slot in range(8):
        h = slot % on.half_volume(dims)
        got = np.empty((3, 3), dtype=np.complex128)
        for a in range(3):
            for b in range(3):
                d = []
                for e in (1.0, 1j):
                    plus = links.copy()
                    plus[slot, a, b, h] += eps * e
                    minus = links.copy()
                    minus[slot, a, b, h] -= eps * e
                    d.append((f(plus) - f(minus)) / (2 * eps))
                got[b, a] = d[0] - 1j * d[1]
        err = max(err, _mat_rel(g[slot, :, :, h], got))
    return err


def force_gauge_covariance(force_fn, dims=(4, 2, 4, 6), seed=52):
    """X -> g X, Y -> g Y (fields at their sites): G_mu(z) -> g(z+mu) G_mu(z) g(z)^dag."""
    ph = si.real_link_field(dims, seed, 1)
    coeffs = [0.5, 1.5]
    xs = si.gaussian_field(dims, 2, seed, 2)
    ys = si.gaussian_field(dims, 2, seed, 3)
    g = _site_gauge(dims, seed + 100)
    f0 = force_fn(dims, ph, coeffs, xs, ys)
    f1 = force_fn(dims, ph, coeffs, on.site_matrices_apply(g[0], xs),
                  on.site_matrices_apply(g[1], ys))
    want = np.empty_like(f0)
    for parity in (0, 1):
        z = on.coords(dims, parity)
        for mu in range(4):
            gf = _g_at(dims, g, on.shifted(dims, z, mu, +1))
            want[2 * mu + parity] = np.einsum("abn,bcn,dcn->adn", gf, f0[2 * mu + parity],
                                              np.conj(g[parity]))
    return _mat_rel(f1, want)


ALL_FORCE_PINS = ("linear_response", "gauge_covariance", "action_derivative")


def run_force_pins(force_fn, first_failure=False):
    """{name: (error, tolerance)}, cheapest first."""
    checks = [
        ("gauge_covariance", lambda: force_gauge_covariance(force_fn), 1e-13),
        ("linear_response", lambda: max(force_linear_response(force_fn, (4, 4, 2, 6)),
                                        force_linear_response(force_fn, (2, 4, 2, 2), seed=53)),
         1e-12),
        ("action_derivative", lambda: force_action_derivative(force_fn), 1e-7),
    ]
    out = {}
    for name, fn, tol in checks:
        err = fn()
        out[name] = (err, tol)
        if first_failure and not err <= tol:
            break
    return out


# --------------------------------------------------------------------------
# Stout smearing (Sec. 2.1 stout-improved fermion action, Sec. 2.3 stout levels).
# Each check takes ``stout_fn(dims, links, rho) -> smeared links (8, 3, 3, Vh)``.
# --------------------------------------------------------------------------


def _as_mats(links):
    return np.transpose(links, (0, 3, 1, 2)).reshape(-1, 3, 3)


def stout_special_unitary(stout_fn, dims=(4, 4, 2, 6), rho=0.2, seed=71):
    """exp(iQ) with Q traceless Hermitian times an SU(3) link is in SU(3)."""
    m = _as_mats(stout_fn(dims, si.su3_links(dims, seed, 0), rho))
    unit = np.max(np.abs(m @ np.conj(np.transpose(m, (0, 2, 1))) - np.eye(3)))
    return max(unit, float(np.max(np.abs(np.linalg.det(m) - 1.0))))


def stout_trivial_fields(stout_fn, dims=(4, 2, 4, 4), seed=72):
    """rho = 0, unit links and pure-gauge links are left unchanged (on a pure-gauge
    field every 3-link path from x to x + mu is U_mu(x), so Omega = 6 rho I, Q = 0)."""
    links = si.su3_links(dims, seed, 0)
    e = _mat_rel(stout_fn(dims, links, 0.0), links)
    u = on.unit_links(dims)
    e = max(e, _mat_rel(stout_fn(dims, u, 0.3), u))
    pg = on.pure_gauge_links(dims, *_site_gauge(dims, seed + 1))
    return max(e, _mat_rel(stout_fn(dims, pg, 0.3), pg))


def stout_gauge_covariance(stout_fn, dims=(4, 4, 4, 2), rho=0.15, seed=73):
    """smear(U^g) = smear(U)^g."""
    links = si.su3_links(dims, seed, 0)
    g = _site_gauge(dims, seed + 100)
    a = stout_fn(dims, on.gauge_transform_links(dims, links, *g), rho)
    b = on.gauge_transform_links(dims, stout_fn(dims, links, rho), *g)
    return _mat_rel(a, b)


def stout_abelian_closed_form(stout_fn, dims=(4, 2, 4, 6), rho=0.35, seed=74):
    """Diagonal links diag(e^{i a}, e^{i b}, e^{-i(a+b)}): every product is diagonal,
    entry by entry a product of phases.  With omega = (C U^dag)_cc for colour c,
    Q_cc = Im(omega_c) - (1/3) sum_d Im(omega_d) and U'_cc = exp(i Q_cc) U_cc;
    the phases of the 3-link paths from x to x + mu are summed here site by site."""
    vh = on.half_volume(dims)
    ang = si.rng(seed, 0).uniform(-np.pi, np.pi, size=(8, 2, vh))
    ph = np.stack([ang[:, 0], ang[:, 1], -(ang[:, 0] + ang[:, 1])], axis=1)   # (8, 3, vh)
    links = np.zeros((8, 3, 3, vh), dtype=np.complex128)
    for c in range(3):
        links[:, c, c, :] = np.exp(1j * ph[:, c, :])
    got = stout_fn(dims, links, rho)
    want = np.zeros_like(links)

    def phase(d, y, c):
        return ph[2 * d + int(on.site_parity(y)[0]), c, int(on.half_index(dims, y)[0])]

    for parity in (0, 1):
        xs = on.coords(dims, parity)
        for h in range(vh):
            x = xs[:, h:h + 1]
            for mu in range(4):
                om = np.zeros(3, dtype=np.complex128)
                for c in range(3):
                    tot = 0.0j
                    xm = on.shifted(dims, x, mu, +1)
                    for nu in range(4):
                        if nu == mu:
                            continue
                        xn = on.shifted(dims, x, nu, +1)
                        xd = on.shifted(dims, x, nu, -1)
                        up = phase(nu, x, c) + phase(mu, xn, c) - phase(nu, xm, c)
                        xdm = on.shifted(dims, xd, mu, +1)
                        down = -phase(nu, xd, c) + phase(mu, xd, c) + phase(nu, xdm, c)
                        tot += np.exp(1j * up) + np.exp(1j * down)
                    om[c] = rho * tot * np.exp(-1j * phase(mu, x, c))
                q = np.imag(om) - np.mean(np.imag(om))
                for c in range(3):
                    want[2 * mu + parity, c, c, h] = np.exp(1j * (q[c] + phase(mu, x, c)))
    return _mat_rel(got, want)


def stout_q_from_forward_paths(stout_q_fn, dims=(4, 4, 2, 4), rho=0.25, seed=75):
    """Q built from the six 3-link paths from x to x + mu written as Wilson lines
    (independent of the staple sum): C = rho sum_nu [U_nu U_mu U_nu^dag paths]."""
    links = si.su3_links(dims, seed, 0)
    q = stout_q_fn(dims, links, rho)
    want = np.empty_like(q)
    for parity in (0, 1):
        x = on.coords(dims, parity)
        for mu in range(4):
            c = np.zeros((3, 3, x.shape[1]), dtype=np.complex128)
            for nu in range(4):
                if nu != mu:
                    c += on.path_product(dims, links, x, [(nu, 1), (mu, 1), (nu, -1)])
                    c += on.path_product(dims, links, x, [(nu, -1), (mu, 1), (nu, 1)])
            om = np.einsum("abn,cbn->acn", rho * c, np.conj(links[2 * mu + parity]))
            a = np.conj(np.transpose(om, (1, 0, 2))) - om
            qq = 0.5j * a
            tr = np.einsum("aan->n", a)
            for i in range(3):
                qq[i, i] -= (1j / 6.0) * tr
            want[2 * mu + parity] = qq
    return _mat_rel(q, want)


def run_stout_pins(stout_fn, first_failure=False):
    checks = [
        ("special_unitary", lambda: stout_special_unitary(stout_fn), 1e-13),
        ("trivial_fields", lambda: stout_trivial_fields(stout_fn), 1e-13),
        ("gauge_covariance", lambda: stout_gauge_covariance(stout_fn), 1e-13),
        ("abelian_closed_form", lambda: stout_abelian_closed_form(stout_fn), 1e-13),
    ]
    out = {}
    for name, fn, tol in checks:
        err = fn()
        out[name] = (err, tol)
        if first_failure and not err <= tol:
            break
    return out


def rel_err(a, b):
    return _rel(a, b)


def vec_rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sqrt(x):
    return math.sqrt(x)
