"""Pins of the two FP64 oracles (NumPy and C) against what the theory fixes.

CPU only.  The oracle is trusted by the GPU parity tests only because of these.
"""
import math

import numpy as np
import pytest

import seeded_inputs as si
from oracle import oracle_np as on

import pins


@pytest.fixture(scope="module")
def impls(corc):
    return {"numpy": (on.dslash, on.standard_phases),
            "c": (corc.dslash, corc.standard_phases)}


@pytest.mark.parametrize("which", ["numpy", "c"])
def test_operator_pins(impls, which):
    dslash, phases_fn = impls[which]
    res = pins.run_operator_pins(dslash, phases_fn)
    for name, (err, tol) in res.items():
        assert err <= tol, f"{which}: pin {name} error {err:.3e} > {tol:.1e}"


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (2, 4, 6, 4)])
def test_normal_operator_hermitian_positive(dims):
    herm, gap = pins.hermitian_positive(on.dslash, dims, mass=0.1)
    assert herm < 1e-14
    assert gap >= -1e-12


def test_free_spectrum_full_4444():
    """All 384 eigenvalues of the free 4^4 normal operator match the closed form."""
    err = pins.free_spectrum(on.dslash, on.standard_phases, (4, 4, 4, 4), mass=0.05)
    assert err < 1e-12


def test_antiperiodic_boundary_matters():
    """Periodic-in-time momenta are not eigenvectors: the boundary sign is present."""
    dims = (4, 4, 4, 4)
    p = [0.0, 0.0, 0.0, 2 * math.pi / 4]
    pw = on.plane_wave(dims, 0, p, [1, 0, 0])
    a = on.apply_normal(dims, on.unit_links(dims), on.standard_phases(dims), 0.1, pw)
    assert np.max(np.abs(a - on.free_eigenvalue(0.1, p) * pw)) > 0.1


def test_n_version_dslash(corc):
    """NumPy and C oracles agree on random inputs, several shapes, multi-RHS."""
    for dims, seed in (((4, 4, 4, 4), 1), ((2, 4, 6, 8), 2), ((6, 2, 4, 4), 3)):
        links = si.su3_links(dims, seed, 0)
        phases = si.real_link_field(dims, seed, 1)
        v = si.gaussian_field(dims, 2, seed, 2)
        for par in (0, 1):
            a = on.dslash(dims, links, phases, par, v)
            b = corc.dslash(dims, links, phases, par, v)
            assert pins.rel_err(b, a) < 1e-14
        an = on.apply_normal(dims, links, phases, 0.3, v[0], sigma=0.2)
        ac = corc.apply_normal(dims, links, phases, 0.3, v[0], sigma=0.2)
        assert pins.rel_err(ac, an) < 1e-14


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 4, 6, 4)])
def test_cg_vs_dense_solve(corc, dims):
    links = si.su3_links(dims, 11, 0)
    phases = on.standard_phases(dims)
    b = si.gaussian_field(dims, 1, 11, 1)[0]
    mass = 0.2
    a = pins.dense_normal(on.dslash, dims, links, phases, mass)
    x_dense = np.linalg.solve(a, b.reshape(-1)).reshape(b.shape)
    x_np, it_np, res_np = on.cg(dims, links, phases, mass, b, tol=1e-13)
    x_c, it_c, res_c, st = corc.cg(dims, links, phases, mass, b, tol=1e-13)
    assert st == 0 and res_c < 1e-12 and res_np < 1e-12
    assert pins.vec_rel(x_np, x_dense) < 1e-11
    assert pins.vec_rel(x_c, x_dense) < 1e-11
    # CG on n = 3 Vh unknowns terminates in at most n steps in exact arithmetic
    assert it_c <= 3 * on.half_volume(dims) + 5


def test_cg_pure_gauge_exact(corc):
    """b = g * plane wave is an exact eigenvector: CG returns b / lambda."""
    dims = (4, 4, 4, 6)
    ge = si.su3_site_field(dims, 21, 0)
    go = si.su3_site_field(dims, 21, 1)
    links = on.pure_gauge_links(dims, ge, go)
    phases = on.standard_phases(dims)
    p = on.momenta(dims, (1, 2, 0, 1))
    b = on.site_matrices_apply(ge, on.plane_wave(dims, 0, p, [1.0, 0.5j, -0.25]))
    lam = on.free_eigenvalue(0.1, p)
    x, it, res, st = corc.cg(dims, links, phases, 0.1, b, tol=1e-12)
    assert st == 0
    assert pins.vec_rel(x, b / lam) < 1e-12
    assert it <= 2  # an eigenvector is solved in one step


def test_cg_warm_restart_and_not_converged(corc):
    dims = (4, 4, 4, 4)
    links = si.su3_links(dims, 31, 0)
    phases = on.standard_phases(dims)
    b = si.gaussian_field(dims, 1, 31, 1)[0]
    x1, it1, _, st1 = corc.cg(dims, links, phases, 0.1, b, tol=1e-10, max_iter=10)
    assert st1 == 1 and it1 == 10
    x2, it2, res2, st2 = corc.cg(dims, links, phases, 0.1, b, tol=1e-10, x0=x1)
    assert st2 == 0 and res2 < 1e-9


def test_cg_iteration_count_random_links(corc):
    """Random links at m = 0.1 on 8^4: about 300 iterations to 1e-10 (recorded, unpinned
    by theory; a sanity range only)."""
    dims = (8, 8, 8, 8)
    links = si.su3_links(dims, 1701, 0, 0)
    phases = on.standard_phases(dims)
    b = si.gaussian_field(dims, 1, 426, 0, 0, 0)[0]
    x, it, res, st = corc.cg(dims, links, phases, 0.1, b, tol=1e-10)
    assert st == 0 and res < 2e-10
    assert 150 < it < 600


def test_mscg_vs_independent_cg(corc):
    """Each multi-shift solution matches an independent CG on its own shifted system."""
    dims = (4, 4, 4, 4)
    links = si.su3_links(dims, 41, 0)
    phases = on.standard_phases(dims)
    b = si.gaussian_field(dims, 1, 41, 1)[0]
    shifts = si.log_shifts(6, 1e-4, 10.0)
    mass = 0.05
    xs, its, res, st = corc.mscg(dims, links, phases, mass, shifts, b, tol=1e-11)
    assert st == 0
    for k, s in enumerate(shifts):
        assert res[k] < 1e-10
        xk, _, rk, stk = corc.cg(dims, links, phases, mass, b, tol=1e-12, sigma=s)
        assert stk == 0
        assert pins.vec_rel(xs[k], xk) < 1e-9
        # and against the NumPy oracle's residual on the returned solution
        assert on.true_relative_residual(dims, links, phases, mass, b, xs[k], sigma=s) < 1e-10
    # larger shifts converge earlier
    assert its[-1] < its[0]


def test_mscg_single_shift_is_cg(corc):
    """With one shift the multi-shift recurrences reduce to plain CG (zeta = 1)."""
    dims = (4, 4, 2, 4)
    links = si.su3_links(dims, 51, 0)
    phases = on.standard_phases(dims)
    b = si.gaussian_field(dims, 1, 51, 1)[0]
    xs, its, res, st = corc.mscg(dims, links, phases, 0.1, [0.3], b, tol=1e-10)
    x, it, r, st2 = corc.cg(dims, links, phases, 0.1, b, tol=1e-10, sigma=0.3)
    assert its[0] == it
    assert pins.vec_rel(xs[0], x) < 1e-13


def test_mscg_shift_order_independent(corc):
    dims = (4, 2, 4, 4)
    links = si.su3_links(dims, 61, 0)
    phases = on.standard_phases(dims)
    b = si.gaussian_field(dims, 1, 61, 1)[0]
    sh = np.array([0.5, 0.01, 2.0])
    x1, _, r1, _ = corc.mscg(dims, links, phases, 0.1, sh, b, tol=1e-11)
    perm = [2, 0, 1]
    x2, _, r2, _ = corc.mscg(dims, links, phases, 0.1, sh[perm], b, tol=1e-11)
    for j, k in enumerate(perm):
        assert pins.vec_rel(x2[j], x1[k]) < 1e-13


try:
    from hypothesis import given, settings
    from hypothesis import strategies as hs
except ImportError:  # pragma: no cover
    given = None

if given is not None:
    _even = hs.sampled_from([2, 4, 6])

    @settings(max_examples=25, deadline=None)
    @given(n0=_even, n1=_even, n2=_even, n3=_even, seed=hs.integers(0, 2**31 - 1))
    def test_random_shapes_anti_hermitian_and_n_version(corc, n0, n1, n2, n3, seed):
        """Any even shape, any seed: anti-Hermiticity, gauge covariance on the NumPy
        oracle, and NumPy == C oracle."""
        dims = (n0, n1, n2, n3)
        assert pins.anti_hermiticity(on.dslash, dims, seed=seed % 1000,
                                     phases=on.standard_phases(dims)) < 1e-14
        links = si.su3_links(dims, seed, 1)
        phases = si.real_link_field(dims, seed, 2)
        v = si.gaussian_field(dims, 1, seed, 3)[0]
        for par in (0, 1):
            assert pins.rel_err(corc.dslash(dims, links, phases, par, v),
                                on.dslash(dims, links, phases, par, v)) < 1e-14
        assert pins.gauge_covariance(on.dslash, dims, seed=seed % 997) < 1e-13


# --------------------------------------------------------------------------
# rational function of the normal operator (RHMC, Eq. rooting / Eq. shlineq)
# --------------------------------------------------------------------------
def test_rational_apply_free_field_closed_form():
    """Unit links: a plane wave is an eigenvector of A with lambda = m^2 + sum sin^2 p,
    so r(A) pw = (a0 + sum_k a_k / (lambda + sigma_k)) pw exactly."""
    dims = (4, 6, 4, 8)
    links = on.unit_links(dims)
    phases = on.standard_phases(dims)
    mass = 0.1
    shifts = [0.0, 0.03, 0.4, 2.5]
    coeffs = [0.7, -0.2, 1.3, 0.05]
    a0 = 0.25
    for n in ((0, 0, 0, 0), (1, 2, 3, 1), (3, 5, 1, 6)):
        p = on.momenta(dims, n)
        pw = on.plane_wave(dims, 0, p, np.array([1.0, 0.5j, -0.25 + 0.1j]))
        lam = on.free_eigenvalue(mass, p)
        want = (a0 + sum(a / (lam + s) for a, s in zip(coeffs, shifts))) * pw
        y, worst = on.rational_apply(dims, links, phases, mass, shifts, coeffs, a0, pw)
        assert worst <= 1e-12
        assert np.max(np.abs(y - want)) <= 1e-10 * np.max(np.abs(want))


def test_rational_apply_partial_fractions():
    """1/((x+s1)(x+s2)) = (1/(x+s1) - 1/(x+s2)) / (s2 - s1): with those coefficients
    (A + s2)(A + s1) y = b, checked with the operator itself on random SU(3) links."""
    dims = (4, 4, 2, 6)
    links = si.su3_links(dims, 31, 0)
    phases = on.standard_phases(dims)
    mass, s1, s2 = 0.2, 0.01, 0.3
    b = si.gaussian_field(dims, 1, 31, 1)[0]
    c = 1.0 / (s2 - s1)
    y, worst = on.rational_apply(dims, links, phases, mass, [s1, s2], [c, -c], 0.0, b)
    assert worst <= 1e-12
    back = on.apply_normal(dims, links, phases, mass,
                           on.apply_normal(dims, links, phases, mass, y, sigma=s1), sigma=s2)
    assert np.linalg.norm(back - b) <= 1e-9 * np.linalg.norm(b)


def test_rational_apply_linear_in_coefficients():
    dims = (2, 4, 2, 4)
    links = si.su3_links(dims, 32, 0)
    phases = on.standard_phases(dims)
    b = si.gaussian_field(dims, 1, 32, 1)[0]
    shifts = [0.0, 0.1, 1.0]
    ca, cb = [1.0, 2.0, -0.5], [0.3, -1.0, 0.25]
    ya, _ = on.rational_apply(dims, links, phases, 0.1, shifts, ca, 0.5, b)
    yb, _ = on.rational_apply(dims, links, phases, 0.1, shifts, cb, -0.2, b)
    yab, _ = on.rational_apply(dims, links, phases, 0.1, shifts,
                               [u + v for u, v in zip(ca, cb)], 0.3, b)
    assert np.max(np.abs(yab - (ya + yb))) <= 1e-10 * np.max(np.abs(yab))


# --------------------------------------------------------------------------
# Staples of the tree-level Symanzik gauge force (Sec. 2.1, Sec. 4.3)
# --------------------------------------------------------------------------


def test_staple_pins():
    res = pins.run_staple_pins(on.staples)
    for name, (err, tol) in res.items():
        assert err <= tol, f"staple pin {name} error {err:.3e} > {tol:.1e}"


def test_path_product_pure_gauge():
    """On U_mu(x) = g(x) g(x+mu)^dag any path from y to z multiplies to g(y) g(z)^dag."""
    dims = (4, 6, 4, 4)
    g = (si.su3_site_field(dims, 27, 0), si.su3_site_field(dims, 27, 1))
    links = on.pure_gauge_links(dims, *g)
    x = on.all_coords(dims)
    steps = [(0, 1), (2, -1), (1, 1), (1, 1), (3, -1), (0, -1), (0, -1), (2, 1)]
    w = on.path_product(dims, links, x, steps)
    end = x.copy()
    for mu, s in steps:
        end = on.shifted(dims, end, mu, s)
    want = np.einsum("abn,cbn->acn", pins._g_at(dims, g, x), np.conj(pins._g_at(dims, g, end)))
    assert np.max(np.abs(w - want)) <= 1e-13


def test_loop_sums_unit_and_counts():
    """Unit links: each loop has trace 3; there are 6 V plaquettes and 12 V rectangles."""
    dims = (4, 4, 6, 4)
    plaq, rect = on.loop_sums(dims, on.unit_links(dims))
    v = on.volume(dims)
    assert plaq == 3.0 * 6 * v and rect == 3.0 * 12 * v


def test_staples_tree_level_weights():
    """Tree-level weights: c1 = -1/12 and c0 + 8 c1 = 1, so the unit-link staple is 8.5 I."""
    assert on.SYMANZIK_C1 == -1.0 / 12.0 and abs(on.SYMANZIK_C0 - 5.0 / 3.0) < 1e-15
    dims = (4, 4, 4, 4)
    s = on.staples(dims, on.unit_links(dims))
    assert np.allclose(s[5], 8.5 * np.eye(3)[:, :, None], rtol=0, atol=1e-14)


def test_staples_at_matches_whole_lattice():
    dims = (4, 6, 2, 4)
    links = si.su3_links(dims, 28, 0)
    full = on.staples(dims, links, 0.8, -0.3)
    hs = [0, 5, 17, 47]
    for slot in range(8):
        part = on.staples_at(dims, links, slot, hs, 0.8, -0.3)
        assert np.array_equal(part, full[slot][:, :, hs])


# --------------------------------------------------------------------------
# Fermion force of the rational action (Sec. 2.2)
# --------------------------------------------------------------------------


def test_force_pins():
    res = pins.run_force_pins(on.force_from_solutions)
    for name, (err, tol) in res.items():
        assert err <= tol, f"force pin {name} error {err:.3e} > {tol:.1e}"


def test_fermion_force_end_to_end_matches_dense_derivative():
    """fermion_force (its own CG solves) agrees with the force from dense solves."""
    dims = (2, 2, 4, 2)
    links = si.su3_links(dims, 54, 0)
    ph = on.standard_phases(dims)
    mass, shifts, coeffs = 0.2, [0.01, 0.3], [1.0, 0.5]
    phi = si.gaussian_field(dims, 1, 54, 1)[0]
    g, xs, ys = on.fermion_force(dims, links, ph, mass, shifts, coeffs, phi)
    _, deo, doe, _ = on.dense_blocks(dims, links, ph)
    a = mass * mass * np.eye(deo.shape[0]) - deo @ doe
    xd = np.array([np.linalg.solve(a + s * np.eye(a.shape[0]), phi.reshape(-1)).reshape(3, -1)
                   for s in shifts])
    yd = np.array([on.d_oe(dims, links, ph, x) for x in xd])
    gd = on.force_from_solutions(dims, ph, coeffs, xd, yd)
    assert np.max(np.abs(g - gd)) <= 1e-9 * np.max(np.abs(gd))


def test_force_sampled_matches_whole_lattice():
    dims = (4, 2, 6, 4)
    ph = si.real_link_field(dims, 55, 0)
    xs = si.gaussian_field(dims, 2, 55, 1)
    ys = si.gaussian_field(dims, 2, 55, 2)
    full = on.force_from_solutions(dims, ph, [0.3, -1.2], xs, ys)
    hs = [0, 7, 30, 47]
    assert np.array_equal(on.force_from_solutions(dims, ph, [0.3, -1.2], xs, ys, hs=hs),
                          full[:, :, :, hs])


# --------------------------------------------------------------------------
# Stout smearing (Sec. 2.1, Sec. 2.3)
# --------------------------------------------------------------------------


def test_stout_pins():
    res = pins.run_stout_pins(on.stout_smear)
    for name, (err, tol) in res.items():
        assert err <= tol, f"stout pin {name} error {err:.3e} > {tol:.1e}"


def test_stout_q_from_forward_paths():
    assert pins.stout_q_from_forward_paths(on.stout_q) <= 1e-14


def test_stout_q_linear_in_rho_and_small_rho():
    """Q is linear in rho, and U'(rho) = U + i rho Q(1) U + O(rho^2)."""
    dims = (4, 2, 4, 4)
    links = si.su3_links(dims, 76, 0)
    q1 = on.stout_q(dims, links, 1.0)
    assert np.max(np.abs(on.stout_q(dims, links, 0.37) - 0.37 * q1)) <= 1e-14
    r = 1e-5
    d = (on.stout_smear(dims, links, r) - links) / r
    want = 1j * np.einsum("sabn,sbcn->sacn", q1, links)
    assert np.max(np.abs(d - want)) <= 1e-3 * np.max(np.abs(want))


def test_stout_at_matches_whole_lattice():
    dims = (4, 2, 4, 6)
    links = si.su3_links(dims, 77, 0)
    full = on.stout_smear(dims, links, 0.15)
    hs = [0, 9, 47]
    for slot in range(8):
        assert np.max(np.abs(on.stout_smear_at(dims, links, slot, hs, 0.15) -
                             full[slot][:, :, hs])) <= 1e-14


# --------------------------------------------------------------------------
# Pure-gauge molecular dynamics (Sec. 4.3, Table 4)
# --------------------------------------------------------------------------


def test_gauge_force_is_the_derivative_of_the_action():
    """F traceless Hermitian, and (S(e^{itX}U) - S(e^{-itX}U)) / 2t = Tr(F X) + O(t^2)
    for random traceless Hermitian X at links of every slot (c0, c1 tree level and
    separately)."""
    from scipy.linalg import expm
    dims, beta = (4, 4, 6, 4), 5.0
    links = si.su3_links(dims, 91, 0)
    x = si.traceless_hermitian_field(dims, 91, 1)
    for c0, c1 in ((on.SYMANZIK_C0, on.SYMANZIK_C1), (1.0, 0.0), (0.0, 1.0)):
        f = on.gauge_force(dims, links, beta, c0, c1)
        assert np.max(np.abs(f - np.conj(np.transpose(f, (0, 2, 1, 3))))) <= 1e-14
        assert np.max(np.abs(np.einsum("saan->sn", f))) <= 1e-13
        t = 1e-4
        for slot in range(8):
            h = (13 * slot + 5) % on.half_volume(dims)

            def s_at(tt):
                lk = links.copy()
                lk[slot, :, :, h] = expm(1j * tt * x[slot, :, :, h]) @ links[slot, :, :, h]
                return on.symanzik_action(dims, lk, beta, c0, c1)

            d = (s_at(t) - s_at(-t)) / (2 * t)
            want = float(np.real(np.trace(f[slot, :, :, h] @ x[slot, :, :, h])))
            assert abs(d - want) <= 1e-6 * max(abs(want), 1.0)


def test_leapfrog_energy_error_scales_as_eps_squared_and_reverses():
    dims, beta = (4, 2, 4, 4), 5.5
    links = si.su3_links(dims, 92, 0)
    mom = si.traceless_hermitian_field(dims, 92, 1)
    h0 = on.md_hamiltonian(dims, links, mom, beta)
    dh = []
    for eps, n in ((0.04, 4), (0.02, 8)):
        u, p = on.leapfrog(dims, links, mom, beta, eps, n)
        dh.append(on.md_hamiltonian(dims, u, p, beta) - h0)
    assert 3.7 <= dh[0] / dh[1] <= 4.3, dh
    # reversibility: flip the momenta, integrate back
    u, p = on.leapfrog(dims, links, mom, beta, 0.02, 8)
    ub, pb = on.leapfrog(dims, u, -p, beta, 0.02, 8)
    assert np.max(np.abs(ub - links)) <= 1e-12 and np.max(np.abs(pb + mom)) <= 1e-12


def test_gauge_force_covariance_and_link_update_unitary():
    dims, beta = (4, 4, 2, 4), 6.0
    links = si.su3_links(dims, 93, 0)
    g = (si.su3_site_field(dims, 93, 1), si.su3_site_field(dims, 93, 2))
    f = on.gauge_force(dims, links, beta)
    fg = on.gauge_force(dims, on.gauge_transform_links(dims, links, *g), beta)
    for parity in (0, 1):
        for mu in range(4):
            want = np.einsum("abn,bcn,dcn->adn", g[parity], f[2 * mu + parity],
                             np.conj(g[parity]))
            assert np.max(np.abs(fg[2 * mu + parity] - want)) <= 1e-13
    u = on.link_update(links, si.traceless_hermitian_field(dims, 93, 3), 0.3)
    m = np.transpose(u, (0, 3, 1, 2)).reshape(-1, 3, 3)
    assert np.max(np.abs(m @ np.conj(np.transpose(m, (0, 2, 1))) - np.eye(3))) <= 1e-14
    assert np.max(np.abs(np.linalg.det(m) - 1)) <= 1e-14


def _complex_field(dims, *seed):
    vh = on.half_volume(dims)
    z = si.rng(*seed).standard_normal((8, 3, 3, vh, 2))
    return z[..., 0] + 1j * z[..., 1]


def test_stout_backprop_is_the_chain_rule():
    """For S(U) = Re sum_l Tr(U'_l(U) M_l) (so dS/dU' = M) the chain rule must give the
    central differences of S in all 18 real directions, at links of every slot, on two
    lattices and weights; rho = 0 maps Sigma' to itself."""
    for dims, rho, seed in (((4, 2, 4, 4), 0.2, 111), ((2, 4, 4, 4), -0.35, 112)):
        links = si.su3_links(dims, seed, 0)
        m = _complex_field(dims, seed, 1)
        sig = on.stout_backprop(dims, links, rho, m)

        def f(lk):
            return float(np.real(np.einsum("sabn,sban->", on.stout_smear(dims, lk, rho), m)))

        eps = 1e-5
        for slot in range(8):
            h = (7 * slot + 3) % on.half_volume(dims)
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
            assert np.max(np.abs(got - sig[slot, :, :, h])) <= 1e-7 * np.max(
                np.abs(sig[slot, :, :, h]))
        assert np.array_equal(on.stout_backprop(dims, links, 0.0, m), m)


def test_stout_backprop_gauge_covariance():
    """dS = Re Tr(dU' Sigma') is gauge invariant when Sigma'_mu(x) transforms as
    g(x+mu) Sigma' g(x)^dag; Sigma then transforms the same way."""
    dims, rho = (4, 4, 2, 4), 0.15
    links = si.su3_links(dims, 113, 0)
    m = _complex_field(dims, 113, 1)
    g = (si.su3_site_field(dims, 113, 2), si.su3_site_field(dims, 113, 3))

    def tr_ends(field):
        out = np.empty_like(field)
        for parity in (0, 1):
            x = on.coords(dims, parity)
            for mu in range(4):
                gf = pins._g_at(dims, g, on.shifted(dims, x, mu, +1))
                out[2 * mu + parity] = np.einsum("abn,bcn,dcn->adn", gf, field[2 * mu + parity],
                                                 np.conj(g[parity]))
        return out

    s0 = on.stout_backprop(dims, links, rho, m)
    s1 = on.stout_backprop(dims, on.gauge_transform_links(dims, links, *g), rho, tr_ends(m))
    assert np.max(np.abs(s1 - tr_ends(s0))) <= 1e-12 * np.max(np.abs(s0))


def test_stout_backprop_at_matches_whole_lattice():
    """The per-link form of the chain rule (for spot checks at 32^4) against the whole
    lattice one, at links of every slot, including lattices with extents of 2 where a
    3-link path crosses the same link twice."""
    for dims in ((4, 4, 2, 6), (2, 4, 4, 2)):
        links = si.su3_links(dims, 114, 0)
        m = _complex_field(dims, 114, 1)
        full = on.stout_backprop(dims, links, 0.15, m)
        vh = on.half_volume(dims)
        hs = [0, 5, vh // 2, vh - 1]
        for slot in range(8):
            part = on.stout_backprop_at(dims, links, 0.15, m, slot, hs)
            assert np.max(np.abs(part - full[slot][:, :, hs])) <= 1e-13 * np.max(np.abs(full))


def test_smeared_fermion_force_is_the_derivative():
    """The force of the rational action on stout-smeared links, S(U) = Re phi^dag
    sum_k a_k (A(U') + sigma_k)^-1 phi with U' = exp(iQ) U: the thin-link fermion force
    on U' passed through the stout chain rule must equal the central differences of S
    (dense solves) in all 18 directions of one link per slot.  This fixes that the two
    pieces share one convention (dS = Re Tr(dU G)) and compose."""
    dims, rho, eps = (2, 2, 2, 4), 0.12, 1e-6
    links = si.su3_links(dims, 115, 0)
    ph = on.standard_phases(dims)
    mass, shifts, coeffs = 0.3, [0.0, 0.05, 0.5], [0.4, 0.8, -0.2]
    phi = si.gaussian_field(dims, 1, 115, 1)[0]

    def solver(lk):
        _, deo, doe, _ = on.dense_blocks(dims, lk, ph)
        a = mass * mass * np.eye(deo.shape[0]) - deo @ doe
        return lambda sig, b: np.linalg.solve(a + sig * np.eye(a.shape[0]),
                                              b.reshape(-1)).reshape(3, -1)

    smeared = on.stout_smear(dims, links, rho)
    sol = solver(smeared)
    xs = np.array([sol(s, phi) for s in shifts])
    ys = np.array([on.d_oe(dims, smeared, ph, x) for x in xs])
    sig = on.stout_backprop(dims, links, rho, on.force_from_solutions(dims, ph, coeffs, xs, ys))

    def f(lk):
        sm = on.stout_smear(dims, lk, rho)
        return on.rational_action(dims, sm, ph, mass, shifts, coeffs, phi, solve=solver(sm))

    for slot in range(8):
        h = (3 * slot + 1) % on.half_volume(dims)
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
        assert np.max(np.abs(got - sig[slot, :, :, h])) <= 1e-6 * np.max(np.abs(sig[slot, :, :, h]))
