"""NumPy FP64 oracle of the even/odd staggered operator, its normal operator and CG.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU
baseline leg of the benchmark, never by the GPU library.  It shares no code with
the GPU path.  It is the second, independent implementation of the same
definitions as ``stag_oracle.c`` (N-version check), plus the brute-force dense
constructions and the closed forms that pin both.

Paper: Bonati et al., arXiv:1701.00426.
  * Sec. 4.1, Eq. lexicographic_eo -- half-lattice index h = floor(lex/2), x0
    fastest, all extents even (applied to both parities).
  * Sec. 4.1 -- vec3_soa field layout [3][Vh]; gauge field as an array of 8
    su3_soa, layout here [8][3][3][Vh], slot 2*mu + parity of the link's start.
  * Sec. 2.2, Eq. diracblock -- M = m + [[0, D_oe], [D_eo, 0]], D_oe^dag = -D_eo.
  * Sec. 2.2, Eq. lineqeo -- (m^2 - D_eo D_oe) phi_e = b_e, Hermitian positive
    definite, solved by CG.
  * Sec. 2.2, Eq. shlineq -- shifted systems (M + sigma_i) phi_i = b; with the
    coefficients of a rational approximation (Eq. rooting, the RHMC algorithm)
    their solutions combine into r(A) b.
  * Sec. 4.3, deo listing -- the operator takes links, in, out and a real
    per-link "backfield" array; here that array carries the staggered phases.
  * Sec. 2.1 (tree-level Symanzik gauge action) and Sec. 4.3 (gauge force:
    staples as products of 3 and 5 links along C-shaped paths) -- Wilson
    lines, the 1x1 and 1x2 loop sums and the staple sum of every link.
  * Sec. 2.2 (forces of the molecular dynamics from the solutions of Eq.
    shlineq) -- the rational pseudofermion action and its derivative with
    respect to every link (thin links; the stout-smearing chain is not here).
  * Sec. 2.1, Sec. 2.3 -- one stout-smearing step (Morningstar-Peardon definition)
    and the chain rule of a force through it.
  * Sec. 4.3 and Table 4 -- the pure-gauge molecular dynamics: the gauge force
    from the staples, momentum and link updates, the leapfrog and its energy.

Everything takes the arrays as given; random inputs come from the seeded
generators, which hold none of this arithmetic.
"""
from __future__ import annotations

import math

import numpy as np

# --------------------------------------------------------------------------
# Geometry (Sec. 4.1, Eq. lexicographic_eo)
# --------------------------------------------------------------------------


def volume(dims) -> int:
    n0, n1, n2, n3 = dims
    return n0 * n1 * n2 * n3


def half_volume(dims) -> int:
    return volume(dims) // 2


def check_dims(dims):
    if len(dims) != 4 or any(int(n) < 2 or int(n) % 2 for n in dims):
        raise ValueError(f"every lattice extent must be even and >= 2, got {dims}")


def lex_index(dims, x):
    """lex(x) = x0 + N0 (x1 + N1 (x2 + N2 x3)); x is (4, ...) integer array."""
    n0, n1, n2, _ = dims
    return x[0] + n0 * (x[1] + n1 * (x[2] + n2 * x[3]))


def half_index(dims, x):
    """h(x) = floor(lex(x) / 2) (Eq. lexicographic_eo)."""
    return lex_index(dims, x) // 2


def site_parity(x):
    return (x[0] + x[1] + x[2] + x[3]) & 1


def coords(dims, parity: int):
    """Coordinates (4, Vh) of the sites of one parity, in half-index order."""
    n0, n1, n2, _ = dims
    h = np.arange(half_volume(dims), dtype=np.int64)
    nh0 = n0 // 2
    x0half = h % nh0
    rest = h // nh0
    x1 = rest % n1
    rest = rest // n1
    x2 = rest % n2
    x3 = rest // n2
    x0 = 2 * x0half + ((parity + x1 + x2 + x3) & 1)
    return np.stack([x0, x1, x2, x3])


def shifted(dims, x, mu: int, step: int):
    """x + step*mu_hat with periodic wrap of the index."""
    y = x.copy()
    y[mu] = (x[mu] + step) % dims[mu]
    return y


# --------------------------------------------------------------------------
# Phases
# --------------------------------------------------------------------------


def eta(x, mu: int):
    """Staggered phase eta_mu(x) = (-1)^(x0 + ... + x_{mu-1})."""
    s = np.zeros_like(x[0])
    for nu in range(mu):
        s = s + x[nu]
    return np.where(s & 1, -1.0, 1.0)


def standard_phases(dims):
    """phases[2*mu + parity, h] = eta_mu(x) * s_mu(x), antiperiodic in x3.

    s_3(x) = -1 on the link leaving x3 = N3 - 1 (time = x3), else +1.
    """
    vh = half_volume(dims)
    ph = np.empty((8, vh), dtype=np.float64)
    for parity in (0, 1):
        x = coords(dims, parity)
        for mu in range(4):
            bc = np.where((x[3] == dims[3] - 1), -1.0, 1.0) if mu == 3 else 1.0
            ph[2 * mu + parity] = eta(x, mu) * bc
    return ph


# --------------------------------------------------------------------------
# The hop (Sec. 2.2 Eq. diracblock; explicit textbook form)
# --------------------------------------------------------------------------


def dslash(dims, links, phases, out_parity: int, vin, hs=None):
    """D restricted to output parity ``out_parity`` (0: D_eo, 1: D_oe).

    (D psi)(x) = 1/2 sum_mu [ phi_mu(x) U_mu(x) psi(x+mu)
                             - phi_mu(x-mu) U_mu(x-mu)^dag psi(x-mu) ]

    links (8, 3, 3, Vh) complex; phases (8, Vh) real; vin (..., 3, Vh) on the
    other parity.  Returns (..., 3, Vh), or (..., 3, len(hs)) for the output
    sites listed in ``hs`` only (sampled checks of large lattices).
    """
    x = coords(dims, out_parity)
    if hs is not None:
        x = x[:, np.asarray(hs, dtype=np.int64)]
    own = half_index(dims, x)
    in_parity = 1 - out_parity
    out = np.zeros(vin.shape[:-1] + (x.shape[1],), dtype=np.complex128)
    for mu in range(4):
        hf = half_index(dims, shifted(dims, x, mu, +1))
        hb = half_index(dims, shifted(dims, x, mu, -1))
        uf = links[2 * mu + out_parity][:, :, own]          # U_mu(x), (3,3,n)
        ub = links[2 * mu + in_parity][:, :, hb]            # U_mu(x-mu)
        pf = phases[2 * mu + out_parity][own]
        pb = phases[2 * mu + in_parity][hb]
        fwd = np.einsum("abh,...bh->...ah", uf, vin[..., :, hf])
        bwd = np.einsum("bah,...bh->...ah", np.conj(ub), vin[..., :, hb])
        out += pf * fwd - pb * bwd
    return 0.5 * out


def d_eo(dims, links, phases, v_odd):
    return dslash(dims, links, phases, 0, v_odd)


def d_oe(dims, links, phases, v_even):
    return dslash(dims, links, phases, 1, v_even)


def apply_normal(dims, links, phases, mass, v_even, sigma=0.0):
    """(m^2 + sigma - D_eo D_oe) v (Eq. lineqeo, shifted as in Eq. shlineq)."""
    t = d_oe(dims, links, phases, v_even)
    return (mass * mass + sigma) * v_even - d_eo(dims, links, phases, t)


# --------------------------------------------------------------------------
# CG (Sec. 2.2): textbook Hestenes-Stiefel
# --------------------------------------------------------------------------


def _re_dot(a, b):
    return float(np.real(np.vdot(a, b)))


def cg(dims, links, phases, mass, b, tol=1e-12, max_iter=100000, sigma=0.0, x0=None):
    """Returns (x, iterations, true relative residual)."""
    x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128).copy()
    r = b - apply_normal(dims, links, phases, mass, x, sigma)
    p = r.copy()
    bb = _re_dot(b, b)
    rr = _re_dot(r, r)
    it = 0
    while rr > tol * tol * bb and it < max_iter:
        q = apply_normal(dims, links, phases, mass, p, sigma)
        alpha = rr / _re_dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = _re_dot(r, r)
        it += 1
        if rr_new <= tol * tol * bb:
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    res = b - apply_normal(dims, links, phases, mass, x, sigma)
    return x, it, math.sqrt(_re_dot(res, res) / bb)


def true_relative_residual(dims, links, phases, mass, b, x, sigma=0.0):
    res = b - apply_normal(dims, links, phases, mass, x, sigma)
    return math.sqrt(_re_dot(res, res) / _re_dot(b, b))


def rational_apply(dims, links, phases, mass, shifts, coeffs, a0, b, tol=1e-12):
    """y = a0 b + sum_k coeffs[k] (m^2 + shifts[k] - D_eo D_oe)^{-1} b.

    The rational function of the normal operator that the RHMC algorithm uses in
    place of the fractional power of Eq. rooting (Sec. 2.2): its poles are the
    shifts of Eq. shlineq, whose solutions are combined with the caller's
    coefficients.  Each shifted system is solved here by plain CG (the definition;
    no multi-shift recurrence).  Returns (y, worst true relative residual)."""
    y = a0 * np.asarray(b, dtype=np.complex128)
    worst = 0.0
    for s, a in zip(shifts, coeffs):
        x, _, res = cg(dims, links, phases, mass, b, tol=tol, sigma=s)
        y = y + a * x
        worst = max(worst, res)
    return y, worst


# --------------------------------------------------------------------------
# Brute force: the full-lattice operator as a dense matrix
# --------------------------------------------------------------------------


def dense_full_operator(dims, links, phases):
    """Dense D on all V sites, 3V x 3V, filled entry by entry from the definition.

    Rows/columns are ordered (site lex index, colour).  Independent of
    ``dslash``: it walks every site and direction once and adds the two hopping
    terms into the matrix.
    """
    n0, n1, n2, n3 = dims
    v = volume(dims)
    vh = v // 2
    d = np.zeros((3 * v, 3 * v), dtype=np.complex128)
    for x3 in range(n3):
        for x2 in range(n2):
            for x1 in range(n1):
                for x0 in range(n0):
                    x = np.array([x0, x1, x2, x3])
                    lx = int(lex_index(dims, x))
                    px = int(site_parity(x))
                    hx = lx // 2
                    for mu in range(4):
                        xf = x.copy()
                        xf[mu] = (x[mu] + 1) % dims[mu]
                        xb = x.copy()
                        xb[mu] = (x[mu] - 1) % dims[mu]
                        lf = int(lex_index(dims, xf))
                        lb = int(lex_index(dims, xb))
                        hb = lb // 2
                        uf = links[2 * mu + px, :, :, hx]
                        ub = links[2 * mu + (1 - px), :, :, hb]
                        pf = phases[2 * mu + px, hx]
                        pb = phases[2 * mu + (1 - px), hb]
                        d[3 * lx:3 * lx + 3, 3 * lf:3 * lf + 3] += 0.5 * pf * uf
                        d[3 * lx:3 * lx + 3, 3 * lb:3 * lb + 3] -= 0.5 * pb * ub.conj().T
    assert vh * 2 == v
    return d


def parity_permutation(dims):
    """Indices into the (lex, colour) ordering giving (parity, colour, h) order.

    Maps the dense full operator onto the [3][Vh] field layout of each parity:
    perm[parity*3*Vh + c*Vh + h] = 3*lex(x(parity, h)) + c.
    """
    vh = half_volume(dims)
    perm = np.empty(6 * vh, dtype=np.int64)
    for parity in (0, 1):
        lx = lex_index(dims, coords(dims, parity))
        for c in range(3):
            perm[parity * 3 * vh + c * vh: parity * 3 * vh + (c + 1) * vh] = 3 * lx + c
    return perm


def dense_blocks(dims, links, phases):
    """(D_ee, D_eo, D_oe, D_oo) dense blocks in the [3][Vh] layout of each parity."""
    d = dense_full_operator(dims, links, phases)
    perm = parity_permutation(dims)
    dp = d[np.ix_(perm, perm)]
    n = 3 * half_volume(dims)
    return dp[:n, :n], dp[:n, n:], dp[n:, :n], dp[n:, n:]


# --------------------------------------------------------------------------
# Closed forms and constructions used by the pins
# --------------------------------------------------------------------------


def unit_links(dims):
    vh = half_volume(dims)
    u = np.zeros((8, 3, 3, vh), dtype=np.complex128)
    for a in range(3):
        u[:, a, a, :] = 1.0
    return u


def momenta(dims, n):
    """p_mu = 2 pi n_mu / N_mu (mu < 3), p_3 = pi (2 n_3 + 1) / N_3 (antiperiodic)."""
    p = [2.0 * math.pi * n[mu] / dims[mu] for mu in range(3)]
    p.append(math.pi * (2 * n[3] + 1) / dims[3])
    return p


def plane_wave(dims, parity, p, colour_vec):
    """psi(x) = c e^{i p.x} on the sites of one parity, shape (3, Vh)."""
    x = coords(dims, parity)
    phase = np.exp(1j * sum(p[mu] * x[mu] for mu in range(4)))
    return np.asarray(colour_vec, dtype=np.complex128)[:, None] * phase[None, :]


def free_doe_plane_wave(dims, p, colour_vec):
    """Closed form of D_oe on a plane wave with unit links and standard phases.

    (D_oe psi)(x) = i c e^{i p.x} sum_mu eta_mu(x) sin p_mu on odd x.
    """
    x = coords(dims, 1)
    s = sum(eta(x, mu) * math.sin(p[mu]) for mu in range(4))
    phase = np.exp(1j * sum(p[mu] * x[mu] for mu in range(4)))
    return 1j * np.asarray(colour_vec, dtype=np.complex128)[:, None] * (s * phase)[None, :]


def free_eigenvalue(mass, p, sigma=0.0):
    """Eigenvalue of m^2 + sigma - D_eo D_oe on a plane wave: m^2 + sigma + sum sin^2 p."""
    return mass * mass + sigma + sum(math.sin(q) ** 2 for q in p)


def free_spectrum(dims, mass):
    """All 3*Vh eigenvalues of the free normal operator, from the closed form.

    On even sites p and p + (pi,pi,pi,pi) give the same function, so each class
    is taken once: n_0 runs over half of its range.
    """
    vals = []
    n0, n1, n2, n3 = dims
    for a in range(n0 // 2):
        for b in range(n1):
            for c in range(n2):
                for d in range(n3):
                    lam = free_eigenvalue(mass, momenta(dims, (a, b, c, d)))
                    vals.extend([lam, lam, lam])
    return np.sort(np.array(vals))


def site_matrices_apply(g, v):
    """(g v)(x) = g(x) v(x); g (3,3,Vh), v (...,3,Vh)."""
    return np.einsum("abh,...bh->...ah", g, v)


def gauge_transform_links(dims, links, g_even, g_odd):
    """U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dag for every link."""
    g = (g_even, g_odd)
    out = np.empty_like(links)
    for parity in (0, 1):
        x = coords(dims, parity)
        for mu in range(4):
            hf = half_index(dims, shifted(dims, x, mu, +1))
            gx = g[parity]
            gf = g[1 - parity][:, :, hf]
            u = links[2 * mu + parity]
            out[2 * mu + parity] = np.einsum(
                "abh,bch,dch->adh", gx, u, np.conj(gf))
    return out


def pure_gauge_links(dims, g_even, g_odd):
    """U_mu(x) = g(x) g(x+mu)^dag: the gauge transform of the unit field."""
    return gauge_transform_links(dims, unit_links(dims), g_even, g_odd)


def translate_field(dims, v, parity, shift_vec):
    """Field on one parity translated by an even shift: w(x) = v(x - s).

    Returns the field on the same parity (the shift is even in every
    component that is nonzero, so parity is preserved when sum(s) is even).
    """
    x = coords(dims, parity)
    src = x.copy()
    for mu in range(4):
        src[mu] = (x[mu] - shift_vec[mu]) % dims[mu]
    hsrc = half_index(dims, src)
    return v[..., hsrc]


def translate_links(dims, links, shift_vec):
    out = np.empty_like(links)
    for parity in (0, 1):
        x = coords(dims, parity)
        src = x.copy()
        for mu in range(4):
            src[mu] = (x[mu] - shift_vec[mu]) % dims[mu]
        hsrc = half_index(dims, src)
        for mu in range(4):
            out[2 * mu + parity] = links[2 * mu + parity][:, :, hsrc]
    return out


# --------------------------------------------------------------------------
# Gauge part: Wilson lines, the loops of the tree-level Symanzik action and
# the staples of its gauge force (Sec. 2.1: tree-level Symanzik gauge action;
# Sec. 4.3: staples as products of 3 and 5 links along C-shaped paths).
# --------------------------------------------------------------------------

# Tree-level Symanzik weights of the 1x1 and 1x2 loops.  The paper names the
# action and cites its origin without printing the numbers; these are the
# standard tree-level values, c0 + 8 c1 = 1 (Wilson normalisation).
SYMANZIK_C1 = -1.0 / 12.0
SYMANZIK_C0 = 1.0 - 8.0 * SYMANZIK_C1


def all_coords(dims):
    """Coordinates (4, V) of every site: the even sites, then the odd ones."""
    return np.concatenate([coords(dims, 0), coords(dims, 1)], axis=1)


def link_matrices(dims, links, y, mu: int):
    """U_mu(y), (3, 3, n), for sites y (4, n) of any parity."""
    u = links[2 * mu + site_parity(y), :, :, half_index(dims, y)]  # (n, 3, 3)
    return np.transpose(u, (1, 2, 0))


def path_product(dims, links, start, steps):
    """Ordered product of the links met along a lattice path, (3, 3, n).

    steps is a sequence of (mu, +1 | -1) taken from each site of ``start``.  A +1
    step from y contributes U_mu(y) and moves to y + mu; a -1 step moves to
    y - mu and contributes U_mu(y - mu)^dag.  Factors multiply from the right in
    path order (a Wilson line from the start to the end of the path).
    """
    y = start.copy()
    n = start.shape[1]
    w = np.repeat(np.eye(3, dtype=np.complex128)[:, :, None], n, axis=2)
    for mu, s in steps:
        if s > 0:
            u = link_matrices(dims, links, y, mu)
            y = shifted(dims, y, mu, +1)
        else:
            y = shifted(dims, y, mu, -1)
            u = np.conj(np.transpose(link_matrices(dims, links, y, mu), (1, 0, 2)))
        w = np.einsum("abn,bcn->acn", w, u)
    return w


def staple_paths(mu: int, nu: int):
    """The C-shaped paths in the (mu, nu) plane that lead from x + mu back to x.

    Two 3-link paths (the rest of the 1x1 loops above and below the link) and
    six 5-link paths (the rest of the 1x2 loops: long side along mu, extended
    forward or backward, and long side along nu, each above or below the link).
    U_mu(x) times any of them is a closed loop through x.
    """
    fw, bw, up, dn = (mu, +1), (mu, -1), (nu, +1), (nu, -1)
    three = [[up, bw, dn], [dn, bw, up]]
    five = [[fw, up, bw, bw, dn], [up, bw, bw, dn, fw], [up, up, bw, dn, dn],
            [fw, dn, bw, bw, up], [dn, bw, bw, up, fw], [dn, dn, bw, up, up]]
    return three, five


def staples(dims, links, c0=SYMANZIK_C0, c1=SYMANZIK_C1):
    """Sigma_mu(x) for every link, (8, 3, 3, Vh) in the gauge-field layout.

    Sigma_mu(x) = sum over nu != mu of c0 (the two 3-link paths) + c1 (the six
    5-link paths) of staple_paths, each a Wilson line from x + mu to x, so that
    U_mu(x) Sigma_mu(x) is the weighted sum of the closed 1x1 and 1x2 loops that
    contain the link.  Written out directly as products along each path.
    """
    check_dims(dims)
    out = np.zeros((8, 3, 3, half_volume(dims)), dtype=np.complex128)
    for parity in (0, 1):
        x = coords(dims, parity)
        for mu in range(4):
            start = shifted(dims, x, mu, +1)
            acc = out[2 * mu + parity]
            for nu in range(4):
                if nu == mu:
                    continue
                three, five = staple_paths(mu, nu)
                for p in three:
                    acc += c0 * path_product(dims, links, start, p)
                for p in five:
                    acc += c1 * path_product(dims, links, start, p)
    return out


def loop_sums(dims, links):
    """(sum of Re Tr over all 1x1 loops, sum of Re Tr over all 1x2 loops).

    Every unoriented loop counted once: the plaquette U_mu U_nu U_mu^dag U_nu^dag
    at x for mu < nu, and the rectangle with its long side (two links) along mu
    and its short side along nu at x for every ordered pair mu != nu.
    """
    x = all_coords(dims)
    plaq = rect = 0.0
    for mu in range(4):
        for nu in range(4):
            if nu == mu:
                continue
            if mu < nu:
                w = path_product(dims, links, x, [(mu, 1), (nu, 1), (mu, -1), (nu, -1)])
                plaq += float(np.sum(np.real(np.einsum("aan->n", w))))
            w = path_product(dims, links, x,
                             [(mu, 1), (mu, 1), (nu, 1), (mu, -1), (mu, -1), (nu, -1)])
            rect += float(np.sum(np.real(np.einsum("aan->n", w))))
    return plaq, rect


def weighted_loop_sum(dims, links, c0=SYMANZIK_C0, c1=SYMANZIK_C1):
    """c0 (1x1 loop sum) + c1 (1x2 loop sum): the link-dependent part of the
    tree-level Symanzik action up to its -beta/3 normalisation and a constant."""
    plaq, rect = loop_sums(dims, links)
    return c0 * plaq + c1 * rect


def staples_at(dims, links, slot: int, hs, c0=SYMANZIK_C0, c1=SYMANZIK_C1):
    """Sigma_mu(x), (3, 3, n), for the links of one slot (2*mu + parity) at the
    half indices hs only: the same sum of path products as ``staples``, for
    spot checks on lattices too large to do whole."""
    mu, parity = slot // 2, slot % 2
    x = coords(dims, parity)[:, np.asarray(hs, dtype=np.int64)]
    start = shifted(dims, x, mu, +1)
    acc = np.zeros((3, 3, x.shape[1]), dtype=np.complex128)
    for nu in range(4):
        if nu == mu:
            continue
        three, five = staple_paths(mu, nu)
        for p in three:
            acc += c0 * path_product(dims, links, start, p)
        for p in five:
            acc += c1 * path_product(dims, links, start, p)
    return acc


# --------------------------------------------------------------------------
# Fermion force of the rational pseudofermion action (Sec. 2.2: the forces of
# the molecular dynamics come from the multi-shift solutions of Eq. shlineq;
# Sec. 4.3: most of that step is spent in the operator).
# --------------------------------------------------------------------------


def rational_action(dims, links, phases, mass, shifts, coeffs, phi, solve=None):
    """S = Re phi^dag sum_k a_k (A + sigma_k)^{-1} phi on the even sites, A the
    normal operator of Eq. lineqeo (the a0 term of the rational function does not
    depend on the links and is left out).  ``solve(sigma, b)`` returns
    (A + sigma)^{-1} b; plain CG to 1e-13 when not given."""
    s = 0.0
    for sig, a in zip(shifts, coeffs):
        if solve is None:
            x, _, _ = cg(dims, links, phases, mass, phi, tol=1e-13, sigma=sig)
        else:
            x = solve(sig, phi)
        s += a * float(np.real(np.vdot(phi, x)))
    return s


def force_from_solutions(dims, phases, coeffs, x_even, y_odd, hs=None):
    """G_mu(z), (8, 3, 3, Vh) in the gauge-field layout, from X_k (even, (n, 3, Vh))
    and Y_k (odd, (n, 3, Vh)):

      z even:  G_mu(z) =  sum_k a_k phi_mu(z) Y_k(z+mu) X_k(z)^dag
      z odd:   G_mu(z) = -sum_k a_k phi_mu(z) X_k(z+mu) Y_k(z)^dag

    With X_k = (A + sigma_k)^{-1} phi and Y_k = D_oe X_k this is the derivative of
    the rational action: A = m^2 - D_eo D_oe gives dS = -sum_k a_k X_k^dag dA X_k
    = sum_k a_k 2 Re(X_k^dag dD_eo Y_k) (D_eo^dag = -D_oe for any links), and a
    link U_mu(z) enters D_eo through the forward term at an even z and the
    backward term at z + mu for an odd z.  So S(U + E) = S(U) + Re Tr(E G) to first
    order when one link U_mu(z) becomes U_mu(z) + E.  For arbitrary X_k, Y_k the
    same G is the exact derivative of sum_k a_k 2 Re(X_k^dag D_eo(U) Y_k), which is
    linear in every link.  With ``hs`` only the links at those half indices (of
    both parities) are computed: (8, 3, 3, len(hs))."""
    sel = np.arange(half_volume(dims)) if hs is None else np.asarray(hs, dtype=np.int64)
    out = np.zeros((8, 3, 3, len(sel)), dtype=np.complex128)
    for parity in (0, 1):
        z = coords(dims, parity)[:, sel]
        for mu in range(4):
            hf = half_index(dims, shifted(dims, z, mu, +1))
            ph = phases[2 * mu + parity][sel]
            acc = out[2 * mu + parity]
            for a, x, y in zip(coeffs, x_even, y_odd):
                if parity == 0:
                    acc += a * ph * np.einsum("an,bn->abn", y[:, hf], np.conj(x[:, sel]))
                else:
                    acc -= a * ph * np.einsum("an,bn->abn", x[:, hf], np.conj(y[:, sel]))
    return out


def fermion_force(dims, links, phases, mass, shifts, coeffs, phi, tol=1e-13):
    """G of ``force_from_solutions`` with X_k solved by plain CG per pole and
    Y_k = D_oe X_k.  Returns (G, X, Y)."""
    xs, ys = [], []
    for sig in shifts:
        x, _, _ = cg(dims, links, phases, mass, phi, tol=tol, sigma=sig)
        xs.append(x)
        ys.append(d_oe(dims, links, phases, x))
    xs, ys = np.array(xs), np.array(ys)
    return force_from_solutions(dims, phases, coeffs, xs, ys), xs, ys


# --------------------------------------------------------------------------
# Stout smearing (Sec. 2.1: the fermion action uses stout-smeared links; Sec. 2.3:
# the configurations of several stout levels U^(k) are kept).  The definition of
# Morningstar and Peardon: C_mu(x) = rho * (sum of the six 3-link paths from x to
# x + mu), Omega = C U^dag, Q = (i/2)(Omega^dag - Omega) - (i/6) Tr(Omega^dag - Omega),
# U' = exp(iQ) U.
# --------------------------------------------------------------------------


def stout_q(dims, links, rho):
    """Q_mu(x), (8, 3, 3, Vh): the traceless Hermitian generator of one stout step
    with isotropic weight rho in all four directions."""
    # the 3-link paths from x to x + mu are the daggers of the staple paths from
    # x + mu back to x, so C = rho * (1x1 staple sum)^dag
    sig = staples(dims, links, 1.0, 0.0)
    c = rho * np.conj(np.transpose(sig, (0, 2, 1, 3)))
    omega = np.einsum("sabn,scbn->sacn", c, np.conj(links))       # C U^dag
    a = np.conj(np.transpose(omega, (0, 2, 1, 3))) - omega         # Omega^dag - Omega
    tr = np.einsum("saan->sn", a)
    q = 0.5j * a
    for i in range(3):
        q[:, i, i, :] -= (1j / 6.0) * tr
    return q


def stout_smear(dims, links, rho):
    """U'_mu(x) = exp(i Q_mu(x)) U_mu(x) for every link (one stout level); the
    exponential by scipy.linalg.expm, matrix by matrix."""
    from scipy.linalg import expm
    q = stout_q(dims, links, rho)
    out = np.empty_like(links)
    for s in range(8):
        for h in range(links.shape[3]):
            out[s, :, :, h] = expm(1j * q[s, :, :, h]) @ links[s, :, :, h]
    return out


def stout_smear_at(dims, links, slot: int, hs, rho):
    """U' at the links of one slot at half indices hs only, (3, 3, n): the same
    definition as ``stout_smear`` with C from the six 3-link paths from x to x + mu
    written as Wilson lines, for spot checks on large lattices."""
    from scipy.linalg import expm
    mu, parity = slot // 2, slot % 2
    hs = np.asarray(hs, dtype=np.int64)
    x = coords(dims, parity)[:, hs]
    c = np.zeros((3, 3, len(hs)), dtype=np.complex128)
    for nu in range(4):
        if nu != mu:
            c += path_product(dims, links, x, [(nu, 1), (mu, 1), (nu, -1)])
            c += path_product(dims, links, x, [(nu, -1), (mu, 1), (nu, 1)])
    u = links[slot][:, :, hs]
    om = np.einsum("abn,cbn->acn", rho * c, np.conj(u))
    a = np.conj(np.transpose(om, (1, 0, 2))) - om
    q = 0.5j * a
    tr = np.einsum("aan->n", a)
    for i in range(3):
        q[i, i] -= (1j / 6.0) * tr
    out = np.empty_like(u)
    for n in range(len(hs)):
        out[:, :, n] = expm(1j * q[:, :, n]) @ u[:, :, n]
    return out


# --------------------------------------------------------------------------
# Pure-gauge molecular dynamics (Sec. 4.3: the gauge cycle evolves momenta and
# links with the gauge force; Table 4 times it per site).  Momenta P_mu(x) are
# traceless Hermitian 3x3 matrices in the link layout (8, 3, 3, Vh); a link moves
# as U -> exp(i eps P) U.
# --------------------------------------------------------------------------


def symanzik_action(dims, links, beta, c0=SYMANZIK_C0, c1=SYMANZIK_C1):
    """S_g = -(beta/3) (c0 sum Re Tr(1x1 loops) + c1 sum Re Tr(1x2 loops)), the
    link-dependent part of the tree-level Symanzik action (constants dropped)."""
    return -(beta / 3.0) * weighted_loop_sum(dims, links, c0, c1)


def traceless_hermitian(a):
    """(a + a^dag)/2 minus its trace / 3, matrix by matrix, (..., 3, 3, n)."""
    h = 0.5 * (a + np.conj(np.swapaxes(a, -3, -2)))
    tr = np.einsum("...aan->...n", h)
    for i in range(3):
        h[..., i, i, :] -= tr / 3.0
    return h


def gauge_force(dims, links, beta, c0=SYMANZIK_C0, c1=SYMANZIK_C1):
    """F_mu(x), traceless Hermitian, defined by dS/dt = Tr(F X) at t = 0 when the
    link moves as U -> exp(i t X) U (X traceless Hermitian).  S depends on the link
    through -(beta/3) Re Tr(U Sigma) (Sigma the staple sum), so
    dS/dt = -(beta/3) Re Tr(i X U Sigma) and F = -(beta/3) traceless Hermitian
    part of (i U Sigma)."""
    m = np.einsum("sabn,sbcn->sacn", links, staples(dims, links, c0, c1))
    return -(beta / 3.0) * traceless_hermitian(1j * m)


def momentum_update(dims, links, mom, beta, eps, c0=SYMANZIK_C0, c1=SYMANZIK_C1):
    """P -> P - eps F(U)."""
    return mom - eps * gauge_force(dims, links, beta, c0, c1)


def link_update(links, mom, eps):
    """U -> exp(i eps P) U for every link (scipy.linalg.expm, matrix by matrix)."""
    from scipy.linalg import expm
    out = np.empty_like(links)
    for s in range(links.shape[0]):
        for h in range(links.shape[3]):
            out[s, :, :, h] = expm(1j * eps * mom[s, :, :, h]) @ links[s, :, :, h]
    return out


def md_hamiltonian(dims, links, mom, beta, c0=SYMANZIK_C0, c1=SYMANZIK_C1):
    """H = 1/2 sum Tr P^2 + S_g."""
    kin = 0.5 * float(np.real(np.einsum("sabn,sban->", mom, mom)))
    return kin + symanzik_action(dims, links, beta, c0, c1)


def leapfrog(dims, links, mom, beta, eps, nsteps, c0=SYMANZIK_C0, c1=SYMANZIK_C1):
    """nsteps leapfrog steps: P half step, (U full step, P full step) ..., P half step."""
    p = momentum_update(dims, links, mom, beta, 0.5 * eps, c0, c1)
    u = links
    for k in range(nsteps):
        u = link_update(u, p, eps)
        p = momentum_update(dims, u, p, beta, eps if k < nsteps - 1 else 0.5 * eps, c0, c1)
    return u, p


def stout_backprop(dims, links, rho, sig_p):
    """The chain rule through one stout step: given Sigma'_l = dS/dU'_l for every link of
    the smeared field U' = exp(iQ) U (convention: dS = Re Tr(dU' Sigma')), returns
    Sigma_l = dS/dU_l for the thin links (same convention), (8, 3, 3, Vh).

    Written out from the definition of the step:
      * through U in exp(iQ) U:            Sigma'_l exp(iQ_l);
      * through Q: with Gamma = L(iQ, U Sigma') (the Frechet derivative of exp, used
        through Tr(L(A, E) M) = Tr(E L(A, M))), dS = Re Tr(i dQ Gamma); Q's definition
        turns that into dS = Re Tr(dOmega G) with
        G = (Gamma - Gamma^dag)/2 + (conj(Tr Gamma) - Tr Gamma)/6 I;
      * Omega = C U^dag: through U^dag, C^dag G^dag; through C, Re Tr(dC U^dag G);
      * C = rho * (3-link paths): every link of every path receives
        rho * (product after it) (U^dag G) (product before it), daggered for a link
        the path walks backwards.
    Pinned by central differences of Re sum Tr(U'(U) M)."""
    from scipy.linalg import expm_frechet
    vh = half_volume(dims)
    sig_s = staples(dims, links, 1.0, 0.0)
    cmat = rho * np.conj(np.transpose(sig_s, (0, 2, 1, 3)))
    q = stout_q(dims, links, rho)
    out = np.zeros_like(links)
    gc = np.empty_like(links)        # U^dag G per link
    for s in range(8):
        for h in range(vh):
            u = links[s, :, :, h]
            e, gam = expm_frechet(1j * q[s, :, :, h], u @ sig_p[s, :, :, h])
            tg = np.trace(gam)
            g = 0.5 * (gam - np.conj(gam.T)) + ((np.conj(tg) - tg) / 6.0) * np.eye(3)
            c = cmat[s, :, :, h]
            out[s, :, :, h] = sig_p[s, :, :, h] @ e + np.conj(c.T) @ np.conj(g.T)
            gc[s, :, :, h] = np.conj(u.T) @ g
    for parity in (0, 1):
        x = coords(dims, parity)
        for mu in range(4):
            g = gc[2 * mu + parity]
            for al in range(4):
                if al == mu:
                    continue
                for steps in ([(al, 1), (mu, 1), (al, -1)], [(al, -1), (mu, 1), (al, 1)]):
                    y = x.copy()
                    for k, (d, sgn) in enumerate(steps):
                        a = path_product(dims, links, x, steps[:k])
                        if sgn > 0:
                            site = y
                            after = shifted(dims, y, d, +1)
                        else:
                            site = shifted(dims, y, d, -1)
                            after = site
                        dd = path_product(dims, links, after, steps[k + 1:])
                        contrib = rho * np.einsum("abn,bcn,cdn->adn", dd, g, a)
                        if sgn < 0:
                            contrib = np.conj(np.transpose(contrib, (1, 0, 2)))
                        slot = 2 * d + site_parity(site)
                        # for fixed (mu, parity, al, path, k) the link sites are a
                        # translate of the sites x: no index repeats
                        hh = half_index(dims, site)
                        for p2 in (0, 1):
                            sel = (site_parity(site) == p2)
                            out[2 * d + p2][:, :, hh[sel]] += contrib[:, :, sel]
                        y = after
    return out


def stout_backprop_at(dims, links, rho, sig_p, slot: int, hs):
    """dS/dU of the thin links of one slot at half indices hs only, (3, 3, n): the
    chain rule of ``stout_backprop`` organised per output link, for spot checks on
    large lattices.  The link's own terms are Sigma' exp(iQ) + C^dag G^dag.  The
    terms through C come from the 3-link paths of other links l' = (mu, x) that walk
    across this link: 6 paths along the link's own direction (it is their middle
    step) and 12 from links of the other directions (it is their first or last
    step, either way); each gives rho * (product after it) (U^dag G at l')
    (product before it), daggered where the path walks the link backwards."""
    from scipy.linalg import expm_frechet
    d, parity = slot // 2, slot % 2
    hs = np.asarray(hs, dtype=np.int64)
    z = coords(dims, parity)[:, hs]
    eye = np.eye(3)

    def terms_at(mu, x):
        """exp(iQ), G, C, U and Sigma' of the links (mu, x), each (3, 3, n)."""
        c = np.zeros((3, 3, x.shape[1]), dtype=np.complex128)
        for nu in range(4):
            if nu != mu:
                c += path_product(dims, links, x, [(nu, 1), (mu, 1), (nu, -1)])
                c += path_product(dims, links, x, [(nu, -1), (mu, 1), (nu, 1)])
        c *= rho
        u = link_matrices(dims, links, x, mu)
        sp = np.transpose(sig_p[2 * mu + site_parity(x), :, :, half_index(dims, x)], (1, 2, 0))
        e, g = np.empty_like(u), np.empty_like(u)
        for i in range(x.shape[1]):
            om = c[:, :, i] @ np.conj(u[:, :, i].T)
            a = np.conj(om.T) - om
            q = 0.5j * a - (1j / 6.0) * np.trace(a) * eye
            e[:, :, i], gam = expm_frechet(1j * q, u[:, :, i] @ sp[:, :, i])
            tg = np.trace(gam)
            g[:, :, i] = 0.5 * (gam - np.conj(gam.T)) + ((np.conj(tg) - tg) / 6.0) * eye
        return e, g, c, u, sp

    e, g, c, u, sp = terms_at(d, z)
    out = np.einsum("abn,bcn->acn", sp, e) + np.einsum(
        "ban,cbn->acn", np.conj(c), np.conj(g))
    for mu in range(4):
        for al in range(4):
            if al == mu:
                continue
            for steps in ([(al, 1), (mu, 1), (al, -1)], [(al, -1), (mu, 1), (al, 1)]):
                for k, (dk, sk) in enumerate(steps):
                    if dk != d:
                        continue
                    # the site x of the path's own link: walking steps[:k] from x
                    # reaches y, and the link crossed next is (d, y) going forward,
                    # (d, y - d) going backward; either must be (d, z)
                    x = z if sk > 0 else shifted(dims, z, d, +1)
                    for dj, sj in reversed(steps[:k]):
                        x = shifted(dims, x, dj, -sj)
                    _, gl, _, ul, _ = terms_at(mu, x)
                    gc = np.einsum("ban,bcn->acn", np.conj(ul), gl)
                    before = path_product(dims, links, x, steps[:k])
                    after = shifted(dims, z, d, +1) if sk > 0 else z
                    rest = path_product(dims, links, after, steps[k + 1:])
                    contrib = rho * np.einsum("abn,bcn,cdn->adn", rest, gc, before)
                    if sk < 0:
                        contrib = np.conj(np.transpose(contrib, (1, 0, 2)))
                    out += contrib
    return out
