"""GPU solvers through the C ABI: FP64 CG, mixed-precision CG with reliable
updates (FP32-12 and BF16-12 links), multi-RHS, multi-shift CG with refinement.

Parity bar: every returned solution has an FP64 true relative residual
|b - A x| / |b| <= 1e-10 recomputed by the oracle, and its distance to the
oracle's own solution is within the conditioning bound (reported)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1701_00426_amd as stg  # noqa: E402
import seeded_inputs as si  # noqa: E402
from oracle import oracle_np as on  # noqa: E402

from gpu_common import rel_norm, say, to_dev  # noqa: E402

TOL = 1e-10


def _problem(dims, seed, nrhs=1):
    links = si.su3_links(dims, 1701, *seed)
    phases = on.standard_phases(dims)
    b = si.gaussian_field(dims, nrhs, 426, *seed)
    return links, phases, b


def _check(corc, dims, links, phases, mass, b, x, stats, sigma=0.0, label=""):
    for j in range(b.shape[0]):
        res = on.true_relative_residual(dims, links, phases, mass, b[j], x[j], sigma=sigma)
        xr, it, r0, st = corc.cg(dims, links, phases, mass, b[j], tol=1e-12, sigma=sigma)
        err = rel_norm(x[j], xr)
        s = stats[j]
        say(f"  {label} rhs {j}: iters {s['iters']} RU {s['reliable_updates']} "
            f"lib resid {s['true_rel_resid']:.2e} oracle resid {res:.2e} |x-x*|/|x*| {err:.2e} "
            f"(oracle iters {it})")
        assert s["status"] == 0
        assert res <= TOL
        assert abs(s["true_rel_resid"] - res) <= 1e-3 * res + 1e-14
        # |x - x*| / |x*| <= kappa |r| / |b|, kappa <= (m^2 + 16) / m^2
        kappa = (mass * mass + sigma + 16.0) / (mass * mass + sigma)
        assert err <= kappa * 2 * TOL


@pytest.mark.parametrize("fmt", ["c128_18", "c128_12"])
@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (4, 6, 8, 10), (2, 2, 2, 2)])
def test_cg_fp64(dims, fmt, corc):
    say(f"cg fp64 {fmt} {dims}")
    links, phases, b = _problem(dims, (0, 0))
    g = stg.pack_gauge(dims, to_dev(links), fmt)
    x, st, stats = stg.cg_solve(g, 0.1, to_dev(b), tol=TOL)
    _check(corc, dims, links, phases, 0.1, b, x.cpu().numpy(), stats, label=fmt)


@pytest.mark.parametrize("lofmt", ["c64_12", "bf16_12"])
def test_cg_mixed(lofmt, corc):
    dims = (8, 8, 8, 8)
    say(f"cg mixed {lofmt} {dims}")
    links, phases, b = _problem(dims, (0, 0))
    dl = to_dev(links)
    hi = stg.pack_gauge(dims, dl, "c128_12")
    lo = stg.pack_gauge(dims, dl, lofmt)
    x, st, stats = stg.cg_solve(hi, 0.1, to_dev(b), lo=lo, tol=TOL)
    assert stats[0]["reliable_updates"] >= 2
    _check(corc, dims, links, phases, 0.1, b, x.cpu().numpy(), stats, label=lofmt)


@pytest.fixture(params=[0, 1, 2, 4], ids=["fields-auto", "fields-1", "fields-2", "fields-4"])
def fields_per_launch(request):
    """The most fields one hop launch takes (0: automatic, 8 without a tuned choice)."""
    key = stg._lib.STG_TUNE_FIELDS_PER_LAUNCH
    old = stg.stg_get_tuning(key)
    stg.stg_set_tuning(key, request.param)
    yield request.param
    stg.stg_set_tuning(key, old)


@pytest.mark.parametrize("nrhs", [5, 8])
@pytest.mark.parametrize("mode", ["f64", "c64_12"])
def test_cg_multi_rhs(mode, nrhs, corc, fields_per_launch):
    """Chunks of 4 + 1 and 8 fields per launch, with the default launch shapes
    (several threads per site: the most blocks, so the most reduction partials), and
    the same systems chunked at most 1, 2 or 4 fields per launch."""
    dims = (4, 6, 4, 8)
    say(f"cg multi-rhs {mode} nrhs={nrhs} fields per launch {fields_per_launch}")
    links, phases, b = _problem(dims, (2, 0), nrhs)
    dl = to_dev(links)
    hi = stg.pack_gauge(dims, dl, "c128_12")
    lo = stg.pack_gauge(dims, dl, mode) if mode != "f64" else None
    x, st, stats = stg.cg_solve(hi, 0.05, to_dev(b), lo=lo, tol=TOL)
    _check(corc, dims, links, phases, 0.05, b, x.cpu().numpy(), stats, label=mode)


@pytest.mark.parametrize("knobs", [(0, 0), (2, 1), (4, 1)], ids=["natural", "G2-spread", "G4-spread"])
@pytest.mark.parametrize("mode", ["f64", "c64_12"])
def test_cg_multi_rhs_layer_order(mode, knobs, corc):
    """8 right-hand sides with the hop's layer order of the sites and the spread
    epilogue (every thread group finishes its share of the fields), solved to the
    oracle-checked true residual."""
    group, spread = knobs
    dims, nrhs = (4, 6, 4, 8), 8
    say(f"cg multi-rhs layer order {mode} G={group} spread={spread}")
    L = stg._lib
    old = {k: stg.stg_get_tuning(k) for k in (L.STG_TUNE_LAYER_GROUP, L.STG_TUNE_SPREAD_EPILOGUE)}
    stg.stg_set_tuning(L.STG_TUNE_LAYER_GROUP, group)
    stg.stg_set_tuning(L.STG_TUNE_SPREAD_EPILOGUE, spread)
    try:
        links, phases, b = _problem(dims, (2, 1), nrhs)
        dl = to_dev(links)
        hi = stg.pack_gauge(dims, dl, "c128_12")
        lo = stg.pack_gauge(dims, dl, mode) if mode != "f64" else None
        x, st, stats = stg.cg_solve(hi, 0.05, to_dev(b), lo=lo, tol=TOL)
        _check(corc, dims, links, phases, 0.05, b, x.cpu().numpy(), stats, label=mode)
    finally:
        for k, v in old.items():
            stg.stg_set_tuning(k, v)


def test_cg_pure_gauge_exact():
    """b = g * plane wave: the GPU CG returns b / lambda (FP64 path)."""
    dims = (4, 4, 6, 8)
    ge = si.su3_site_field(dims, 21, 0)
    go = si.su3_site_field(dims, 21, 1)
    links = on.pure_gauge_links(dims, ge, go)
    p = on.momenta(dims, (1, 2, 0, 1))
    b = on.site_matrices_apply(ge, on.plane_wave(dims, 0, p, [1.0, 0.5j, -0.25]))[None]
    lam = on.free_eigenvalue(0.1, p)
    g = stg.pack_gauge(dims, to_dev(links), "c128_12")
    x, st, stats = stg.cg_solve(g, 0.1, to_dev(b), tol=1e-12)
    err = rel_norm(x.cpu().numpy(), b / lam)
    say(f"pure gauge: iters {stats[0]['iters']} err {err:.2e}")
    assert err < 1e-12
    assert stats[0]["iters"] <= 2


def test_cg_not_converged_then_warm_restart(corc):
    dims = (8, 8, 8, 8)
    links, phases, b = _problem(dims, (3, 0))
    g = stg.pack_gauge(dims, to_dev(links), "c128_12")
    bd = to_dev(b)
    x, st, stats = stg.cg_solve(g, 0.1, bd, tol=TOL, max_iter=10, check_status=False)
    assert st == 1 and stats[0]["status"] == 1 and stats[0]["iters"] == 10
    res10 = on.true_relative_residual(dims, links, phases, 0.1, b[0], x.cpu().numpy()[0])
    assert abs(stats[0]["true_rel_resid"] - res10) < 1e-6 * res10
    x2, st2, stats2 = stg.cg_solve(g, 0.1, bd, x=x, tol=TOL)
    assert st2 == 0
    _check(corc, dims, links, phases, 0.1, b, x2.cpu().numpy(), stats2, label="warm")


def test_cg_zero_rhs():
    dims = (4, 4, 4, 4)
    links, phases, b = _problem(dims, (4, 0), 2)
    b[1] = 0
    g = stg.pack_gauge(dims, to_dev(links), "c128_12")
    x0 = to_dev(np.ones_like(b))
    x, st, stats = stg.cg_solve(g, 0.1, to_dev(b), x=x0, tol=TOL)
    assert st == 0
    assert torch.count_nonzero(x[1]).item() == 0
    assert on.true_relative_residual(dims, links, phases, 0.1, b[0], x.cpu().numpy()[0]) <= TOL


def test_cg_breakdown_on_nan():
    dims = (4, 4, 4, 4)
    links, phases, b = _problem(dims, (5, 0))
    b[0, 1, 3] = np.nan
    g = stg.pack_gauge(dims, to_dev(links), "c128_12")
    x, st, stats = stg.cg_solve(g, 0.1, to_dev(b), tol=TOL, check_status=False)
    assert st == 2 and stats[0]["status"] == 2


def test_cg_bitwise_reproducible():
    dims = (8, 8, 8, 8)
    links, phases, b = _problem(dims, (6, 0))
    dl = to_dev(links)
    hi = stg.pack_gauge(dims, dl, "c128_12")
    lo = stg.pack_gauge(dims, dl, "c64_12")
    bd = to_dev(b)
    xa, _, sa = stg.cg_solve(hi, 0.1, bd, lo=lo, tol=TOL)
    xb, _, sb = stg.cg_solve(hi, 0.1, bd, lo=lo, tol=TOL)
    assert torch.equal(xa, xb) and sa[0]["iters"] == sb[0]["iters"]


@pytest.mark.parametrize("mode", ["f64", "c64_12"])
def test_multishift(mode, corc, fields_per_launch):
    dims = (4, 6, 4, 8)
    nrhs = 2
    shifts = si.log_shifts(6, 1e-4, 10.0)
    mass = 0.05
    say(f"multishift {mode} shifts={len(shifts)} nrhs={nrhs}")
    links, phases, b = _problem(dims, (7, 0), nrhs)
    dl = to_dev(links)
    hi = stg.pack_gauge(dims, dl, "c128_12")
    lo = stg.pack_gauge(dims, dl, mode) if mode != "f64" else None
    x, st, stats = stg.multishift_cg_solve(hi, mass, shifts, to_dev(b), lo=lo, tol=TOL)
    xn = x.cpu().numpy()
    for k, s in enumerate(shifts):
        _check(corc, dims, links, phases, mass, b, xn[k], stats[k], sigma=s,
               label=f"{mode} shift {s:.1e}")
    # the multi-shift stage retires large shifts earlier
    assert stats[-1][0]["iters"] <= stats[0][0]["iters"]
    if mode == "f64":
        # the FP64 multi-shift stage itself reaches the target: the refinement's first
        # true-residual check finishes almost every system (one update), so the shifted
        # solutions' last steps and the retirement logic are right
        rus = [s["reliable_updates"] for row in stats for s in row]
        say(f"  refinement updates per system: {rus}")
        assert max(rus) <= 2 and sum(r == 1 for r in rus) >= len(rus) // 2


@pytest.mark.parametrize("tps", [2, 4])
@pytest.mark.parametrize("mode", ["f64", "c64_12", "bf16_12"])
def test_cg_threads_per_site(mode, tps, corc):
    """CG with every hop (plain, normal-operator and true-residual epilogues) in the
    kernel that shares a site's directions among 2 or 4 threads; 3 RHS."""
    dims = (8, 4, 6, 8)
    key = stg._lib.STG_TUNE_THREADS_PER_SITE
    old = stg.stg_get_tuning(key)
    stg.stg_set_tuning(key, tps)
    try:
        links, phases, b = _problem(dims, (8, tps), 3)
        dl = to_dev(links)
        hi = stg.pack_gauge(dims, dl, "c128_12")
        lo = stg.pack_gauge(dims, dl, mode) if mode != "f64" else None
        x, st, stats = stg.cg_solve(hi, 0.1, to_dev(b), lo=lo, tol=TOL)
        _check(corc, dims, links, phases, 0.1, b, x.cpu().numpy(), stats,
               label=f"{mode} tps={tps}")
    finally:
        stg.stg_set_tuning(key, old)


# --------------------------------------------------------------------------
# rational function of the normal operator (RHMC: Eq. rooting via Eq. shlineq)
# --------------------------------------------------------------------------
def _rational_bound(dims, links, phases, mass, shifts, coeffs, b, y_ref):
    """|y - y*| <= sum_k |a_k| |x_k - x_k*| <= sum_k |a_k| kappa_k 2 tol |x_k*|."""
    tot = 0.0
    for s, a in zip(shifts, coeffs):
        xk, _, _ = on.cg(dims, links, phases, mass, b, tol=1e-12, sigma=s)
        kappa = (mass * mass + s + 16.0) / (mass * mass + s)
        tot += abs(a) * kappa * 2 * TOL * np.linalg.norm(xk)
    return tot / np.linalg.norm(y_ref)


@pytest.mark.parametrize("mode", ["f64", "c64_12", "bf16_12"])
def test_rational_apply(mode, corc):
    dims = (4, 6, 4, 8)
    shifts = [0.0, 0.003, 0.05, 0.8, 6.0]
    coeffs = [0.11, 0.4, -0.27, 1.9, 7.5]
    a0, mass, nrhs = 0.35, 0.05, 2
    say(f"rational {mode} poles={len(shifts)} nrhs={nrhs}")
    links, phases, b = _problem(dims, (9, 0), nrhs)
    dl = to_dev(links)
    hi = stg.pack_gauge(dims, dl, "c128_12")
    lo = stg.pack_gauge(dims, dl, mode) if mode != "f64" else None
    y, st, stats = stg.rational_apply(hi, mass, shifts, coeffs, a0, to_dev(b), lo=lo, tol=TOL)
    assert st == 0
    yn = y.cpu().numpy()
    for k in range(len(shifts)):
        for j in range(nrhs):
            assert stats[k][j]["status"] == 0 and stats[k][j]["true_rel_resid"] <= TOL
    for j in range(nrhs):
        want, worst = on.rational_apply(dims, links, phases, mass, shifts, coeffs, a0, b[j])
        err = rel_norm(yn[j], want)
        bound = _rational_bound(dims, links, phases, mass, shifts, coeffs, b[j], want)
        say(f"  rhs {j}: |y - y*|/|y*| = {err:.2e} (bound {bound:.2e})")
        assert err <= bound


def test_rational_apply_free_field_and_identity():
    """Unit links: r(A) on a plane wave is the closed-form scalar times the wave; on
    random links, coefficients of a partial-fraction pair give (A+s1)^-1 (A+s2)^-1 b,
    checked by applying (A+s2)(A+s1) with the oracle; a0 alone returns a0 b exactly."""
    dims = (4, 4, 6, 8)
    mass = 0.1
    links = on.unit_links(dims)
    p = on.momenta(dims, (1, 2, 3, 1))
    pw = on.plane_wave(dims, 0, p, np.array([1.0, 0.5j, -0.25 + 0.1j]))[None]
    lam = on.free_eigenvalue(mass, p)
    shifts, coeffs, a0 = [0.0, 0.2, 3.0], [0.5, -0.3, 2.0], 0.125
    g = stg.pack_gauge(dims, to_dev(links), "c128_12")
    y, st, _ = stg.rational_apply(g, mass, shifts, coeffs, a0, to_dev(pw), tol=1e-12)
    want = (a0 + sum(a / (lam + s) for a, s in zip(coeffs, shifts))) * pw
    err = rel_norm(y.cpu().numpy(), want)
    say(f"rational free field: err {err:.2e}")
    assert err <= 1e-10
    # partial fractions on random SU(3) links
    links = si.su3_links(dims, 41, 0)
    phases = on.standard_phases(dims)
    b = si.gaussian_field(dims, 1, 41, 1)
    s1, s2 = 0.01, 0.4
    c = 1.0 / (s2 - s1)
    g = stg.pack_gauge(dims, to_dev(links), "c128_12")
    y, st, _ = stg.rational_apply(g, mass, [s1, s2], [c, -c], 0.0, to_dev(b), tol=1e-12)
    yn = y.cpu().numpy()[0]
    back = on.apply_normal(dims, links, phases, mass,
                           on.apply_normal(dims, links, phases, mass, yn, sigma=s1), sigma=s2)
    ident = np.linalg.norm(back - b[0]) / np.linalg.norm(b[0])
    say(f"rational partial fractions: |(A+s2)(A+s1) y - b|/|b| = {ident:.2e}")
    assert ident <= 1e-9
    # a0 only
    bd = to_dev(b)
    y0, st, _ = stg.rational_apply(g, mass, [0.5], [0.0], 0.75, bd, tol=1e-10)
    assert torch.equal(y0, 0.75 * bd)


def test_tuned_fields_per_launch_reaches_the_solvers(corc, tmp_path):
    """A fields-per-launch choice in the autotuner's table (here read from a cache
    line: at most 2 fields per launch for this lattice and FP64-12) is what the
    solver chunks by when no setting overrides it; the solutions still meet the
    oracle-recomputed residual."""
    dims, nrhs = (4, 6, 4, 8), 5
    key = stg._lib.STG_TUNE_FIELDS_PER_LAUNCH
    old = stg.stg_get_tuning(key)
    stg.stg_set_tuning(key, 0)
    cache = tmp_path / "fields.jsonl"
    cache.write_text('{"arch": "gfx950", "dims": [4, 6, 4, 8], "fmt": 1, '
                     '"fields_per_launch": 2, "us_per_field": 1.0}\n')
    lib = stg.library()
    lib.stg_autotune_clear()
    try:
        assert stg.stg_autotune_load(str(cache)) == 1
        assert stg.stg_autotune_fields_lookup(dims, stg.STG_LINK_C128_12) == 2
        links, phases, b = _problem(dims, (3, 0), nrhs)
        hi = stg.pack_gauge(dims, to_dev(links), "c128_12")
        x, st, stats = stg.cg_solve(hi, 0.05, to_dev(b), tol=TOL)
        _check(corc, dims, links, phases, 0.05, b, x.cpu().numpy(), stats, label="tuned cap 2")
    finally:
        lib.stg_autotune_clear()
        stg.stg_set_tuning(key, old)
