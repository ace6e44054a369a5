"""GPU solvers in the single-reduction form of CG (Chronopoulos and Gear,
STG_TUNE_CG_FORM = 2) through the C ABI: FP64 and mixed precision (FP32-12, BF16-12)
on one and several right-hand sides, on a small lattice (one field: the reductions
finished inside the update, three launches per iteration) and above that size
(finalize kernel), the iteration cap with a warm restart, a NaN breakdown, a
pure-gauge eigenvector, bitwise reproducibility, and the multi-shift solver whose
refinement stage runs in this form.

Parity bar as for the classic form: every returned solution has an FP64 true
relative residual <= 1e-10 recomputed by the oracle and lies within the
conditioning bound of the oracle's own solution; iteration counts stay within 10 %
of the classic form's (the two forms are the same iteration in exact arithmetic)."""
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


@pytest.fixture
def cg_form():
    key = stg._lib.STG_TUNE_CG_FORM
    old = stg.stg_get_tuning(key)

    def set_(v):
        stg.stg_set_tuning(key, v)

    yield set_
    stg.stg_set_tuning(key, old)


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
        kappa = (mass * mass + sigma + 16.0) / (mass * mass + sigma)
        assert err <= kappa * 2 * TOL


# (4, 6, 8, 10): Vh = 960, the fused path for one field; (16, 16, 16, 18): Vh = 36864,
# above the fused limit, so one field goes through the finalize kernel
@pytest.mark.parametrize("nrhs", [1, 3, 8])
@pytest.mark.parametrize("mode", ["f64", "c64_12", "bf16_12"])
@pytest.mark.parametrize("dims", [(4, 6, 8, 10), (16, 16, 16, 18)])
def test_cgcg_solve(dims, mode, nrhs, corc, cg_form):
    if dims[3] == 18 and nrhs == 8:
        pytest.skip("the 8-field case is covered on the small lattice (oracle time)")
    mass = 0.05 if dims[3] == 10 else 0.2
    say(f"cgcg {mode} {dims} nrhs={nrhs}")
    links, phases, b = _problem(dims, (40, nrhs), nrhs)
    dl = to_dev(links)
    hi = stg.pack_gauge(dims, dl, "c128_12")
    lo = stg.pack_gauge(dims, dl, mode) if mode != "f64" else None
    bd = to_dev(b)
    cg_form(1)
    _, st1, s1 = stg.cg_solve(hi, mass, bd, lo=lo, tol=TOL)
    cg_form(2)
    x, st, stats = stg.cg_solve(hi, mass, bd, lo=lo, tol=TOL)
    assert st == 0 and st1 == 0
    _check(corc, dims, links, phases, mass, b, x.cpu().numpy(), stats, label=f"cgcg {mode}")
    for a, c in zip(s1, stats):
        say(f"  iterations classic {a['iters']} single-reduction {c['iters']}")
        assert abs(a["iters"] - c["iters"]) <= max(8, 0.1 * a["iters"])


def test_cgcg_not_converged_then_warm_restart(corc, cg_form):
    cg_form(2)
    dims = (8, 8, 8, 8)
    links, phases, b = _problem(dims, (41, 0))
    g = stg.pack_gauge(dims, to_dev(links), "c128_12")
    bd = to_dev(b)
    x, st, stats = stg.cg_solve(g, 0.1, bd, tol=TOL, max_iter=10, check_status=False)
    assert st == 1 and stats[0]["status"] == 1 and stats[0]["iters"] == 10
    res10 = on.true_relative_residual(dims, links, phases, 0.1, b[0], x.cpu().numpy()[0])
    assert abs(stats[0]["true_rel_resid"] - res10) < 1e-6 * res10
    x2, st2, stats2 = stg.cg_solve(g, 0.1, bd, x=x, tol=TOL)
    assert st2 == 0
    _check(corc, dims, links, phases, 0.1, b, x2.cpu().numpy(), stats2, label="warm")


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (16, 16, 16, 18)])
def test_cgcg_breakdown_on_nan(dims, cg_form):
    cg_form(2)
    links, phases, b = _problem(dims, (42, 0))
    b[0, 1, 3] = np.nan
    g = stg.pack_gauge(dims, to_dev(links), "c128_12")
    x, st, stats = stg.cg_solve(g, 0.1, to_dev(b), tol=TOL, check_status=False)
    assert st == 2 and stats[0]["status"] == 2


def test_cgcg_pure_gauge_exact(cg_form):
    """b = g * plane wave: the solution b / lambda after one update."""
    cg_form(2)
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
    say(f"pure gauge (single reduction): iters {stats[0]['iters']} err {err:.2e}")
    assert err < 1e-12
    assert stats[0]["iters"] <= 2


def test_cgcg_bitwise_reproducible(cg_form):
    cg_form(2)
    dims = (8, 8, 8, 8)
    links, phases, b = _problem(dims, (43, 0))
    dl = to_dev(links)
    hi = stg.pack_gauge(dims, dl, "c128_12")
    lo = stg.pack_gauge(dims, dl, "c64_12")
    bd = to_dev(b)
    xa, _, sa = stg.cg_solve(hi, 0.1, bd, lo=lo, tol=TOL)
    xb, _, sb = stg.cg_solve(hi, 0.1, bd, lo=lo, tol=TOL)
    assert torch.equal(xa, xb) and sa[0]["iters"] == sb[0]["iters"]


@pytest.mark.parametrize("mode", ["f64", "c64_12"])
def test_cgcg_multishift(mode, corc, cg_form):
    """The multi-shift solver with its refinement stage in the single-reduction form."""
    cg_form(2)
    dims = (4, 6, 4, 8)
    nrhs = 2
    shifts = si.log_shifts(6, 1e-4, 10.0)
    mass = 0.05
    links, phases, b = _problem(dims, (44, 0), nrhs)
    dl = to_dev(links)
    hi = stg.pack_gauge(dims, dl, "c128_12")
    lo = stg.pack_gauge(dims, dl, mode) if mode != "f64" else None
    x, st, stats = stg.multishift_cg_solve(hi, mass, shifts, to_dev(b), lo=lo, tol=TOL)
    assert st == 0
    xn = x.cpu().numpy()
    for k, s in enumerate(shifts):
        for j in range(nrhs):
            res = on.true_relative_residual(dims, links, phases, mass, b[j], xn[k, j], sigma=s)
            assert res <= TOL
