"""GPU parity of the staggered hop, the normal operator, link packing and the
compensated dot products, through the C ABI, against the FP64 oracle."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1701_00426_amd as stg  # noqa: E402
import seeded_inputs as si  # noqa: E402
from oracle import oracle_np as on  # noqa: E402

from gpu_common import DEV, TOL, TOL_ARITH, rel_max, rel_norm, say, stored_links, to_dev  # noqa: E402

SHAPES = [(2, 2, 2, 2), (4, 4, 4, 4), (8, 8, 8, 8), (4, 6, 8, 10), (6, 4, 2, 10), (2, 8, 2, 6)]


def _bf16_bits(x):
    """Round-to-nearest-even of float64 values to bfloat16 bit patterns (exact)."""
    m, e = np.frexp(x)
    y = np.ldexp(np.rint(m * 256.0) / 256.0, e)
    return (y.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


@pytest.mark.parametrize("dims", [(4, 6, 4, 8), (2, 2, 2, 2)])
def test_pack_links_exact(dims, corc):
    say(f"pack_links {dims}")
    links = si.su3_links(dims, 5, 5)
    vh = on.half_volume(dims)
    dl = to_dev(links)
    two = links[:, :2]                                     # (8, 2, 3, Vh)
    got12 = stg.stg_pack_links(dims, dl, "c128_12").cpu().numpy().view(np.complex128)
    assert np.array_equal(got12.reshape(8, 2, 3, vh), two)
    got32 = stg.stg_pack_links(dims, dl, "c64_12").cpu().numpy().view(np.float32)
    e = two.reshape(8, 6, vh).astype(np.complex64)         # RNE per component
    want32 = np.stack([e[:, 0::2], e[:, 1::2]], axis=-1)   # (8, 3, Vh, 2) complex64
    assert np.array_equal(got32, want32.view(np.float32).reshape(-1))
    gotbf = stg.stg_pack_links(dims, dl, "bf16_12").cpu().numpy().view(np.uint16)
    e6 = two.reshape(8, 6, vh)
    bits = np.stack([_bf16_bits(e6.real), _bf16_bits(e6.imag)], axis=-1)  # (8, 6, Vh, 2)
    first = bits[:, :4].transpose(0, 2, 1, 3).reshape(8, vh, 8)
    second = bits[:, 4:].transpose(0, 2, 1, 3).reshape(8, vh, 4)
    want = np.concatenate([first.reshape(-1), second.reshape(-1)])
    assert np.array_equal(gotbf, want)


@pytest.mark.parametrize("tps", [0, 1])
@pytest.mark.parametrize("fmt", ["c128_18", "c128_12", "c64_12", "bf16_12"])
@pytest.mark.parametrize("dims", SHAPES)
def test_hop_parity(dims, fmt, tps, corc, tuning):
    """D_eo and D_oe on random SU(3) links, standard phases computed in-kernel, with
    the automatic launch shape and with one thread per site."""
    say(f"hop {fmt} {dims} tps={tps}")
    tuning(stg._lib.STG_TUNE_THREADS_PER_SITE, tps)
    links = si.su3_links(dims, 1701, 7, 0)
    phases = on.standard_phases(dims)
    g = stg.pack_gauge(dims, to_dev(links), fmt)
    cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
    for par, fn, name in ((0, stg.dirac_apply_eo, "eo"), (1, stg.dirac_apply_oe, "oe")):
        v = si.gaussian_field(dims, 1, 426, 7, par)
        out = fn(g, to_dev(v).to(cdt))
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.complex128)
        want = corc.dslash(dims, links, phases, par, v)
        err = rel_max(got, want)
        say(f"  D_{name} max rel err {err:.2e} (norm {rel_norm(got, want):.2e})")
        assert err <= TOL[fmt]


@pytest.fixture
def staged_neighbours():
    """Neighbour staging on, with one thread per site (the kernel that stages)."""
    keys = (stg._lib.STG_TUNE_STAGE_NEIGHBOURS, stg._lib.STG_TUNE_THREADS_PER_SITE)
    old = [stg.stg_get_tuning(k) for k in keys]
    stg.stg_set_tuning(keys[0], 1)
    stg.stg_set_tuning(keys[1], 1)
    yield
    for k, v in zip(keys, old):
        stg.stg_set_tuning(k, v)


@pytest.mark.parametrize("spt", [1, 2])
@pytest.mark.parametrize("nrhs", [1, 2, 3])
@pytest.mark.parametrize("fmt", ["c128_18", "c128_12", "c64_12", "bf16_12"])
@pytest.mark.parametrize("dims", [(4, 6, 8, 10), (6, 4, 2, 10), (2, 2, 2, 2), (16, 2, 18, 2),
                                  (128, 2, 2, 4), (132, 2, 2, 2)])
def test_hop_staged_neighbours(dims, fmt, nrhs, spt, corc, staged_neighbours):
    """The hop with x0/x1 neighbours read from an LDS copy of the block's rows
    (one or two fields per launch, N0 <= 128; wider rows fall back to the plain
    kernel) against the oracle, with one and two chunks of sites per block."""
    say(f"hop staged {fmt} {dims} nrhs={nrhs} spt={spt}")
    key = stg._lib.STG_TUNE_SITES_PER_THREAD
    old = stg.stg_get_tuning(key)
    stg.stg_set_tuning(key, spt)
    try:
        links = si.su3_links(dims, 1701, 8, 0)
        phases = on.standard_phases(dims)
        g = stg.pack_gauge(dims, to_dev(links), fmt)
        cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
        for par, fn in ((0, stg.dirac_apply_eo), (1, stg.dirac_apply_oe)):
            v = si.gaussian_field(dims, nrhs, 426, 8, par)
            got = fn(g, to_dev(v).to(cdt)).cpu().numpy().astype(np.complex128)
            want = corc.dslash(dims, links, phases, par, v)
            for j in range(nrhs):
                assert rel_max(got[j], want[j]) <= TOL[fmt]
    finally:
        stg.stg_set_tuning(key, old)


@pytest.fixture
def tuning():
    """Sets hop tuning knobs for one test and restores them afterwards."""
    saved = {}

    def set_(key, value):
        if key not in saved:
            saved[key] = stg.stg_get_tuning(key)
        stg.stg_set_tuning(key, value)

    yield set_
    for key, value in saved.items():
        stg.stg_set_tuning(key, value)


@pytest.mark.parametrize("tps", [2, 4])
@pytest.mark.parametrize("nrhs", [1, 2, 3, 8, 13])
@pytest.mark.parametrize("fmt", ["c128_18", "c128_12", "c64_12", "bf16_12"])
@pytest.mark.parametrize("dims", [(4, 6, 8, 10), (6, 4, 2, 10), (2, 2, 2, 2), (10, 2, 4, 2)])
def test_hop_threads_per_site(dims, fmt, nrhs, tps, corc, tuning):
    """The hop with the directions of a site shared by 2 or 4 threads (partials
    combined in LDS; FP64 with 8 fields at 4 threads falls back to one thread) for
    both parities, explicit and standard phases, against the oracle."""
    say(f"hop tps={tps} {fmt} {dims} nrhs={nrhs}")
    tuning(stg._lib.STG_TUNE_THREADS_PER_SITE, tps)
    links = si.su3_links(dims, 1701, 9, 0)
    phases = on.standard_phases(dims)
    cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
    for explicit in (False, True):
        ph = si.real_link_field(dims, 9, 1) if explicit else phases
        g = stg.pack_gauge(dims, to_dev(links), fmt,
                           phases_f64=to_dev(ph) if explicit else None)
        for par, fn in ((0, stg.dirac_apply_eo), (1, stg.dirac_apply_oe)):
            v = si.gaussian_field(dims, nrhs, 426, 9, par)
            got = fn(g, to_dev(v).to(cdt)).cpu().numpy().astype(np.complex128)
            want = corc.dslash(dims, links, ph, par, v)
            for j in range(nrhs):
                assert rel_max(got[j], want[j]) <= TOL[fmt]


@pytest.mark.parametrize("group", [0, 2, 3, 4])
@pytest.mark.parametrize("tps", [1, 2, 4])
@pytest.mark.parametrize("fmt", ["c128_12", "c64_12", "bf16_12"])
@pytest.mark.parametrize("dims", [(4, 6, 8, 12), (6, 4, 2, 10), (2, 2, 2, 2)])
def test_hop_layer_order_and_spread_epilogue(dims, fmt, tps, group, corc, tuning):
    """The layer order of the output sites (G x3 planes per group) and the spread
    epilogue (every thread group finishes its share of the fields): D_oe, D_eo and
    the normal operator of 8 and 4 fields against the oracle; the spread epilogue
    gives results bitwise equal to group 0 finishing every field."""
    say(f"layer order G={group} tps={tps} {fmt} {dims}")
    L = stg._lib
    tuning(L.STG_TUNE_THREADS_PER_SITE, tps)
    tuning(L.STG_TUNE_LAYER_GROUP, group)
    links = si.su3_links(dims, 1701, 14, 0)
    phases = on.standard_phases(dims)
    g = stg.pack_gauge(dims, to_dev(links), fmt)
    cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
    for nrhs in (8, 4):
        v = si.gaussian_field(dims, nrhs, 426, 14, nrhs)
        dv = to_dev(v).to(cdt)
        res = {}
        for spread in (0, 1):
            tuning(L.STG_TUNE_SPREAD_EPILOGUE, spread)
            res[spread] = [stg.dirac_apply_oe(g, dv).cpu().numpy(),
                           stg.dirac_apply_eo(g, dv).cpu().numpy(),
                           stg.stg_apply_normal(g, 0.2, dv, sigma=0.01).cpu().numpy()]
        for a, b in zip(res[0], res[1]):
            assert np.array_equal(a, b)
        oe, eo, nm = (x.astype(np.complex128) for x in res[1])
        want_oe = corc.dslash(dims, links, phases, 1, v)
        want_eo = corc.dslash(dims, links, phases, 0, v)
        for j in range(nrhs):
            assert rel_max(oe[j], want_oe[j]) <= TOL[fmt]
            assert rel_max(eo[j], want_eo[j]) <= TOL[fmt]
            want_nm = corc.apply_normal(dims, links, phases, 0.2, v[j], sigma=0.01)
            assert rel_max(nm[j], want_nm) <= TOL[fmt]


@pytest.mark.parametrize("tps", [2, 4])
@pytest.mark.parametrize("fmt", ["c128_12", "c64_12"])
def test_apply_normal_threads_per_site(fmt, tps, corc, tuning):
    """The normal-operator epilogue (q = diag p - D_eo D_oe p) in the shared-site kernel."""
    dims = (4, 6, 4, 6)
    tuning(stg._lib.STG_TUNE_THREADS_PER_SITE, tps)
    links = si.su3_links(dims, 11, 1)
    phases = on.standard_phases(dims)
    g = stg.pack_gauge(dims, to_dev(links), fmt)
    cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
    v = si.gaussian_field(dims, 5, 11, 2)
    got = stg.stg_apply_normal(g, 0.3, to_dev(v).to(cdt), sigma=0.05).cpu().numpy()
    for j in range(5):
        want = corc.apply_normal(dims, links, phases, 0.3, v[j], sigma=0.05)
        assert rel_max(got[j].astype(np.complex128), want) <= TOL[fmt]


@pytest.mark.parametrize("fmt", ["c128_12", "c64_12"])
def test_hop_explicit_phases(fmt, corc):
    """Arbitrary real per-link phases read from memory (the paper's backfield array)."""
    dims = (4, 6, 2, 8)
    say(f"hop explicit phases {fmt} {dims}")
    links = si.su3_links(dims, 3, 3)
    phases = si.real_link_field(dims, 3, 4)
    g = stg.pack_gauge(dims, to_dev(links), fmt, phases_f64=to_dev(phases))
    cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
    for par in (0, 1):
        v = si.gaussian_field(dims, 2, 3, 5 + par)
        fn = stg.dirac_apply_eo if par == 0 else stg.dirac_apply_oe
        got = fn(g, to_dev(v).to(cdt)).cpu().numpy().astype(np.complex128)
        want = corc.dslash(dims, links, phases, par, v)
        assert rel_max(got, want) <= TOL[fmt]


@pytest.mark.parametrize("tps", [0, 1])
@pytest.mark.parametrize("nrhs", [2, 3, 5, 8, 11])
@pytest.mark.parametrize("fmt", ["c128_12", "c64_12"])
def test_hop_multi_rhs(nrhs, fmt, tps, corc, tuning):
    """Several fields per launch (chunks of 8/4/3/2/1): each equals its own hop."""
    dims = (4, 4, 6, 4)
    say(f"hop multi-rhs {fmt} nrhs={nrhs} tps={tps}")
    tuning(stg._lib.STG_TUNE_THREADS_PER_SITE, tps)
    links = si.su3_links(dims, 9, nrhs)
    phases = on.standard_phases(dims)
    g = stg.pack_gauge(dims, to_dev(links), fmt)
    cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
    v = si.gaussian_field(dims, nrhs, 9, 1)
    got = stg.dirac_apply_oe(g, to_dev(v).to(cdt)).cpu().numpy().astype(np.complex128)
    want = corc.dslash(dims, links, phases, 1, v)
    for j in range(nrhs):
        assert rel_max(got[j], want[j]) <= TOL[fmt]
    # the last field alone: the same values up to the order of additions (the
    # launch shape may differ with the number of fields)
    single = stg.dirac_apply_oe(g, to_dev(v[nrhs - 1:]).to(cdt)).cpu().numpy()
    assert rel_max(single[0].astype(np.complex128), got[nrhs - 1]) <= \
        (1e-14 if fmt == "c128_12" else 1e-6)


@pytest.mark.parametrize("cap", [1, 2, 4, 8])
@pytest.mark.parametrize("fmt", ["c128_12", "c64_12"])
def test_fields_per_launch(fmt, cap, corc, tuning):
    """11 fields chunked at most 1, 2, 4 or 8 per launch: D_oe, D_eo and the normal
    operator of every field match the oracle."""
    dims, nrhs = (6, 4, 2, 10), 11
    say(f"fields per launch {cap} {fmt}")
    tuning(stg._lib.STG_TUNE_FIELDS_PER_LAUNCH, cap)
    links = si.su3_links(dims, 13, 0)
    phases = on.standard_phases(dims)
    g = stg.pack_gauge(dims, to_dev(links), fmt)
    cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
    v = si.gaussian_field(dims, nrhs, 13, 1)
    dv = to_dev(v).to(cdt)
    oe = stg.dirac_apply_oe(g, dv).cpu().numpy().astype(np.complex128)
    eo = stg.dirac_apply_eo(g, dv).cpu().numpy().astype(np.complex128)
    nm = stg.stg_apply_normal(g, 0.2, dv).cpu().numpy().astype(np.complex128)
    want_oe = corc.dslash(dims, links, phases, 1, v)
    want_eo = corc.dslash(dims, links, phases, 0, v)
    for j in range(nrhs):
        assert rel_max(oe[j], want_oe[j]) <= TOL[fmt]
        assert rel_max(eo[j], want_eo[j]) <= TOL[fmt]
        assert rel_max(nm[j], corc.apply_normal(dims, links, phases, 0.2, v[j])) <= TOL[fmt]


@pytest.mark.parametrize("fmt", ["c128_12", "c64_12", "bf16_12"])
def test_apply_normal(fmt, corc):
    dims = (4, 6, 4, 6)
    say(f"apply_normal {fmt}")
    links = si.su3_links(dims, 11, 0)
    phases = on.standard_phases(dims)
    g = stg.pack_gauge(dims, to_dev(links), fmt)
    cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
    v = si.gaussian_field(dims, 3, 11, 1)
    got = stg.stg_apply_normal(g, 0.3, to_dev(v).to(cdt), sigma=0.05).cpu().numpy()
    for j in range(3):
        want = corc.apply_normal(dims, links, phases, 0.3, v[j], sigma=0.05)
        assert rel_max(got[j].astype(np.complex128), want) <= TOL[fmt]


def test_anti_hermiticity_full_size():
    """32^4 FP64-12 (the benchmark configuration): <chi, D_eo psi> = -<D_oe chi, psi>,
    evaluated with the library's compensated dot products."""
    dims = (32, 32, 32, 32)
    say(f"anti-hermiticity {dims}")
    links = si.su3_links(dims, 1701, 1, 0)
    g = stg.pack_gauge(dims, to_dev(links), "c128_12")
    chi = to_dev(si.gaussian_field(dims, 1, 1, 2))
    psi = to_dev(si.gaussian_field(dims, 1, 1, 3))
    a = stg.stg_dot(chi, stg.dirac_apply_eo(g, psi))[0]
    b = stg.stg_dot(stg.dirac_apply_oe(g, chi), psi)[0]
    nrm = math.sqrt(stg.stg_dot(chi, chi)[0].real * stg.stg_dot(psi, psi)[0].real)
    say(f"  |a + b| / |chi||psi| = {abs(a + b) / nrm:.2e}")
    assert abs(a + b) / nrm < 1e-13


@pytest.mark.parametrize("fmt", ["c128_12", "c64_12", "bf16_12"])
def test_hop_sampled_full_size(fmt):
    """32^4 in the launch configuration the benchmark times: 4096 sampled output sites
    of D_eo and D_oe against the oracle evaluated site by site; the compressed formats
    also against the oracle on the links as stored and the complex64 input, where
    only the FP32 arithmetic differs."""
    dims = (32, 32, 32, 32)
    say(f"sampled full size {fmt} {dims}")
    links = si.su3_links(dims, 1701, 1, 0)
    phases = on.standard_phases(dims)
    g = stg.pack_gauge(dims, to_dev(links), fmt)
    cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
    vh = on.half_volume(dims)
    rng = np.random.default_rng(5)
    hs = np.concatenate([rng.choice(vh, 4000, replace=False),
                         np.arange(48), vh - 1 - np.arange(48)])
    stored = stored_links(links, fmt) if fmt in TOL_ARITH else None
    for par in (0, 1):
        v = si.gaussian_field(dims, 1, 426, 1, par)
        fn = stg.dirac_apply_eo if par == 0 else stg.dirac_apply_oe
        vd = to_dev(v).to(cdt)
        out = fn(g, vd).cpu().numpy().astype(np.complex128)
        want = on.dslash(dims, links, phases, par, v, hs=hs)
        err = rel_max(out[..., hs], want)
        say(f"  parity {par} sampled max rel err {err:.2e}")
        assert err <= TOL[fmt]
        if stored is not None:
            v32 = vd.cpu().numpy().astype(np.complex128)
            want_s = on.dslash(dims, stored, phases, par, v32, hs=hs)
            err_s = rel_max(out[..., hs], want_s)
            say(f"  parity {par} vs oracle on the stored links: {err_s:.2e}")
            assert err_s <= TOL_ARITH[fmt]


@pytest.mark.parametrize("nrhs", [1, 3, 8])
@pytest.mark.parametrize("fmt", ["c64_12", "bf16_12"])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 8, 8, 8), (4, 6, 8, 10)])
def test_hop_against_stored_links(dims, fmt, nrhs, corc):
    """Every output entry of D_eo and D_oe for the FP32 formats against the FP64
    oracle on the links as the format stores them (row 2 rebuilt from the rounded
    rows) and on the complex64 input: the FP32 arithmetic alone, to 1e-6."""
    say(f"hop vs stored links {fmt} {dims} nrhs={nrhs}")
    links = si.su3_links(dims, 1701, 9, 0)
    phases = on.standard_phases(dims)
    stored = stored_links(links, fmt)
    g = stg.pack_gauge(dims, to_dev(links), fmt)
    for par in (0, 1):
        v = si.gaussian_field(dims, nrhs, 426, 9, par)
        vd = to_dev(v).to(torch.complex64)
        fn = stg.dirac_apply_eo if par == 0 else stg.dirac_apply_oe
        got = fn(g, vd).cpu().numpy().astype(np.complex128)
        v32 = vd.cpu().numpy().astype(np.complex128)
        want = corc.dslash(dims, stored, phases, par, v32)
        for j in range(nrhs):
            assert rel_max(got[j], want[j]) <= TOL_ARITH[fmt], (par, j)


def test_pure_gauge_eigenvector_gpu():
    """U = g(x) g(x+mu)^dag: the GPU normal operator maps g * plane wave to lambda times it."""
    dims = (4, 6, 4, 8)
    ge = si.su3_site_field(dims, 4, 0)
    go = si.su3_site_field(dims, 4, 1)
    links = on.pure_gauge_links(dims, ge, go)
    for fmt in ("c128_18", "c128_12", "c64_12"):
        g = stg.pack_gauge(dims, to_dev(links), fmt)
        for n in ((1, 2, 0, 3), (0, 0, 0, 0), (1, 5, 3, 7)):
            p = on.momenta(dims, n)
            v = on.site_matrices_apply(ge, on.plane_wave(dims, 0, p, [1.0, -0.5j, 0.25]))
            cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
            got = stg.stg_apply_normal(g, 0.1, to_dev(v[None]).to(cdt)).cpu().numpy()[0]
            lam = on.free_eigenvalue(0.1, p)
            err = float(np.max(np.abs(got - lam * v)))
            assert err < (1e-12 if fmt.startswith("c128") else 1e-6), (fmt, n, err)


def test_dot_compensated_vs_fsum():
    """Ill-conditioned sums: the library's dot agrees with math.fsum (correctly rounded)."""
    rng = np.random.default_rng(3)
    n = 3 * 20000 + 17
    for trial in range(4):
        x = rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))
        x = np.concatenate([x, -x[: n // 2]])            # heavy cancellation
        x[-1] += 1.0
        xc = (x + 0j).astype(np.complex128)
        y = np.ones_like(xc)
        got = stg.stg_dot(to_dev(xc[None]), to_dev(y[None]))[0].real
        want = math.fsum(x.tolist())
        say(f"  trial {trial}: dot {got!r} fsum {want!r}")
        assert abs(got - want) <= 4 * np.spacing(abs(want)) + 1e-300


def test_dot_fp32_products_exact():
    rng = np.random.default_rng(4)
    x = (rng.standard_normal((2, 3000)) + 1j * rng.standard_normal((2, 3000))).astype(np.complex64)
    y = (rng.standard_normal((2, 3000)) + 1j * rng.standard_normal((2, 3000))).astype(np.complex64)
    got = stg.stg_dot(to_dev(x), to_dev(y))
    for j in range(2):
        xd = x[j].astype(np.complex128)
        yd = y[j].astype(np.complex128)
        prod = np.conj(xd) * yd
        want = complex(math.fsum(prod.real.tolist()), math.fsum(prod.imag.tolist()))
        assert abs(got[j] - want) <= 4 * np.spacing(abs(want))


def test_deterministic_hop_and_dot():
    dims = (8, 8, 8, 8)
    links = si.su3_links(dims, 8, 8)
    g = stg.pack_gauge(dims, to_dev(links), "c128_12")
    v = to_dev(si.gaussian_field(dims, 1, 8, 9))
    a = stg.dirac_apply_eo(g, v)
    b = stg.dirac_apply_eo(g, v)
    assert torch.equal(a, b)
    assert stg.stg_dot(a, v) == stg.stg_dot(b, v)


@pytest.mark.parametrize("fmt,nrhs", [("c64_12", 1), ("c64_12", 3), ("c128_12", 2),
                                      ("bf16_12", 1), ("c64_12", 8), ("c128_12", 5)])
def test_autotune_choice_and_parity(fmt, nrhs, corc, tmp_path):
    """stg_autotune times the launch shapes on the caller's buffers, keeps a valid
    choice in the process-wide table and the cache file (read back by
    stg_autotune_load), with several fields also the fields per launch, and the hop
    launched with those choices matches the oracle."""
    dims = (8, 6, 4, 10)
    say(f"autotune {fmt} nrhs={nrhs}")
    links = si.su3_links(dims, 1701, 12, 0)
    phases = on.standard_phases(dims)
    g = stg.pack_gauge(dims, to_dev(links), fmt)
    cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
    cache = tmp_path / "tune.jsonl"
    lib = stg.library()
    lib.stg_autotune_clear()
    try:
        choice = stg.stg_autotune(g, nrhs, cache_path=str(cache))
        say(f"  choice {choice}")
        assert choice["xcd_remap"] in (0, 1)
        assert choice["sites_per_thread"] in (1, 2, 4, 8)
        assert choice["stage_neighbours"] in (0, 1)
        assert choice["threads_per_site"] in (1, 2, 4)
        assert choice["us"] > 0
        if choice["threads_per_site"] > 1:
            assert choice["sites_per_thread"] == 1 and choice["stage_neighbours"] == 0
        if nrhs >= 2:
            assert choice["fields_per_launch"] in (1, 2, 4, 8)
        v = si.gaussian_field(dims, nrhs, 426, 12, 1)
        got = stg.dirac_apply_eo(g, to_dev(v).to(cdt)).cpu().numpy().astype(np.complex128)
        want = corc.dslash(dims, links, phases, 0, v)
        for j in range(nrhs):
            assert rel_max(got[j], want[j]) <= TOL[fmt]
        lib.stg_autotune_clear()
        assert stg.stg_autotune_lookup(dims, g.fmt, choice_nr(nrhs)) is None
        assert stg.stg_autotune_fields_lookup(dims, g.fmt) is None
        assert stg.stg_autotune_load(str(cache)) == (2 if nrhs >= 2 else 1)
        again = stg.stg_autotune_lookup(dims, g.fmt, choice_nr(nrhs))
        shape_keys = [k for k in choice if k not in ("us", "fields_per_launch")]
        assert {k: again[k] for k in shape_keys} == {k: choice[k] for k in shape_keys}
        assert abs(again["us"] - choice["us"]) <= 1e-3
        if nrhs >= 2:
            assert stg.stg_autotune_fields_lookup(dims, g.fmt) == choice["fields_per_launch"]
    finally:
        lib.stg_autotune_clear()


def choice_nr(nrhs):
    """Fields per launch of the first chunk of nrhs fields (8, 4, or nrhs below 4)."""
    return 8 if nrhs >= 8 else 4 if nrhs >= 4 else nrhs


def test_hop_sampled_links_above_4gib():
    """The largest buffers: FP64-18 links on 48^3 x 72 take 4.59 GB, so the byte
    offsets of the last sites' links do not fit in 32 bits.  D_eo and D_oe at sampled
    output sites, the last 64 half-sites included, against the oracle site by site."""
    dims = (48, 48, 48, 72)
    vh = on.half_volume(dims)
    assert 8 * 9 * 16 * vh > 2 ** 32
    say(f"generating {dims} links ({8 * 9 * 16 * vh / 1e9:.2f} GB)")
    links = si.su3_links(dims, 1701, 14, 0)
    phases = on.standard_phases(dims)
    g = stg.pack_gauge(dims, to_dev(links), "c128_18")
    rng = np.random.default_rng(14)
    hs = np.concatenate([rng.choice(vh, 2000, replace=False), np.arange(32),
                         vh - 1 - np.arange(64)])
    for par in (0, 1):
        v = si.gaussian_field(dims, 1, 14, 1, par)
        fn = stg.dirac_apply_eo if par == 0 else stg.dirac_apply_oe
        out = fn(g, to_dev(v))
        got = out[..., torch.from_numpy(hs).to(out.device)].cpu().numpy()
        want = on.dslash(dims, links, phases, par, v, hs=hs)
        err = rel_max(got, want)
        say(f"  parity {par}: sampled max rel err {err:.2e}")
        assert err <= TOL["c128_18"]
