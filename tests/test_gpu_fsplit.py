"""GPU parity of the field-split hop (several fields per launch split over the waves
of a block, the block's links shared through LDS; STG_TUNE_FIELD_SPLIT) against the
FP64 oracle: D_oe, D_eo and the normal operator for 2, 3, 4 and 8 fields, one and
two fields per wave, the automatic choice and the split turned off, half-index and
layer order, lattices whose half volume is and is not a multiple of the 64-site
block; and CG with 8 right-hand sides on it."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1701_00426_amd as stg  # noqa: E402
import seeded_inputs as si  # noqa: E402
from oracle import oracle_np as on  # noqa: E402

from gpu_common import TOL, rel_max, say, to_dev  # noqa: E402


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


# Vh: 960 (15 blocks of 64), 240 (ragged: 3.75 blocks), 8 (one partial block),
# 1536 with N3 = 12 for the layer order
DIMS = [(4, 6, 8, 10), (6, 4, 2, 10), (2, 2, 2, 2), (4, 4, 8, 12)]


@pytest.mark.parametrize("group", [0, 3])
@pytest.mark.parametrize("fpw", [1, 2, 0, -1])
@pytest.mark.parametrize("fmt", ["c128_12", "c64_12", "bf16_12"])
@pytest.mark.parametrize("dims", DIMS)
def test_fsplit_hop_and_normal(dims, fmt, fpw, group, corc, tuning):
    L = stg._lib
    tuning(L.STG_TUNE_FIELD_SPLIT, fpw)
    tuning(L.STG_TUNE_LAYER_GROUP, group)
    links = si.su3_links(dims, 1701, 31, 0)
    phases = on.standard_phases(dims)
    g = stg.pack_gauge(dims, to_dev(links), fmt)
    cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
    for nrhs in (8, 4, 3, 2):
        if fpw > 0 and nrhs % fpw:
            continue
        say(f"fsplit {fmt} {dims} nrhs={nrhs} fields/wave={fpw} G={group}")
        v = si.gaussian_field(dims, nrhs, 426, 31, nrhs)
        dv = to_dev(v).to(cdt)
        oe = stg.dirac_apply_oe(g, dv).cpu().numpy().astype(np.complex128)
        eo = stg.dirac_apply_eo(g, dv).cpu().numpy().astype(np.complex128)
        nm = stg.stg_apply_normal(g, 0.2, dv, sigma=0.01).cpu().numpy().astype(np.complex128)
        want_oe = corc.dslash(dims, links, phases, 1, v)
        want_eo = corc.dslash(dims, links, phases, 0, v)
        for j in range(nrhs):
            assert rel_max(oe[j], want_oe[j]) <= TOL[fmt]
            assert rel_max(eo[j], want_eo[j]) <= TOL[fmt]
            want_nm = corc.apply_normal(dims, links, phases, 0.2, v[j], sigma=0.01)
            assert rel_max(nm[j], want_nm) <= TOL[fmt]


@pytest.mark.parametrize("fpw", [1, 2])
@pytest.mark.parametrize("fmt", ["c128_12", "c64_12"])
def test_fsplit_explicit_phases(fmt, fpw, corc, tuning):
    """Arbitrary real per-link phases read from memory, 8 fields."""
    dims = (4, 6, 2, 8)
    tuning(stg._lib.STG_TUNE_FIELD_SPLIT, fpw)
    links = si.su3_links(dims, 1701, 32, 0)
    ph = si.real_link_field(dims, 32, 1)
    g = stg.pack_gauge(dims, to_dev(links), fmt, phases_f64=to_dev(ph))
    cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
    for par, fn in ((0, stg.dirac_apply_eo), (1, stg.dirac_apply_oe)):
        v = si.gaussian_field(dims, 8, 426, 32, par)
        got = fn(g, to_dev(v).to(cdt)).cpu().numpy().astype(np.complex128)
        want = corc.dslash(dims, links, ph, par, v)
        for j in range(8):
            assert rel_max(got[j], want[j]) <= TOL[fmt]


@pytest.mark.parametrize("fpw", [1, 2])
@pytest.mark.parametrize("mode", ["f64", "c64_12", "bf16_12"])
def test_fsplit_cg_multi_rhs(mode, fpw, corc, tuning):
    """8 right-hand sides solved with the field-split hop to the oracle-checked FP64
    true residual 1e-10."""
    dims, nrhs, mass = (4, 6, 4, 8), 8, 0.05
    say(f"fsplit cg {mode} fields/wave={fpw}")
    tuning(stg._lib.STG_TUNE_FIELD_SPLIT, fpw)
    links = si.su3_links(dims, 1701, 33, 0)
    phases = on.standard_phases(dims)
    b = si.gaussian_field(dims, nrhs, 426, 33, 0)
    dl = to_dev(links)
    hi = stg.pack_gauge(dims, dl, "c128_12")
    lo = stg.pack_gauge(dims, dl, mode) if mode != "f64" else None
    x, st, stats = stg.cg_solve(hi, mass, to_dev(b), lo=lo, tol=1e-10)
    assert st == 0
    xn = x.cpu().numpy()
    for j in range(nrhs):
        res = on.true_relative_residual(dims, links, phases, mass, b[j], xn[j])
        say(f"  rhs {j}: iters {stats[j]['iters']} oracle resid {res:.2e}")
        assert stats[j]["status"] == 0 and res <= 1e-10
