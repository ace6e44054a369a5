"""GPU staples of the tree-level Symanzik gauge force (gauge_staples) against the
FP64 oracle.

Parity: every entry of Sigma_mu(x) for every link on small lattices (one and
several 64-link blocks, a ragged last block, several x0/x1/x2 tiles of the
kernel's visiting order, extents of 2 where the 1x2 paths wrap onto themselves),
with one and two threads per link, and sampled links at 32^4 computed one by one
by the oracle.

Inputs of the oracle are the links as the format holds them: FP64-18 as given;
the 12-real formats keep rows 0 and 1 (FP64 exactly, FP32 rounded to nearest even,
BF16 rounded to nearest even to 8 significant bits) and rebuild row 2 as
conj(row0 x row1), done here in FP64.

Tolerances (max |GPU - oracle| over all entries, absolute; entries of a staple are
bounded by the weight sum 6|c0| + 18|c1| since every path is a product of unitary
matrices):  each 3x3 product of unitary matrices has entry errors <= 3 * 2 u with
u the unit roundoff of the arithmetic, a 5-link path takes 4 products, the 24 paths
add with their weights, and the reconstruction of row 2 adds a few u per link; 64 u
times the weight sum covers this with margin.  FP64: u = 2^-53; FP32: u = 2^-24.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1701_00426_amd as stg  # noqa: E402
import seeded_inputs as si  # noqa: E402
from oracle import oracle_np as on  # noqa: E402

from gpu_common import say, to_dev  # noqa: E402

C0, C1 = on.SYMANZIK_C0, on.SYMANZIK_C1
UNIT = {"c128_18": 2.0 ** -53, "c128_12": 2.0 ** -53, "c64_12": 2.0 ** -24, "bf16_12": 2.0 ** -24}
FORMATS = list(UNIT)


def _tol(fmt, c0, c1):
    return 64 * UNIT[fmt] * (6 * abs(c0) + 18 * abs(c1))


def _bf16(x):
    """Round float64 values to bfloat16 (8 significant bits), nearest even."""
    m, e = np.frexp(x)
    return np.ldexp(np.rint(m * 256.0), e - 8)


def as_stored(links, fmt):
    """The full matrices the kernel works with for links given in FP64."""
    if fmt == "c128_18":
        return links
    r = links[:, :2].copy()
    if fmt == "c64_12":
        r = r.astype(np.complex64).astype(np.complex128)
    elif fmt == "bf16_12":
        r = _bf16(r.real) + 1j * _bf16(r.imag)
    out = np.empty_like(links)
    out[:, :2] = r
    out[:, 2] = np.conj(np.cross(r[:, 0], r[:, 1], axis=1))
    return out


def gpu_staples(dims, links, fmt, c0=C0, c1=C1):
    gauge = stg.pack_gauge(dims, to_dev(links), fmt)
    s = stg.gauge_staples(gauge, c0, c1)
    torch.cuda.synchronize()
    return s.cpu().numpy().astype(np.complex128)


@pytest.fixture(params=[0, 1, 2], ids=["threads-auto", "threads-1", "threads-2"])
def staple_threads(request):
    """Threads per link of the staple kernel: automatic (2 for FP64 links, 1 for FP32
    ones), one thread, or the two sides of the link on separate waves."""
    key = stg._lib.STG_TUNE_STAPLE_THREADS
    old = stg.stg_get_tuning(key)
    stg.stg_set_tuning(key, request.param)
    yield request.param
    stg.stg_set_tuning(key, old)


@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (6, 4, 2, 10), (4, 6, 8, 10),
                                  (2, 8, 4, 6), (34, 4, 6, 2), (32, 8, 4, 6)])
def test_staples_parity(dims, fmt, staple_threads):
    links = si.su3_links(dims, 1701, 40, sum(dims))
    got = gpu_staples(dims, links, fmt)
    want = on.staples(dims, as_stored(links, fmt))
    err = float(np.max(np.abs(got - want)))
    say(f"staples {fmt} {dims} threads={staple_threads}: max abs err {err:.3e} "
        f"(tol {_tol(fmt, C0, C1):.1e})")
    assert err <= _tol(fmt, C0, C1)


@pytest.mark.parametrize("c0,c1", [(1.0, 0.0), (0.0, 1.0), (0.7, 0.45), (-2.5, 3.0)])
def test_staples_weights(c0, c1):
    dims = (4, 4, 6, 4)
    links = si.su3_links(dims, 1701, 41, 0)
    got = gpu_staples(dims, links, "c128_18", c0, c1)
    want = on.staples(dims, links, c0, c1)
    assert float(np.max(np.abs(got - want))) <= _tol("c128_18", c0, c1)


@pytest.mark.parametrize("fmt", FORMATS)
def test_staples_unit_links(fmt):
    """Unit links: (6 c0 + 18 c1) I on every link, in every format."""
    dims = (4, 2, 4, 6)
    got = gpu_staples(dims, on.unit_links(dims), fmt)
    want = np.zeros_like(got)
    for a in range(3):
        want[:, a, a, :] = 6 * C0 + 18 * C1
    assert float(np.max(np.abs(got - want))) <= _tol(fmt, C0, C1)


def test_staples_launch_shape_and_repeat_identical():
    """The XCD block order changes only which CU computes a link: bitwise equal
    results, and two calls agree bitwise (with the automatic threads per link)."""
    dims = (8, 4, 4, 6)
    links = si.su3_links(dims, 1701, 42, 0)
    gauge = stg.pack_gauge(dims, to_dev(links), "c128_12")
    key = stg._lib.STG_TUNE_XCD_REMAP
    old = stg.stg_get_tuning(key)
    try:
        outs = []
        for remap in (0, 1, 1):
            stg.stg_set_tuning(key, remap)
            outs.append(stg.gauge_staples(gauge).clone())
        torch.cuda.synchronize()
    finally:
        stg.stg_set_tuning(key, old)
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[1], outs[2])


def test_staples_output_argument_checked():
    dims = (4, 4, 4, 4)
    gauge = stg.pack_gauge(dims, to_dev(si.su3_links(dims, 1701, 43, 0)), "c64_12")
    wrong = torch.empty((8, 3, 3, on.half_volume(dims)), dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):
        stg.gauge_staples(gauge, out=wrong)
    out = torch.empty((8, 3, 3, on.half_volume(dims)), dtype=torch.complex64, device="cuda")
    assert stg.gauge_staples(gauge, out=out) is out


@pytest.fixture(scope="module")
def big_links():
    dims = (32, 32, 32, 32)
    say("generating 32^4 links")
    return dims, si.su3_links(dims, 1701, 44, 0)


@pytest.mark.parametrize("fmt", ["c128_12", "c128_18", "c64_12", "bf16_12"])
def test_staples_32_4_sampled(big_links, fmt):
    """32^4 (the size the benchmark times): every slot, sampled links including both
    ends of the half-index range, against the oracle link by link."""
    dims, links = big_links
    gauge = stg.pack_gauge(dims, to_dev(links), fmt)
    s = stg.gauge_staples(gauge)
    torch.cuda.synchronize()
    vh = on.half_volume(dims)
    pick = np.concatenate([[0, 1, vh - 1], si.rng(45, 0).integers(0, vh, size=40)])
    stored = None
    err = 0.0
    for slot in range(8):
        got = s[slot][:, :, torch.from_numpy(pick).to(s.device)].cpu().numpy()
        if fmt.startswith("c128"):
            want = on.staples_at(dims, links, slot, pick)
        else:
            if stored is None:
                stored = as_stored(links, fmt)
            want = on.staples_at(dims, stored, slot, pick)
        err = max(err, float(np.max(np.abs(got.astype(np.complex128) - want))))
    say(f"staples 32^4 {fmt}: max abs err over {8 * len(pick)} links {err:.3e}")
    assert err <= _tol(fmt, C0, C1)
