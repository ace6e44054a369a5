"""GPU pure-gauge molecular dynamics (gauge_momentum_update, gauge_link_update) against
the FP64 oracle.

Parity: the momentum update P - eps F(U) and the link update exp(i eps P) U entry by
entry on small lattices (FP64-18 and FP64-12 links, one and two threads per link),
at sampled links of 32^4, and whole leapfrog trajectories against the oracle's, with
the energy error and reversibility measured on the GPU's own trajectory.

Tolerances: F entries are bounded by (beta/3)(6|c0| + 18|c1|) (products of unitary
matrices), and the kernel's sums agree with the oracle's to a few units of 2^-53
per product: 64 u times that bound times eps, plus the rounding of P.  exp(i eps P) U
agrees with scipy's expm to ~1e-15 (entries of modulus <= 1): 1e-13.
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

U53 = 2.0 ** -53
BETA, EPS = 5.5, 0.02


def _as_stored(links, fmt):
    if fmt == "c128_18":
        return links
    out = links.copy()
    out[:, 2] = np.conj(np.cross(links[:, 0], links[:, 1], axis=1))
    return out


def _mom_tol(beta, eps, c0=on.SYMANZIK_C0, c1=on.SYMANZIK_C1):
    return 64 * U53 * (beta / 3.0) * (6 * abs(c0) + 18 * abs(c1)) * abs(eps) + 16 * U53 * 4


@pytest.fixture(params=[0, 1, 2], ids=["threads-auto", "threads-1", "threads-2"])
def staple_threads(request):
    key = stg._lib.STG_TUNE_STAPLE_THREADS
    old = stg.stg_get_tuning(key)
    stg.stg_set_tuning(key, request.param)
    yield request.param
    stg.stg_set_tuning(key, old)


@pytest.mark.parametrize("fmt", ["c128_18", "c128_12"])
@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (6, 4, 2, 10), (32, 8, 4, 6)])
def test_momentum_update_parity(dims, fmt, staple_threads):
    links = si.su3_links(dims, 1701, 95, sum(dims))
    mom = si.traceless_hermitian_field(dims, 96, sum(dims))
    gauge = stg.pack_gauge(dims, to_dev(links), fmt)
    p = to_dev(mom)
    stg.gauge_momentum_update(gauge, p, BETA, EPS)
    torch.cuda.synchronize()
    want = on.momentum_update(dims, _as_stored(links, fmt), mom, BETA, EPS)
    err = float(np.max(np.abs(p.cpu().numpy() - want)))
    say(f"momentum update {fmt} {dims} threads={staple_threads}: max abs err {err:.2e}")
    assert err <= _mom_tol(BETA, EPS)


@pytest.mark.parametrize("fmt", ["c128_18", "c128_12"])
@pytest.mark.parametrize("eps", [0.02, -0.5, 0.0])
def test_link_update_parity(fmt, eps):
    dims = (4, 6, 2, 4)
    links = si.su3_links(dims, 1701, 97, 0)
    mom = si.traceless_hermitian_field(dims, 98, 0)
    gauge = stg.pack_gauge(dims, to_dev(links), fmt)
    stg.gauge_link_update(gauge, to_dev(mom), eps)
    torch.cuda.synchronize()
    want = on.link_update(_as_stored(links, fmt), mom, eps)
    got = gauge.links.cpu().numpy()
    if fmt == "c128_12":
        # the packed 12-real field is a raw byte buffer: rows 0 and 1 as complex128
        got = got.view(np.complex128).reshape(8, 2, 3, -1)
        want = want[:, :2]
    err = float(np.max(np.abs(got - want)))
    say(f"link update {fmt} eps={eps}: max abs err {err:.2e}")
    assert err <= 1e-13


def _gpu_leapfrog(gauge, p, beta, eps, n):
    stg.gauge_momentum_update(gauge, p, beta, 0.5 * eps)
    for k in range(n):
        stg.gauge_link_update(gauge, p, eps)
        stg.gauge_momentum_update(gauge, p, beta, eps if k < n - 1 else 0.5 * eps)


def test_leapfrog_matches_oracle_conserves_and_reverses():
    """The GPU trajectory equals the oracle's; its energy error falls by ~4 when eps
    halves (second-order integrator; random links give large forces, so dH itself is
    not small at these eps); flipping the momenta and integrating back returns to the
    start."""
    dims, n = (4, 2, 4, 4), 6
    links = si.su3_links(dims, 1701, 99, 0)
    mom = si.traceless_hermitian_field(dims, 100, 0)
    h0 = on.md_hamiltonian(dims, links, mom, BETA)
    dhs = []
    for eps, steps in ((2 * EPS, n // 2), (EPS, n)):
        g2 = stg.pack_gauge(dims, to_dev(links), "c128_18")
        p2 = to_dev(mom)
        _gpu_leapfrog(g2, p2, BETA, eps, steps)
        torch.cuda.synchronize()
        dhs.append(on.md_hamiltonian(dims, g2.links.cpu().numpy(), p2.cpu().numpy(), BETA) - h0)
    gauge = stg.pack_gauge(dims, to_dev(links), "c128_18")
    p = to_dev(mom)
    _gpu_leapfrog(gauge, p, BETA, EPS, n)
    torch.cuda.synchronize()
    u1, p1 = gauge.links.cpu().numpy(), p.cpu().numpy()
    uo, po = on.leapfrog(dims, links, mom, BETA, EPS, n)
    eu, ep = float(np.max(np.abs(u1 - uo))), float(np.max(np.abs(p1 - po)))
    say(f"leapfrog: |U - U_oracle| {eu:.2e}, |P - P_oracle| {ep:.2e}, dH {dhs}")
    assert eu <= 1e-11 and ep <= 1e-11
    assert 3.5 <= dhs[0] / dhs[1] <= 4.5
    p.neg_()
    _gpu_leapfrog(gauge, p, BETA, EPS, n)
    torch.cuda.synchronize()
    er = float(np.max(np.abs(gauge.links.cpu().numpy() - links)))
    ep0 = float(np.max(np.abs(p.cpu().numpy() + mom)))
    say(f"leapfrog reversed: |U - U0| {er:.2e}, |P + P0| {ep0:.2e}")
    assert er <= 1e-11 and ep0 <= 1e-11


def test_momentum_update_32_4_sampled():
    dims = (32, 32, 32, 32)
    say("generating 32^4 links and momenta")
    links = si.su3_links(dims, 1701, 101, 0)
    vh = on.half_volume(dims)
    mom = np.zeros((8, 3, 3, vh), dtype=np.complex128)
    gauge = stg.pack_gauge(dims, to_dev(links), "c128_12")
    p = to_dev(mom)
    stg.gauge_momentum_update(gauge, p, BETA, EPS)
    torch.cuda.synchronize()
    pick = np.concatenate([[0, 1, vh - 1], si.rng(102, 0).integers(0, vh, size=40)])
    err = 0.0
    for slot in range(8):
        sig = on.staples_at(dims, links, slot, pick)
        m = np.einsum("abn,bcn->acn", links[slot][:, :, pick], sig)
        want = EPS * (BETA / 3.0) * on.traceless_hermitian(1j * m)
        got = p[slot][:, :, torch.from_numpy(pick).to(p.device)].cpu().numpy()
        err = max(err, float(np.max(np.abs(got - want))))
    say(f"momentum update 32^4 sampled: max abs err {err:.2e}")
    assert err <= _mom_tol(BETA, EPS)


U24 = 2.0 ** -24


def _as_stored_c64(links):
    """FP32-12 links as the kernel sees them: rows 0 and 1 rounded to complex64, row 2
    rebuilt as conj(row0 x row1) (here in FP64)."""
    out = links.copy()
    out[:, :2] = links[:, :2].astype(np.complex64).astype(np.complex128)
    out[:, 2] = np.conj(np.cross(out[:, 0], out[:, 1], axis=1))
    return out


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 10), (32, 8, 4, 6)])
def test_momentum_update_fp32(dims, staple_threads):
    """Single-precision molecular dynamics: FP32-12 links, complex64 momenta, FP32
    arithmetic; tolerance 64 u (u = 2^-24) on the force term and on the momenta."""
    links = si.su3_links(dims, 1701, 103, sum(dims))
    mom = si.traceless_hermitian_field(dims, 104, sum(dims)).astype(np.complex64)
    gauge = stg.pack_gauge(dims, to_dev(links), "c64_12")
    p = to_dev(mom)
    stg.gauge_momentum_update(gauge, p, BETA, EPS)
    torch.cuda.synchronize()
    want = on.momentum_update(dims, _as_stored_c64(links), mom.astype(np.complex128), BETA, EPS)
    err = float(np.max(np.abs(p.cpu().numpy().astype(np.complex128) - want)))
    tol = 64 * U24 * ((BETA / 3.0) * 8.5 * EPS + float(np.max(np.abs(mom))))
    say(f"momentum update FP32 {dims} threads={staple_threads}: max abs err {err:.2e} "
        f"(tol {tol:.1e})")
    assert err <= tol


def test_link_update_fp32():
    dims = (4, 6, 2, 4)
    links = si.su3_links(dims, 1701, 105, 0)
    mom = si.traceless_hermitian_field(dims, 106, 0).astype(np.complex64)
    gauge = stg.pack_gauge(dims, to_dev(links), "c64_12")
    stg.gauge_link_update(gauge, to_dev(mom), 0.05)
    torch.cuda.synchronize()
    want = on.link_update(_as_stored_c64(links), mom.astype(np.complex128), 0.05)[:, :2]
    # memory order: slot, chunk k, site, pair; chunk k holds entries 2k, 2k+1 of
    # (U00 U01 U02 U10 U11 U12)
    vh = on.half_volume(dims)
    got = gauge.links.cpu().numpy().view(np.complex64).reshape(8, 3, vh, 2)
    got = np.transpose(got, (0, 1, 3, 2)).reshape(8, 6, vh).reshape(8, 2, 3, vh)
    err = float(np.max(np.abs(got.astype(np.complex128) - want)))
    say(f"link update FP32: max abs err {err:.2e}")
    assert err <= 32 * U24


@pytest.mark.parametrize("fmt", ["c128_12", "c64_12"])
def test_md_step_32_4_sampled(fmt):
    """One step as the benchmark times it at 32^4 (beta 5.5, eps 0.01, FP64-12 with
    complex128 momenta or FP32-12 with complex64 ones): the momentum update from
    nonzero momenta, then the link update with the new momenta; sampled links of every
    slot against the oracle link by link."""
    dims, beta, eps = (32, 32, 32, 32), 5.5, 0.01
    say(f"generating 32^4 links and momenta ({fmt})")
    links = si.su3_links(dims, 1701, 107, 0)
    mom = si.traceless_hermitian_field(dims, 108, 0)
    vh = on.half_volume(dims)
    fp64 = fmt == "c128_12"
    if not fp64:
        mom = mom.astype(np.complex64).astype(np.complex128)
    stored = _as_stored(links, fmt) if fp64 else _as_stored_c64(links)
    gauge = stg.pack_gauge(dims, to_dev(links), fmt)
    p = to_dev(mom if fp64 else mom.astype(np.complex64))
    stg.gauge_momentum_update(gauge, p, beta, eps)
    stg.gauge_link_update(gauge, p, eps)
    torch.cuda.synchronize()
    pick = np.concatenate([[0, 1, vh - 1], si.rng(109, 0).integers(0, vh, size=24)])
    idx = torch.from_numpy(pick).to(p.device)
    if fp64:
        u_now = gauge.links.cpu().numpy().view(np.complex128).reshape(8, 2, 3, vh)
        ptol = _mom_tol(beta, eps)
        utol = 1e-13 + abs(eps) * 3 * ptol
    else:
        u_now = gauge.links.cpu().numpy().view(np.complex64).reshape(8, 3, vh, 2)
        u_now = np.transpose(u_now, (0, 1, 3, 2)).reshape(8, 2, 3, vh)
        ptol = 64 * U24 * ((beta / 3.0) * 8.5 * eps + float(np.max(np.abs(mom))))
        utol = 32 * U24 + abs(eps) * 3 * ptol
    ep = eu = 0.0
    for slot in range(8):
        sig = on.staples_at(dims, stored, slot, pick)
        m = np.einsum("abn,bcn->acn", stored[slot][:, :, pick], sig)
        p1 = mom[slot][:, :, pick] + eps * (beta / 3.0) * on.traceless_hermitian(1j * m)
        u1 = on.link_update(stored[slot][None, :, :, pick], p1[None], eps)[0]
        got_p = p[slot][:, :, idx].cpu().numpy().astype(np.complex128)
        ep = max(ep, float(np.max(np.abs(got_p - p1))))
        eu = max(eu, float(np.max(np.abs(u_now[slot][:, :, pick].astype(np.complex128) - u1[:2]))))
    say(f"MD step 32^4 {fmt}: momenta max abs err {ep:.2e} (tol {ptol:.1e}), links {eu:.2e} "
        f"(tol {utol:.1e})")
    assert ep <= ptol and eu <= utol
