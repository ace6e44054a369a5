"""The operator-side entry points under HIP graph capture.

dirac_apply_eo / dirac_apply_oe, stg_apply_normal, gauge_staples, fermion_force,
stout_smear, stout_force_backprop and the molecular-dynamics pair
gauge_momentum_update + gauge_link_update only enqueue kernels on the caller's stream
(no allocation, no copy, no memset, no host synchronisation), so a caller can record
them into a graph and replay it.  Each graph is replayed several times with eager work
and synchronisations in between, and every replay must equal the eager calls bitwise
(the same kernels in the same order).  The solvers read convergence flags on the host
and are not capturable by design.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1701_00426_amd as stg  # noqa: E402
import seeded_inputs as si  # noqa: E402

from gpu_common import say, to_dev  # noqa: E402

REPLAYS = 3


def _capture(fn):
    """Warm fn up on a side stream, then record one call of it into a graph."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def _busy_eager():
    """Unrelated eager work between replays."""
    a = torch.randn(1 << 20, device="cuda")
    (a * 2.0 + 1.0).sum().item()


def test_operators_in_a_graph():
    dims, rho, mass = (4, 6, 2, 8), 0.15, 0.1
    vh = stg.half_volume(dims)
    links = to_dev(si.su3_links(dims, 1701, 130, 0))
    gauge = stg.pack_gauge(dims, links, "c128_12")
    v_odd = to_dev(si.gaussian_field(dims, 2, 131, 0))
    v_even = to_dev(si.gaussian_field(dims, 2, 132, 0))
    xs = to_dev(si.gaussian_field(dims, 3, 133, 0))
    coeffs = [0.5, -0.25, 1.0]
    sp = torch.randn((8, 3, 3, vh), dtype=torch.complex128, device="cuda")

    outs = {
        "eo": torch.empty_like(v_even), "oe": torch.empty_like(v_odd),
        "normal": torch.empty_like(v_even), "tmp": torch.empty_like(v_odd),
        "staples": torch.empty((8, 3, 3, vh), dtype=torch.complex128, device="cuda"),
        "force": torch.empty((8, 3, 3, vh), dtype=torch.complex128, device="cuda"),
        "y": torch.empty_like(xs),
        "stout": torch.empty((8, 3, 3, vh), dtype=torch.complex128, device="cuda"),
        "back": torch.empty((8, 3, 3, vh), dtype=torch.complex128, device="cuda"),
        "ws": torch.empty((8, 3, 3, vh), dtype=torch.complex128, device="cuda"),
    }

    def calls():
        stg.dirac_apply_eo(gauge, v_odd, outs["eo"])
        stg.dirac_apply_oe(gauge, v_even, outs["oe"])
        stg.stg_apply_normal(gauge, mass, v_even, out_even=outs["normal"], tmp_odd=outs["tmp"])
        stg.gauge_staples(gauge, out=outs["staples"])
        stg.fermion_force(gauge, coeffs, xs, y_odd=outs["y"], out=outs["force"])
        stg.stout_smear(gauge, rho, out=outs["stout"])
        stg.stout_force_backprop(gauge, rho, sp, out=outs["back"], ws=outs["ws"])

    calls()
    torch.cuda.synchronize()
    want = {k: v.clone() for k, v in outs.items() if k not in ("tmp", "ws")}
    g = _capture(calls)
    for r in range(REPLAYS):
        for v in outs.values():
            v.fill_(float("nan"))
        _busy_eager()
        g.replay()
        torch.cuda.synchronize()
        for k, w in want.items():
            assert torch.equal(outs[k], w), f"replay {r}: {k} differs"
        say(f"replay {r}: all {len(want)} outputs bitwise equal to the eager calls")


@pytest.mark.parametrize("fmt", ["c128_12", "c64_12"])
def test_md_step_in_a_graph(fmt):
    """An MD step (momentum update, then link update) recorded once: every replay
    advances the state exactly as one more eager step does."""
    dims, beta, eps = (4, 4, 6, 4), 5.5, 0.02
    links = to_dev(si.su3_links(dims, 1701, 134, 0))
    mom0 = si.traceless_hermitian_field(dims, 135, 0)
    cdt = torch.complex128 if fmt == "c128_12" else torch.complex64
    g_graph = stg.pack_gauge(dims, links, fmt)
    g_eager = stg.pack_gauge(dims, links, fmt)
    p_graph = to_dev(mom0).to(cdt)
    p_eager = p_graph.clone()

    def step(gauge, p):
        stg.gauge_momentum_update(gauge, p, beta, eps)
        stg.gauge_link_update(gauge, p, eps)

    # the warm-up call is one step on the graph's state (capture records, runs nothing)
    graph = _capture(lambda: step(g_graph, p_graph))
    step(g_eager, p_eager)
    torch.cuda.synchronize()
    assert torch.equal(g_graph.links, g_eager.links) and torch.equal(p_graph, p_eager)
    for r in range(REPLAYS):
        _busy_eager()
        graph.replay()
        step(g_eager, p_eager)
        torch.cuda.synchronize()
        assert torch.equal(g_graph.links, g_eager.links), f"replay {r}: links differ"
        assert torch.equal(p_graph, p_eager), f"replay {r}: momenta differ"
    say(f"MD step {fmt}: {REPLAYS} replays bitwise equal to eager steps")
    assert np.isfinite(p_graph.abs().max().item())
