"""Planted mistakes in a copy of the NumPy oracle must each fail at least one pin.

This shows the pins are strong enough that a plausible slip in the oracle (a
dropped term, a wrong sign or index, a transposed operand, a wrong phase or
boundary sign, a wrong normalisation) cannot pass unnoticed.  CPU only.
"""
import numpy as np
import pytest

from oracle import oracle_np as on

import pins


def make_dslash(mutation):
    def dslash(dims, links, phases, out_parity, vin):
        x = on.coords(dims, out_parity)
        in_parity = 1 - out_parity
        out = np.zeros(vin.shape, dtype=np.complex128)
        for mu in range(4):
            if mutation == "drop_direction" and mu == 2:
                continue
            step_f = 1
            if mutation == "wrong_neighbour" and mu == 1:
                step_f = -1 if out_parity == 0 else 1
            hf = on.half_index(dims, on.shifted(dims, x, mu, step_f))
            hb = on.half_index(dims, on.shifted(dims, x, mu, -1))
            uf = links[2 * mu + out_parity]
            ub = links[2 * mu + in_parity][:, :, hb]
            if mutation == "wrong_slot":
                ub = links[2 * mu + out_parity][:, :, hb]
            pf = phases[2 * mu + out_parity]
            pb = phases[2 * mu + in_parity][hb]
            if mutation == "backward_phase_at_x":
                pb = phases[2 * mu + out_parity]
            if mutation == "transposed_forward":
                fwd = np.einsum("bah,...bh->...ah", uf, vin[..., :, hf])
            else:
                fwd = np.einsum("abh,...bh->...ah", uf, vin[..., :, hf])
            if mutation == "no_dagger":
                bwd = np.einsum("abh,...bh->...ah", ub, vin[..., :, hb])
            elif mutation == "transpose_no_conj":
                bwd = np.einsum("bah,...bh->...ah", ub, vin[..., :, hb])
            else:
                bwd = np.einsum("bah,...bh->...ah", np.conj(ub), vin[..., :, hb])
            if mutation == "plus_backward":
                out += pf * fwd + pb * bwd
            else:
                out += pf * fwd - pb * bwd
        scale = 1.0 if mutation == "no_half" else 0.5
        return scale * out
    return dslash


def make_phases(mutation):
    def phases_fn(dims):
        ph = on.standard_phases(dims)
        if mutation == "periodic_time":
            for parity in (0, 1):
                x = on.coords(dims, parity)
                ph[6 + parity] = on.eta(x, 3)
        elif mutation == "eta_inclusive":
            for parity in (0, 1):
                x = on.coords(dims, parity)
                for mu in range(4):
                    s = sum(x[nu] for nu in range(mu + 1))
                    e = np.where(s & 1, -1.0, 1.0)
                    if mu == 3:
                        e = e * np.where(x[3] == dims[3] - 1, -1.0, 1.0)
                    ph[2 * mu + parity] = e
        elif mutation == "no_phases":
            ph[:] = 1.0
        elif mutation == "boundary_on_x2":
            for parity in (0, 1):
                x = on.coords(dims, parity)
                ph[6 + parity] = on.eta(x, 3)
                ph[4 + parity] = on.eta(x, 2) * np.where(x[2] == dims[2] - 1, -1.0, 1.0)
        return ph
    return phases_fn


OPERATOR_MUTANTS = ["drop_direction", "wrong_neighbour", "wrong_slot", "backward_phase_at_x",
                    "transposed_forward", "no_dagger", "transpose_no_conj", "plus_backward",
                    "no_half"]
PHASE_MUTANTS = ["periodic_time", "eta_inclusive", "no_phases", "boundary_on_x2"]


def _failed(res):
    return [name for name, (err, tol) in res.items() if not err <= tol]


def test_unmutated_copy_passes():
    res = pins.run_operator_pins(make_dslash(None), make_phases(None))
    assert _failed(res) == []


@pytest.mark.parametrize("mutation", OPERATOR_MUTANTS)
def test_operator_mutant_detected(mutation):
    res = pins.run_operator_pins(make_dslash(mutation), on.standard_phases)
    assert _failed(res), f"planted mistake {mutation} passed every pin"


@pytest.mark.parametrize("mutation", PHASE_MUTANTS)
def test_phase_mutant_detected(mutation):
    res = pins.run_operator_pins(on.dslash, make_phases(mutation))
    assert _failed(res), f"planted phase mistake {mutation} passed every pin"


# --------------------------------------------------------------------------
# Staples: planted mistakes in a copy of the staple sum
# --------------------------------------------------------------------------


def _path_product(dims, links, start, steps, mutation):
    y = start.copy()
    w = np.repeat(np.eye(3, dtype=np.complex128)[:, :, None], start.shape[1], axis=2)
    for mu, s in steps:
        if s > 0:
            u = on.link_matrices(dims, links, y, mu)
            y = on.shifted(dims, y, mu, +1)
        else:
            y = on.shifted(dims, y, mu, -1)
            u = on.link_matrices(dims, links, y, mu)
            if mutation == "transpose_no_conj":
                u = np.transpose(u, (1, 0, 2))
            elif mutation != "no_dagger":
                u = np.conj(np.transpose(u, (1, 0, 2)))
        if mutation == "reversed_product":
            w = np.einsum("abn,bcn->acn", u, w)
        else:
            w = np.einsum("abn,bcn->acn", w, u)
    return w


def make_staples(mutation):
    def staples_fn(dims, links, c0, c1):
        out = np.zeros((8, 3, 3, on.half_volume(dims)), dtype=np.complex128)
        for parity in (0, 1):
            x = on.coords(dims, parity)
            for mu in range(4):
                start = x if mutation == "start_at_x" else on.shifted(dims, x, mu, +1)
                for nu in range(4):
                    if nu == mu:
                        continue
                    three, five = on.staple_paths(mu, nu)
                    if mutation == "drop_lower_plaquette":
                        three = three[:1]
                    if mutation == "drop_tall":
                        five = [five[0], five[1], five[3], five[4]]
                    if mutation == "rect_ends_wrong":
                        five = [p[:-1] + [(mu, -1)] if p[-1] == (mu, 1) else p for p in five]
                    if mutation == "tall_along_mu":
                        five = five[:2] + [[(mu, 1), (mu, 1), (nu, 1), (mu, -1), (nu, -1)]] \
                            + five[3:]
                    w3, w5 = (c1, c0) if mutation == "swapped_weights" else (c0, c1)
                    for p in three:
                        out[2 * mu + parity] += w3 * _path_product(dims, links, start, p,
                                                                   mutation)
                    for p in five:
                        out[2 * mu + parity] += w5 * _path_product(dims, links, start, p,
                                                                   mutation)
        return out
    return staples_fn


STAPLE_MUTANTS = ["start_at_x", "drop_lower_plaquette", "drop_tall", "rect_ends_wrong",
                  "tall_along_mu", "swapped_weights", "no_dagger", "transpose_no_conj",
                  "reversed_product"]


def test_unmutated_staple_copy_passes():
    assert _failed(pins.run_staple_pins(make_staples(None))) == []


@pytest.mark.parametrize("mutation", STAPLE_MUTANTS)
def test_staple_mutant_detected(mutation):
    res = pins.run_staple_pins(make_staples(mutation), first_failure=True)
    assert _failed(res), f"planted staple mistake {mutation} passed every pin"


# --------------------------------------------------------------------------
# Fermion force: planted mistakes in a copy of the outer-product formula
# --------------------------------------------------------------------------


def make_force(mutation):
    def force_fn(dims, phases, coeffs, x_even, y_odd):
        out = np.zeros((8, 3, 3, on.half_volume(dims)), dtype=np.complex128)
        for parity in (0, 1):
            z = on.coords(dims, parity)
            for mu in range(4):
                step = -1 if mutation == "backward_neighbour" and mu == 2 else 1
                hf = on.half_index(dims, on.shifted(dims, z, mu, step))
                ph = phases[2 * mu + parity]
                if mutation == "no_phase":
                    ph = 1.0
                if mutation == "phase_at_neighbour":
                    ph = phases[2 * mu + 1 - parity][hf]
                for a, x, y in zip(coeffs, x_even, y_odd):
                    if parity == 0:
                        t = np.einsum("an,bn->abn", y[:, hf], np.conj(x))
                        if mutation == "transposed_outer":
                            t = np.einsum("an,bn->abn", np.conj(x), y[:, hf])
                        out[2 * mu] += a * ph * t
                    else:
                        t = np.einsum("an,bn->abn", x[:, hf], np.conj(y))
                        if mutation == "conj_swapped":
                            t = np.einsum("an,bn->abn", np.conj(x[:, hf]), y)
                        sign = 1.0 if mutation == "odd_sign" else -1.0
                        out[2 * mu + 1] += sign * a * ph * t
        if mutation == "half":
            out *= 0.5
        return out
    return force_fn


FORCE_MUTANTS = ["backward_neighbour", "no_phase", "phase_at_neighbour", "transposed_outer",
                 "conj_swapped", "odd_sign", "half"]


def test_unmutated_force_copy_passes():
    assert _failed(pins.run_force_pins(make_force(None))) == []


@pytest.mark.parametrize("mutation", FORCE_MUTANTS)
def test_force_mutant_detected(mutation):
    res = pins.run_force_pins(make_force(mutation), first_failure=True)
    assert _failed(res), f"planted force mistake {mutation} passed every pin"


# --------------------------------------------------------------------------
# Stout smearing: planted mistakes in a copy of the smearing step
# --------------------------------------------------------------------------


def make_stout(mutation):
    from scipy.linalg import expm

    def stout_fn(dims, links, rho):
        c1 = 1.0 if mutation == "with_rectangles" else 0.0
        sig = on.staples(dims, links, 1.0, c1)
        c = rho * (sig if mutation == "staple_not_daggered"
                   else np.conj(np.transpose(sig, (0, 2, 1, 3))))
        if mutation == "omega_udag_c":
            om = np.einsum("sban,sbcn->sacn", np.conj(links), c)
        else:
            om = np.einsum("sabn,scbn->sacn", c, np.conj(links))
        a = np.conj(np.transpose(om, (0, 2, 1, 3))) - om
        q = 0.5j * a
        if mutation != "no_trace":
            tr = np.einsum("saan->sn", a)
            for i in range(3):
                q[:, i, i, :] -= (1j / 6.0) * tr
        sign = -1.0 if mutation == "minus_q" else 1.0
        out = np.empty_like(links)
        for s in range(8):
            for h in range(links.shape[3]):
                e = expm(sign * 1j * q[s, :, :, h])
                u = links[s, :, :, h]
                out[s, :, :, h] = u @ e if mutation == "right_multiply" else e @ u
        return out
    return stout_fn


STOUT_MUTANTS = ["with_rectangles", "staple_not_daggered", "omega_udag_c", "no_trace", "minus_q",
                 "right_multiply"]


def test_unmutated_stout_copy_passes():
    assert _failed(pins.run_stout_pins(make_stout(None))) == []


@pytest.mark.parametrize("mutation", STOUT_MUTANTS)
def test_stout_mutant_detected(mutation):
    res = pins.run_stout_pins(make_stout(mutation), first_failure=True)
    assert _failed(res), f"planted stout mistake {mutation} passed every pin"
