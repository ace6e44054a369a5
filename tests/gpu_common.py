"""Helpers shared by the GPU tests: device inputs and error figures."""
import sys

import numpy as np
import torch

import seeded_inputs as si
from oracle import oracle_np as on

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel_max(got, want):
    """max |got - want| / max |want|."""
    return float(np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-300))


def rel_norm(got, want):
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def setup(dims, seed, nrhs=1, parity_field=True):
    links = si.su3_links(dims, 1701, *seed)
    phases = on.standard_phases(dims)
    v = si.gaussian_field(dims, nrhs, 426, *seed)
    return links, phases, v


# Tolerances of the GPU hop against the FP64 oracle (max-norm relative):
#  FP64 formats: 1e-12 (the contract of the FP64 path).
#  FP32-12: unit roundoff u = 2^-24 ~ 6e-8 on links, fields and each of the ~30
#    operations per output entry (measured ~1-3e-7); 1e-6.
#  BF16-12: links rounded to 8 significant bits, u = 2^-9 ~ 2e-3; 1e-2.  Against the
#    oracle evaluated on the links as stored (dequantized, row 2 rebuilt in FP64) and
#    on the complex64 input, only the FP32 arithmetic differs: TOL_ARITH.
TOL = {"c128_18": 1e-12, "c128_12": 1e-12, "c64_12": 1e-6, "bf16_12": 1e-2}
TOL_ARITH = {"c64_12": 1e-6, "bf16_12": 1e-6}


def _round_bf16(x):
    """Round-to-nearest-even of float64 values to bfloat16, returned as float64."""
    m, e = np.frexp(x)
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def stored_links(links, fmt):
    """The full FP64 links the kernel of a 12-real format works on: rows 0 and 1 as
    stored (rounded to FP32 or BF16, round to nearest even), row 2 rebuilt as
    conj(row0 x row1) in FP64 (Sec. 2.3)."""
    two = links[:, :2]
    if fmt == "c64_12":
        two = two.astype(np.complex64).astype(np.complex128)
    elif fmt == "bf16_12":
        two = _round_bf16(two.real) + 1j * _round_bf16(two.imag)
    else:
        raise ValueError(fmt)
    out = np.empty_like(links)
    out[:, :2] = two
    r0, r1 = two[:, 0], two[:, 1]                      # (8, 3 columns, Vh)
    out[:, 2] = np.conj(np.stack([r0[:, 1] * r1[:, 2] - r0[:, 2] * r1[:, 1],
                                  r0[:, 2] * r1[:, 0] - r0[:, 0] * r1[:, 2],
                                  r0[:, 0] * r1[:, 1] - r0[:, 1] * r1[:, 0]], axis=1))
    return out
