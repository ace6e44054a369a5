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
#    operations per output entry; 2e-6 bounds the accumulated rounding with margin.
#  BF16-12: links rounded to 8 significant bits, u = 2^-9 ~ 2e-3; 1e-2.
TOL = {"c128_18": 1e-12, "c128_12": 1e-12, "c64_12": 2e-6, "bf16_12": 1e-2}
