"""FP64 CPU oracle of the even/odd staggered operator and its solvers.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library never
imports, links or calls it, and this package imports nothing from the GPU
library.

Two independent implementations of the same definitions (arXiv:1701.00426,
Sec. 2.2 Eqs. diracblock / lineqeo / shlineq, Sec. 4.1 layouts):
  * ``oracle_np``  -- NumPy, vectorised over sites, plus dense brute force and
    closed forms;
  * ``stag_oracle.c`` -- plain C99 ``double complex`` with OpenMP over sites,
    wrapped here through ctypes (``COracle``), fast enough for full-size samples
    and for the CPU baseline timing.

Parity status: every function is pinned by the tests under ``tests/`` marked
``not gpu`` (anti-Hermiticity, free-field closed form and full spectrum, gauge
covariance, pure-gauge eigenvectors, dense brute force, translation, multi-shift
vs independent CG, N-version NumPy vs C, planted-mistake detection).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import oracle_np  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstag_oracle.so")
SRC_PATH = os.path.join(_HERE, "stag_oracle.c")


def build(verbose: bool = False, native_dir: str = "") -> str:
    """Compile stag_oracle.c into libstag_oracle.so (plain gcc, OpenMP).

    With native_dir the library is built with -O3 -march=native into that folder
    (the CPU baseline builds it on the host it times; -march=native code may not
    run on another CPU, so the tests' copy keeps the portable flags).  The source
    is ISO C99, so gcc contracts no multiply-add: both builds round alike."""
    if native_dir:
        out = os.path.join(native_dir, "libstag_oracle_native.so")
        flags = ["-O3", "-march=native"]
    else:
        out = LIB_PATH
        flags = ["-O2"]
    cmd = ["gcc", *flags, "-std=c99", "-fopenmp", "-shared", "-fPIC", SRC_PATH,
           "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class COracle:
    """ctypes wrapper of libstag_oracle.so (builds it if it is missing)."""

    def __init__(self, path: str = LIB_PATH):
        if not os.path.exists(path):
            build()
        lib = ctypes.CDLL(path)
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_num_threads.argtypes = []
        lib.orc_set_num_threads.restype = None
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        lib.orc_half_volume.restype = ctypes.c_long
        lib.orc_half_volume.argtypes = [_P]
        lib.orc_standard_phases.argtypes = [_P, _P]
        lib.orc_dslash.argtypes = [_P, _P, _P, _I, _P, _P]
        lib.orc_apply_normal.argtypes = [_P, _P, _P, _D, _D, _P, _P, _P]
        lib.orc_cg.restype = _I
        lib.orc_cg.argtypes = [_P, _P, _P, _D, _D, _P, _P, _D, _I, _P, _P]
        lib.orc_mscg.restype = _I
        lib.orc_mscg.argtypes = [_P, _P, _P, _D, _I, _P, _P, _P, _D, _I, _P, _P]
        self.lib = lib

    def num_threads(self) -> int:
        return int(self.lib.orc_num_threads())

    def set_num_threads(self, n: int) -> None:
        self.lib.orc_set_num_threads(int(n))

    @staticmethod
    def _dims(dims):
        return np.ascontiguousarray(np.asarray(dims, dtype=np.int32))

    @staticmethod
    def _c128(a):
        return np.ascontiguousarray(a, dtype=np.complex128)

    @staticmethod
    def _f64(a):
        return np.ascontiguousarray(a, dtype=np.float64)

    def standard_phases(self, dims):
        d = self._dims(dims)
        vh = int(self.lib.orc_half_volume(_ptr(d)))
        ph = np.empty((8, vh), dtype=np.float64)
        self.lib.orc_standard_phases(_ptr(d), _ptr(ph))
        return ph

    def dslash(self, dims, links, phases, out_parity, vin):
        d = self._dims(dims)
        links = self._c128(links)
        phases = self._f64(phases)
        vin = self._c128(vin)
        out = np.empty_like(vin)
        flat_in = vin.reshape(-1, *vin.shape[-2:])
        flat_out = out.reshape(-1, *vin.shape[-2:])
        for i in range(flat_in.shape[0]):
            src = np.ascontiguousarray(flat_in[i])
            dst = np.empty_like(src)
            self.lib.orc_dslash(_ptr(d), _ptr(links), _ptr(phases), int(out_parity),
                                _ptr(src), _ptr(dst))
            flat_out[i] = dst
        return out

    def d_eo(self, dims, links, phases, v_odd):
        return self.dslash(dims, links, phases, 0, v_odd)

    def d_oe(self, dims, links, phases, v_even):
        return self.dslash(dims, links, phases, 1, v_even)

    def apply_normal(self, dims, links, phases, mass, v_even, sigma=0.0):
        d = self._dims(dims)
        links = self._c128(links)
        phases = self._f64(phases)
        v = self._c128(v_even)
        out = np.empty_like(v)
        tmp = np.empty_like(v)
        self.lib.orc_apply_normal(_ptr(d), _ptr(links), _ptr(phases), float(mass), float(sigma),
                                  _ptr(v), _ptr(out), _ptr(tmp))
        return out

    def cg(self, dims, links, phases, mass, b, tol=1e-12, max_iter=100000, sigma=0.0, x0=None):
        """Returns (x, iterations, true relative residual, status)."""
        d = self._dims(dims)
        links = self._c128(links)
        phases = self._f64(phases)
        b = self._c128(b)
        x = np.zeros_like(b) if x0 is None else self._c128(x0).copy()
        it = ctypes.c_int(0)
        res = ctypes.c_double(0.0)
        st = self.lib.orc_cg(_ptr(d), _ptr(links), _ptr(phases), float(mass), float(sigma),
                             _ptr(b), _ptr(x), float(tol), int(max_iter),
                             ctypes.byref(it), ctypes.byref(res))
        return x, it.value, res.value, st

    def mscg(self, dims, links, phases, mass, shifts, b, tol=1e-10, max_iter=100000):
        """Returns (x[nshift], iterations[nshift], true residuals[nshift], status)."""
        d = self._dims(dims)
        links = self._c128(links)
        phases = self._f64(phases)
        b = self._c128(b)
        sh = self._f64(shifts)
        ns = sh.shape[0]
        x = np.zeros((ns,) + b.shape, dtype=np.complex128)
        its = np.zeros(ns, dtype=np.int32)
        res = np.zeros(ns, dtype=np.float64)
        st = self.lib.orc_mscg(_ptr(d), _ptr(links), _ptr(phases), float(mass), int(ns), _ptr(sh),
                               _ptr(b), _ptr(x), float(tol), int(max_iter), _ptr(its), _ptr(res))
        return x, its, res, st
