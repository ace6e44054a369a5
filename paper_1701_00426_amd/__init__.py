"""MI355X (gfx950) staggered-fermion library: the even/odd staggered Dirac operator
D_eo / D_oe and the CG / multi-shift CG solves of (m^2 - D_eo D_oe) x = b.

Paper: Bonati et al., "Design and optimization of a portable LQCD Monte Carlo
code using OpenACC", arXiv:1701.00426 (Sec. 2.2 Eqs. diracblock / lineqeo /
shlineq; Sec. 2.3 and Sec. 4.1 data layouts; Sec. 4.3 deo / doe).

This module is a thin binding over the C ABI in include/stagmi.h: it passes
device pointers of torch tensors and the current HIP stream to the library and
checks the returned status.  Every step of the operator and the solvers runs in
the library's HIP kernels; nothing here computes.  The functions carry the names
of the C entry points.

Layouts (see include/stagmi.h): links complex128 (8, 3, 3, Vh) before packing,
phases float64 (8, Vh) or None for the standard staggered phases, fields
(nrhs, 3, Vh) complex128 or complex64.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import torch

from . import _lib
from ._lib import (STG_C64, STG_C128, STG_CG_F64, STG_CG_MIXED, STG_LINK_BF16_12,  # noqa: F401
                   STG_LINK_C64_12, STG_LINK_C128_12, STG_LINK_C128_18, StgError)

__all__ = [
    "Gauge", "pack_gauge", "stg_links_bytes", "stg_pack_links", "stg_pack_phases",
    "dirac_apply_eo", "dirac_apply_oe", "stg_apply_normal", "stg_apply_normal_noalloc",
    "stg_dot", "cg_solve",
    "multishift_cg_solve", "stg_workspace_bytes", "library", "stg_set_tuning", "stg_get_tuning",
    "cg_solve_batch", "rational_apply", "stg_rational_workspace_bytes", "stg_autotune",
    "stg_autotune_load", "stg_autotune_lookup", "stg_autotune_fields_lookup", "gauge_staples", "SYMANZIK_C0", "SYMANZIK_C1",
    "fermion_force", "stout_smear", "gauge_momentum_update", "gauge_link_update",
    "stout_force_backprop",
]

# tree-level Symanzik weights of the 1x1 and 1x2 loops: c1 = -1/12, c0 + 8 c1 = 1
SYMANZIK_C1 = -1.0 / 12.0
SYMANZIK_C0 = 1.0 - 8.0 * SYMANZIK_C1

FORMAT_NAMES = {"c128_18": STG_LINK_C128_18, "c128_12": STG_LINK_C128_12,
                "c64_12": STG_LINK_C64_12, "bf16_12": STG_LINK_BF16_12}


def library():
    """The loaded libstagmi.so (raises if it has not been built)."""
    return _lib.load()


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _field_type(t: torch.Tensor) -> int:
    if t.dtype == torch.complex128:
        return STG_C128
    if t.dtype == torch.complex64:
        return STG_C64
    raise ValueError(f"fields are complex128 or complex64, got {t.dtype}")


def _nrhs(t: torch.Tensor, vh: int) -> int:
    if t.dim() == 2:
        if tuple(t.shape) != (3, vh):
            raise ValueError(f"field shape {tuple(t.shape)} != (3, {vh})")
        return 1
    if t.dim() != 3 or tuple(t.shape[1:]) != (3, vh):
        raise ValueError(f"field shape {tuple(t.shape)} != (nrhs, 3, {vh})")
    return int(t.shape[0])


def half_volume(dims) -> int:
    v = 1
    for d in dims:
        v *= int(d)
    return v // 2


@dataclass
class Gauge:
    """A gauge field in one storage format, with its (optional) phase array.

    ``links`` is a device tensor holding the format's bytes; ``phases`` a device
    float64 (C128 formats) or float32 (FP32 formats) tensor (8, Vh), or None for
    the standard staggered phases computed inside the kernels.
    """
    dims: tuple
    links: torch.Tensor
    fmt: int
    phases: Optional[torch.Tensor] = None

    def c(self) -> _lib.StgGauge:
        g = _lib.StgGauge()
        g.links = self.links.data_ptr()
        g.fmt = int(self.fmt)
        g.phases = self.phases.data_ptr() if self.phases is not None else None
        return g

    @property
    def field(self) -> int:
        return STG_C128 if self.fmt in (STG_LINK_C128_18, STG_LINK_C128_12) else STG_C64


def stg_set_tuning(key: int, value: int) -> None:
    """Sets a launch-shape choice of the hop kernels (speed only, not results)."""
    _lib.check("stg_set_tuning", library().stg_set_tuning(int(key), int(value)))


def stg_get_tuning(key: int) -> int:
    v = ctypes.c_int(0)
    _lib.check("stg_get_tuning", library().stg_get_tuning(int(key), ctypes.byref(v)))
    return v.value


def stg_links_bytes(dims, fmt) -> int:
    n = ctypes.c_size_t(0)
    _lib.check("stg_links_bytes", library().stg_links_bytes(
        ctypes.byref(_lib.lattice(dims)), int(fmt), ctypes.byref(n)))
    return n.value


def stg_pack_links(dims, links_c128_18: torch.Tensor, fmt, stream=None) -> torch.Tensor:
    """Packs full complex128 links (8, 3, 3, Vh) on the GPU into format ``fmt``."""
    fmt = FORMAT_NAMES.get(fmt, fmt)
    vh = half_volume(dims)
    if links_c128_18.dtype != torch.complex128 or tuple(links_c128_18.shape) != (8, 3, 3, vh):
        raise ValueError("links must be complex128 (8, 3, 3, Vh)")
    out = torch.empty(stg_links_bytes(dims, fmt), dtype=torch.uint8, device=links_c128_18.device)
    _lib.check("stg_pack_links", library().stg_pack_links(
        ctypes.byref(_lib.lattice(dims)), _ptr(links_c128_18), int(fmt), _ptr(out),
        _stream(stream)))
    return out


def stg_pack_phases(dims, phases_f64: torch.Tensor, field, stream=None) -> torch.Tensor:
    vh = half_volume(dims)
    if phases_f64.dtype != torch.float64 or tuple(phases_f64.shape) != (8, vh):
        raise ValueError("phases must be float64 (8, Vh)")
    dt = torch.float64 if field == STG_C128 else torch.float32
    out = torch.empty((8, vh), dtype=dt, device=phases_f64.device)
    _lib.check("stg_pack_phases", library().stg_pack_phases(
        ctypes.byref(_lib.lattice(dims)), _ptr(phases_f64), int(field), _ptr(out),
        _stream(stream)))
    return out


def pack_gauge(dims, links_c128_18: torch.Tensor, fmt, phases_f64: Optional[torch.Tensor] = None,
               stream=None) -> Gauge:
    """Gauge field in format ``fmt`` (name or code) from full complex128 links on the GPU."""
    fmt = FORMAT_NAMES.get(fmt, fmt)
    if fmt == STG_LINK_C128_18:
        links = links_c128_18.contiguous()
    else:
        links = stg_pack_links(dims, links_c128_18, fmt, stream)
    ph = None
    if phases_f64 is not None:
        field = STG_C128 if fmt in (STG_LINK_C128_18, STG_LINK_C128_12) else STG_C64
        ph = stg_pack_phases(dims, phases_f64, field, stream)
    return Gauge(tuple(int(d) for d in dims), links, fmt, ph)


def _apply(name, gauge: Gauge, vin: torch.Tensor, out: Optional[torch.Tensor], stream):
    vh = half_volume(gauge.dims)
    nrhs = _nrhs(vin, vh)
    if out is None:
        out = torch.empty_like(vin)
    if out.dtype != vin.dtype or out.shape != vin.shape:
        raise ValueError("out must match in")
    g = gauge.c()
    fn = getattr(library(), name)
    _lib.check(name, fn(ctypes.byref(_lib.lattice(gauge.dims)), ctypes.byref(g), _field_type(vin),
                        nrhs, _ptr(vin), _ptr(out), _stream(stream)))
    return out


def dirac_apply_eo(gauge: Gauge, in_odd: torch.Tensor, out_even: Optional[torch.Tensor] = None,
                   stream=None) -> torch.Tensor:
    """out_even = D_eo in_odd (asynchronous on the stream)."""
    return _apply("dirac_apply_eo", gauge, in_odd, out_even, stream)


def dirac_apply_oe(gauge: Gauge, in_even: torch.Tensor, out_odd: Optional[torch.Tensor] = None,
                   stream=None) -> torch.Tensor:
    """out_odd = D_oe in_even (asynchronous on the stream)."""
    return _apply("dirac_apply_oe", gauge, in_even, out_odd, stream)


def gauge_staples(gauge: Gauge, c0: float = SYMANZIK_C0, c1: float = SYMANZIK_C1,
                  out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Staples Sigma_mu(x) of every link, (8, 3, 3, Vh): complex128 for the FP64
    link formats, complex64 for the FP32 ones (asynchronous on the stream)."""
    vh = half_volume(gauge.dims)
    dtype = torch.complex128 if gauge.field == STG_C128 else torch.complex64
    if out is None:
        out = torch.empty((8, 3, 3, vh), dtype=dtype, device=gauge.links.device)
    elif out.dtype != dtype or tuple(out.shape) != (8, 3, 3, vh) or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous {dtype} tensor of shape (8, 3, 3, {vh})")
    g = gauge.c()
    _lib.check("gauge_staples", library().gauge_staples(
        ctypes.byref(_lib.lattice(gauge.dims)), ctypes.byref(g), float(c0), float(c1), _ptr(out),
        _stream(stream)))
    return out


def fermion_force(gauge: Gauge, coeffs, x_even: torch.Tensor, y_odd: Optional[torch.Tensor] = None,
                  out: Optional[torch.Tensor] = None, stream=None):
    """Derivative G_mu(z) of S = Re phi^dag sum_k a_k X_k with respect to every link,
    from the solutions X_k (complex128, (nshift, 3, Vh)); returns (G (8, 3, 3, Vh),
    Y = D_oe X).  Asynchronous on the stream."""
    vh = half_volume(gauge.dims)
    coeffs = [float(c) for c in coeffs]
    n = len(coeffs)
    if x_even.dtype != torch.complex128 or tuple(x_even.shape) != (n, 3, vh) or \
            not x_even.is_contiguous():
        raise ValueError(f"x_even must be a contiguous complex128 tensor of shape ({n}, 3, {vh})")
    y_odd = torch.empty_like(x_even) if y_odd is None else y_odd
    if out is None:
        out = torch.empty((8, 3, 3, vh), dtype=torch.complex128, device=x_even.device)
    arr = (ctypes.c_double * max(n, 1))(*coeffs)
    g = gauge.c()
    _lib.check("fermion_force", library().fermion_force(
        ctypes.byref(_lib.lattice(gauge.dims)), ctypes.byref(g), n, arr, _ptr(x_even),
        _ptr(y_odd), _ptr(out), _stream(stream)))
    return out, y_odd


def stout_smear(gauge: Gauge, rho: float, out: Optional[torch.Tensor] = None,
                stream=None) -> torch.Tensor:
    """One stout-smearing step of every link: complex128 (8, 3, 3, Vh), the full
    FP64 link layout (asynchronous on the stream)."""
    vh = half_volume(gauge.dims)
    if out is None:
        out = torch.empty((8, 3, 3, vh), dtype=torch.complex128, device=gauge.links.device)
    elif out.dtype != torch.complex128 or tuple(out.shape) != (8, 3, 3, vh) or \
            not out.is_contiguous():
        raise ValueError(f"out must be a contiguous complex128 tensor of shape (8, 3, 3, {vh})")
    g = gauge.c()
    _lib.check("stout_smear", library().stout_smear(
        ctypes.byref(_lib.lattice(gauge.dims)), ctypes.byref(g), float(rho), _ptr(out),
        _stream(stream)))
    return out


def _check_mom(gauge: Gauge, mom: torch.Tensor):
    vh = half_volume(gauge.dims)
    dt = torch.complex64 if gauge.fmt == STG_LINK_C64_12 else torch.complex128
    if mom.dtype != dt or tuple(mom.shape) != (8, 3, 3, vh) or not mom.is_contiguous():
        raise ValueError(f"mom must be a contiguous {dt} tensor of shape (8, 3, 3, {vh})")


def gauge_momentum_update(gauge: Gauge, mom: torch.Tensor, beta: float, eps: float,
                          c0: float = SYMANZIK_C0, c1: float = SYMANZIK_C1,
                          stream=None) -> torch.Tensor:
    """P <- P - eps F(U) in place for the tree-level Symanzik gauge force (FP64 links and
    complex128 momenta, or FP32-12 links and complex64 momenta)."""
    _check_mom(gauge, mom)
    g = gauge.c()
    _lib.check("gauge_momentum_update", library().gauge_momentum_update(
        ctypes.byref(_lib.lattice(gauge.dims)), ctypes.byref(g), float(beta), float(c0),
        float(c1), float(eps), _ptr(mom), _stream(stream)))
    return mom


def gauge_link_update(gauge: Gauge, mom: torch.Tensor, eps: float, stream=None) -> Gauge:
    """U <- exp(i eps P) U in place on gauge.links (FP64 formats or FP32-12)."""
    _check_mom(gauge, mom)
    _lib.check("gauge_link_update", library().gauge_link_update(
        ctypes.byref(_lib.lattice(gauge.dims)), int(gauge.fmt), _ptr(gauge.links), float(eps),
        _ptr(mom), _stream(stream)))
    return gauge


def stout_force_backprop(gauge: Gauge, rho: float, sigma_smeared: torch.Tensor,
                         out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                         stream=None) -> torch.Tensor:
    """dS/dU for the thin links from dS/dU' of the links smeared once with weight rho
    (complex128 (8, 3, 3, Vh) each; asynchronous on the stream)."""
    vh = half_volume(gauge.dims)
    shape = (8, 3, 3, vh)
    if sigma_smeared.dtype != torch.complex128 or tuple(sigma_smeared.shape) != shape or \
            not sigma_smeared.is_contiguous():
        raise ValueError(f"sigma_smeared must be a contiguous complex128 tensor of shape {shape}")
    out = torch.empty(shape, dtype=torch.complex128, device=sigma_smeared.device) \
        if out is None else out
    ws = torch.empty(shape, dtype=torch.complex128, device=sigma_smeared.device) \
        if ws is None else ws
    g = gauge.c()
    _lib.check("stout_force_backprop", library().stout_force_backprop(
        ctypes.byref(_lib.lattice(gauge.dims)), ctypes.byref(g), float(rho),
        _ptr(sigma_smeared), _ptr(out), _ptr(ws), _stream(stream)))
    return out


def stg_apply_normal(gauge: Gauge, mass: float, in_even: torch.Tensor, sigma: float = 0.0,
                     out_even: Optional[torch.Tensor] = None,
                     tmp_odd: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """out = (mass^2 + sigma) in - D_eo D_oe in."""
    vh = half_volume(gauge.dims)
    nrhs = _nrhs(in_even, vh)
    out_even = torch.empty_like(in_even) if out_even is None else out_even
    tmp_odd = torch.empty_like(in_even) if tmp_odd is None else tmp_odd
    g = gauge.c()
    _lib.check("stg_apply_normal", library().stg_apply_normal(
        ctypes.byref(_lib.lattice(gauge.dims)), ctypes.byref(g), _field_type(in_even), nrhs,
        float(mass), float(sigma), _ptr(in_even), _ptr(out_even), _ptr(tmp_odd), _stream(stream)))
    return out_even


def stg_apply_normal_noalloc(gauge: Gauge, mass: float, in_even: torch.Tensor,
                             out_even: torch.Tensor, sigma: float = 0.0,
                             stream=None) -> torch.Tensor:
    """out = (mass^2 + sigma) in - D_eo D_oe in, the odd intermediate in the library's
    fixed device scratch array (no allocation by the call; out_even is the caller's)."""
    vh = half_volume(gauge.dims)
    nrhs = _nrhs(in_even, vh)
    g = gauge.c()
    _lib.check("stg_apply_normal_noalloc", library().stg_apply_normal_noalloc(
        ctypes.byref(_lib.lattice(gauge.dims)), ctypes.byref(g), _field_type(in_even), nrhs,
        float(mass), float(sigma), _ptr(in_even), _ptr(out_even), _stream(stream)))
    return out_even


def stg_dot(x: torch.Tensor, y: torch.Tensor, stream=None):
    """Compensated <x_j, y_j> over the last dims, one complex per leading index."""
    if x.dtype != y.dtype or x.shape != y.shape:
        raise ValueError("x and y must have the same dtype and shape")
    nvec = int(x.shape[0]) if x.dim() > 1 else 1
    n = x.numel() // nvec
    lib = library()
    ws = torch.empty(lib.stg_dot_workspace_bytes(), dtype=torch.uint8, device=x.device)
    res = (ctypes.c_double * (2 * nvec))()
    _lib.check("stg_dot", lib.stg_dot(_field_type(x), nvec, n, _ptr(x), _ptr(y), res, _ptr(ws),
                                      ws.numel(), _stream(stream)))
    return [complex(res[2 * j], res[2 * j + 1]) for j in range(nvec)]


def stg_workspace_bytes(dims, nrhs, nshift=0, mode=STG_CG_F64) -> int:
    n = ctypes.c_size_t(0)
    _lib.check("stg_workspace_bytes", library().stg_workspace_bytes(
        ctypes.byref(_lib.lattice(dims)), int(nrhs), int(nshift), int(mode), ctypes.byref(n)))
    return n.value


def cg_params(**kw) -> _lib.StgCgParams:
    p = _lib.StgCgParams()
    library().stg_cg_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def cg_solve(hi: Gauge, mass: float, b: torch.Tensor, x: Optional[torch.Tensor] = None,
             lo: Optional[Gauge] = None, ws: Optional[torch.Tensor] = None, stream=None,
             check_status: bool = True, **params):
    """Solves (mass^2 - D_eo D_oe) x = b for every RHS of b (complex128 (nrhs, 3, Vh)).

    ``x`` holds the initial guess (zero if None) and receives the solution.
    Mixed precision when ``lo`` is given (mode STG_CG_MIXED) unless ``mode`` is
    passed.  Returns (x, status, list of per-RHS stats dicts).
    """
    vh = half_volume(hi.dims)
    if b.dtype != torch.complex128:
        raise ValueError("b must be complex128")
    nrhs = _nrhs(b, vh)
    if x is None:
        x = torch.zeros_like(b)
    params.setdefault("mode", STG_CG_MIXED if lo is not None else STG_CG_F64)
    prm = cg_params(**params)
    need = stg_workspace_bytes(hi.dims, nrhs, 0, prm.mode)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=b.device)
    stats = (_lib.StgCgStats * nrhs)()
    g_hi = hi.c()
    g_lo = lo.c() if lo is not None else None
    st = library().cg_solve(
        ctypes.byref(_lib.lattice(hi.dims)), ctypes.byref(g_hi),
        ctypes.byref(g_lo) if g_lo is not None else None, float(mass), nrhs, _ptr(b), _ptr(x),
        ctypes.byref(prm), _ptr(ws), ws.numel(), stats, _stream(stream))
    if check_status:
        _lib.check("cg_solve", st, ok=(_lib.STG_OK,))
    return x, st, [s.as_dict() for s in stats]


def multishift_cg_solve(hi: Gauge, mass: float, shifts, b: torch.Tensor,
                        lo: Optional[Gauge] = None, ws: Optional[torch.Tensor] = None,
                        stream=None, check_status: bool = True, **params):
    """Solves (mass^2 + sigma_k - D_eo D_oe) x_k = b_j for all shifts and RHS.

    Returns (x complex128 (nshift, nrhs, 3, Vh), status, stats[nshift][nrhs]).
    """
    vh = half_volume(hi.dims)
    if b.dtype != torch.complex128:
        raise ValueError("b must be complex128")
    nrhs = _nrhs(b, vh)
    shifts = [float(s) for s in shifts]
    ns = len(shifts)
    x = torch.zeros((ns, nrhs, 3, vh), dtype=torch.complex128, device=b.device)
    params.setdefault("mode", STG_CG_MIXED if lo is not None else STG_CG_F64)
    prm = cg_params(**params)
    need = stg_workspace_bytes(hi.dims, nrhs, ns, prm.mode)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=b.device)
    stats = (_lib.StgCgStats * (ns * nrhs))()
    sh = (ctypes.c_double * ns)(*shifts)
    g_hi = hi.c()
    g_lo = lo.c() if lo is not None else None
    st = library().multishift_cg_solve(
        ctypes.byref(_lib.lattice(hi.dims)), ctypes.byref(g_hi),
        ctypes.byref(g_lo) if g_lo is not None else None, float(mass), ns, sh, nrhs, _ptr(b),
        _ptr(x), ctypes.byref(prm), _ptr(ws), ws.numel(), stats, _stream(stream))
    if check_status:
        _lib.check("multishift_cg_solve", st, ok=(_lib.STG_OK,))
    out = [[stats[k * nrhs + j].as_dict() for j in range(nrhs)] for k in range(ns)]
    return x, st, out


def stg_rational_workspace_bytes(dims, nrhs: int, nshift: int, mode: int) -> int:
    n = ctypes.c_size_t(0)
    _lib.check("stg_rational_workspace_bytes", library().stg_rational_workspace_bytes(
        ctypes.byref(_lib.lattice(dims)), int(nrhs), int(nshift), int(mode), ctypes.byref(n)))
    return n.value


def rational_apply(hi: Gauge, mass: float, shifts, coeffs, a0: float, b: torch.Tensor,
                   lo: Optional[Gauge] = None, ws: Optional[torch.Tensor] = None, stream=None,
                   check_status: bool = True, **params):
    """y_j = a0 b_j + sum_k coeffs[k] (mass^2 + shifts[k] - D_eo D_oe)^{-1} b_j.

    Returns (y complex128 (nrhs, 3, Vh), status, stats[nshift][nrhs]).
    """
    vh = half_volume(hi.dims)
    if b.dtype != torch.complex128:
        raise ValueError("b must be complex128")
    nrhs = _nrhs(b, vh)
    shifts = [float(s) for s in shifts]
    coeffs = [float(c) for c in coeffs]
    if len(coeffs) != len(shifts):
        raise ValueError("one coefficient per shift")
    ns = len(shifts)
    y = torch.empty_like(b)
    params.setdefault("mode", STG_CG_MIXED if lo is not None else STG_CG_F64)
    prm = cg_params(**params)
    need = stg_rational_workspace_bytes(hi.dims, nrhs, ns, prm.mode)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=b.device)
    stats = (_lib.StgCgStats * (ns * nrhs))()
    sh = (ctypes.c_double * ns)(*shifts)
    co = (ctypes.c_double * ns)(*coeffs)
    g_hi = hi.c()
    g_lo = lo.c() if lo is not None else None
    st = library().rational_apply(
        ctypes.byref(_lib.lattice(hi.dims)), ctypes.byref(g_hi),
        ctypes.byref(g_lo) if g_lo is not None else None, float(mass), ns, sh, co, float(a0),
        nrhs, _ptr(b), _ptr(y), ctypes.byref(prm), _ptr(ws), ws.numel(), stats, _stream(stream))
    if check_status:
        _lib.check("rational_apply", st, ok=(_lib.STG_OK,))
    out = [[stats[k * nrhs + j].as_dict() for j in range(nrhs)] for k in range(ns)]
    return y, st, out


def cg_solve_batch(solves, mode=None, ws: Optional[torch.Tensor] = None, stream=None,
                   check_status: bool = True, **params):
    """Uneven batch: every entry of ``solves`` is a dict with ``hi`` (Gauge, FP64),
    ``lo`` (Gauge, FP32 formats; mixed mode), ``mass``, ``b`` (complex128 (nrhs, 3, Vh))
    and optionally ``x`` (initial guess, receives the solution).

    Returns (list of x, status, list of per-solve lists of per-RHS stats dicts).
    """
    n = len(solves)
    if mode is None:
        mode = STG_CG_MIXED if all(sv.get("lo") is not None for sv in solves) else STG_CG_F64
    descs = (_lib.StgSolveDesc * n)()
    xs = []
    keep = []
    nsys = 0
    for i, sv in enumerate(solves):
        hi, lo, b = sv["hi"], sv.get("lo"), sv["b"]
        vh = half_volume(hi.dims)
        nrhs = _nrhs(b, vh)
        if b.dtype != torch.complex128:
            raise ValueError("b must be complex128")
        x = sv.get("x")
        if x is None:
            x = torch.zeros_like(b)
        xs.append(x)
        d = descs[i]
        d.lat = _lib.lattice(hi.dims)
        d.hi = hi.c()
        if lo is not None:
            d.lo = lo.c()
        d.mass = float(sv["mass"])
        d.nrhs = nrhs
        d.b = b.data_ptr()
        d.x = x.data_ptr()
        keep.append((b, x))
        nsys += nrhs
    params["mode"] = mode
    prm = cg_params(**params)
    lib = library()
    need = ctypes.c_size_t(0)
    _lib.check("stg_batch_workspace_bytes", lib.stg_batch_workspace_bytes(
        n, descs, int(mode), ctypes.byref(need)))
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(need.value, dtype=torch.uint8, device=solves[0]["b"].device)
    stats = (_lib.StgCgStats * nsys)()
    st = lib.cg_solve_batch(n, descs, ctypes.byref(prm), _ptr(ws), ws.numel(), stats,
                            _stream(stream))
    if check_status:
        _lib.check("cg_solve_batch", st, ok=(_lib.STG_OK,))
    out, k = [], 0
    for sv in solves:
        nr = _nrhs(sv["b"], half_volume(sv["hi"].dims))
        out.append([stats[k + j].as_dict() for j in range(nr)])
        k += nr
    return xs, st, out


def stg_autotune(gauge: Gauge, nrhs: int = 1, cache_path: Optional[str] = None, stream=None):
    """Times the hop launch shapes for this gauge field and nrhs fields per launch and
    keeps the fastest (process-wide; appended to cache_path when given).  Returns the
    choice as a dict."""
    vh = half_volume(gauge.dims)
    cdt = torch.complex128 if gauge.field == STG_C128 else torch.complex64
    vin = torch.zeros((nrhs, 3, vh), dtype=cdt, device=gauge.links.device)
    out = torch.empty_like(vin)
    g = gauge.c()
    lib = library()
    _lib.check("stg_autotune", lib.stg_autotune(
        ctypes.byref(_lib.lattice(gauge.dims)), ctypes.byref(g), int(gauge.field), int(nrhs),
        _ptr(vin), _ptr(out), cache_path.encode() if cache_path else None, _stream(stream)))
    nr = 8 if nrhs >= 8 else 4 if nrhs >= 4 else nrhs
    choice = stg_autotune_lookup(gauge.dims, gauge.fmt, nr)
    if nrhs >= 2:
        choice["fields_per_launch"] = stg_autotune_fields_lookup(gauge.dims, gauge.fmt)
    return choice


def stg_autotune_load(cache_path: str) -> int:
    n = ctypes.c_int(0)
    _lib.check("stg_autotune_load", library().stg_autotune_load(cache_path.encode(),
                                                                ctypes.byref(n)))
    return n.value


def stg_autotune_fields_lookup(dims, fmt):
    """The stored fields per launch (1, 2, 4 or 8) for (dims, fmt), or None."""
    v = ctypes.c_int(0)
    st = library().stg_autotune_fields_lookup(ctypes.byref(_lib.lattice(dims)), int(fmt),
                                              ctypes.byref(v))
    if st == _lib.STG_NOT_CONVERGED:
        return None
    _lib.check("stg_autotune_fields_lookup", st)
    return v.value


def stg_autotune_lookup(dims, fmt, nr: int = 1):
    """The stored launch shape for (dims, fmt, nr), or None."""
    c = _lib.StgTuneChoice()
    st = library().stg_autotune_lookup(ctypes.byref(_lib.lattice(dims)), int(fmt), int(nr),
                                       ctypes.byref(c))
    if st == _lib.STG_NOT_CONVERGED:
        return None
    _lib.check("stg_autotune_lookup", st)
    return c.as_dict()
