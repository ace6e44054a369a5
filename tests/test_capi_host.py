"""The C-ABI library on the host (no GPU): it loads, exports every entry point that
include/stagmi.h declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1701_00426_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1701_00426_amd import build
        build.build()
    return _lib.load()


def header_functions():
    text = open(os.path.join(ROOT, "include", "stagmi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_exports_every_declared_symbol(lib):
    from paper_1701_00426_amd import _lib
    names = header_functions()
    assert len(names) >= 14, names
    for n in names:
        assert hasattr(lib, n), f"libstagmi.so does not export {n}"
    # the Python binding declares exactly the header's surface
    assert sorted(_lib.SIGNATURES) == names


def test_version_and_status_strings(lib):
    assert lib.stg_version() >> 16 == 1
    for code in (0, 1, 2, -1, -2, -3):
        assert lib.stg_status_string(code)
    assert b"unknown" in lib.stg_status_string(12345)


def _lat(dims):
    from paper_1701_00426_amd import _lib
    return _lib.lattice(dims)


@pytest.mark.parametrize("dims,ok", [((4, 4, 4, 4), True), ((32, 32, 32, 32), True),
                                     ((3, 4, 4, 4), False), ((4, 4, 4, 0), False),
                                     ((4, 4, 4, -2), False), ((2, 2, 2, 2), True)])
def test_links_bytes(lib, dims, ok):
    n = ctypes.c_size_t(0)
    rc = lib.stg_links_bytes(ctypes.byref(_lat(dims)), 0, ctypes.byref(n))
    if ok:
        vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
        assert rc == 0 and n.value == 8 * 9 * vh * 16
        for fmt, per in ((1, 96), (2, 48), (3, 24)):
            assert lib.stg_links_bytes(ctypes.byref(_lat(dims)), fmt, ctypes.byref(n)) == 0
            assert n.value == 8 * vh * per
    else:
        assert rc == -1


def test_invalid_arguments_rejected_on_host(lib):
    from paper_1701_00426_amd import _lib
    lat = _lat((4, 4, 4, 4))
    g = _lib.StgGauge()
    g.links = 0x1000
    g.fmt = 0
    g.phases = None
    # null field pointers
    assert lib.dirac_apply_eo(ctypes.byref(lat), ctypes.byref(g), 0, 1, None, None, None) == -1
    # misaligned
    assert lib.dirac_apply_oe(ctypes.byref(lat), ctypes.byref(g), 0, 1, 0x1008, 0x100000,
                              None) == -1
    # aliasing input and output
    assert lib.dirac_apply_oe(ctypes.byref(lat), ctypes.byref(g), 0, 1, 0x200000, 0x200000,
                              None) == -1
    # precision mismatch: FP64 links with complex64 fields
    assert lib.dirac_apply_eo(ctypes.byref(lat), ctypes.byref(g), 1, 1, 0x200000, 0x400000,
                              None) == -1
    # nrhs < 1
    assert lib.dirac_apply_eo(ctypes.byref(lat), ctypes.byref(g), 0, 0, 0x200000, 0x400000,
                              None) == -1
    # odd extent
    bad = _lat((5, 4, 4, 4))
    assert lib.dirac_apply_eo(ctypes.byref(bad), ctypes.byref(g), 0, 1, 0x200000, 0x400000,
                              None) == -1
    assert b"even" in lib.stg_last_error()


def test_solver_arguments_rejected_on_host(lib):
    from paper_1701_00426_amd import _lib
    lat = _lat((4, 4, 4, 4))
    g = _lib.StgGauge()
    g.links = 0x1000
    g.fmt = 0
    prm = _lib.StgCgParams()
    lib.stg_cg_default_params(ctypes.byref(prm))
    assert prm.tol == 1e-10 and prm.max_iter == 100000 and abs(prm.delta - 0.1) < 1e-15
    stats = (_lib.StgCgStats * 1)()
    need = ctypes.c_size_t(0)
    assert lib.stg_workspace_bytes(ctypes.byref(lat), 1, 0, 0, ctypes.byref(need)) == 0
    assert need.value > 0
    # workspace too small
    rc = lib.cg_solve(ctypes.byref(lat), ctypes.byref(g), None, 0.1, 1, 0x200000, 0x400000,
                      ctypes.byref(prm), 0x10000000, 16, stats, None)
    assert rc == -3
    # mixed mode without a low-precision gauge field
    prm.mode = 1
    rc = lib.cg_solve(ctypes.byref(lat), ctypes.byref(g), None, 0.1, 1, 0x200000, 0x400000,
                      ctypes.byref(prm), 0x10000000, 1 << 30, stats, None)
    assert rc == -1
    # bad tolerance
    prm.mode = 0
    prm.tol = 0.0
    rc = lib.cg_solve(ctypes.byref(lat), ctypes.byref(g), None, 0.1, 1, 0x200000, 0x400000,
                      ctypes.byref(prm), 0x10000000, 1 << 30, stats, None)
    assert rc == -1
    # negative shift
    prm.tol = 1e-10
    sh = (ctypes.c_double * 2)(0.1, -1.0)
    rc = lib.multishift_cg_solve(ctypes.byref(lat), ctypes.byref(g), None, 0.1, 2, sh, 1,
                                 0x200000, 0x400000, ctypes.byref(prm), 0x10000000, 1 << 30,
                                 stats, None)
    assert rc == -1
    # multi-shift workspace is at least the refinement's
    ms = ctypes.c_size_t(0)
    assert lib.stg_workspace_bytes(ctypes.byref(lat), 2, 4, 1, ctypes.byref(ms)) == 0
    cg8 = ctypes.c_size_t(0)
    assert lib.stg_workspace_bytes(ctypes.byref(lat), 8, 0, 1, ctypes.byref(cg8)) == 0
    assert ms.value >= cg8.value


def test_rational_arguments_rejected_on_host(lib):
    """rational_apply checks its arguments before any GPU work."""
    from paper_1701_00426_amd import _lib
    lat = _lat((4, 4, 4, 4))
    g = _lib.StgGauge()
    g.links = 0x1000
    g.fmt = 0
    prm = _lib.StgCgParams()
    lib.stg_cg_default_params(ctypes.byref(prm))
    stats = (_lib.StgCgStats * 2)()
    sh = (ctypes.c_double * 2)(0.1, 1.0)
    co = (ctypes.c_double * 2)(0.5, 0.25)
    need = ctypes.c_size_t(0)
    assert lib.stg_rational_workspace_bytes(ctypes.byref(lat), 1, 2, 0, ctypes.byref(need)) == 0
    ms = ctypes.c_size_t(0)
    assert lib.stg_workspace_bytes(ctypes.byref(lat), 1, 2, 0, ctypes.byref(ms)) == 0
    # the shifted solutions (2 x 128 sites x 3 x 16 B) plus the coefficients come first
    assert need.value >= ms.value + 2 * 128 * 3 * 16
    assert lib.stg_rational_workspace_bytes(ctypes.byref(lat), 1, 0, 0, ctypes.byref(need)) == -1

    def call(nshift=2, shifts=sh, coeffs=co, a0=0.5, ws_bytes=1 << 30):
        return lib.rational_apply(ctypes.byref(lat), ctypes.byref(g), None, 0.1, nshift, shifts,
                                  coeffs, a0, 1, 0x200000, 0x400000, ctypes.byref(prm),
                                  0x10000000, ws_bytes, stats, None)

    assert call(nshift=0) == -1
    assert call(coeffs=None) == -1
    assert call(shifts=(ctypes.c_double * 2)(0.1, -1.0)) == -1
    assert call(coeffs=(ctypes.c_double * 2)(0.1, float("nan"))) == -1
    assert call(a0=float("inf")) == -1
    assert call(ws_bytes=64) == -3


def test_product_does_not_import_oracle():
    """The GPU package never imports the oracle; the oracle never imports the package."""
    pkg = os.path.join(ROOT, "paper_1701_00426_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower().replace("oracle-free", ""), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c")):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_1701_00426_amd" not in text and "stagmi" not in text, f


def test_autotune_cache_roundtrip(lib, tmp_path):
    """The cache file format is read back into the table; unknown keys report 1.
    Lines written before a field existed read as that field's default."""
    from paper_1701_00426_amd import _lib
    lat = _lat((32, 32, 32, 32))
    lat8 = _lat((8, 8, 8, 8))
    lib.stg_autotune_clear()
    c = _lib.StgTuneChoice()
    assert lib.stg_autotune_lookup(ctypes.byref(lat), 1, 1, ctypes.byref(c)) == 1
    f = tmp_path / "tune.jsonl"
    head = '{"arch": "gfx950", "dims": '
    f.write_text(
        head + '[32, 32, 32, 32], "fmt": 1, "nr": 1, "xcd_remap": 0, '
        '"sites_per_thread": 2, "us": 87.5}\n'
        'not a line of the cache\n'
        + head + '[32, 32, 32, 32], "fmt": 1, "nr": 1, "xcd_remap": 1, '
        '"sites_per_thread": 4, "stage_neighbours": 1, "threads_per_site": 1, "us": 80.25}\n'
        + head + '[8, 8, 8, 8], "fmt": 2, "nr": 4, "xcd_remap": 1, '
        '"sites_per_thread": 3, "us": 1.0}\n'
        + head + '[8, 8, 8, 8], "fmt": 2, "nr": 2, "xcd_remap": 1, '
        '"sites_per_thread": 1, "stage_neighbours": 2, "us": 1.0}\n'
        + head + '[8, 8, 8, 8], "fmt": 2, "nr": 8, "xcd_remap": 1, '
        '"sites_per_thread": 1, "stage_neighbours": 0, "threads_per_site": 3, "us": 1.0}\n'
        + '{"arch": "gfx942", "dims": [8, 8, 8, 8], "fmt": 2, "nr": 1, "xcd_remap": 1, '
        '"sites_per_thread": 1, "us": 1.0}\n'
        + head + '[8, 8, 8, 8], "fmt": 2, "nr": 1, "xcd_remap": 0, '
        '"sites_per_thread": 2, "us": 3.5}\n'
        + head + '[8, 8, 8, 8], "fmt": 3, "nr": 2, "xcd_remap": 1, '
        '"sites_per_thread": 1, "stage_neighbours": 0, "threads_per_site": 4, "us": 2.25}\n')
    n = ctypes.c_int(0)
    assert lib.stg_autotune_load(str(f).encode(), ctypes.byref(n)) == 0
    # skipped: the malformed line, sites per thread 3, staging 2, threads per site 3,
    # another architecture
    assert n.value == 4
    assert lib.stg_autotune_lookup(ctypes.byref(lat), 1, 1, ctypes.byref(c)) == 0
    assert (c.xcd_remap, c.sites_per_thread, c.stage_neighbours, c.threads_per_site,
            c.us) == (1, 4, 1, 1, 80.25)
    assert lib.stg_autotune_lookup(ctypes.byref(lat8), 2, 1, ctypes.byref(c)) == 0
    assert (c.xcd_remap, c.sites_per_thread, c.stage_neighbours, c.threads_per_site,
            c.us) == (0, 2, 0, 1, 3.5)
    assert lib.stg_autotune_lookup(ctypes.byref(lat8), 3, 2, ctypes.byref(c)) == 0
    assert (c.threads_per_site, c.us) == (4, 2.25)
    for fmt, nr in ((2, 4), (2, 2), (2, 8)):
        assert lib.stg_autotune_lookup(ctypes.byref(lat8), fmt, nr, ctypes.byref(c)) == 1
    assert lib.stg_autotune_load(b"/nonexistent/file", ctypes.byref(n)) == -1
    lib.stg_autotune_clear()
    assert lib.stg_autotune_lookup(ctypes.byref(lat), 1, 1, ctypes.byref(c)) == 1


def test_autotune_fields_cache_roundtrip(lib, tmp_path):
    """Fields-per-launch lines of the cache: read into their own table (later lines
    win, caps other than 1, 2, 4, 8 skipped), looked up per (lattice, format), and
    emptied by stg_autotune_clear together with the shapes."""
    lat = _lat((32, 32, 32, 32))
    lat8 = _lat((8, 8, 8, 8))
    lib.stg_autotune_clear()
    v = ctypes.c_int(-1)
    assert lib.stg_autotune_fields_lookup(ctypes.byref(lat), 2, ctypes.byref(v)) == 1
    assert lib.stg_autotune_fields_lookup(ctypes.byref(lat), 2, None) == -1
    assert lib.stg_autotune_fields_lookup(None, 2, ctypes.byref(v)) == -1
    bad = _lat((8, 8, 8, 7))
    assert lib.stg_autotune_fields_lookup(ctypes.byref(bad), 2, ctypes.byref(v)) == -1
    head = '{"arch": "gfx950", "dims": '
    f = tmp_path / "fields.jsonl"
    f.write_text(
        head + '[32, 32, 32, 32], "fmt": 2, "fields_per_launch": 4, "us_per_field": 9.5}\n'
        + head + '[32, 32, 32, 32], "fmt": 2, "fields_per_launch": 8, "us_per_field": 9.1}\n'
        + head + '[8, 8, 8, 8], "fmt": 1, "fields_per_launch": 3, "us_per_field": 1.0}\n'
        + head + '[8, 8, 8, 8], "fmt": 3, "fields_per_launch": 2, "us_per_field": 1.5}\n'
        + head + '[8, 8, 8, 8], "fmt": 3, "nr": 1, "xcd_remap": 0, '
        '"sites_per_thread": 1, "us": 2.0}\n')
    n = ctypes.c_int(0)
    assert lib.stg_autotune_load(str(f).encode(), ctypes.byref(n)) == 0
    assert n.value == 4  # the cap of 3 is skipped
    assert lib.stg_autotune_fields_lookup(ctypes.byref(lat), 2, ctypes.byref(v)) == 0
    assert v.value == 8
    assert lib.stg_autotune_fields_lookup(ctypes.byref(lat8), 3, ctypes.byref(v)) == 0
    assert v.value == 2
    assert lib.stg_autotune_fields_lookup(ctypes.byref(lat8), 1, ctypes.byref(v)) == 1
    from paper_1701_00426_amd import _lib
    c = _lib.StgTuneChoice()
    assert lib.stg_autotune_lookup(ctypes.byref(lat8), 3, 1, ctypes.byref(c)) == 0
    lib.stg_autotune_clear()
    assert lib.stg_autotune_fields_lookup(ctypes.byref(lat8), 3, ctypes.byref(v)) == 1
    assert lib.stg_autotune_lookup(ctypes.byref(lat8), 3, 1, ctypes.byref(c)) == 1


def test_tuning_knobs(lib):
    v = ctypes.c_int(-1)
    assert lib.stg_get_tuning(0, ctypes.byref(v)) == 0 and v.value == 1
    assert lib.stg_set_tuning(1, 3) == -1
    assert lib.stg_set_tuning(1, 2) == 0
    assert lib.stg_get_tuning(1, ctypes.byref(v)) == 0 and v.value == 2
    assert lib.stg_set_tuning(1, 1) == 0
    assert lib.stg_set_tuning(11, 1) == -1 and lib.stg_set_tuning(-1, 1) == -1
    # neighbour staging: 0 or 1, off by default
    assert lib.stg_get_tuning(2, ctypes.byref(v)) == 0 and v.value == 0
    assert lib.stg_set_tuning(2, 2) == -1
    assert lib.stg_set_tuning(2, 1) == 0
    assert lib.stg_get_tuning(2, ctypes.byref(v)) == 0 and v.value == 1
    assert lib.stg_set_tuning(2, 0) == 0
    # threads per site: 0 (automatic, the default), 1, 2 or 4
    assert lib.stg_get_tuning(3, ctypes.byref(v)) == 0 and v.value == 0
    assert lib.stg_set_tuning(3, 3) == -1
    assert lib.stg_set_tuning(3, 4) == 0
    assert lib.stg_get_tuning(3, ctypes.byref(v)) == 0 and v.value == 4
    assert lib.stg_set_tuning(3, 0) == 0
    # threads per link of the staple kernel: 0 (automatic), 1 or 2
    assert lib.stg_get_tuning(4, ctypes.byref(v)) == 0 and v.value == 0
    assert lib.stg_set_tuning(4, 3) == -1 and lib.stg_set_tuning(4, -1) == -1
    assert lib.stg_set_tuning(4, 1) == 0
    assert lib.stg_get_tuning(4, ctypes.byref(v)) == 0 and v.value == 1
    assert lib.stg_set_tuning(4, 0) == 0
    # tile shape of the pencil order: 0 .. 5
    assert lib.stg_get_tuning(5, ctypes.byref(v)) == 0 and v.value == 0
    assert lib.stg_set_tuning(5, 6) == -1 and lib.stg_set_tuning(5, -1) == -1
    assert lib.stg_set_tuning(5, 4) == 0
    assert lib.stg_get_tuning(5, ctypes.byref(v)) == 0 and v.value == 4
    assert lib.stg_set_tuning(5, 0) == 0
    # fields per launch: 0 (automatic), 1, 2, 4 or 8
    assert lib.stg_get_tuning(6, ctypes.byref(v)) == 0 and v.value == 0
    for bad in (3, 5, 16, -1):
        assert lib.stg_set_tuning(6, bad) == -1
    for good in (1, 2, 4, 8):
        assert lib.stg_set_tuning(6, good) == 0
        assert lib.stg_get_tuning(6, ctypes.byref(v)) == 0 and v.value == good
    assert lib.stg_set_tuning(6, 0) == 0
    # layer order: 0 (half-index order) or planes per group 1 .. 1024
    assert lib.stg_get_tuning(7, ctypes.byref(v)) == 0
    default = v.value
    assert lib.stg_set_tuning(7, -1) == -1 and lib.stg_set_tuning(7, 1025) == -1
    for good in (0, 1, 4, 1024):
        assert lib.stg_set_tuning(7, good) == 0
        assert lib.stg_get_tuning(7, ctypes.byref(v)) == 0 and v.value == good
    assert lib.stg_set_tuning(7, default) == 0
    # spread epilogue: 0 or 1
    assert lib.stg_get_tuning(8, ctypes.byref(v)) == 0
    default = v.value
    assert lib.stg_set_tuning(8, 2) == -1 and lib.stg_set_tuning(8, -1) == -1
    for good in (0, 1):
        assert lib.stg_set_tuning(8, good) == 0
        assert lib.stg_get_tuning(8, ctypes.byref(v)) == 0 and v.value == good
    assert lib.stg_set_tuning(8, default) == 0
    # field split: 0 (automatic, the default), -1 (off), 1 or 2 fields per wave
    assert lib.stg_get_tuning(9, ctypes.byref(v)) == 0 and v.value == 0
    assert lib.stg_set_tuning(9, 3) == -1 and lib.stg_set_tuning(9, -2) == -1
    for good in (1, 2, -1, 0):
        assert lib.stg_set_tuning(9, good) == 0
        assert lib.stg_get_tuning(9, ctypes.byref(v)) == 0 and v.value == good
    # CG form: 0 (automatic, the default), 1 (two reductions) or 2 (one reduction)
    assert lib.stg_get_tuning(10, ctypes.byref(v)) == 0 and v.value == 0
    assert lib.stg_set_tuning(10, 3) == -1 and lib.stg_set_tuning(10, -1) == -1
    for good in (2, 1, 0):
        assert lib.stg_set_tuning(10, good) == 0
        assert lib.stg_get_tuning(10, ctypes.byref(v)) == 0 and v.value == good


def test_cg_default_params(lib):
    from paper_1701_00426_amd import _lib
    p = _lib.StgCgParams()
    lib.stg_cg_default_params(ctypes.byref(p))
    assert p.tol == 1e-10 and p.max_iter == 100000 and p.mode == 0
    assert p.delta == 0.1 and p.poll_every == 0 and p.restart == -1


def test_staple_arguments_rejected_on_host(lib):
    """gauge_staples checks its arguments before any GPU work."""
    from paper_1701_00426_amd import _lib
    lat = _lat((4, 4, 4, 4))
    g = _lib.StgGauge()
    g.links = 0x1000
    g.fmt = 0

    def call(lattice=lat, gauge=g, c0=5.0 / 3.0, c1=-1.0 / 12.0, out=0x10000000):
        return lib.gauge_staples(ctypes.byref(lattice), ctypes.byref(gauge) if gauge else None,
                                 c0, c1, out, None)

    assert call(lattice=_lat((4, 3, 4, 4))) == -1
    assert call(gauge=None) == -1
    assert call(out=None) == -1
    assert call(out=0x10000008) == -1          # not 16-byte aligned
    assert call(out=0x1000 + 64) == -1         # overlaps the links
    assert call(c0=float("nan")) == -1
    assert call(c1=float("inf")) == -1
    bad = _lib.StgGauge()
    bad.links = 0x1000
    bad.fmt = 7
    assert call(gauge=bad) == -1
    assert b"format" in lib.stg_last_error()


def test_force_arguments_rejected_on_host(lib):
    """fermion_force checks its arguments before any GPU work."""
    from paper_1701_00426_amd import _lib
    lat = _lat((4, 4, 4, 4))
    g = _lib.StgGauge()
    g.links = 0x1000
    g.fmt = 1
    co = (ctypes.c_double * 2)(0.5, 0.25)

    # every call below must fail its checks: none may reach a launch
    def call(gauge=g, n=2, coeffs=co, x=0x1000000, y=0x2000000, out=0x3000000):
        return lib.fermion_force(ctypes.byref(lat), ctypes.byref(gauge), n, coeffs, x, y, out,
                                 None)

    assert call(n=0) == -1
    assert call(coeffs=None) == -1
    assert call(coeffs=(ctypes.c_double * 2)(0.5, float("nan"))) == -1
    assert call(x=None) == -1 and call(out=0x3000008) == -1
    assert call(y=0x1000000 + 64) == -1               # y overlaps x
    assert call(out=0x2000000 + 64) == -1             # out overlaps y
    f32 = _lib.StgGauge()
    f32.links = 0x1000
    f32.fmt = 2                                       # FP32 links: not for the force
    assert call(gauge=f32) == -1


def test_stout_arguments_rejected_on_host(lib):
    """stout_smear checks its arguments before any GPU work (every call here fails)."""
    from paper_1701_00426_amd import _lib
    lat = _lat((4, 4, 4, 4))
    g = _lib.StgGauge()
    g.links = 0x1000
    g.fmt = 0

    def call(gauge=g, rho=0.15, out=0x10000000):
        return lib.stout_smear(ctypes.byref(lat), ctypes.byref(gauge), rho, out, None)

    assert call(rho=float("nan")) == -1
    assert call(out=None) == -1 and call(out=0x10000004) == -1
    assert call(out=0x1000 + 4096) == -1           # overlaps the links
    f32 = _lib.StgGauge()
    f32.links = 0x1000
    f32.fmt = 2
    assert call(gauge=f32) == -1


def test_md_arguments_rejected_on_host(lib):
    """gauge_momentum_update and gauge_link_update check their arguments before any
    GPU work (every call here fails)."""
    from paper_1701_00426_amd import _lib
    lat = _lat((4, 4, 4, 4))
    g = _lib.StgGauge()
    g.links = 0x1000
    g.fmt = 1

    def mom_call(gauge=g, beta=5.0, eps=0.01, mom=0x10000000):
        return lib.gauge_momentum_update(ctypes.byref(lat), ctypes.byref(gauge), beta,
                                         5.0 / 3.0, -1.0 / 12.0, eps, mom, None)

    assert mom_call(beta=float("nan")) == -1 and mom_call(eps=float("inf")) == -1
    assert mom_call(mom=None) == -1 and mom_call(mom=0x1000 + 32) == -1
    f32 = _lib.StgGauge()
    f32.links = 0x1000
    f32.fmt = 3
    assert mom_call(gauge=f32) == -1

    def link_call(fmt=0, links=0x1000, eps=0.01, mom=0x10000000):
        return lib.gauge_link_update(ctypes.byref(lat), fmt, links, eps, mom, None)

    assert link_call(fmt=3) == -1 and link_call(fmt=9) == -1
    assert link_call(eps=float("nan")) == -1
    assert link_call(links=None) == -1 and link_call(mom=0x1008) == -1
    assert link_call(mom=0x1000 + 4096) == -1         # overlaps the links


def test_stout_backprop_arguments_rejected_on_host(lib):
    """stout_force_backprop checks its arguments before any GPU work (every call fails)."""
    from paper_1701_00426_amd import _lib
    lat = _lat((4, 4, 4, 4))
    g = _lib.StgGauge()
    g.links = 0x1000
    g.fmt = 0
    mb = 8 * 9 * 128 * 16

    def call(gauge=g, rho=0.15, sp=0x1000000, out=0x2000000, ws=0x3000000):
        return lib.stout_force_backprop(ctypes.byref(lat), ctypes.byref(gauge), rho, sp, out, ws,
                                        None)

    assert call(rho=float("nan")) == -1
    assert call(sp=None) == -1 and call(ws=0x3000008) == -1
    assert call(out=0x1000000 + mb - 16) == -1      # out overlaps sigma_smeared
    assert call(ws=0x1000 + 64) == -1               # ws overlaps the links
    f32 = _lib.StgGauge()
    f32.links = 0x1000
    f32.fmt = 2
    assert call(gauge=f32) == -1
