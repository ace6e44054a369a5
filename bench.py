"""Benchmark of the even/odd staggered operator and its CG solves on one MI355X.

Workload (the plain FP64 configuration at scale): 32^4 lattice, seeded random
SU(3) links with standard staggered phases and antiperiodic time boundary,
m = 0.01, one complex Gaussian even-site right-hand side.

  * value: D_eo apply bandwidth in GB/s at FP64 with 12-real links (the paper's
    storage), algorithmic bytes / mean kernel duration, measured with HIP events
    on the library's stream over back-to-back applies that rotate through three
    link/field copies (1.36 GB working set, above the 256 MB Infinity Cache).
  * a step: CG solves of (m^2 - D_eo D_oe) x = b to |r|/|b| <= 1e-10: FP64; mixed
    precision with FP32-12 inner links and FP64 reliable updates, for one RHS and
    for eight RHS in one call; mixed precision with BF16-12 inner links.
  * roofline: the dominant kernel (the hop) against the 8 TB/s HBM peak.
  * cpu_baseline: the FP64 C oracle's D_eo on the host cores, bounded sample.

Prints one JSON line.  `python bench.py --gpus N` with N > 1 exits with a
message: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "D_eo apply GB/s (% HBM peak); mixed vs FP64 CG time to |r|/|b|<1e-10 per RHS"
HBM_PEAK_GBS = 8000.0
DIMS = (32, 32, 32, 32)
MASS = 0.01
TOL = 1e-10
# algorithmic bytes per output site of one hop: 8 links + 1 input + 1 output vector
BYTES_PER_SITE = {"c128_18": 8 * 144 + 48 + 48, "c128_12": 8 * 96 + 48 + 48,
                  "c64_12": 8 * 48 + 24 + 24, "bf16_12": 8 * 24 + 24 + 24}
# The naive byte model of a hop: every neighbour vector read separately (8 per site),
# no reuse through the caches.
NAIVE_BYTES_PER_SITE = {"c128_18": 8 * 144 + 8 * 48 + 48, "c128_12": 8 * 96 + 8 * 48 + 48,
                        "c64_12": 8 * 48 + 8 * 24 + 24, "bf16_12": 8 * 24 + 8 * 24 + 24}
FLOPS_PER_SITE = 570  # 8 SU(3) mat-vecs (66) + 7 colour-vector sums (6); reconstruction excluded
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hop_traffic_32x32x32x32.json")
KERNEL_SOURCES = ["paper_1701_00426_amd/csrc/hop.hip",
                  "paper_1701_00426_amd/csrc/hop_core.hpp",
                  "paper_1701_00426_amd/csrc/kernels.hpp",
                  "paper_1701_00426_amd/csrc/device_common.hpp"]


STAPLE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "staples_traffic_32x32x32x32.json")
STAPLE_SOURCES = ["paper_1701_00426_amd/csrc/staple.hip",
                  "paper_1701_00426_amd/csrc/staple.hpp",
                  "paper_1701_00426_amd/csrc/pencil.hpp",
                  "paper_1701_00426_amd/csrc/kernels.hpp",
                  "paper_1701_00426_amd/csrc/device_common.hpp"]


def kernel_hash(sources=None) -> str:
    h = hashlib.sha256()
    for f in (sources or KERNEL_SOURCES):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path, sources):
    """HBM bytes per launch from a committed PMC summary, or None when the kernel
    sources have changed since the counters were taken."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        tr = json.load(fh)
    if tr.get("kernel_hash") != kernel_hash(sources):
        return None
    return tr.get("bytes_per_launch")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_applies(stg, torch, gauges, fields, outs, parity, n):
    """Mean duration (s) of one hop over n back-to-back launches rotating copies."""
    fn = stg.dirac_apply_eo if parity == 0 else stg.dirac_apply_oe
    stream = torch.cuda.current_stream()
    for i in range(3):
        fn(gauges[i % len(gauges)], fields[i % len(fields)], outs[i % len(outs)])
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for i in range(n):
        k = i % len(gauges)
        fn(gauges[k], fields[k % len(fields)], outs[k % len(outs)])
    t1.record(stream)
    t1.synchronize()
    return t0.elapsed_time(t1) * 1e-3 / n


def time_pack(stg, torch, links, dims, fmt, reps=20):
    """stg_pack_links from full complex128 links into one compressed format: HIP-event
    mean over reps calls after one warm-up; GB/s of the bytes read (144 B per link)
    plus the bytes written (the packed field)."""
    stg.stg_pack_links(dims, links, fmt)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(reps):
        out = stg.stg_pack_links(dims, links, fmt)
    t1.record(stream)
    t1.synchronize()
    dt = t0.elapsed_time(t1) * 1e-3 / reps
    nbytes = links.numel() * links.element_size() + out.numel()
    return {"us": round(dt * 1e6, 2), "GBs": round(nbytes / dt / 1e9, 1),
            "bytes": int(nbytes)}


def _native_oracle():
    """The C oracle compiled with -O3 -march=native on this host (a private copy: the
    tests keep the portable build)."""
    import tempfile
    import oracle
    return oracle.COracle(oracle.build(native_dir=tempfile.mkdtemp(prefix="stg_oracle_")))


def cpu_baseline(links, b, vh, seconds=10.0, one_core_seconds=4.0):
    """The FP64 C oracle's D_eo on the host cores, bounded samples on all cores and
    on one core; the metric's unit (GB/s on the same byte model as value)."""
    from oracle import oracle_np as on
    orc = _native_oracle()
    phases = on.standard_phases(DIMS)
    cores = orc.num_threads()

    def sample(budget):
        t = time.perf_counter()
        orc.d_eo(DIMS, links, phases, b)
        one = time.perf_counter() - t
        n = max(1, min(50, int(budget / max(one, 1e-3))))
        t = time.perf_counter()
        for _ in range(n):
            orc.d_eo(DIMS, links, phases, b)
        return n, (time.perf_counter() - t) / n

    n, dt = sample(seconds)
    orc.set_num_threads(1)
    n1, dt1 = sample(one_core_seconds)
    orc.set_num_threads(cores)
    gbs = BYTES_PER_SITE["c128_12"] * vh / dt / 1e9
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} D_eo applies of the FP64 C oracle (gcc -O3 -march=native, OpenMP "
                      f"over {cores} threads, full 3x3 links) at 32^4, {dt * 1e3:.1f} ms each, "
                      f"same byte model as value (864 B/site); one core: {n1} applies, "
                      f"{dt1 * 1e3:.1f} ms each",
            "ms_per_apply": round(dt * 1e3, 3),
            "one_core": {"GBs": round(BYTES_PER_SITE["c128_12"] * vh / dt1 / 1e9, 3),
                         "ms_per_apply": round(dt1 * 1e3, 3), "applies": n1}}


def oracle_solution(links, b, tol=1e-12):
    """x* = the FP64 C oracle's own CG solution of the benchmark system to |r|/|b| <=
    tol on all host cores (textbook CG on the full 3x3 links), and its time to
    solution: the CPU time-to-solution figure of the FP64 solve."""
    import numpy as np
    from oracle import oracle_np as on
    import threading
    orc = _native_oracle()
    phases = on.standard_phases(DIMS)
    done = threading.Event()

    def ticker():  # progress lines while the C call runs (it releases the GIL)
        while not done.wait(20.0):
            log(f"  oracle CG running, {time.perf_counter() - t:.0f} s")

    t = time.perf_counter()
    th = threading.Thread(target=ticker, daemon=True)
    th.start()
    try:
        x, iters, res, st = orc.cg(DIMS, links, phases, MASS, b, tol=tol, max_iter=20000)
    finally:
        done.set()
        th.join()
    dt = time.perf_counter() - t
    del np
    return x, {"tol": tol, "status": int(st), "iters": int(iters), "true_rel_resid": res,
               "seconds": round(dt, 2), "cores": orc.num_threads(),
               "build": "gcc -O3 -march=native -fopenmp (dslash over OpenMP threads)"}


def copy_ceiling(torch, nbytes=1 << 30, reps=20):
    """Read + write GB/s of a plain 1 GiB device copy (HIP events): the practical
    ceiling a streaming kernel reaches on this GPU."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    t1.synchronize()
    dt = t0.elapsed_time(t1) * 1e-3 / reps
    del src, dst
    torch.cuda.empty_cache()
    return round(2 * nbytes / dt / 1e9, 1)


def read_ceiling(torch, nbytes=1 << 30, reps=20):
    """Read GB/s of the fastest of a few plain read-only library reductions over three
    rotating 1 GiB device buffers (beyond the Infinity Cache; HIP events): a floor on
    the practical ceiling of a read-dominated stream on this GPU."""
    bufs = [torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0") for _ in range(3)]
    ops = {"dot": lambda i: torch.dot(bufs[i % 3], bufs[(i + 1) % 3]),
           "sum": lambda i: bufs[i % 3].sum(),
           "rowsum": lambda i: bufs[i % 3].view(-1, 4096).sum(1),
           "amax": lambda i: bufs[i % 3].amax()}
    best = {}
    for name, op in ops.items():
        for i in range(3):
            op(i)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for i in range(reps):
            op(i)
        t1.record()
        t1.synchronize()
        dt = t0.elapsed_time(t1) * 1e-3 / reps
        read = 2 * nbytes if name == "dot" else nbytes
        best[name] = round(read / dt / 1e9, 1)
    del bufs
    torch.cuda.empty_cache()
    return max(best.values()), best


def calibrate_copy():
    """A plain device-to-device copy of 1 GiB, 10 times: FETCH_SIZE / WRITE_SIZE per
    dispatch of this kernel against the known 1 GiB read and 1 GiB write give the
    scale factor of the counters."""
    import torch
    n = 1 << 30
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 10
    print(json.dumps({"calibrate_copy_bytes_read": n, "bytes_written": n,
                      "GBs_read_plus_write": round(2 * n / dt / 1e9, 1)}), flush=True)


def bench_multishift():
    """24^3 x 48, m = 0.005, 16 shifts log-spaced in [1e-4, 10], 8 RHS in one solve:
    multi-shift stage in FP32 (FP32-12 links) then per-(shift, RHS) mixed refinement to
    the FP64 true residual 1e-10."""
    import torch
    import paper_1701_00426_amd as stg
    import seeded_inputs as si
    dims, mass, nrhs = (24, 24, 24, 48), 0.005, 8
    shifts = si.log_shifts(16, 1e-4, 10.0)
    dev = torch.device("cuda:0")
    log("generating 24^3x48 inputs")
    links = torch.from_numpy(si.su3_links(dims, 1701, 4, 0)).to(dev)
    b = torch.from_numpy(si.gaussian_field(dims, nrhs, 426, 4, 0)).to(dev)
    hi = stg.pack_gauge(dims, links, "c128_12")
    lo = stg.pack_gauge(dims, links, "c64_12")
    ws = torch.empty(stg.stg_workspace_bytes(dims, nrhs, len(shifts), stg.STG_CG_MIXED),
                     dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, st, stats = stg.multishift_cg_solve(hi, mass, shifts, b, lo=lo, ws=ws,
                                           tol=TOL)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    flat = [s for row in stats for s in row]
    out = {"workload": "multishift 24^3x48 m=0.005, 16 shifts in [1e-4, 10], 8 RHS, FP32-12 + "
                       "FP64 refinement to 1e-10",
           "status": st, "seconds": round(dt, 3), "s_per_rhs": round(dt / nrhs, 4),
           "worst_true_rel_resid": max(s["true_rel_resid"] for s in flat),
           "iters_smallest_shift": max(s["iters"] for s in stats[0]),
           "iters_largest_shift": max(s["iters"] for s in stats[-1]),
           "refine_reliable_updates_max": max(s["reliable_updates"] for s in flat),
           "workspace_GB": round(ws.numel() / 1e9, 2)}
    out["ms_stage_bytes"] = multishift_stage_bytes(dims, stats, 8)
    print(json.dumps(out), flush=True)


def multishift_stage_bytes(dims, stats, elem):
    """Algorithmic bytes of the multi-shift stage (each datum once per kernel), from
    the iterations each (shift, RHS) system took part in (stats[k][j]["ms_iters"]):
    the operator (two hops per iteration; one link read per launch serves the 8
    fields of a launch) against the vector kernels, the shift update above all.
    elem: bytes per complex entry of the stage's vectors (8 for FP32)."""
    vh = 1
    for d in dims:
        vh *= d
    vh //= 2
    vec = 3 * elem                                # one colour vector per site
    nshift, nrhs = len(stats), len(stats[0])
    base = [max(stats[k][j]["ms_iters"] for k in range(nshift)) for j in range(nrhs)]
    shift_iters = sum(stats[k][j]["ms_iters"] for k in range(nshift) for j in range(nrhs))
    launches = sum(max(base[j0:j0 + 8]) for j0 in range(0, nrhs, 8))   # 8 fields per launch
    link_bytes = 8 * 6 * elem                      # FP32-12: 48 B per link, 8 per site
    hops = vh * (2 * launches * link_bytes + sum(base) * (2 * vec + 3 * vec))
    r_update = vh * sum(base) * 3 * vec            # r, q read, r written
    # base p: r, p read, p written; each (shift, RHS) still in the stage: p_k, x_k read,
    # x_k and p_k written (r is re-read by every shift's blocks from L2: counted once)
    p_update = vh * (sum(base) * 3 * vec + shift_iters * 4 * vec)
    return {"hop_launch_pairs": launches, "base_iters": base, "shift_iters_total": shift_iters,
            "hops": hops, "ms_r_update": r_update, "ms_p_update": p_update,
            "model": "hops: 2 x 8 links x 48 B per launch + per field 2 x (in + out) + p; "
                     "ms_r_update: 3 vectors per field; ms_p_update: 3 vectors per field + "
                     "4 vectors per (shift, RHS) iteration; vector = 24 B per site"}


def bench_rational():
    """The multi-shift workload of bench_multishift combined into a rational function
    of the normal operator: y = a0 b + sum_k a_k (A + sigma_k)^-1 b with synthetic
    coefficients a_k = 1 / (1 + k), a0 = 0.5 (a caller's RHMC approximation would
    supply its own), 8 RHS, FP32-12 multi-shift stage + FP64 refinement to 1e-10."""
    import torch
    import paper_1701_00426_amd as stg
    import seeded_inputs as si
    dims, mass, nrhs = (24, 24, 24, 48), 0.005, 8
    shifts = si.log_shifts(16, 1e-4, 10.0)
    coeffs = [1.0 / (1 + k) for k in range(len(shifts))]
    dev = torch.device("cuda:0")
    log("generating 24^3x48 inputs")
    links = torch.from_numpy(si.su3_links(dims, 1701, 4, 0)).to(dev)
    b = torch.from_numpy(si.gaussian_field(dims, nrhs, 426, 4, 0)).to(dev)
    hi = stg.pack_gauge(dims, links, "c128_12")
    lo = stg.pack_gauge(dims, links, "c64_12")
    ws = torch.empty(stg.stg_rational_workspace_bytes(dims, nrhs, len(shifts), stg.STG_CG_MIXED),
                     dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y, st, stats = stg.rational_apply(hi, mass, shifts, coeffs, 0.5, b, lo=lo, ws=ws, tol=TOL)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    flat = [s for row in stats for s in row]
    vh = stg.half_volume(dims)
    out = {"workload": "rational function a0 b + sum_k a_k (A + sigma_k)^-1 b, 24^3x48 "
                       "m=0.005, 16 poles in [1e-4, 10], 8 RHS, FP32-12 + FP64 refinement "
                       "to 1e-10",
           "status": st, "seconds": round(dt, 3), "s_per_rhs": round(dt / nrhs, 4),
           "worst_true_rel_resid": max(s["true_rel_resid"] for s in flat),
           "sum_kernel_bytes": (len(shifts) + 2) * 16 * 3 * vh * nrhs,
           "workspace_GB": round(ws.numel() / 1e9, 2)}
    print(json.dumps(out), flush=True)


def _batch_run(shapes_masses, label, form=0):
    """One cg_solve_batch (mixed FP32-12; STG_TUNE_CG_FORM `form` for the batch) over the
    solves, against the same solves launched one after another with cg_solve in the
    automatic form; nrhs_i = 1 + (i mod 4)."""
    import torch
    import paper_1701_00426_amd as stg
    import seeded_inputs as si
    dev = torch.device("cuda:0")
    solves = []
    for i, (dims, m) in enumerate(shapes_masses):
        nrhs = 1 + (i % 4)
        links = torch.from_numpy(si.su3_links(dims, 1701, 5, i)).to(dev)
        b = torch.from_numpy(si.gaussian_field(dims, nrhs, 426, 5, i)).to(dev)
        solves.append(dict(hi=stg.pack_gauge(dims, links, "c128_12"),
                           lo=stg.pack_gauge(dims, links, "c64_12"), mass=m, b=b))
        del links
    torch.cuda.synchronize()
    stg.stg_set_tuning(stg._lib.STG_TUNE_CG_FORM, form)
    t0 = time.perf_counter()
    xs, st, stats = stg.cg_solve_batch(solves, tol=TOL)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    stg.stg_set_tuning(stg._lib.STG_TUNE_CG_FORM, 0)
    t1 = time.perf_counter()
    worst_single = 0.0
    for sv in solves:
        _, s1, st1 = stg.cg_solve(sv["hi"], sv["mass"], sv["b"], lo=sv["lo"], tol=TOL)
        worst_single = max(worst_single, max(q["true_rel_resid"] for q in st1))
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t1
    flat = [q for row in stats for q in row]
    out = {"workload": label, "cg_form": form, "status": st, "makespan_s": round(t_batch, 3),
           "sequential_cg_solve_s": round(t_seq, 3),
           "speedup_vs_sequential": round(t_seq / t_batch, 3),
           "worst_true_rel_resid": max(q["true_rel_resid"] for q in flat),
           "worst_true_rel_resid_sequential": worst_single,
           "max_iters": max(q["iters"] for q in flat), "nsys": len(flat)}
    print(json.dumps(out), flush=True)


def bench_batch(form=0):
    """12 solves: two each on 8^4, 12^4, 16^4, 16^3x32, 24^4, 32^4 at m = 0.01 and 0.05."""
    shapes = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16), (16, 16, 16, 32),
              (24, 24, 24, 24), (32, 32, 32, 32)]
    _batch_run([(d, m) for d in shapes for m in (0.01, 0.05)],
               "uneven batch: 12 solves (8^4, 12^4, 16^4, 16^3x32, 24^4, 32^4 x m in "
               "{0.01, 0.05}), 30 RHS, FP32-12 + FP64 reliable updates, tol 1e-10", form)


def bench_batch_small(form=0):
    """48 small solves: 16 each on 8^4, 12^4 and 16^4 at m in {0.05, 0.1}: the regime the
    batch is for, where one launch per kernel and solve is all overhead."""
    shapes = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16)]
    _batch_run([(d, (0.05, 0.1)[k % 2]) for d in shapes for k in range(16)],
               "uneven batch of small lattices: 48 solves (16 each on 8^4, 12^4, 16^4, m in "
               "{0.05, 0.1}), 120 RHS, FP32-12 + FP64 reliable updates, tol 1e-10", form)


# The paper's Table 3 lattices, written N0 x N1 x N2 x N3 with time last, and its
# per-site times on other hardware [ns]: (K80 GPU SP, DP, P100 SP, DP).
PAPER_TABLE3 = {(32, 32, 8, 32): (4.19, 8.51, 1.77, 3.07), (32, 32, 32, 8): (4.15, 8.39, 1.22, 2.48),
                (24, 24, 24, 24): (4.43, 8.62, 1.58, 2.90), (32, 32, 32, 32): (4.02, 9.54, 1.32, 2.40),
                (32, 32, 32, 36): (4.03, 8.48, 1.46, 2.54)}


def bench_shapes():
    """D_eo on the paper's Table 3 lattice shapes at FP64-12 and FP32-12: default launch
    shape and the autotuner's choice; ns per site as (t(D_eo) + t(D_oe)) / V."""
    import torch
    import paper_1701_00426_amd as stg
    import seeded_inputs as si
    dev = torch.device("cuda:0")
    rows = []
    for dims, paper in PAPER_TABLE3.items():
        vh = stg.half_volume(dims)
        links = torch.from_numpy(si.su3_links(dims, 1701, 6, 0)).to(dev)
        b = torch.from_numpy(si.gaussian_field(dims, 1, 426, 6, 0)).to(dev)
        for fmt in ("c128_12", "c64_12"):
            cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
            gauges = [stg.pack_gauge(dims, links if i == 0 else links.clone(), fmt)
                      for i in range(3)]
            fields = [b.to(cdt).clone() for _ in range(3)]
            outs = [torch.empty_like(fields[0]) for _ in range(3)]
            stg.library().stg_autotune_clear()
            t_def = time_applies(stg, torch, gauges, fields, outs, 0, 200)
            t_def_oe = time_applies(stg, torch, gauges, fields, outs, 1, 200)
            choice = stg.stg_autotune(gauges[0], 1)
            t_tun = time_applies(stg, torch, gauges, fields, outs, 0, 200)
            t_tun_oe = time_applies(stg, torch, gauges, fields, outs, 1, 200)
            bps = BYTES_PER_SITE[fmt]
            rows.append({"lattice": "x".join(map(str, dims)), "format": fmt,
                         "deo_us_default": round(t_def * 1e6, 2),
                         "GBs_default": round(bps * vh / t_def / 1e9, 1),
                         "deo_us_tuned": round(t_tun * 1e6, 2),
                         "GBs_tuned": round(bps * vh / t_tun / 1e9, 1),
                         "tuned": {k: v for k, v in choice.items() if k != "us"},
                         "ns_per_site": round((t_tun + t_tun_oe) * 1e9 / (2 * vh), 4),
                         "paper_ns_per_site_K80_P100": paper[1::2] if fmt == "c128_12"
                         else paper[0::2]})
            log(json.dumps(rows[-1]))
            del gauges, fields, outs
        del links
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "paper Table 3 shapes, D_eo FP64-12 / FP32-12", "rows": rows}),
          flush=True)


# Staples of the tree-level Symanzik gauge force.  Flops of the kernel's factored
# evaluation per link: per neighbouring direction and side, 8 SU(3) products into a
# fresh matrix (27 complex multiplies + 18 complex adds = 198 flops) and 3 into an
# accumulator (216 flops) plus the weighting (72 flops): 2304; x 2 sides x 3
# directions = 13824 (row-2 reconstruction of the 12-real formats not counted).
STAPLE_FLOPS_PER_LINK = 13824
# Vector FMA peak without packed-FP32 instructions: 256 CUs x 4 SIMDs x 16 lanes x
# 2 flops x 2.4 GHz, the same for FP64 and for unpacked FP32.
ALU_PEAK_TFLOPS = 78.6
# Paper Table 4: ns per site of the pure-gauge MD step (whose most expensive part is
# the staples) on NVIDIA GK201 (K80) and P100: context only, a different quantity.
PAPER_TABLE4 = {(32, 32, 8, 32): (193.79, 51.80), (32, 32, 32, 8): (190.39, 51.69),
                (24, 24, 24, 24): (212.04, 53.74), (32, 32, 32, 32): (201.82, 51.72),
                (32, 32, 32, 36): (208.54, 52.62)}
STAPLE_LINK_BYTES = {"c128_18": 144, "c128_12": 96, "c64_12": 48, "bf16_12": 24}
# threads per link gauge_staples takes by default (2 for FP64 links, 1 for FP32 ones)
STAPLE_DEFAULT_THREADS = {"c128_18": 2, "c128_12": 2, "c64_12": 1, "bf16_12": 1}


def time_staples(stg, torch, gauges, outs, n):
    """Mean duration (s) of one gauge_staples launch over n back-to-back launches
    rotating link copies, HIP events on the launching stream."""
    stream = torch.cuda.current_stream()
    for i in range(3):
        stg.gauge_staples(gauges[i % len(gauges)], out=outs[i % len(outs)])
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for i in range(n):
        stg.gauge_staples(gauges[i % len(gauges)], out=outs[i % len(outs)])
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / 1e3 / n


def staple_cpu_baseline(dims=(8, 8, 8, 8)):
    """The NumPy oracle's staples of a whole 8^4 lattice (all 4 directions), timed
    on the host: ns per site."""
    import seeded_inputs as si
    from oracle import oracle_np as on
    links = si.su3_links(dims, 1701, 7, 1)
    t0 = time.perf_counter()
    reps = 0
    while True:
        on.staples(dims, links)
        reps += 1
        if time.perf_counter() - t0 > 5.0:
            break
    dt = (time.perf_counter() - t0) / reps
    v = 2 * on.half_volume(dims)
    return {"value": round(dt * 1e9 / v, 1), "unit": "ns/site", "cores": 1, "kind": "oracle",
            "sample": f"NumPy oracle, whole {'x'.join(map(str, dims))} lattice, {reps} passes"}


def bench_staples(profile=False, no_cpu=False, applies=100):
    """Staples of every link (gauge_staples) on the paper's Table 4 lattice shapes at
    FP64-12 and FP32-12, and at 32^4 in every format; ns per site = t / V (all four
    directions in one launch).  The first line printed is the 32^4 FP64-12 one with
    its ALU roofline."""
    import torch
    import paper_1701_00426_amd as stg
    import seeded_inputs as si
    dev = torch.device("cuda:0")
    shapes = [(32, 32, 32, 32)] if profile else list(PAPER_TABLE4)
    rows = []
    head = None
    for dims in shapes:
        vh = stg.half_volume(dims)
        links = torch.from_numpy(si.su3_links(dims, 1701, 7, 0)).to(dev)
        fmts = ["c128_12"] if profile else (
            ["c128_12", "c128_18", "c64_12", "bf16_12"] if dims == (32, 32, 32, 32)
            else ["c128_12", "c64_12"])
        key = stg._lib.STG_TUNE_STAPLE_THREADS
        runs = [(fmt, 0) for fmt in fmts]
        if dims == (32, 32, 32, 32) and not profile:
            # the non-default threads per link too, for comparison
            runs = [(fmt, t) for fmt in fmts for t in (0, 3 - STAPLE_DEFAULT_THREADS[fmt])]
        cur = None
        for fmt, threads in runs:
            if cur != fmt:
                gauges = [stg.pack_gauge(dims, links if i == 0 else links.clone(), fmt)
                          for i in range(2)]
                cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
                outs = [torch.empty((8, 3, 3, vh), dtype=cdt, device=dev) for _ in range(2)]
                cur = fmt
            stg.stg_set_tuning(key, threads)
            dt = time_staples(stg, torch, gauges, outs, applies)
            stg.stg_set_tuning(key, 0)
            tflops = STAPLE_FLOPS_PER_LINK * 8 * vh / dt / 1e12
            row = {"lattice": "x".join(map(str, dims)), "format": fmt,
                   "threads_per_link": threads or STAPLE_DEFAULT_THREADS[fmt],
                   "launch_us": round(dt * 1e6, 2),
                   "ns_per_site": round(dt * 1e9 / (2 * vh), 4),
                   "TFLOPs": round(tflops, 2), "frac_alu": round(tflops / ALU_PEAK_TFLOPS, 4),
                   "algorithmic_GBs": round((STAPLE_LINK_BYTES[fmt] + (144 if cdt ==
                                             torch.complex128 else 72)) * 8 * vh / dt / 1e9, 1),
                   "paper_gauge_md_ns_per_site_K80_P100": PAPER_TABLE4[dims]}
            rows.append(row)
            log(json.dumps(row))
            if dims == (32, 32, 32, 32) and fmt == "c128_12" and threads == 0:
                head = row
        del gauges, outs, links
        torch.cuda.empty_cache()
    out = {"workload": "staples of the tree-level Symanzik gauge force, every link, "
                       "paper Table 4 shapes", "rows": rows}
    if head is not None:
        out["roofline"] = {"bound": "alu", "kernel": "staple_kernel<double, FP64-12> 32^4",
                           "achieved": head["TFLOPs"], "peak": ALU_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": head["frac_alu"],
                           "traffic": measured_traffic(STAPLE_TRAFFIC_FILE, STAPLE_SOURCES),
                           "kernel_hash": kernel_hash(STAPLE_SOURCES)}
    if not no_cpu and not profile:
        out["cpu_baseline"] = staple_cpu_baseline()
    print(json.dumps(out), flush=True)


def bench_force(profile=False, applies=50):
    """fermion_force at 32^4 with 16 poles (one pseudofermion of the multi-shift
    workload): the D_oe hops of the 16 solutions plus the outer-product kernel.
    The solutions are seeded Gaussian fields (the cost does not depend on the
    values).  Reports the whole call, the hops alone (dirac_apply_oe on the 16
    fields) and the difference, the force kernel, with its algorithmic GB/s."""
    import torch
    import paper_1701_00426_amd as stg
    import seeded_inputs as si
    dev = torch.device("cuda:0")
    dims, n = (32, 32, 32, 32), 16
    vh = stg.half_volume(dims)
    links = torch.from_numpy(si.su3_links(dims, 1701, 8, 0)).to(dev)
    gauge = stg.pack_gauge(dims, links, "c128_12")
    xs = torch.from_numpy(si.gaussian_field(dims, n, 426, 8, 0)).to(dev)
    coeffs = [1.0 / (1 + k) for k in range(n)]
    y = torch.empty_like(xs)
    out = torch.empty((8, 3, 3, vh), dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(reps):
            fn()
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / 1e3 / reps

    t_all = timed(lambda: stg.fermion_force(gauge, coeffs, xs, y_odd=y, out=out), applies)
    if profile:
        print(json.dumps({"profile": "fermion_force 32^4 16 poles", "calls": applies,
                          "mean_call_us": round(t_all * 1e6, 2)}), flush=True)
        return
    t_hop = timed(lambda: stg.dirac_apply_oe(gauge, xs, y), applies)
    t_force = t_all - t_hop
    force_bytes = (2 * n * 48 + 8 * 144) * vh
    print(json.dumps({
        "workload": "fermion force, 32^4, 16 poles, FP64-12 links: D_oe of the 16 solutions "
                    "+ outer-product kernel",
        "call_ms": round(t_all * 1e3, 3), "doe_16_fields_ms": round(t_hop * 1e3, 3),
        "force_kernel_ms": round(t_force * 1e3, 3),
        "force_kernel_algorithmic_bytes": force_bytes,
        "force_kernel_GBs": round(force_bytes / t_force / 1e9, 1),
        "force_kernel_frac_hbm": round(force_bytes / t_force / 1e9 / HBM_PEAK_GBS, 4),
        "ns_per_site": round(t_all * 1e9 / (2 * vh), 3)}), flush=True)


# One stout-smearing step per link: 12 SU(3) products for the six 3-link paths
# (2484 flop), Omega (198), Q^2 and Tr Q^3 (261), exp(iQ) = f0 + f1 Q + f2 Q^2 (189)
# and exp(iQ) U (198), plus the weighting: about 3375 flop (trigonometric functions
# and the row-2 reconstruction of FP64-12 links not counted).
STOUT_FLOPS_PER_LINK = 3375


def bench_stout(profile=False, applies=100):
    """Two stout levels (rho = 0.15) of a 32^4 FP64-12 gauge field: level 1 reads
    FP64-12 links, level 2 the FP64-18 output of level 1; HIP events per level."""
    import torch
    import paper_1701_00426_amd as stg
    import seeded_inputs as si
    dev = torch.device("cuda:0")
    dims = (32, 32, 32, 32)
    vh = stg.half_volume(dims)
    links = torch.from_numpy(si.su3_links(dims, 1701, 9, 0)).to(dev)
    g0 = stg.pack_gauge(dims, links, "c128_12")
    del links
    u1 = torch.empty((8, 3, 3, vh), dtype=torch.complex128, device=dev)
    u2 = torch.empty_like(u1)
    g1 = stg.pack_gauge(dims, u1, "c128_18")
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(reps):
            fn()
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / 1e3 / reps

    t1 = timed(lambda: stg.stout_smear(g0, 0.15, out=u1), applies)
    if profile:
        print(json.dumps({"profile": "stout level FP64-12 -> FP64-18, 32^4", "calls": applies,
                          "mean_launch_us": round(t1 * 1e6, 2)}), flush=True)
        return
    t2 = timed(lambda: stg.stout_smear(g1, 0.15, out=u2), applies)
    rows = []
    for label, t, lb in (("level 1 (FP64-12 in)", t1, 96), ("level 2 (FP64-18 in)", t2, 144)):
        tf = STOUT_FLOPS_PER_LINK * 8 * vh / t / 1e12
        rows.append({"step": label, "launch_us": round(t * 1e6, 2),
                     "ns_per_site": round(t * 1e9 / (2 * vh), 4), "TFLOPs": round(tf, 2),
                     "frac_alu": round(tf / ALU_PEAK_TFLOPS, 4),
                     "algorithmic_GBs": round((lb + 144) * 8 * vh / t / 1e9, 1),
                     "frac_hbm": round((lb + 144) * 8 * vh / t / 1e9 / HBM_PEAK_GBS, 4)})
    print(json.dumps({"workload": "stout smearing, 32^4, rho = 0.15, two levels",
                      "rows": rows}), flush=True)


def bench_tiles(applies=30):
    """The pencil tile shapes (STG_TUNE_PENCIL_TILE 0 .. 5) at 32^4 for the kernels that
    visit links or sites in pencil order: the fermion force with 16 poles (whole call),
    staples FP64-12 (2 threads per link) and FP32-12, and one stout level from FP64-12
    links."""
    import torch
    import paper_1701_00426_amd as stg
    import seeded_inputs as si
    dev = torch.device("cuda:0")
    dims = (32, 32, 32, 32)
    vh = stg.half_volume(dims)
    links = torch.from_numpy(si.su3_links(dims, 1701, 7, 0)).to(dev)
    g64 = [stg.pack_gauge(dims, links if i == 0 else links.clone(), "c128_12") for i in range(2)]
    g32 = [stg.pack_gauge(dims, links.clone(), "c64_12") for _ in range(2)]
    del links
    o64 = [torch.empty((8, 3, 3, vh), dtype=torch.complex128, device=dev) for _ in range(2)]
    o32 = [torch.empty((8, 3, 3, vh), dtype=torch.complex64, device=dev) for _ in range(2)]
    stream = torch.cuda.current_stream()
    key = stg._lib.STG_TUNE_PENCIL_TILE
    names = ["32x2x4", "32x4x2", "16x4x4", "16x8x4", "8x8x8", "32x8x2"]

    def timed(fn):
        for i in range(3):
            fn(i)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for i in range(applies):
            fn(i)
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / 1e3 / applies

    xs = torch.from_numpy(si.gaussian_field(dims, 16, 426, 8, 0)).to(dev)
    ys = torch.empty_like(xs)
    fo = torch.empty((8, 3, 3, vh), dtype=torch.complex128, device=dev)
    coeffs = [1.0 / (1 + k) for k in range(16)]
    rows = []
    for shape, name in enumerate(names):
        stg.stg_set_tuning(key, shape)
        rows.append({
            "force_16_poles_us": round(1e6 * timed(
                lambda i: stg.fermion_force(g64[i % 2], coeffs, xs, y_odd=ys, out=fo)), 1),
            "tile": name,
            "staples_fp64_12_us": round(1e6 * timed(
                lambda i: stg.gauge_staples(g64[i % 2], out=o64[i % 2])), 1),
            "staples_fp32_12_us": round(1e6 * timed(
                lambda i: stg.gauge_staples(g32[i % 2], out=o32[i % 2])), 1),
            "stout_fp64_12_us": round(1e6 * timed(
                lambda i: stg.stout_smear(g64[i % 2], 0.15, out=o64[i % 2])), 1)})
        log(json.dumps(rows[-1]))
    stg.stg_set_tuning(key, 0)
    print(json.dumps({"workload": "pencil tile shapes at 32^4", "rows": rows}), flush=True)


def bench_small(reps=5):
    """The small configuration: 8^4, m = 0.1, FP64-18 links, one RHS (latency-bound:
    1.8 MB per hop).  Hop and normal-operator times (HIP events), FP64 CG to 1e-10:
    wall time per solve (best of reps) and per iteration; the FP64 C oracle's CG on the
    same inputs on the host cores as the CPU baseline."""
    import numpy as np
    import torch
    import paper_1701_00426_amd as stg
    import seeded_inputs as si
    import oracle
    from oracle import oracle_np as on
    dev = torch.device("cuda:0")
    dims, mass = (8, 8, 8, 8), 0.1
    links_np = si.su3_links(dims, 1701, 1, 0)
    b_np = si.gaussian_field(dims, 1, 426, 1, 0, 0)
    gauge = stg.pack_gauge(dims, torch.from_numpy(links_np).to(dev), "c128_18")
    b = torch.from_numpy(b_np).to(dev)
    stream = torch.cuda.current_stream()

    def timed(fn, n=2000):
        for _ in range(20):
            fn()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(n):
            fn()
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / 1e3 / n

    out = torch.empty_like(b)
    tmp = torch.empty_like(b)
    t_eo = timed(lambda: stg.dirac_apply_eo(gauge, b, out))
    t_n = timed(lambda: stg.stg_apply_normal(gauge, mass, b, out_even=out, tmp_odd=tmp))
    best = None
    key = stg._lib.STG_TUNE_CG_FORM
    stg.stg_set_tuning(key, 1)  # the classic form first
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st, stats = stg.cg_solve(gauge, mass, b, tol=TOL)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if best is None or dt < best[0]:
            best = (dt, stats[0])
    dt, s0 = best
    # the same solve in the single-reduction form of CG (the default for one field)
    stg.stg_set_tuning(key, 2)
    cbest = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xg, stg_, statsg = stg.cg_solve(gauge, mass, b, tol=TOL)
        torch.cuda.synchronize()
        tg = time.perf_counter() - t0
        if cbest is None or tg < cbest[0]:
            cbest = (tg, statsg[0])
    stg.stg_set_tuning(key, 0)
    # the same solve through the uneven-batch runner (iterations replayed from a hipGraph)
    bbest = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xb, stb, statsb = stg.cg_solve_batch([dict(hi=gauge, mass=mass, b=b)], tol=TOL)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        if bbest is None or tb < bbest[0]:
            bbest = (tb, statsb[0][0])
    # the same CG with the launch shape the autotuner picks for this lattice
    choice = stg.stg_autotune(gauge, 1)
    t_eo_tuned = timed(lambda: stg.dirac_apply_eo(gauge, b, out))
    tbest = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st, stats = stg.cg_solve(gauge, mass, b, tol=TOL)
        torch.cuda.synchronize()
        tt = time.perf_counter() - t0
        if tbest is None or tt < tbest[0]:
            tbest = (tt, stats[0])
    stg.library().stg_autotune_clear()
    orc = oracle.COracle()
    ph = on.standard_phases(dims)
    t0 = time.perf_counter()
    xc, itc, resc, stc = orc.cg(dims, links_np, ph, mass, b_np[0], tol=TOL)
    tc = time.perf_counter() - t0
    print(json.dumps({
        "workload": "8^4, m = 0.1, FP64-18 links, 1 RHS: hop, normal operator, FP64 CG to 1e-10",
        "deo_us": round(t_eo * 1e6, 2), "normal_op_us": round(t_n * 1e6, 2),
        "deo_GBs": round(BYTES_PER_SITE["c128_18"] * stg.half_volume(dims) / t_eo / 1e9, 1),
        "cg_classic_ms": round(dt * 1e3, 3), "cg_classic_iters": s0["iters"],
        "cg_classic_us_per_iter": round(dt * 1e6 / s0["iters"], 2),
        "cg_classic_true_rel_resid": s0["true_rel_resid"],
        "cg_single_reduction_ms": round(cbest[0] * 1e3, 3),
        "cg_single_reduction_iters": cbest[1]["iters"],
        "cg_single_reduction_us_per_iter": round(cbest[0] * 1e6 / cbest[1]["iters"], 2),
        "cg_single_reduction_true_rel_resid": cbest[1]["true_rel_resid"],
        "tuned_shape": {k: v for k, v in choice.items() if k != "us"},
        "deo_us_tuned": round(t_eo_tuned * 1e6, 2),
        "cg_ms_tuned": round(tbest[0] * 1e3, 3),
        "cg_us_per_iter_tuned": round(tbest[0] * 1e6 / tbest[1]["iters"], 2),
        "batch_runner_ms": round(bbest[0] * 1e3, 3), "batch_runner_iters": bbest[1]["iters"],
        "batch_runner_us_per_iter": round(bbest[0] * 1e6 / bbest[1]["iters"], 2),
        "cpu_baseline": {"value": round(tc * 1e3, 2), "unit": "ms per CG solve", "cores":
                         orc.num_threads(), "kind": "oracle",
                         "sample": f"the FP64 C oracle's CG on the same 8^4 system, {itc} "
                                   f"iterations, true residual {resc:.2e}"}}), flush=True)


def bench_md(applies=50, profile=False):
    """One pure-gauge molecular-dynamics step (momentum update with the tree-level
    Symanzik force, then link update) on the paper's Table 4 shapes: FP64-12 links with
    FP64 momenta, and the single-precision variant (FP32-12 links, complex64 momenta);
    ns per site = step time / V, beside Table 4 (context)."""
    import torch
    import paper_1701_00426_amd as stg
    import seeded_inputs as si
    dev = torch.device("cuda:0")
    beta, eps = 5.5, 0.01
    rows = []
    stream = torch.cuda.current_stream()
    shapes = [(32, 32, 32, 32)] if profile else list(PAPER_TABLE4)
    for dims in shapes:
        vh = stg.half_volume(dims)
        links = torch.from_numpy(si.su3_links(dims, 1701, 10, 0)).to(dev)
        mom64 = torch.from_numpy(si.traceless_hermitian_field(dims, 426, 10, 0)).to(dev)
        row = {"lattice": "x".join(map(str, dims))}
        for fmt in (("c128_12",) if profile else ("c128_12", "c64_12")):
            gauge = stg.pack_gauge(dims, links, fmt)
            mom = mom64 if fmt == "c128_12" else mom64.to(torch.complex64)

            def step():
                stg.gauge_momentum_update(gauge, mom, beta, eps)
                stg.gauge_link_update(gauge, mom, eps)

            for _ in range(3):
                step()
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record(stream)
            for _ in range(applies):
                step()
            t1.record(stream)
            torch.cuda.synchronize()
            dt = t0.elapsed_time(t1) / 1e3 / applies
            tag = "fp64" if fmt == "c128_12" else "fp32"
            row[f"step_us_{tag}"] = round(dt * 1e6, 1)
            row[f"ns_per_site_{tag}"] = round(dt * 1e9 / (2 * vh), 3)
            del gauge, mom
        row["paper_gauge_md_ns_per_site_K80_P100"] = PAPER_TABLE4[dims]
        rows.append(row)
        log(json.dumps(rows[-1]))
        del links, mom64
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "pure-gauge MD step (tree-level Symanzik force, momentum + "
                                  "link update), FP64-12 and FP32-12 links, paper Table 4 "
                                  "shapes",
                      "rows": rows}), flush=True)


def bench_stout_force(applies=20):
    """The force through one stout level (stout_force_backprop) at 32^4: FP64-12 thin
    links, rho = 0.15, a seeded Gaussian dS/dU'; two passes per call.  HIP events."""
    import torch
    import paper_1701_00426_amd as stg
    import seeded_inputs as si
    dev = torch.device("cuda:0")
    dims = (32, 32, 32, 32)
    vh = stg.half_volume(dims)
    links = torch.from_numpy(si.su3_links(dims, 1701, 11, 0)).to(dev)
    gauge = stg.pack_gauge(dims, links, "c128_12")
    del links
    z = si.rng(426, 11, 0).standard_normal((8, 3, 3, vh, 2))
    sp = torch.from_numpy(z[..., 0] + 1j * z[..., 1]).to(dev)
    del z
    out = torch.empty_like(sp)
    ws = torch.empty_like(sp)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        stg.stout_force_backprop(gauge, 0.15, sp, out=out, ws=ws)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(applies):
        stg.stout_force_backprop(gauge, 0.15, sp, out=out, ws=ws)
    t1.record(stream)
    torch.cuda.synchronize()
    dt = t0.elapsed_time(t1) / 1e3 / applies
    print(json.dumps({"workload": "force through one stout level, 32^4, FP64-12 thin links, "
                                  "rho = 0.15", "call_us": round(dt * 1e6, 1),
                      "ns_per_site": round(dt * 1e9 / (2 * vh), 3)}), flush=True)


# Launch-shape variants of the hop compared under one kernel trace: (format, fields,
# knob settings).  Each runs the same number of back-to-back D_eo launches.
VARIANTS = [
    ("c128_12", 1, {"tps": 1, "stage": 0, "xcd": 1}, "default"),
    ("c128_12", 1, {"tps": 1, "stage": 0, "xcd": 0}, "plain block order"),
    ("c128_12", 1, {"tps": 1, "stage": 1, "xcd": 1}, "LDS neighbour staging"),
    ("c128_12", 1, {"tps": 4, "stage": 0, "xcd": 1}, "4 threads per site"),
    ("c64_12", 1, {"tps": 1, "stage": 0, "xcd": 1}, "default"),
    ("c64_12", 1, {"tps": 1, "stage": 1, "xcd": 1}, "LDS neighbour staging"),
    ("c64_12", 1, {"tps": 4, "stage": 0, "xcd": 1}, "4 threads per site"),
    ("c64_12", 8, {"tps": 1, "stage": 0, "xcd": 1}, "1 thread per site"),
    ("c64_12", 8, {"tps": 2, "stage": 0, "xcd": 1}, "2 threads per site"),
    ("c64_12", 8, {"tps": 4, "stage": 0, "xcd": 1}, "default (4 threads per site)"),
    ("bf16_12", 1, {"tps": 1, "stage": 0, "xcd": 1}, "1 thread per site"),
    ("bf16_12", 1, {"tps": 4, "stage": 0, "xcd": 1}, "default (4 threads per site)"),
]


def profile_variants(applies=100):
    """For rocprofv3: the hop variants of VARIANTS at 32^4, `applies` D_eo launches each,
    in order; prints one JSON line per variant with its HIP-event mean."""
    import torch
    import paper_1701_00426_amd as stg
    import seeded_inputs as si
    dev = torch.device("cuda:0")
    vh = stg.half_volume(DIMS)
    links = torch.from_numpy(si.su3_links(DIMS, 1701, 2, 0)).to(dev)
    b8 = torch.from_numpy(si.gaussian_field(DIMS, 8, 426, 2, 0, 0)).to(dev)
    L = stg._lib
    keys = {"tps": L.STG_TUNE_THREADS_PER_SITE, "stage": L.STG_TUNE_STAGE_NEIGHBOURS,
            "xcd": L.STG_TUNE_XCD_REMAP}
    cache = {}
    for fmt, nr, knobs, label in VARIANTS:
        if fmt not in cache:
            cache.clear()
            torch.cuda.empty_cache()
            cache[fmt] = [stg.pack_gauge(DIMS, links if i == 0 else links.clone(), fmt)
                          for i in range(3)]
        gauges = cache[fmt]
        cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
        fields = [b8[:nr].to(cdt).clone() for _ in range(3)]
        outs = [torch.empty_like(fields[0]) for _ in range(3)]
        for k, v in knobs.items():
            stg.stg_set_tuning(keys[k], v)
        dt = time_applies(stg, torch, gauges, fields, outs, 0, applies)
        stg.stg_set_tuning(keys["tps"], 0)
        stg.stg_set_tuning(keys["stage"], 0)
        stg.stg_set_tuning(keys["xcd"], 1)
        links_b = {"c128_12": 768, "c64_12": 384, "bf16_12": 192}[fmt]
        field_b = 96 if fmt.startswith("c128") else 48
        gbs = (links_b + nr * field_b) * vh / dt / 1e9
        print(json.dumps({"format": fmt, "fields": nr, "variant": label, "knobs": knobs,
                          "mean_launch_us": round(dt * 1e6, 2), "GBs": round(gbs, 1)}), flush=True)
        del fields, outs


# Launch shapes of the hop with 8 fields per launch at 32^4 (D_eo; normal operator):
# threads per site, layer order (x3 planes per group, 0: half-index order) and the
# spread epilogue.
MULTIFIELD_VARIANTS = [
    ("c64_12", {"tps": 4, "group": 0, "spread": 0}, "default (4 threads per site)"),
    ("c64_12", {"tps": 4, "group": 4, "spread": 0}, "layer order G=4"),
    ("c64_12", {"tps": 4, "group": 8, "spread": 0}, "layer order G=8"),
    ("c64_12", {"tps": 4, "group": 0, "spread": 1}, "spread epilogue"),
    ("c64_12", {"tps": 4, "group": 4, "spread": 1}, "layer order G=4 + spread"),
    ("c64_12", {"tps": 4, "group": 8, "spread": 1}, "layer order G=8 + spread"),
    ("c64_12", {"tps": 2, "group": 8, "spread": 1}, "2 threads, G=8 + spread"),
    ("c128_12", {"tps": 2, "group": 0, "spread": 0}, "default (2 threads per site)"),
    ("c128_12", {"tps": 2, "group": 4, "spread": 0}, "layer order G=4"),
    ("c128_12", {"tps": 2, "group": 8, "spread": 0}, "layer order G=8"),
    ("c128_12", {"tps": 2, "group": 8, "spread": 1}, "layer order G=8 + spread"),
    ("c128_12", {"tps": 1, "group": 8, "spread": 0}, "1 thread, G=8"),
    ("c64_12", {}, "automatic"),
    ("c64_12", {"fsplit": 1, "group": 0}, "fields split, 1 per wave"),
    ("c64_12", {"fsplit": 2, "group": 0}, "fields split, 2 per wave"),
    ("c64_12", {"fsplit": 1, "group": 4}, "fields split, 1 per wave, G=4"),
    ("c64_12", {"fsplit": 2, "group": 4}, "fields split, 2 per wave, G=4"),
    ("c128_12", {"fsplit": 1, "group": 0}, "fields split, 1 per wave"),
    ("c128_12", {"fsplit": 1, "group": 4}, "fields split, 1 per wave, G=4"),
    ("c128_12", {"fsplit": 2, "group": 0}, "fields split, 2 per wave"),
    ("bf16_12", {"tps": 4, "group": 0, "spread": 0}, "default (4 threads per site)"),
    ("bf16_12", {"tps": 4, "group": 8, "spread": 1}, "layer order G=8 + spread"),
    ("bf16_12", {"fsplit": 1, "group": 0}, "fields split, 1 per wave"),
    ("bf16_12", {"fsplit": 2, "group": 0}, "fields split, 2 per wave"),
    ("bf16_12", {"fsplit": 1, "group": 4}, "fields split, 1 per wave, G=4"),
    ("c128_12", {}, "automatic"),
    ("bf16_12", {}, "automatic"),
]


def profile_multifield(only=None, applies=100, nfields=8):
    """For rocprofv3: D_eo and the normal operator with `nfields` fields per launch at 32^4 in the
    launch shapes of MULTIFIELD_VARIANTS (all, or the indices in the list `only`, in its order
    and with its repeats), rotating
    three link/field copies; one JSON line per variant with HIP-event means and GB/s of
    the algorithmic bytes (links once + nfields x (in + out) for D_eo)."""
    import torch
    import paper_1701_00426_amd as stg
    import seeded_inputs as si
    dev = torch.device("cuda:0")
    vh = stg.half_volume(DIMS)
    links = torch.from_numpy(si.su3_links(DIMS, 1701, 2, 0)).to(dev)
    b8 = torch.from_numpy(si.gaussian_field(DIMS, nfields, 426, 2, 0, 0)).to(dev)
    L = stg._lib
    keys = {"tps": L.STG_TUNE_THREADS_PER_SITE, "group": L.STG_TUNE_LAYER_GROUP,
            "spread": L.STG_TUNE_SPREAD_EPILOGUE, "fsplit": L.STG_TUNE_FIELD_SPLIT}
    cache = {}
    stream = torch.cuda.current_stream()
    order = range(len(MULTIFIELD_VARIANTS)) if only is None else only
    for idx in order:
        fmt, knobs, label = MULTIFIELD_VARIANTS[idx]
        if fmt not in cache:
            cache.clear()
            torch.cuda.empty_cache()
            cache[fmt] = [stg.pack_gauge(DIMS, links if i == 0 else links.clone(), fmt)
                          for i in range(3)]
        gauges = cache[fmt]
        cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
        fields = [b8.to(cdt).clone() for _ in range(3)]
        outs = [torch.empty_like(fields[0]) for _ in range(3)]
        tmps = [torch.empty_like(fields[0]) for _ in range(3)]
        for k, v in knobs.items():
            stg.stg_set_tuning(keys[k], v)
        log(f"variant {idx}: {fmt} {label}")
        dt = time_applies(stg, torch, gauges, fields, outs, 0, applies)
        for i in range(3):
            stg.stg_apply_normal(gauges[i], MASS, fields[i], out_even=outs[i], tmp_odd=tmps[i])
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for i in range(applies):
            stg.stg_apply_normal(gauges[i % 3], MASS, fields[i % 3], out_even=outs[i % 3],
                                 tmp_odd=tmps[i % 3])
        t1.record(stream)
        t1.synchronize()
        dn = t0.elapsed_time(t1) * 1e-3 / applies
        for k in keys.values():
            stg.stg_set_tuning(k, 0)
        links_b = {"c128_12": 768, "c64_12": 384, "bf16_12": 192}[fmt]
        field_b = 96 if fmt.startswith("c128") else 48
        byts = (links_b + nfields * field_b) * vh
        print(json.dumps({"variant": idx, "format": fmt, "fields": nfields, "label": label,
                          "knobs": knobs, "deo_us": round(dt * 1e6, 2),
                          "deo_GBs": round(byts / dt / 1e9, 1),
                          "deo_frac_hbm": round(byts / dt / 1e9 / HBM_PEAK_GBS, 4),
                          "normal_us": round(dn * 1e6, 2),
                          "algorithmic_bytes_deo": byts}), flush=True)
        del fields, outs, tmps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--applies", type=int, default=300)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--profile", action="store_true",
                    help="for rocprofv3: only the dominant kernel's timed loop (FP64-12 D_eo)")
    ap.add_argument("--profile-cg", action="store_true",
                    help="for rocprofv3: one FP64 CG and one mixed CG solve only")
    ap.add_argument("--workload", choices=["main", "multishift", "rational", "batch",
                                           "batch-small", "shapes", "staples", "force",
                                           "stout", "tiles", "small", "md",
                                           "stoutforce"],
                    default="main",
                    help="main: the 32^4 line; multishift: 24^3x48, 16 shifts x 8 RHS; "
                         "rational: the same shifts combined into r(A) b; "
                         "batch: 12 solves on 8^4 .. 32^4 in one cg_solve_batch; "
                         "batch-small: 48 solves on 8^4 .. 16^4; "
                         "staples: gauge-force staples on the Table 4 shapes; "
                         "force: fermion force from 16 multi-shift solutions at 32^4; "
                         "stout: two stout-smearing levels at 32^4; "
                         "tiles: the pencil tile shapes of the staple and stout kernels; "
                         "small: 8^4 FP64-18 hop and CG (latency-bound); "
                         "md: the pure-gauge MD step on the Table 4 shapes; "
                         "stoutforce: the force through one stout level at 32^4")
    ap.add_argument("--profile-md", action="store_true",
                    help="for rocprofv3: only the 32^4 MD-step loop")
    ap.add_argument("--profile-stout", action="store_true",
                    help="for rocprofv3: only the 32^4 level-1 stout loop")
    ap.add_argument("--profile-force", action="store_true",
                    help="for rocprofv3: only the 32^4 fermion_force loop")
    ap.add_argument("--profile-staples", action="store_true",
                    help="for rocprofv3: only the 32^4 FP64-12 staple loop")
    ap.add_argument("--profile-variants", action="store_true",
                    help="for rocprofv3: the hop's launch-shape variants at 32^4, in order")
    ap.add_argument("--profile-multifield", nargs="?", const="all", default=None,
                    metavar="VARIANTS",
                    help="for rocprofv3: the 8-field hop launch shapes at 32^4 (all, or "
                         "comma-separated indices of MULTIFIELD_VARIANTS)")
    ap.add_argument("--mf-fields", type=int, default=8, choices=[2, 3, 4, 8],
                    help="fields per launch of --profile-multifield")
    ap.add_argument("--cg-form", type=int, default=0, choices=[0, 1, 2],
                    help="STG_TUNE_CG_FORM for the solves: 0 automatic, 1 classic (two "
                         "reductions per iteration), 2 single reduction")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="for rocprofv3 --pmc: a plain 1 GiB device copy, to scale byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(no halo exchange between slabs); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.profile_variants:
        profile_variants()
        return
    if args.profile_multifield is not None:
        pm = args.profile_multifield
        profile_multifield(None if pm == "all" else [int(v) for v in pm.split(",")],
                           nfields=args.mf_fields)
        return
    if args.workload == "multishift":
        bench_multishift()
        return
    if args.workload == "rational":
        bench_rational()
        return
    if args.workload == "batch":
        bench_batch(args.cg_form)
        return
    if args.workload == "batch-small":
        bench_batch_small(args.cg_form)
        return
    if args.workload == "shapes":
        bench_shapes()
        return
    if args.workload == "stoutforce":
        bench_stout_force()
        return
    if args.workload == "md" or args.profile_md:
        bench_md(profile=args.profile_md)
        return
    if args.workload == "small":
        bench_small()
        return
    if args.workload == "tiles":
        bench_tiles()
        return
    if args.workload == "stout" or args.profile_stout:
        bench_stout(profile=args.profile_stout)
        return
    if args.workload == "force" or args.profile_force:
        bench_force(profile=args.profile_force)
        return
    if args.workload == "staples" or args.profile_staples:
        bench_staples(profile=args.profile_staples, no_cpu=args.no_cpu)
        return

    import numpy as np
    import torch

    import paper_1701_00426_amd as stg
    import seeded_inputs as si

    stg.library()
    dev = torch.device("cuda:0")
    vh = stg.half_volume(DIMS)
    log(f"generating 32^4 inputs (Vh={vh})")
    links_np = si.su3_links(DIMS, 1701, 2, 0)
    b_np = si.gaussian_field(DIMS, 1, 426, 2, 0, 0)
    links = torch.from_numpy(links_np).to(dev)
    b = torch.from_numpy(b_np).to(dev)
    stg.stg_set_tuning(stg._lib.STG_TUNE_CG_FORM, args.cg_form)

    # ---- operator bandwidth (value + roofline) ----------------------------------------
    variants = {}
    hop_time = {}
    fmts = ("c128_12",) if args.profile else ("c128_12", "c128_18", "c64_12", "bf16_12")
    if args.profile_cg:
        fmts = ()
    for fmt in fmts:
        cdt = torch.complex128 if fmt.startswith("c128") else torch.complex64
        ncopy = 3
        gauges = [stg.pack_gauge(DIMS, links if i == 0 else links.clone(), fmt)
                  for i in range(ncopy)]
        fields = [b.to(cdt).clone() for _ in range(ncopy)]
        outs = [torch.empty_like(fields[0]) for _ in range(ncopy)]
        ws_bytes = sum(g.links.numel() * g.links.element_size() for g in gauges) + \
            2 * ncopy * fields[0].numel() * fields[0].element_size()
        res = {}
        pars = ((0, "D_eo"),) if args.profile else ((0, "D_eo"), (1, "D_oe"))
        for par, name in pars:
            dt = time_applies(stg, torch, gauges, fields, outs, par, args.applies)
            gbs = BYTES_PER_SITE[fmt] * vh / dt / 1e9
            res[name] = {"us": round(dt * 1e6, 2), "GBs": round(gbs, 1),
                         "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                         "naive_GBs": round(NAIVE_BYTES_PER_SITE[fmt] * vh / dt / 1e9, 1),
                         "GFLOPs": round(FLOPS_PER_SITE * vh / dt / 1e9, 1),
                         "ns_per_site": round(dt * 1e9 / vh, 4)}
            hop_time[(fmt, name)] = dt
        if fmt == "c128_12" and not args.profile:
            # the same launches with the plain block order, for comparison
            stg.stg_set_tuning(stg._lib.STG_TUNE_XCD_REMAP, 0)
            dt0 = time_applies(stg, torch, gauges, fields, outs, 0, args.applies)
            stg.stg_set_tuning(stg._lib.STG_TUNE_XCD_REMAP, 1)
            res["D_eo_plain_block_order"] = {"us": round(dt0 * 1e6, 2),
                                             "GBs": round(BYTES_PER_SITE[fmt] * vh / dt0 / 1e9, 1)}
        res["working_set_GB"] = round(ws_bytes / 1e9, 3)
        res["bytes_per_site"] = BYTES_PER_SITE[fmt]
        variants[fmt] = res
        log(f"{fmt}: " + ", ".join(f"{k} {v['us']} us {v['GBs']} GB/s"
                                   for k, v in res.items() if isinstance(v, dict)))
        del gauges, fields, outs
        torch.cuda.empty_cache()

    # ---- link packing (once per gauge configuration, timed apart from the steps) -------
    pack = {}
    if not args.profile and not args.profile_cg:
        for fmt in ("c128_12", "c64_12", "bf16_12"):
            pack[fmt] = time_pack(stg, torch, links, DIMS, fmt)
        log("pack: " + ", ".join(f"{k} {v['us']} us {v['GBs']} GB/s" for k, v in pack.items()))

    if args.profile:
        dt = hop_time[("c128_12", "D_eo")]
        print(json.dumps({"profile": "hop D_eo FP64-12 32^4", "applies": args.applies,
                          "mean_launch_us": round(dt * 1e6, 3),
                          "GBs": round(BYTES_PER_SITE["c128_12"] * vh / dt / 1e9, 1),
                          "kernel_hash": kernel_hash()}), flush=True)
        return

    # ---- the steps: FP64 CG and mixed CG to 1e-10 ------------------------------------
    hi = stg.pack_gauge(DIMS, links, "c128_12")
    lo = stg.pack_gauge(DIMS, links, "c64_12")
    ws64 = torch.empty(stg.stg_workspace_bytes(DIMS, 1, 0, stg.STG_CG_F64), dtype=torch.uint8,
                       device=dev)
    wsmx = torch.empty(stg.stg_workspace_bytes(DIMS, 1, 0, stg.STG_CG_MIXED),
                       dtype=torch.uint8, device=dev)
    lo16 = stg.pack_gauge(DIMS, links, "bf16_12")
    wsbf = torch.empty_like(wsmx)
    x64 = torch.zeros_like(b)
    xmx = torch.zeros_like(b)
    xbf = torch.zeros_like(b)
    nb = 8
    b8_np = si.gaussian_field(DIMS, nb, 426, 2, 1, 0)
    b8_np[0] = b_np[0]  # the first of the 8 RHS is the single-RHS b: one x* serves both
    b8 = torch.from_numpy(b8_np).to(dev)
    x8 = torch.zeros_like(b8)
    ws8 = torch.empty(stg.stg_workspace_bytes(DIMS, nb, 0, stg.STG_CG_MIXED), dtype=torch.uint8,
                      device=dev)

    failures = []

    def step():
        s3 = s4 = 0
        x64.zero_()
        xmx.zero_()
        xbf.zero_()
        x8.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, s1, st1 = stg.cg_solve(hi, MASS, b, x=x64, ws=ws64, tol=TOL)
        t1 = time.perf_counter()
        _, s2, st2 = stg.cg_solve(hi, MASS, b, x=xmx, lo=lo, ws=wsmx, tol=TOL)
        t2 = time.perf_counter()
        st3 = st4 = None
        if not args.profile_cg:
            _, s3, st3 = stg.cg_solve(hi, MASS, b8, x=x8, lo=lo, ws=ws8, tol=TOL)
        t3 = time.perf_counter()
        if not args.profile_cg:
            _, s4, st4 = stg.cg_solve(hi, MASS, b, x=xbf, lo=lo16, ws=wsbf, tol=TOL)
        t4 = time.perf_counter()
        for name, status, stats in (("fp64", s1, st1), ("mixed_fp32", s2, st2),
                                    ("mixed_fp32_8rhs", s3 if st3 else 0, st3 or []),
                                    ("mixed_bf16", s4 if st4 else 0, st4 or [])):
            bad = [q for q in stats if q["status"] != 0 or not q["true_rel_resid"] <= TOL]
            if status != 0 or bad:
                failures.append({"solve": name, "status": status,
                                 "stats": bad[:2] if bad else stats[:1]})
        return t1 - t0, t2 - t1, st1[0], st2[0], t3 - t2, st3, t4 - t3, st4

    if args.profile_cg:
        r = step()
        print(json.dumps({"profile": "CG 32^4", "cg_form": args.cg_form,
                          "fp64_s": round(r[0], 4), "mixed_s": round(r[1], 4),
                          "fp64_iters": r[2]["iters"], "mixed_iters": r[3]["iters"]}), flush=True)
        return
    copy_gbs = copy_ceiling(torch)
    read_gbs, read_ops = read_ceiling(torch)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    runs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    if failures:
        print(json.dumps({"error": "a timed solve did not reach |r|/|b| <= 1e-10",
                          "failures": failures[:4]}), file=sys.stderr, flush=True)
        sys.exit(1)
    t64 = min(r[0] for r in runs)
    tmx = min(r[1] for r in runs)
    t8 = min(r[4] for r in runs)
    tbf = min(r[6] for r in runs)
    st64, stmx, st8, stbf = runs[-1][2], runs[-1][3], runs[-1][5], runs[-1][7][0]

    # ---- dominant kernel roofline --------------------------------------------------
    dt = hop_time[("c128_12", "D_eo")]
    achieved = BYTES_PER_SITE["c128_12"] * vh / dt / 1e9
    traffic = trace_us = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("kernel_hash") == kernel_hash():
            traffic = tr.get("bytes_per_launch")
            trace_us = tr.get("trace_mean_launch_us")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "hop_kernel<double, FMT_C128_12, std phases, NR=1, EPI_PLAIN> (D_eo)",
                "algorithmic_bytes_per_launch": BYTES_PER_SITE["c128_12"] * vh,
                "mean_launch_us": round(dt * 1e6, 2),
                "timing": f"HIP events on the library's stream around {args.applies} back-to-back "
                          "launches rotating three link/field copies, in this run",
                # the rocprofv3 kernel-trace average of the same kernel in the committed
                # profile (same sources), and the fraction it gives
                "trace_mean_launch_us": trace_us,
                "trace_frac": (round(BYTES_PER_SITE["c128_12"] * vh / (trace_us * 1e3)
                                     / HBM_PEAK_GBS, 4) if trace_us else None)}

    out = {
        "metric": METRIC,
        "value": round(achieved, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total / max(args.steps, 1) * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "32^4 random SU(3), m=0.01: FP64-12 D_eo apply; FP64 CG, "
                               "mixed FP32-12 CG (1 and 8 RHS) and mixed BF16-12 CG "
                               "to |r|/|b|<=1e-10",
                   "lattice": list(DIMS), "mass": MASS, "nrhs": 1, "tol": TOL,
                   "links": "random SU(3) (Haar), standard phases, antiperiodic t"},
        "hbm_frac": round(achieved / HBM_PEAK_GBS, 4),
        "copy_ceiling_GBs": copy_gbs,
        "read_ceiling_GBs": read_gbs,
        "read_ceiling_ops_GBs": read_ops,
        "frac_of_read_ceiling": round(achieved / read_gbs, 4),
        "cg_fp64_s_per_rhs": round(t64, 4),
        "cg_mixed_s_per_rhs": round(tmx, 4),
        "mixed_speedup": round(t64 / tmx, 3),
        "cg_mixed_batch8_s_per_rhs": round(t8 / nb, 4),
        "batched_mixed_speedup": round(t64 / (t8 / nb), 3),
        "cg_mixed_batch8": {"iters": max(x["iters"] for x in st8),
                            "worst_true_rel_resid": max(x["true_rel_resid"] for x in st8),
                            "reliable_updates": max(x["reliable_updates"] for x in st8)},
        "cg_mixed_bf16_s_per_rhs": round(tbf, 4),
        "mixed_bf16_speedup": round(t64 / tbf, 3),
        "cg_mixed_bf16": {"iters": stbf["iters"], "true_rel_resid": stbf["true_rel_resid"],
                          "reliable_updates": stbf["reliable_updates"]},
        "cg_fp64": {"iters": st64["iters"], "true_rel_resid": st64["true_rel_resid"],
                    "reliable_updates": st64["reliable_updates"]},
        "cg_mixed": {"iters": stmx["iters"], "true_rel_resid": stmx["true_rel_resid"],
                     "reliable_updates": stmx["reliable_updates"]},
        "operator_variants": variants,
        "pack_links": pack,
        "roofline": roofline,
    }
    if not args.no_cpu and not args.profile:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(links_np, b_np, vh)
        log("oracle CG to 1e-12 on the host cores (x*)")
        xs, info = oracle_solution(links_np, b_np[0])
        out["cpu_baseline"]["cg_fp64_time_to_solution"] = info
        xsn = float(np.linalg.norm(xs))
        sols = {"fp64": x64[0], "mixed_fp32_12": xmx[0], "mixed_bf16_12": xbf[0],
                "mixed_fp32_12_8rhs_rhs0": x8[0]}
        kappa = (MASS * MASS + 16.0) / (MASS * MASS)
        out["error_vs_oracle_solution"] = {
            k: float(np.linalg.norm(v.cpu().numpy() - xs) / xsn) for k, v in sols.items()}
        out["error_vs_oracle_solution"]["bound_2kappa_tol"] = 2 * kappa * TOL
        out["error_vs_oracle_solution"]["x_star"] = (
            f"oracle FP64 CG to |r|/|b| <= 1e-12 ({info['iters']} iterations, true residual "
            f"{info['true_rel_resid']:.2e}); the last timed step's solutions")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    del np


if __name__ == "__main__":
    main()
