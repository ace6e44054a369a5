// capi.cpp -- the C ABI of include/stagmi.h: argument checks, dispatch of the hop
// and vector kernels, workspace carving, and the host side of the solvers.
//
// Paper: arXiv:1701.00426, Sec. 2.2 (Eqs. diracblock, lineqeo, shlineq: the
// operator, the even/odd normal equations and the shifted systems), Sec. 4.1
// (layouts), Sec. 4.3 (deo/doe).  The solver loop keeps alpha and beta on the
// device; the host enqueues a batch of iterations, then reads the per-system
// flags once, and enqueues the FP64 true-residual update of any parked system.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/stagmi.h"
#include "batch.hpp"
#include "force.hpp"
#include "kernels.hpp"
#include "solver_state.hpp"
#include "staple.hpp"
#include "tune.hpp"

using namespace stg;

namespace {

thread_local std::string g_last_error;

// launch-shape choice of the hop kernels (stg_set_tuning)
int g_xcd_remap = 1;
int g_sites_per_thread = 1;
int g_stage_neighbours = 0;
int g_threads_per_site = 0;  // 0: by format and fields
int g_staple_threads = 0;    // 0: by format
int g_pencil_tile = 0;       // tile shape of the pencil order (pencil.hpp)
int g_fields_per_launch = 0; // 0: the autotuned choice for the lattice and format, else 8
int g_layer_group = 0;       // 0: half-index order; G: layer order, G x3 planes per group
int g_spread_epilogue = 0;   // 1: split hops with fields a multiple of the threads per
                             // site finish the fields on every thread group
int g_cg_form = 0;           // CG iteration: 0 automatic, 1 two reductions (classic),
                             // 2 one reduction (Chronopoulos-Gear)
int g_field_split = 0;       // several fields per launch split over the waves of a block:
                             // 1 or 2 fields per wave, 0: automatic, -1: off

int hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return STG_HIP_ERROR;
}

#define HIP_TRY(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

int invalid(const char *why) {
    g_last_error = why;
    return STG_INVALID_ARG;
}

// A launch the library itself set up wrongly (never the caller's arguments).
int internal(const char *why) {
    g_last_error = why;
    return STG_HIP_ERROR;
}

#define HOP_TRY(call)                                                  \
    do {                                                               \
        if ((call) != 0) return internal("hop launch refused: " #call); \
    } while (0)

#define VEC_TRY(call)                                                       \
    do {                                                                    \
        if ((call) != 0) return internal("vector kernel not built: " #call); \
    } while (0)

bool make_geom(const stg_lattice *lat, Geom &g) {
    if (!lat) return false;
    uint64_t v = 1;
    for (int mu = 0; mu < 4; ++mu) {
        int32_t n = lat->dims[mu];
        if (n < 2 || (n & 1) || n > 65536) return false;
        g.N[mu] = (uint32_t)n;
        v *= (uint64_t)n;
    }
    if (v / 2 >= (1ull << 30)) return false;  // half indices and strides stay in 32 bits
    g.nh0 = g.N[0] / 2;
    g.Vh = (uint32_t)(v / 2);
    g.stride[0] = 1;
    g.stride[1] = g.nh0;
    g.stride[2] = g.nh0 * g.N[1];
    g.stride[3] = g.nh0 * g.N[1] * g.N[2];
    return true;
}

bool aligned16(const void *p) { return p && (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

size_t link_bytes(const Geom &g, int fmt) {
    const size_t vh = g.Vh;
    switch (fmt) {
        case STG_LINK_C128_18: return 8 * 9 * vh * 16;
        case STG_LINK_C128_12: return 8 * 6 * vh * 16;
        case STG_LINK_C64_12: return 8 * 3 * vh * 16;
        case STG_LINK_BF16_12: return 8 * vh * 24;
        default: return 0;
    }
}

bool fmt_matches(int fmt, int field) {
    if (field == STG_C128) return fmt == STG_LINK_C128_18 || fmt == STG_LINK_C128_12;
    if (field == STG_C64) return fmt == STG_LINK_C64_12 || fmt == STG_LINK_BF16_12;
    return false;
}

size_t field_elem(int field) { return field == STG_C128 ? 16 : 8; }

int check_gauge(const Geom &g, const stg_gauge *gauge, int field) {
    if (!gauge) return invalid("gauge is NULL");
    if (!fmt_matches(gauge->fmt, field))
        return invalid("gauge format does not match the field precision");
    if (!aligned16(gauge->links)) return invalid("links NULL or not 16-byte aligned");
    if (gauge->phases && (reinterpret_cast<uintptr_t>(gauge->phases) & 7u))
        return invalid("phases not 8-byte aligned");
    (void)g;
    return STG_OK;
}

// Planes per group of the layer order for a requested G: the largest divisor of N3
// not above it (0 keeps the half-index order).
uint32_t layer_group_for(const Geom &g, int want) {
    if (want <= 0) return 0;
    for (uint32_t d = std::min<uint32_t>((uint32_t)want, g.N[3]); d > 1; --d)
        if (g.N[3] % d == 0) return d;
    return 0;
}

HopArgs base_hop(const Geom &g, const stg_gauge *gauge) {
    HopArgs a;
    std::memset(&a, 0, sizeof(a));
    a.geom = g;
    a.links = gauge->links;
    a.phases = gauge->phases;
    a.fstride = (size_t)3 * g.Vh;
    a.xcd_remap = g_xcd_remap;
    a.sites_per_thread = (uint32_t)g_sites_per_thread;
    a.stage_neighbours = (uint32_t)g_stage_neighbours;
    a.threads_per_site = (uint32_t)g_threads_per_site;
    a.layer_group = layer_group_for(g, g_layer_group);
    a.layer_group_auto = g_layer_group == 0 ? layer_group_for(g, 4) : 0;
    a.spread_epilogue = (uint32_t)g_spread_epilogue;
    a.fields_per_wave = g_field_split;
    return a;
}

// Launches a hop with the launch shape the autotuner chose for this lattice,
// format and chunk (process-wide defaults when it has not seen the key).
int hop(HopArgs a, int fmt, int nr, int epi, hipStream_t stream) {
    TuneChoice c;
    if (tune_lookup(a.geom, fmt, nr, c)) {
        a.xcd_remap = c.xcd_remap;
        a.sites_per_thread = (uint32_t)c.sites_per_thread;
        a.stage_neighbours = (uint32_t)c.stage_neighbours;
        // the autotuner times the plain hop; epilogues keep their own default
        if (epi == EPI_PLAIN) a.threads_per_site = (uint32_t)c.threads_per_site;
    }
    return launch_hop(a, fmt, nr, epi, stream);
}

// Largest supported chunk of fields for one kernel launch (8, 4, 3, 2 or 1: each
// launch reads the links once for all its fields), at most cap (1, 2, 4 or 8).
int chunk_of(int remaining, int cap = 8) {
    const int c = std::min(remaining, cap);
    if (c >= 8) return 8;
    if (c >= 4) return 4;
    return c;
}

// Fields per launch for hops on this lattice and link format: the caller's setting,
// else the autotuner's choice, else 8.
int field_cap(const Geom &g, int fmt) {
    if (g_fields_per_launch) return g_fields_per_launch;
    int cap;
    return fields_lookup(g, fmt, cap) ? cap : 8;
}

int hop_plain(const Geom &g, const stg_gauge *gauge, int field, int nrhs, const void *in,
              void *out, int out_parity, hipStream_t stream) {
    const size_t fb = (size_t)3 * g.Vh * field_elem(field);
    HopArgs a = base_hop(g, gauge);
    a.out_parity = out_parity;
    a.op = OP_NONE;
    const int cap = field_cap(g, gauge->fmt);
    for (int j0 = 0; j0 < nrhs;) {
        int nr = chunk_of(nrhs - j0, cap);
        a.in = reinterpret_cast<const char *>(in) + j0 * fb;
        a.out = reinterpret_cast<char *>(out) + j0 * fb;
        if (hop(a, gauge->fmt, nr, EPI_PLAIN, stream)) return invalid("unsupported hop");
        j0 += nr;
    }
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

int apply_dirac(const stg_lattice *lat, const stg_gauge *gauge, int field, int nrhs,
                const void *in, void *out, int out_parity, stg_stream_t stream) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    if (field != STG_C128 && field != STG_C64) return invalid("unknown field type");
    int rc = check_gauge(g, gauge, field);
    if (rc) return rc;
    if (nrhs < 1) return invalid("nrhs < 1");
    if (!aligned16(in) || !aligned16(out)) return invalid("field NULL or not 16-byte aligned");
    const size_t fb = (size_t)nrhs * 3 * g.Vh * field_elem(field);
    if (overlap(in, fb, out, fb)) return invalid("input and output overlap");
    return hop_plain(g, gauge, field, nrhs, in, out, out_parity, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Carver {
    char *base;
    size_t off = 0;
    void *take(size_t bytes) {
        void *p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    }
};

struct CgWork {
    Ctl *ctl;
    SysState *state;      // the solver state the next kernel reads
    SysState *state_alt;  // single-field solves: the other buffer of the double-buffered state
    double *partials;
    double *partials2;    // single-field solves: |r|^2 partials (partials holds <p, A p>)
    double *rr_partials;  // single-reduction CG: |r|^2 partials of the last update, per
                          // system, [2 buffers][nsys][site blocks][2]
    int rr_cur = 0;       // buffer of rr_partials the next update reads (one-field fused)
    // inner precision (FP64 mode: double fields; MIXED: float fields); s = A p of the
    // single-reduction CG
    void *x_in, *p, *r, *q, *t, *s;
    // FP64 fields for the true residual (MIXED only; F64 mode aliases r / t)
    void *r64, *t64;
    size_t bytes;
};

size_t partial_count(const Geom &g) {
    // doubles for the (sum, error) pairs: NR <= 8 per block of the site kernels (the
    // hop with 4 threads per site has the most blocks), 2 per dot block
    size_t sites = (size_t)2 * 8 * hop_max_blocks(g.Vh);
    size_t dots = (size_t)2 * 2 * dot_blocks((size_t)3 * g.Vh);
    return std::max(sites, dots);
}

CgWork carve_cg(const Geom &g, int nsys, int mode, void *ws) {
    Carver c{reinterpret_cast<char *>(ws)};
    CgWork w;
    const size_t f64 = (size_t)nsys * 3 * g.Vh * 16;
    const size_t f32 = (size_t)nsys * 3 * g.Vh * 8;
    w.ctl = (Ctl *)c.take(sizeof(Ctl));
    w.state = (SysState *)c.take(sizeof(SysState) * (size_t)nsys);
    w.state_alt = (SysState *)c.take(sizeof(SysState) * (size_t)nsys);
    w.partials = (double *)c.take(sizeof(double) * partial_count(g));
    w.partials2 = (double *)c.take(sizeof(double) * partial_count(g));
    w.rr_partials = (double *)c.take(sizeof(double) * 2 * 2 * (size_t)nsys * site_blocks(g.Vh));
    if (mode == STG_CG_F64) {
        w.x_in = nullptr;  // the caller's x
        w.p = c.take(f64);
        w.r = c.take(f64);
        w.q = c.take(f64);
        w.t = c.take(f64);
        w.s = c.take(f64);
        w.r64 = w.r;
        w.t64 = w.t;
    } else {
        w.x_in = c.take(f32);
        w.p = c.take(f32);
        w.r = c.take(f32);
        w.q = c.take(f32);
        w.t = c.take(f32);
        w.s = c.take(f32);
        w.r64 = c.take(f64);
        w.t64 = c.take(f64);
    }
    w.bytes = c.off;
    return w;
}

// ---------------------------------------------------------------------------
// CG driver shared by cg_solve (and the refinement stage of the multi-shift solve)
// ---------------------------------------------------------------------------
// Restart choice of the reliable update: -1 (auto) restarts the search direction
// when the inner operator stores its links in BF16, whose rounding error is large
// enough that the kept direction loses conjugacy and stalls the iteration at small
// mass; FP32 links keep the direction.
int resolve_restart(int restart, int mode, const stg_gauge *lo) {
    if (restart >= 0) return restart ? 1 : 0;
    return (mode == STG_CG_MIXED && lo && lo->fmt == STG_LINK_BF16_12) ? 1 : 0;
}

// The form of the CG iteration (STG_TUNE_CG_FORM).  Automatic: the single-reduction
// form for a solve of one field, where it saves a finalize kernel and a vector pass
// launch per iteration (measured on MI355X: 8^4 FP64 20.6 -> 17.2 us per iteration;
// 32^4 FP32-12 inner iteration 116.6 -> 111.6 us), the classic one for several fields,
// where it measured no faster.
bool cg_single_reduction(int nsys) { return g_cg_form == 2 || (g_cg_form == 0 && nsys == 1); }

struct CgProblem {
    Geom g;
    const stg_gauge *hi;
    const stg_gauge *lo;
    int mode;
    int nsys;
    const void *b;     // complex128 [nsys][3][Vh]
    void *x;           // complex128 [nsys][3][Vh], guess in, solution out
    std::vector<double> diag;  // m^2 + sigma per system
    stg_cg_params prm;
    int group = 0;     // systems s share b[s % group] (multi-shift refinement); 0: group = nsys
    int cap = 8;       // fields per launch (field_cap of the inner links)
    bool cgcg = false; // the single-reduction form of the iteration
    int chunk(int j0) const {
        const int g = group > 0 ? group : nsys;
        return chunk_of(std::min(nsys - j0, g - j0 % g), cap);
    }
    const void *b_at(int j0, size_t fb64) const {
        const int g = group > 0 ? group : nsys;
        return (const char *)b + (size_t)(j0 % g) * fb64;
    }
};

// One CG iteration for every chunk of systems that still has a running system in
// the flags snapshot `st` (systems leave the running state only inside the
// iteration, and re-enter it only through a reliable update, after which the host
// reads fresh flags: a snapshot one chunk old never skips a running system).
//
// A solve of one field on a small lattice runs the iteration in four kernels: D_oe,
// D_eo with the normal-operator epilogue and <p, q> partials, the x / r update that
// finishes alpha from those partials in every block, and the p update that finishes
// |r|^2 and takes the beta step in every block.  Its state is double-buffered (the p
// update writes the next iteration's copy), so w.state and w.state_alt swap after
// each iteration.  Several fields, and one field on a large lattice, keep the
// finalize kernels (one block per field) between the producers and consumers: there
// every block of a consumer would re-read all the producer's partials before its
// first vector load (measured at 32^4 on MI355X, one field: the p update took 21.0 us
// in FP32 and 24.4 us in FP64 that way, against about 7 and 14 us plus a 4.6 us
// finalize), while on a small lattice every kernel sits at the launch floor and the
// saved launches win (8^4 FP64: 19.6 us per iteration against 21.9-26.1 with six).
constexpr uint32_t kFusedFinishMaxVh = 32768;  // half sites: 16^4 and below

// The single-reduction form (Chronopoulos and Gear, solver_state.hpp cgcg_step) runs
// the iteration in four kernels: t = D_oe r, w = A r with the <r, w> partials (the
// normal-operator epilogue on r), the finalize kernel (alpha and beta from <r, w> and
// the |r|^2 partials of the previous update), and one vector update (p, s = A p, x,
// r) that leaves the |r|^2 partials for the next iteration; a field on a small lattice
// finishes both sums in the update's blocks instead, three kernels per iteration.
int enqueue_cgcg_iteration(const CgProblem &P, CgWork &w, const std::vector<SysState> &st,
                           hipStream_t s) {
    const bool f64 = P.mode == STG_CG_F64;
    const stg_gauge *gg = f64 ? P.hi : P.lo;
    const size_t fb = (size_t)3 * P.g.Vh * (f64 ? 16 : 8);
    void *xin = f64 ? P.x : w.x_in;
    const bool fused = P.nsys == 1 && P.g.Vh <= kFusedFinishMaxVh;
    const uint32_t nbu = site_blocks(P.g.Vh);                 // blocks of the update kernel
    const size_t rr_buf = (size_t)2 * P.nsys * nbu;           // doubles per rr_partials buffer
    for (int j0 = 0; j0 < P.nsys;) {
        const int nr = P.chunk(j0);
        bool any = false;
        for (int j = j0; j < j0 + nr; ++j) any = any || (st[j].flags & SYS_RUNNING);
        if (!any) {
            j0 += nr;
            continue;
        }
        const size_t o = j0 * fb;
        HopArgs a = base_hop(P.g, gg);
        a.gate_running = 1;
        a.ctl = w.ctl;
        a.state = w.state + j0;
        a.partials = w.partials;
        a.partial_pairs = partial_count(P.g) / 2;
        // t = D_oe r
        a.out_parity = 1;
        a.op = OP_NONE;
        a.in = (const char *)w.r + o;
        a.out = (char *)w.t + o;
        HOP_TRY(hop(a, gg->fmt, nr, EPI_PLAIN, s));
        // w = diag r - D_eo t (into q) ; <r, w> partials
        uint32_t hop_blocks = 0;
        a.out_parity = 0;
        a.op = OP_CGCG;
        a.in = (const char *)w.t + o;
        a.out = (char *)w.q + o;
        a.aux0 = (const char *)w.r + o;
        a.defer_finish = 1;
        a.grid_out = &hop_blocks;
        HOP_TRY(hop(a, gg->fmt, nr, EPI_NORMAL, s));
        VecArgs v;
        std::memset(&v, 0, sizeof(v));
        v.Vh = P.g.Vh;
        v.fstride = (size_t)3 * P.g.Vh;
        v.x = (char *)xin + o;
        v.p = (char *)w.p + o;
        v.r = (char *)w.r + o;
        v.w = (const char *)w.q + o;
        v.s = (char *)w.s + o;
        v.state = w.state + j0;
        v.ctl = w.ctl;
        v.gate_running = 1;
        if (fused) {
            v.fin_partials = w.partials;
            v.fin_blocks = hop_blocks;
            v.fin_partials2 = w.rr_partials + (size_t)w.rr_cur * rr_buf;
            v.fin_blocks2 = nbu;
            v.partials = w.rr_partials + (size_t)(w.rr_cur ^ 1) * rr_buf;
            v.state_out = w.state_alt;
            VEC_TRY(launch_cgcg_update_fused(v, f64, s));
            std::swap(w.state, w.state_alt);
            w.rr_cur ^= 1;
        } else {
            double *rrp = w.rr_partials + (size_t)2 * j0 * nbu;
            FinArgs f{w.partials, hop_blocks, nr, OP_CGCG, 1, w.ctl, w.state + j0, nullptr,
                      rrp, nbu};
            VEC_TRY(launch_finalize(f, s));
            v.partials = rrp;
            VEC_TRY(launch_cgcg_update(v, f64, nr, s));
        }
        j0 += nr;
    }
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

int enqueue_inner_iteration(const CgProblem &P, CgWork &w, const std::vector<SysState> &st,
                            hipStream_t s) {
    if (P.cgcg) return enqueue_cgcg_iteration(P, w, st, s);
    const bool f64 = P.mode == STG_CG_F64;
    const stg_gauge *gg = f64 ? P.hi : P.lo;
    const size_t fb = (size_t)3 * P.g.Vh * (f64 ? 16 : 8);
    void *xin = f64 ? P.x : w.x_in;
    const bool fused = P.nsys == 1 && P.g.Vh <= kFusedFinishMaxVh;
    for (int j0 = 0; j0 < P.nsys;) {
        const int nr = P.chunk(j0);
        bool any = false;
        for (int j = j0; j < j0 + nr; ++j) any = any || (st[j].flags & SYS_RUNNING);
        if (!any) {
            j0 += nr;
            continue;
        }
        const size_t o = j0 * fb;
        HopArgs a = base_hop(P.g, gg);
        a.gate_running = 1;
        a.ctl = w.ctl;
        a.state = w.state + j0;
        a.partials = w.partials;
        a.partial_pairs = partial_count(P.g) / 2;
        // t = D_oe p
        a.out_parity = 1;
        a.op = OP_NONE;
        a.in = (const char *)w.p + o;
        a.out = (char *)w.t + o;
        HOP_TRY(hop(a, gg->fmt, nr, EPI_PLAIN, s));
        // q = diag p - D_eo t ; <p, q> -> alpha
        uint32_t hop_blocks = 0;
        a.out_parity = 0;
        a.op = OP_ALPHA;
        a.in = (const char *)w.t + o;
        a.out = (char *)w.q + o;
        a.aux0 = (const char *)w.p + o;
        a.defer_finish = fused ? 1 : 0;
        a.grid_out = &hop_blocks;
        HOP_TRY(hop(a, gg->fmt, nr, EPI_NORMAL, s));
        // x += alpha p, r -= alpha q ; |r|^2 -> beta / park ; p = r + beta p
        VecArgs v;
        std::memset(&v, 0, sizeof(v));
        v.Vh = P.g.Vh;
        v.fstride = (size_t)3 * P.g.Vh;
        v.x = (char *)xin + o;
        v.p = (char *)w.p + o;
        v.r = (char *)w.r + o;
        v.q = (const char *)w.q + o;
        v.state = w.state + j0;
        v.ctl = w.ctl;
        v.partials = w.partials;
        v.gate_running = 1;
        if (fused) {
            v.fin_partials = w.partials;
            v.fin_blocks = hop_blocks;
            v.partials = w.partials2;
            VEC_TRY(launch_cg_update_fused(v, f64, s));
            v.fin_partials = w.partials2;
            v.fin_blocks = site_blocks(P.g.Vh);
            v.state_out = w.state_alt;
            VEC_TRY(launch_p_update_fused(v, f64, s));
            std::swap(w.state, w.state_alt);
        } else {
            VEC_TRY(launch_cg_update(v, f64, nr, s));
            VEC_TRY(launch_p_update(v, f64, nr, s));
        }
        j0 += nr;
    }
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

// FP64 true-residual update of every parked system: x64 += x_inner (MIXED),
// r64 = b - A x64, then resume from r64 or finish.
int enqueue_reliable_update(const CgProblem &P, const CgWork &w, hipStream_t s) {
    const bool f64 = P.mode == STG_CG_F64;
    const size_t fb64 = (size_t)3 * P.g.Vh * 16;
    const size_t fbin = (size_t)3 * P.g.Vh * (f64 ? 16 : 8);
    for (int j0 = 0; j0 < P.nsys;) {
        const int nr = P.chunk(j0);
        VecArgs v;
        std::memset(&v, 0, sizeof(v));
        v.Vh = P.g.Vh;
        v.fstride = (size_t)3 * P.g.Vh;
        v.state = w.state + j0;
        v.ctl = w.ctl;
        v.partials = w.partials;
        v.x64 = (char *)P.x + j0 * fb64;
        if (!f64) {
            v.x = (char *)w.x_in + j0 * fbin;
            VEC_TRY(launch_ru_accumulate(v, nr, s));
        }
        HopArgs a = base_hop(P.g, P.hi);
        a.ctl = w.ctl;
        a.state = w.state + j0;
        a.partials = w.partials;
        a.partial_pairs = partial_count(P.g) / 2;
        a.out_parity = 1;
        a.op = OP_NONE;
        a.in = (const char *)P.x + j0 * fb64;
        a.out = (char *)w.t64 + j0 * fb64;
        HOP_TRY(hop(a, P.hi->fmt, nr, EPI_PLAIN, s));
        a.out_parity = 0;
        a.op = OP_RU;
        a.in = (const char *)w.t64 + j0 * fb64;
        a.out = (char *)w.r64 + j0 * fb64;
        a.aux0 = (const char *)P.x + j0 * fb64;
        a.aux1 = P.b_at(j0, fb64);
        HOP_TRY(hop(a, P.hi->fmt, nr, EPI_RESID, s));
        v.r64 = (const char *)w.r64 + j0 * fb64;
        v.r = (char *)w.r + j0 * fbin;
        v.p = (char *)w.p + j0 * fbin;
        // the single-reduction update applies beta itself: only the inner r is rebuilt
        // (nothing to do in FP64, where r is the true residual already)
        v.skip_p = P.cgcg ? 1 : 0;
        if (!(P.cgcg && f64)) VEC_TRY(launch_ru_resume(v, f64, nr, s));
        j0 += nr;
    }
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

// Pinned host buffers for the pipelined flag snapshots (grown on demand, kept
// for the life of the thread).
struct PinnedSnapshots {
    SysState *buf = nullptr;
    size_t cap = 0;  // SysState entries per slot
    hipEvent_t ev[2] = {nullptr, nullptr};
};
thread_local PinnedSnapshots g_snap;

int snapshots_ready(int nsys) {
    if (!g_snap.ev[0]) {
        HIP_TRY(hipEventCreateWithFlags(&g_snap.ev[0], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&g_snap.ev[1], hipEventDisableTiming));
    }
    if ((size_t)nsys > g_snap.cap) {
        if (g_snap.buf) HIP_TRY(hipHostFree(g_snap.buf));
        g_snap.buf = nullptr;
        g_snap.cap = 0;
        size_t cap = std::max<size_t>(64, (size_t)nsys);
        HIP_TRY(hipHostMalloc((void **)&g_snap.buf, 2 * cap * sizeof(SysState), 0));
        g_snap.cap = cap;
    }
    return STG_OK;
}

// Queues a copy of the flags into pinned slot `slot` and records its event.
int snapshot_enqueue(const SysState *dev, int nsys, int slot, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(g_snap.buf + (size_t)slot * g_snap.cap, dev, sizeof(SysState) * nsys,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(g_snap.ev[slot], s));
    return STG_OK;
}

int snapshot_wait(int nsys, int slot, std::vector<SysState> &st) {
    HIP_TRY(hipEventSynchronize(g_snap.ev[slot]));
    std::memcpy(st.data(), g_snap.buf + (size_t)slot * g_snap.cap, sizeof(SysState) * nsys);
    return STG_OK;
}

// Guards the host loops against a device state that stops advancing while some
// system is still marked running (the loops decide from the per-system flags):
// after kStallSnapshots snapshots without any change of the iteration counts or
// flags the solve returns an error instead of waiting forever.
constexpr int kStallSnapshots = 4;

struct StallGuard {
    long long last = -1;
    int same = 0;
    bool stalled(const std::vector<SysState> &st) {
        long long sig = 0;
        for (const SysState &q : st) sig = sig * 1000003LL + q.iter * 64LL + q.flags;
        same = (sig == last) ? same + 1 : 0;
        last = sig;
        return same >= kStallSnapshots;
    }
};

int stall_error() {
    g_last_error = "the solver state stopped advancing with systems still running";
    return STG_HIP_ERROR;
}

int read_states_n(const SysState *dev, int nsys, std::vector<SysState> &st, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(st.data(), dev, sizeof(SysState) * nsys, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return STG_OK;
}

int read_states(const CgWork &w, int nsys, std::vector<SysState> &st, hipStream_t s) {
    return read_states_n(w.state, nsys, st, s);
}

int run_cg(const CgProblem &P, CgWork w, stg_cg_stats *stats, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const int n = P.nsys;
    const bool f64 = P.mode == STG_CG_F64;
    const size_t fbin = (size_t)3 * P.g.Vh * (f64 ? 16 : 8);
    const size_t fb64 = (size_t)3 * P.g.Vh * 16;

    // initial state: every system parked with beta = 0, so the first update
    // computes r = b - A x0 and sets p = r
    std::vector<SysState> st(n);
    for (int j = 0; j < n; ++j) {
        SysState &q = st[j];
        std::memset(&q, 0, sizeof(q));
        q.diag = P.diag[j];
        q.tol2bb = P.prm.tol * P.prm.tol;  // times |b|^2 on the device
        q.delta2 = f64 ? 0.0 : P.prm.delta * P.prm.delta;
        q.flags = SYS_RU_PENDING;
        q.restart = resolve_restart(P.prm.restart, P.mode, P.lo);
        q.gid = j;
        q.max_iter = P.prm.max_iter;
    }
    Ctl ctl0;
    std::memset(&ctl0, 0, sizeof(ctl0));
    HIP_TRY(hipMemcpyAsync(w.ctl, &ctl0, sizeof(Ctl), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w.state, st.data(), sizeof(SysState) * n, hipMemcpyHostToDevice, s));
    launch_zero(w.p, (size_t)n * fbin, s);
    if (P.cgcg) launch_zero(w.s, (size_t)n * fbin, s);
    if (!f64) launch_zero(w.x_in, (size_t)n * fbin, s);
    for (int j = 0; j < n; ++j) {
        const void *bj = P.b_at(j, fb64);
        launch_dot(1, 1, (size_t)3 * P.g.Vh, bj, bj, w.partials, w.ctl, OP_INIT_BB,
                   w.state + j, nullptr, s);
    }
    HIP_TRY(hipGetLastError());
    int rc = read_states(w, n, st, s);
    if (rc) return rc;
    // b = 0: the solution is x = 0;  non-finite |b|^2: breakdown before any iteration
    bool any_zero = false;
    for (int j = 0; j < n; ++j) {
        if (!(st[j].bb < 1.0e300)) {
            any_zero = true;
            st[j].flags = SYS_BREAKDOWN;
            st[j].rr_true = st[j].bb;
        } else if (!(st[j].bb > 0.0)) {
            any_zero = true;
            st[j].flags = SYS_DONE;
            st[j].rr_true = 0.0;
            launch_zero((char *)P.x + j * fb64, fb64, s);
        }
    }
    if (any_zero)
        HIP_TRY(hipMemcpyAsync(w.state, st.data(), sizeof(SysState) * n, hipMemcpyHostToDevice, s));
    rc = enqueue_reliable_update(P, w, s);
    if (rc) return rc;

    int poll = P.prm.poll_every;
    if (poll <= 0) poll = (int)std::min<uint32_t>(64, std::max<uint32_t>(8, (1u << 22) / P.g.Vh));
    int status_all = STG_OK;
    rc = snapshots_ready(n);
    if (rc) return rc;
    // Pipelined polling: chunk c+1 is queued before the flags copied after chunk c
    // are read, so the GPU never waits for the host.  A parked system (reliable
    // update due) sees its update after at most one more chunk, in which it does
    // not iterate; the update itself drains the stream and restarts the pipeline.
    rc = read_states(w, n, st, s);
    if (rc) return rc;
    int slot = 0, pend = -1;  // pend: slot of a queued snapshot not read yet
    StallGuard guard;
    for (;;) {
        int running = 0, pending = 0;
        for (int j = 0; j < n; ++j) {
            if (st[j].flags & SYS_RUNNING) ++running;
            if (st[j].flags & SYS_RU_PENDING) ++pending;
        }
        if (pending) {
            if (pend >= 0) {
                rc = snapshot_wait(n, pend, st);  // the chunk queued after it: done, unused
                if (rc) return rc;
                pend = -1;
            }
            rc = enqueue_reliable_update(P, w, s);
            if (rc) return rc;
            rc = read_states(w, n, st, s);
            if (rc) return rc;
            continue;
        }
        if (running == 0) break;
        if (guard.stalled(st)) {
            (void)hipStreamSynchronize(s);
            return stall_error();
        }
        for (int i = 0; i < poll; ++i) {
            rc = enqueue_inner_iteration(P, w, st, s);
            if (rc) return rc;
        }
        rc = snapshot_enqueue(w.state, n, slot, s);
        if (rc) return rc;
        if (pend >= 0) {
            rc = snapshot_wait(n, pend, st);  // flags one chunk behind the queue
            if (rc) return rc;
        }
        pend = slot;
        slot ^= 1;
    }
    HIP_TRY(hipStreamSynchronize(s));
    rc = read_states(w, n, st, s);
    if (rc) return rc;
    // systems stopped by the iteration cap: fold the inner solution into x and
    // compute their true residual
    bool any_open = false;
    for (int j = 0; j < n; ++j)
        if (st[j].flags & (SYS_RUNNING | SYS_CAPPED)) {
            st[j].flags = SYS_RU_PENDING;
            st[j].restart = 1;
            any_open = true;
        }
    if (any_open) {
        HIP_TRY(hipMemcpyAsync(w.state, st.data(), sizeof(SysState) * n, hipMemcpyHostToDevice, s));
        rc = enqueue_reliable_update(P, w, s);
        if (rc) return rc;
        rc = read_states(w, n, st, s);
        if (rc) return rc;
    }
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int j = 0; j < n; ++j) {
        int stj;
        if (st[j].flags & SYS_DONE)
            stj = STG_OK;
        else if (st[j].flags & SYS_BREAKDOWN)
            stj = STG_BREAKDOWN;
        else
            stj = STG_NOT_CONVERGED;
        if (stats) {
            stats[j].iters = st[j].iter;
            stats[j].reliable_updates = st[j].n_ru;
            stats[j].status = stj;
            stats[j].converged_iter = (stj == STG_OK) ? st[j].conv_iter : -1;
            stats[j].true_rel_resid = st[j].bb > 0.0   ? std::sqrt(st[j].rr_true / st[j].bb)
                                      : st[j].bb == 0.0 ? 0.0
                                                        : std::nan("");
            stats[j].seconds = secs;
            stats[j].ms_iters = 0;
        }
        if (stj == STG_BREAKDOWN || (stj == STG_NOT_CONVERGED && status_all == STG_OK))
            status_all = stj;
    }
    return status_all;
}

int check_solver_common(const stg_lattice *lat, Geom &g, const stg_gauge *hi, const stg_gauge *lo,
                        int mode, int nrhs, const void *b, void *x, const stg_cg_params *prm) {
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    if (!prm) return invalid("params is NULL");
    if (mode != STG_CG_F64 && mode != STG_CG_MIXED) return invalid("unknown solver mode");
    if (!(prm->tol > 0.0) || prm->max_iter < 1) return invalid("tol must be > 0, max_iter >= 1");
    if (mode == STG_CG_MIXED && !(prm->delta > 0.0 && prm->delta < 1.0))
        return invalid("delta must be in (0, 1)");
    if (nrhs < 1) return invalid("nrhs < 1");
    int rc = check_gauge(g, hi, STG_C128);
    if (rc) return rc;
    if (mode == STG_CG_MIXED) {
        rc = check_gauge(g, lo, STG_C64);
        if (rc) return rc;
    }
    if (!aligned16(b) || !aligned16(x)) return invalid("b or x NULL or not 16-byte aligned");
    return STG_OK;
}


// ---------------------------------------------------------------------------
// multi-shift CG (Sec. 2.2, Eq. shlineq)
// ---------------------------------------------------------------------------

// Target of the multi-shift stage in mixed mode: FP32 vectors cannot carry the
// shifted solutions below about this relative residual; the refinement stage
// takes every system from there to the FP64 tolerance.
constexpr double kMsTolMixed = 1e-6;

struct MsWork {
    Ctl *ctl;
    SysState *state;      // one per RHS: the base system
    ShiftState *shift;    // [nshift][nrhs]
    double *partials;
    void *p, *r, *q, *t;  // base vectors, inner precision, [nrhs]
    void *xs, *ps;        // shifted solutions and directions, inner precision, [nshift][nrhs]
    size_t bytes;
};

MsWork carve_ms(const Geom &g, int nrhs, int nshift, int mode, void *ws) {
    Carver c{reinterpret_cast<char *>(ws)};
    MsWork w;
    const size_t e = mode == STG_CG_F64 ? 16 : 8;
    const size_t f1 = (size_t)nrhs * 3 * g.Vh * e;
    w.ctl = (Ctl *)c.take(sizeof(Ctl));
    w.state = (SysState *)c.take(sizeof(SysState) * (size_t)nrhs);
    w.shift = (ShiftState *)c.take(sizeof(ShiftState) * (size_t)nrhs * nshift);
    w.partials = (double *)c.take(sizeof(double) * partial_count(g));
    w.p = c.take(f1);
    w.r = c.take(f1);
    w.q = c.take(f1);
    w.t = c.take(f1);
    w.xs = c.take(f1 * nshift);
    w.ps = c.take(f1 * nshift);
    w.bytes = c.off;
    return w;
}

size_t ms_workspace(const Geom &g, int nrhs, int nshift, int mode) {
    return std::max(carve_ms(g, nrhs, nshift, mode, nullptr).bytes,
                    carve_cg(g, nrhs * nshift, mode, nullptr).bytes);
}

int enqueue_ms_iteration(const Geom &g, const stg_gauge *gg, int f64, int nrhs, int nshift,
                         const MsWork &w, hipStream_t s) {
    const size_t fb = (size_t)3 * g.Vh * (f64 ? 16 : 8);
    const int cap = field_cap(g, gg->fmt);
    for (int j0 = 0; j0 < nrhs;) {
        const int nr = chunk_of(nrhs - j0, cap);
        const size_t o = j0 * fb;
        HopArgs a = base_hop(g, gg);
        a.gate_running = 1;
        a.ctl = w.ctl;
        a.state = w.state + j0;
        a.partials = w.partials;
        a.partial_pairs = partial_count(g) / 2;
        a.out_parity = 1;
        a.op = OP_NONE;
        a.in = (const char *)w.p + o;
        a.out = (char *)w.t + o;
        HOP_TRY(hop(a, gg->fmt, nr, EPI_PLAIN, s));
        a.out_parity = 0;
        a.op = OP_MS_ALPHA;
        a.in = (const char *)w.t + o;
        a.out = (char *)w.q + o;
        a.aux0 = (const char *)w.p + o;
        HOP_TRY(hop(a, gg->fmt, nr, EPI_NORMAL, s));
        VecArgs v;
        std::memset(&v, 0, sizeof(v));
        v.Vh = g.Vh;
        v.fstride = (size_t)3 * g.Vh;
        v.p = (char *)w.p + o;
        v.r = (char *)w.r + o;
        v.q = (const char *)w.q + o;
        v.xs = (char *)w.xs + o;
        v.ps = (char *)w.ps + o;
        v.kstride = (size_t)nrhs * 3 * g.Vh;
        v.nshift = nshift;
        v.state = w.state + j0;
        v.ctl = w.ctl;
        v.partials = w.partials;
        v.gate_running = 1;
        VEC_TRY(launch_ms_r_update(v, f64, nr, s));
        VEC_TRY(launch_ms_p_update(v, f64, nr, s));
        j0 += nr;
    }
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

int run_mscg(const Geom &g, const stg_gauge *hi, const stg_gauge *lo, double mass, int nshift,
             const double *shifts, int nrhs, const void *b, void *x, const stg_cg_params &prm,
             void *ws, stg_cg_stats *stats, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const int mode = prm.mode;
    const int f64 = mode == STG_CG_F64;
    const stg_gauge *gg = f64 ? hi : lo;
    const size_t fb64 = (size_t)3 * g.Vh * 16;
    const size_t fbin = (size_t)3 * g.Vh * (f64 ? 16 : 8);
    const size_t n1 = (size_t)3 * g.Vh;  // complex entries per field
    int k0 = 0;
    for (int k = 1; k < nshift; ++k)
        if (shifts[k] < shifts[k0]) k0 = k;
    const double sigma0 = shifts[k0];
    const double tol_ms = f64 ? prm.tol : std::max(prm.tol, kMsTolMixed);

    MsWork w = carve_ms(g, nrhs, nshift, mode, ws);
    // host-side initial state
    Ctl ctl0;
    std::memset(&ctl0, 0, sizeof(ctl0));
    ctl0.n_running = nrhs;
    ctl0.nshift = nshift;
    ctl0.nrhs = nrhs;
    ctl0.ms = w.shift;
    std::vector<SysState> st(nrhs);
    for (int j = 0; j < nrhs; ++j) {
        SysState &q = st[j];
        std::memset(&q, 0, sizeof(q));
        q.diag = mass * mass + sigma0;
        q.tol2bb = tol_ms * tol_ms;
        q.flags = SYS_RUNNING;
        q.gid = j;
        q.max_iter = prm.max_iter;
        q.alpha_prev = 1.0;
        q.beta_prev = 0.0;
    }
    std::vector<ShiftState> zs((size_t)nshift * nrhs);
    for (int k = 0; k < nshift; ++k)
        for (int j = 0; j < nrhs; ++j) {
            ShiftState &z = zs[(size_t)k * nrhs + j];
            std::memset(&z, 0, sizeof(z));
            z.delta = shifts[k] - sigma0;
            z.zeta = z.zeta_prev = z.zeta_next = 1.0;
            z.active = 1;
        }
    HIP_TRY(hipMemcpyAsync(w.ctl, &ctl0, sizeof(Ctl), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w.state, st.data(), sizeof(SysState) * nrhs, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w.shift, zs.data(), sizeof(ShiftState) * zs.size(),
                           hipMemcpyHostToDevice, s));
    // r = p = b, p_k = b, x_k = 0  (in the inner precision)
    if (f64) {
        HIP_TRY(hipMemcpyAsync(w.r, b, nrhs * fb64, hipMemcpyDeviceToDevice, s));
    } else {
        launch_c128_to_c64((size_t)nrhs * n1, b, w.r, s);
    }
    HIP_TRY(hipMemcpyAsync(w.p, w.r, nrhs * fbin, hipMemcpyDeviceToDevice, s));
    for (int k = 0; k < nshift; ++k)
        HIP_TRY(hipMemcpyAsync((char *)w.ps + (size_t)k * nrhs * fbin, w.r, nrhs * fbin,
                               hipMemcpyDeviceToDevice, s));
    launch_zero(w.xs, (size_t)nshift * nrhs * fbin, s);
    for (int j = 0; j < nrhs; ++j) {
        const void *bj = (const char *)b + j * fb64;
        launch_dot(1, 1, n1, bj, bj, w.partials, w.ctl, OP_INIT_BB, w.state + j, nullptr, s);
    }
    HIP_TRY(hipGetLastError());
    int rc = read_states_n(w.state, nrhs, st, s);
    if (rc) return rc;
    bool any_zero = false;
    for (int j = 0; j < nrhs; ++j) {
        if (!(st[j].bb < 1.0e300)) {
            // non-finite |b|^2
            any_zero = true;
            st[j].flags = SYS_BREAKDOWN;
        } else if (!(st[j].bb > 0.0)) {
            // b = 0: every x_k stays 0
            any_zero = true;
            st[j].flags = SYS_DONE;
        }
    }
    if (any_zero) {
        int nrun = 0;
        for (int j = 0; j < nrhs; ++j) nrun += (st[j].flags & SYS_RUNNING) ? 1 : 0;
        ctl0.n_running = nrun;
        HIP_TRY(hipMemcpyAsync(w.ctl, &ctl0, sizeof(Ctl), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(w.state, st.data(), sizeof(SysState) * nrhs, hipMemcpyHostToDevice,
                               s));
    }
    int poll = prm.poll_every;
    if (poll <= 0) poll = (int)std::min<uint32_t>(64, std::max<uint32_t>(8, (1u << 22) / g.Vh));
    rc = snapshots_ready(nrhs);
    if (rc) return rc;
    rc = read_states_n(w.state, nrhs, st, s);
    if (rc) return rc;
    // pipelined polling as in the CG loop (no reliable updates in this stage; the
    // iteration cap is enforced on the device)
    int slot = 0, pend = -1;
    StallGuard guard;
    for (;;) {
        int running = 0;
        for (int j = 0; j < nrhs; ++j)
            running += (st[j].flags & (SYS_RUNNING | SYS_FINISHING)) ? 1 : 0;
        if (running == 0) break;
        if (guard.stalled(st)) {
            (void)hipStreamSynchronize(s);
            return stall_error();
        }
        for (int i = 0; i < poll; ++i) {
            rc = enqueue_ms_iteration(g, gg, f64, nrhs, nshift, w, s);
            if (rc) return rc;
        }
        rc = snapshot_enqueue(w.state, nrhs, slot, s);
        if (rc) return rc;
        if (pend >= 0) {
            rc = snapshot_wait(nrhs, pend, st);
            if (rc) return rc;
        }
        pend = slot;
        slot ^= 1;
    }
    HIP_TRY(hipStreamSynchronize(s));
    rc = read_states_n(w.state, nrhs, st, s);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(zs.data(), w.shift, sizeof(ShiftState) * zs.size(),
                           hipMemcpyDeviceToHost, s));
    // shifted solutions -> x (complex128, [nshift][nrhs])
    if (f64)
        HIP_TRY(hipMemcpyAsync(x, w.xs, (size_t)nshift * nrhs * fb64, hipMemcpyDeviceToDevice, s));
    else
        launch_c64_to_c128((size_t)nshift * nrhs * n1, w.xs, x, s);
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<SysState> base = st;

    // refinement: every (shift, RHS) system warm-started from its multi-shift
    // solution, solved to the FP64 tolerance with its own diagonal
    CgProblem P;
    P.g = g;
    P.hi = hi;
    P.lo = lo;
    P.mode = mode;
    P.nsys = nshift * nrhs;
    P.b = b;
    P.x = x;
    P.group = nrhs;
    P.cap = field_cap(g, mode == STG_CG_F64 ? hi->fmt : lo->fmt);
    P.cgcg = cg_single_reduction(P.nsys);
    P.diag.resize(P.nsys);
    for (int k = 0; k < nshift; ++k)
        for (int j = 0; j < nrhs; ++j) P.diag[(size_t)k * nrhs + j] = mass * mass + shifts[k];
    P.prm = prm;
    CgWork cw = carve_cg(g, P.nsys, mode, ws);
    std::vector<stg_cg_stats> rs(P.nsys);
    const int status = run_cg(P, cw, rs.data(), s);
    if (status < 0) return status;
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int k = 0; k < nshift; ++k)
        for (int j = 0; j < nrhs; ++j) {
            const size_t i = (size_t)k * nrhs + j;
            const ShiftState &z = zs[i];
            const int ms_it = z.active ? base[j].iter : z.conv_iter;
            stats[i] = rs[i];
            stats[i].iters = ms_it + rs[i].iters;
            stats[i].ms_iters = ms_it;
            stats[i].converged_iter =
                rs[i].status == STG_OK ? ms_it + std::max(0, rs[i].converged_iter) : -1;
            stats[i].seconds = secs;
        }
    return status;
}


// ---------------------------------------------------------------------------
// uneven batch: many lattices per launch, CG iterations replayed from a hipGraph
// ---------------------------------------------------------------------------
struct BatchPlan {
    std::vector<BSolve> solves;
    std::vector<BTile> sorted;    // every tile, grouped by class
    std::vector<BTile> tiles;     // the tiles launched: grouped by class, see classes
    std::vector<BClass> classes;  // contiguous tile ranges of one (fields, threads per site)
    std::vector<BSysRef> sysref;
    uint32_t nsys = 0, npairs = 0;
    // device tables and state (in the workspace)
    Ctl *ctl = nullptr;
    SysState *state = nullptr;
    BSolve *d_solves = nullptr;
    BTile *d_tiles = nullptr;
    BSysRef *d_sysref = nullptr;
    double *partials = nullptr;
    double *partials2 = nullptr;  // the single-reduction update's |r|^2 partials
    bool cgcg = true;             // iteration in the single-reduction form
    size_t bytes = 0;
};

// Threads per site of a batch tile's hop for a solve's lattice, inner link format and
// chunk of fields: the autotuner's choice when it has timed that key, else the
// library's default for the normal-operator hop (several for several fields or a
// small lattice, else one).
uint8_t batch_tile_tps(const Geom &g, int fmt, int nr) {
    TuneChoice c;
    int tps = tune_lookup(g, fmt, nr, c) ? c.threads_per_site
                                         : default_threads_per_site(fmt, nr, EPI_NORMAL, g.Vh);
    if (g_threads_per_site) tps = g_threads_per_site;  // the caller's process-wide choice
    return (uint8_t)((tps == 2 || tps == 4) ? tps : 1);
}

// Lays out the batch in ws (ws == nullptr: size only).  Tiles are grouped by class
// (fields per tile, threads per site: one hop launch each); within a class they follow
// the solve order, then the RHS chunks (4 while at least 4 remain, then the rest) of
// each solve, then the site blocks.
// The hop gives each XCD one contiguous run of a class's tiles (xcd_block).  Reorder
// the class range [begin, end) so that run x holds the x-th eighth of every group of
// tiles with one solve and chunk of fields: every XCD then works on every solve as
// long as it runs, and its share of a solve is consecutive sites, whose neighbour
// lines meet in that XCD's L2.
void deal_over_xcds(std::vector<BTile> &tiles, uint32_t begin, uint32_t end) {
    std::vector<std::pair<uint32_t, uint32_t>> groups;
    for (uint32_t k = begin; k < end;) {
        uint32_t e = k + 1;
        while (e < end && tiles[e].solve == tiles[k].solve && tiles[e].j0 == tiles[k].j0) ++e;
        groups.emplace_back(k, e);
        k = e;
    }
    std::vector<BTile> out;
    out.reserve(end - begin);
    for (uint32_t x = 0; x < kXcds; ++x)
        for (const auto &gr : groups) {
            const uint64_t m = gr.second - gr.first;
            for (uint64_t k = gr.first + m * x / kXcds; k < gr.first + m * (x + 1) / kXcds; ++k)
                out.push_back(tiles[k]);
        }
    std::copy(out.begin(), out.end(), tiles.begin() + begin);
}

// A system that converged or broke down never runs again.
bool system_final(const SysState &q) {
    return (q.flags & (SYS_DONE | SYS_BREAKDOWN)) &&
           !(q.flags & (SYS_RUNNING | SYS_RU_PENDING | SYS_RESUME));
}

bool tile_finished(const BatchPlan &B, const BTile &t, const std::vector<SysState> &st) {
    const uint32_t k0 = B.solves[t.solve].sys0 + t.j0;
    for (uint32_t j = 0; j < t.nr; ++j)
        if (!system_final(st[k0 + j])) return false;
    return true;
}

// The launched tile table: the tiles of B.sorted (all of them, or with st the ones
// holding a system that is not final), in classes, each class dealt over the XCDs.
void arrange_tiles(BatchPlan &B, const std::vector<SysState> *st) {
    B.tiles.clear();
    for (const BTile &t : B.sorted)
        if (!st || !tile_finished(B, t, *st)) B.tiles.push_back(t);
    B.classes.clear();
    for (uint32_t k = 0; k < (uint32_t)B.tiles.size(); ++k) {
        const BTile &t = B.tiles[k];
        const BSolve &S = B.solves[t.solve];
        const int lo = S.lo_phases == nullptr, hi = S.hi_phases == nullptr;
        const BClass *c = B.classes.empty() ? nullptr : &B.classes.back();
        if (!c || c->nr != t.nr || c->tps != t.tps || c->std_lo != lo || c->std_hi != hi)
            B.classes.push_back(BClass{k, k, t.nr, t.tps, lo, hi});
        B.classes.back().end = k + 1;
    }
    for (const BClass &cl : B.classes) deal_over_xcds(B.tiles, cl.begin, cl.end);
}

// Class order of the tiles: fields, threads per site, then the phase kinds.
int tile_class_key(const BatchPlan &B, const BTile &t) {
    const BSolve &S = B.solves[t.solve];
    return ((t.nr * 8 + t.tps) * 2 + (S.lo_phases == nullptr)) * 2 + (S.hi_phases == nullptr);
}

// Whether dropping the finished tiles pays for a new graph: a quarter of the launched
// tiles, or a whole class (two hop launches per iteration), would go.
bool prune_pays(const BatchPlan &B, const std::vector<SysState> &st) {
    size_t live = 0;
    size_t live_classes = 0;
    for (const BClass &cl : B.classes) {
        size_t n = 0;
        for (uint32_t k = cl.begin; k < cl.end; ++k) n += tile_finished(B, B.tiles[k], st) ? 0 : 1;
        live += n;
        live_classes += n ? 1 : 0;
    }
    return live > 0 && (4 * live <= 3 * B.tiles.size() || live_classes < B.classes.size());
}

int plan_batch(int nsolve, const stg_solve_desc *d, int mode, void *ws, BatchPlan &B) {
    const bool f64 = mode == STG_CG_F64;
    Carver c{reinterpret_cast<char *>(ws)};
    B.solves.assign(nsolve, BSolve{});
    B.tiles.clear();
    B.sysref.clear();
    uint32_t sys = 0, pairs = 0;
    for (int i = 0; i < nsolve; ++i) {
        Geom g;
        if (!make_geom(&d[i].lat, g)) return invalid("batch: lattice extents must be even, >= 2");
        if (d[i].nrhs < 1) return invalid("batch: nrhs < 1");
        BSolve &S = B.solves[i];
        S.g = g;
        S.nrhs = (uint32_t)d[i].nrhs;
        S.sys0 = sys;
        S.nblk = site_blocks(g.Vh);
        S.part0 = pairs;
        S.hi_phases = d[i].hi.phases;  // the tile classes depend on the phase kinds
        S.lo_phases = f64 ? nullptr : d[i].lo.phases;
        pairs += S.nblk * S.nrhs;
        for (int j = 0; j < d[i].nrhs; ++j) B.sysref.push_back(BSysRef{(uint32_t)i, (uint32_t)j});
        sys += S.nrhs;
        const int fmt_in = f64 ? d[i].hi.fmt : d[i].lo.fmt;
        for (int j0 = 0; j0 < d[i].nrhs;) {
            int rem = d[i].nrhs - j0;
            int nr = rem >= 4 ? 4 : rem;
            const uint8_t tps = batch_tile_tps(g, fmt_in, nr);
            for (uint32_t blk = 0; blk < S.nblk; ++blk)
                B.tiles.push_back(BTile{(uint32_t)i, blk, (uint16_t)j0, (uint8_t)nr, tps});
            j0 += nr;
        }
    }
    // group the tiles by class, keeping their order within a class
    std::stable_sort(B.tiles.begin(), B.tiles.end(), [&B](const BTile &x, const BTile &y) {
        return tile_class_key(B, x) < tile_class_key(B, y);
    });
    B.sorted = B.tiles;
    arrange_tiles(B, nullptr);
    B.nsys = sys;
    B.npairs = pairs;
    B.ctl = (Ctl *)c.take(sizeof(Ctl));
    B.state = (SysState *)c.take(sizeof(SysState) * sys);
    B.d_solves = (BSolve *)c.take(sizeof(BSolve) * nsolve);
    B.d_tiles = (BTile *)c.take(sizeof(BTile) * B.tiles.size());
    B.d_sysref = (BSysRef *)c.take(sizeof(BSysRef) * sys);
    B.partials = (double *)c.take(sizeof(double) * 2 * kTileSlots * (size_t)pairs);
    B.partials2 = (double *)c.take(sizeof(double) * 2 * kTileSlots * (size_t)pairs);
    for (int i = 0; i < nsolve; ++i) {
        BSolve &S = B.solves[i];
        const size_t n1 = (size_t)S.nrhs * 3 * S.g.Vh;
        const size_t fin = n1 * (f64 ? 16 : 8);
        S.hi_links = d[i].hi.links;
        S.lo_links = f64 ? nullptr : d[i].lo.links;
        S.b = d[i].b;
        S.x64 = d[i].x;
        S.p = c.take(fin);
        S.r = c.take(fin);
        S.q = c.take(fin);
        S.t = c.take(fin);
        S.s = c.take(fin);
        if (f64) {
            S.xin = d[i].x;
            S.r64 = S.r;
            S.t64 = S.t;
        } else {
            S.xin = c.take(fin);
            S.r64 = c.take(n1 * 16);
            S.t64 = c.take(n1 * 16);
        }
    }
    B.bytes = c.off;
    return STG_OK;
}

BArgs batch_args(const BatchPlan &B, int gate, int tile_mask) {
    BArgs a;
    std::memset(&a, 0, sizeof(a));
    a.solves = B.d_solves;
    a.tiles = B.d_tiles;
    a.sysref = B.d_sysref;
    a.state = B.state;
    a.ctl = B.ctl;
    a.partials = B.partials;
    a.partials2 = B.partials2;
    a.ntiles = (uint32_t)B.tiles.size();
    a.nsys = B.nsys;
    a.grid = a.ntiles;  // one block per tile
    a.gate_running = gate;
    a.tile_mask = tile_mask;
    return a;
}

int enqueue_batch_iteration(const BatchPlan &B, int f64, int fmt_in, hipStream_t s) {
    BArgs a = batch_args(B, 1, SYS_RUNNING);
    a.use_hi = f64;
    if (B.cgcg) {
        // single-reduction form: t = D_oe r; w = diag r - D_eo t (into q) with <r, w>;
        // alpha and beta from <r, w> and the last update's |r|^2; one vector update
        a.out_parity = 1;
        a.f_in = BF_R;
        a.f_out = BF_T;
        HOP_TRY(launch_bhop(a, B.classes.data(), (int)B.classes.size(), fmt_in, EPI_PLAIN, s));
        a.out_parity = 0;
        a.f_in = BF_T;
        a.f_out = BF_Q;
        a.f_aux0 = BF_R;
        HOP_TRY(launch_bhop(a, B.classes.data(), (int)B.classes.size(), fmt_in, EPI_NORMAL, s));
        VEC_TRY(launch_bfinalize(a, OP_CGCG, s));
        VEC_TRY(launch_bcgcg_update(a, f64, s));
        HIP_TRY(hipGetLastError());
        return STG_OK;
    }
    a.out_parity = 1;  // t = D_oe p
    a.f_in = BF_P;
    a.f_out = BF_T;
    HOP_TRY(launch_bhop(a, B.classes.data(), (int)B.classes.size(), fmt_in, EPI_PLAIN, s));
    a.out_parity = 0;  // q = diag p - D_eo t; <p, q>
    a.f_in = BF_T;
    a.f_out = BF_Q;
    a.f_aux0 = BF_P;
    HOP_TRY(launch_bhop(a, B.classes.data(), (int)B.classes.size(), fmt_in, EPI_NORMAL, s));
    VEC_TRY(launch_bfinalize(a, OP_ALPHA, s));
    VEC_TRY(launch_bcg_update(a, f64, s));
    VEC_TRY(launch_bfinalize(a, OP_BETA, s));
    VEC_TRY(launch_bp_update(a, f64, s));
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

int enqueue_batch_update(const BatchPlan &B, int f64, int fmt_hi, hipStream_t s) {
    BArgs a = batch_args(B, 0, SYS_RU_PENDING);
    if (!f64) VEC_TRY(launch_bru_accumulate(a, s));
    a.use_hi = 1;
    a.out_parity = 1;
    a.f_in = BF_X64;
    a.f_out = BF_T64;
    HOP_TRY(launch_bhop(a, B.classes.data(), (int)B.classes.size(), fmt_hi, EPI_PLAIN, s));
    a.out_parity = 0;
    a.f_in = BF_T64;
    a.f_out = BF_R64;
    a.f_aux0 = BF_X64;
    HOP_TRY(launch_bhop(a, B.classes.data(), (int)B.classes.size(), fmt_hi, EPI_RESID, s));
    VEC_TRY(launch_bfinalize(a, OP_RU, s));
    a.tile_mask = SYS_RESUME;
    // the single-reduction update applies beta to p and s itself, so a resume only
    // rebuilds the inner r (nothing at all in FP64, where r is the true residual)
    a.skip_p = B.cgcg ? 1 : 0;
    if (!(B.cgcg && f64)) VEC_TRY(launch_bru_resume(a, f64, s));
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

thread_local hipStream_t g_capture_stream = nullptr;

// K inner iterations of the whole batch, captured into one executable graph.
int capture_batch(const BatchPlan &B, int f64, int fmt_in, int K, hipGraph_t &graph,
                  hipGraphExec_t &exec) {
    graph = nullptr;
    exec = nullptr;
    if (!g_capture_stream) HIP_TRY(hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < K; ++i) {
        const int rc = enqueue_batch_iteration(B, f64, fmt_in, g_capture_stream);
        if (rc) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(g_capture_stream, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            return rc;
        }
    }
    HIP_TRY(hipStreamEndCapture(g_capture_stream, &graph));
    hipError_t ge = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ge != hipSuccess) {
        (void)hipGraphDestroy(graph);
        graph = nullptr;
        exec = nullptr;
        return hip_fail(ge, "hipGraphInstantiate");
    }
    return STG_OK;
}

int run_cg_batch(int nsolve, const stg_solve_desc *d, const stg_cg_params &prm, void *ws,
                 stg_cg_stats *stats, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const int mode = prm.mode;
    const int f64 = mode == STG_CG_F64;
    BatchPlan B;
    int rc = plan_batch(nsolve, d, mode, ws, B);
    if (rc) return rc;
    // the classic form unless the single-reduction one is asked for: on the 12-lattice
    // benchmark (same box, same sources) the batch took 1.233 s in the classic form and
    // 1.264 s in the single-reduction one, whose extra step per reliable update and
    // per solve outweighed the finalize launch it saves
    B.cgcg = g_cg_form == 2;
    const int fmt_hi = d[0].hi.fmt;
    const int fmt_in = f64 ? fmt_hi : d[0].lo.fmt;
    const int n = (int)B.nsys;
    HIP_TRY(hipMemcpyAsync(B.d_solves, B.solves.data(), sizeof(BSolve) * nsolve,
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(B.d_tiles, B.tiles.data(), sizeof(BTile) * B.tiles.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(B.d_sysref, B.sysref.data(), sizeof(BSysRef) * n,
                           hipMemcpyHostToDevice, s));
    std::vector<SysState> st(n);
    for (int k = 0; k < n; ++k) {
        const stg_solve_desc &di = d[B.sysref[k].solve];
        SysState &q = st[k];
        std::memset(&q, 0, sizeof(q));
        q.diag = di.mass * di.mass;
        q.tol2bb = prm.tol * prm.tol;
        q.delta2 = f64 ? 0.0 : prm.delta * prm.delta;
        q.flags = SYS_RU_PENDING;
        q.restart = resolve_restart(prm.restart, prm.mode, f64 ? nullptr : &di.lo);
        q.gid = k;
        q.max_iter = prm.max_iter;
    }
    Ctl ctl0;
    std::memset(&ctl0, 0, sizeof(ctl0));
    HIP_TRY(hipMemcpyAsync(B.ctl, &ctl0, sizeof(Ctl), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(B.state, st.data(), sizeof(SysState) * n, hipMemcpyHostToDevice, s));
    for (int i = 0; i < nsolve; ++i) {
        const BSolve &S = B.solves[i];
        const size_t fin = (size_t)S.nrhs * 3 * S.g.Vh * (f64 ? 16 : 8);
        launch_zero(S.p, fin, s);
        launch_zero(S.s, fin, s);  // beta = 0 multiplies it in the first step
        if (!f64) launch_zero(S.xin, fin, s);
    }
    {
        BArgs a = batch_args(B, 0, 0);
        launch_bnorm_b(a, s);
        launch_bfinalize(a, OP_INIT_BB, s);
    }
    HIP_TRY(hipGetLastError());
    rc = read_states_n(B.state, n, st, s);
    if (rc) return rc;
    bool fix = false;
    for (int k = 0; k < n; ++k) {
        const BSolve &S = B.solves[B.sysref[k].solve];
        const size_t fb = (size_t)3 * S.g.Vh * 16;
        if (!(st[k].bb < 1.0e300)) {
            fix = true;
            st[k].flags = SYS_BREAKDOWN;
            st[k].rr_true = st[k].bb;
        } else if (!(st[k].bb > 0.0)) {
            fix = true;
            st[k].flags = SYS_DONE;
            st[k].rr_true = 0.0;
            launch_zero((char *)S.x64 + B.sysref[k].j * fb, fb, s);
        }
    }
    if (fix) HIP_TRY(hipMemcpyAsync(B.state, st.data(), sizeof(SysState) * n, hipMemcpyHostToDevice, s));
    rc = enqueue_batch_update(B, f64, fmt_hi, s);
    if (rc) return rc;

    // K inner iterations of the whole batch, captured and replayed; captured again
    // over the remaining tiles when finished solves leave enough of them idle
    int K = prm.poll_every > 0 ? prm.poll_every : 16;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    rc = capture_batch(B, f64, fmt_in, K, graph, exec);
    if (rc) return rc;
    int replays = 0;
    rc = snapshots_ready(n);
    if (!rc) rc = read_states_n(B.state, n, st, s);
    int slot = 0, pend = -1;
    StallGuard guard;
    while (!rc) {
        int running = 0, pending = 0;
        for (int k = 0; k < n; ++k) {
            if (st[k].flags & SYS_RUNNING) ++running;
            if (st[k].flags & SYS_RU_PENDING) ++pending;
        }
        if (pending) {
            if (pend >= 0) {
                rc = snapshot_wait(n, pend, st);
                if (rc) break;
                pend = -1;
            }
            rc = enqueue_batch_update(B, f64, fmt_hi, s);
            if (!rc) rc = read_states_n(B.state, n, st, s);
            continue;
        }
        if (running == 0) break;
        if (guard.stalled(st)) {
            rc = stall_error();
            break;
        }
        if (prune_pays(B, st)) {
            // the replay in flight still reads the old tile table
            hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess) {
                rc = hip_fail(e, "hipStreamSynchronize");
                break;
            }
            if (pend >= 0) {
                rc = snapshot_wait(n, pend, st);
                if (rc) break;
                pend = -1;
            }
            arrange_tiles(B, &st);
            e = hipMemcpyAsync(B.d_tiles, B.tiles.data(), sizeof(BTile) * B.tiles.size(),
                               hipMemcpyHostToDevice, s);
            if (e != hipSuccess) {
                rc = hip_fail(e, "hipMemcpyAsync");
                break;
            }
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            rc = capture_batch(B, f64, fmt_in, K, graph, exec);
            if (rc) break;
        }
        hipError_t le = hipGraphLaunch(exec, s);
        if (le != hipSuccess) {
            rc = hip_fail(le, "hipGraphLaunch");
            break;
        }
        ++replays;
        rc = snapshot_enqueue(B.state, n, slot, s);
        if (rc) break;
        if (pend >= 0) rc = snapshot_wait(n, pend, st);
        pend = slot;
        slot ^= 1;
    }
    if (!rc) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) return rc;
    rc = read_states_n(B.state, n, st, s);
    if (rc) return rc;
    bool open = false;
    for (int k = 0; k < n; ++k)
        if (st[k].flags & (SYS_RUNNING | SYS_CAPPED)) {
            st[k].flags = SYS_RU_PENDING;
            st[k].restart = 1;
            open = true;
        }
    if (open) {
        HIP_TRY(hipMemcpyAsync(B.state, st.data(), sizeof(SysState) * n, hipMemcpyHostToDevice, s));
        rc = enqueue_batch_update(B, f64, fmt_hi, s);
        if (rc) return rc;
        rc = read_states_n(B.state, n, st, s);
        if (rc) return rc;
    }
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int status_all = STG_OK;
    for (int k = 0; k < n; ++k) {
        int stk = (st[k].flags & SYS_DONE) ? STG_OK
                  : (st[k].flags & SYS_BREAKDOWN) ? STG_BREAKDOWN
                                                  : STG_NOT_CONVERGED;
        stats[k].iters = st[k].iter;
        stats[k].reliable_updates = st[k].n_ru;
        stats[k].status = stk;
        stats[k].converged_iter = stk == STG_OK ? st[k].conv_iter : -1;
        stats[k].true_rel_resid = st[k].bb > 0.0   ? std::sqrt(st[k].rr_true / st[k].bb)
                                  : st[k].bb == 0.0 ? 0.0
                                                    : std::nan("");
        stats[k].seconds = secs;
        stats[k].ms_iters = 0;
        if (stk == STG_BREAKDOWN || (stk == STG_NOT_CONVERGED && status_all == STG_OK))
            status_all = stk;
    }
    (void)replays;
    return status_all;
}

int check_batch(int nsolve, const stg_solve_desc *d, const stg_cg_params *prm) {
    if (nsolve < 1 || !d) return invalid("batch: nsolve >= 1 and descs non-NULL");
    if (!prm) return invalid("params is NULL");
    if (prm->mode != STG_CG_F64 && prm->mode != STG_CG_MIXED) return invalid("unknown solver mode");
    if (!(prm->tol > 0.0) || prm->max_iter < 1) return invalid("tol must be > 0, max_iter >= 1");
    if (prm->mode == STG_CG_MIXED && !(prm->delta > 0.0 && prm->delta < 1.0))
        return invalid("delta must be in (0, 1)");
    for (int i = 0; i < nsolve; ++i) {
        Geom g;
        if (!make_geom(&d[i].lat, g)) return invalid("batch: lattice extents must be even, >= 2");
        if (d[i].nrhs < 1) return invalid("batch: nrhs < 1");
        int rc = check_gauge(g, &d[i].hi, STG_C128);
        if (rc) return rc;
        if (d[i].hi.fmt != d[0].hi.fmt) return invalid("batch: every hi gauge field has one format");
        if (prm->mode == STG_CG_MIXED) {
            rc = check_gauge(g, &d[i].lo, STG_C64);
            if (rc) return rc;
            if (d[i].lo.fmt != d[0].lo.fmt)
                return invalid("batch: every lo gauge field has one format");
        }
        if (!aligned16(d[i].b) || !aligned16(d[i].x)) return invalid("batch: b or x misaligned");
        const size_t fb = (size_t)d[i].nrhs * 3 * g.Vh * 16;
        if (overlap(d[i].b, fb, d[i].x, fb)) return invalid("batch: b and x overlap");
    }
    return STG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// normal operator
// ---------------------------------------------------------------------------
namespace {

int check_normal(const stg_lattice *lat, const stg_gauge *gauge, int field, int nrhs,
                 const void *in_even, const void *out_even, Geom &g) {
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    if (field != STG_C128 && field != STG_C64) return invalid("unknown field type");
    int rc = check_gauge(g, gauge, field);
    if (rc) return rc;
    if (nrhs < 1) return invalid("nrhs < 1");
    if (!aligned16(in_even) || !aligned16(out_even))
        return invalid("field NULL or not 16-byte aligned");
    const size_t fb = (size_t)nrhs * 3 * g.Vh * field_elem(field);
    if (overlap(in_even, fb, out_even, fb)) return invalid("fields overlap");
    return STG_OK;
}

// out = diag in - D_eo D_oe in, with tmp (odd parity, same shape) receiving D_oe in.
int apply_normal(const Geom &g, const stg_gauge *gauge, int field, int nrhs, double mass,
                 double sigma, const void *in_even, void *out_even, void *tmp_odd,
                 hipStream_t s) {
    int rc = hop_plain(g, gauge, field, nrhs, in_even, tmp_odd, 1, s);
    if (rc) return rc;
    const size_t f1 = (size_t)3 * g.Vh * field_elem(field);
    HopArgs a = base_hop(g, gauge);
    a.out_parity = 0;
    a.op = OP_NONE;
    a.diag = mass * mass + sigma;
    const int cap = field_cap(g, gauge->fmt);
    for (int j0 = 0; j0 < nrhs;) {
        int nr = chunk_of(nrhs - j0, cap);
        a.in = (const char *)tmp_odd + j0 * f1;
        a.out = (char *)out_even + j0 * f1;
        a.aux0 = (const char *)in_even + j0 * f1;
        HOP_TRY(hop(a, gauge->fmt, nr, EPI_NORMAL, s));
        j0 += nr;
    }
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

}  // namespace

// ===========================================================================
// exported
// ===========================================================================
extern "C" {

int stg_version(void) { return (1 << 16) | 0; }

const char *stg_status_string(int status) {
    switch (status) {
        case STG_OK: return "ok";
        case STG_NOT_CONVERGED: return "not converged (iteration cap reached)";
        case STG_BREAKDOWN: return "breakdown (non-finite scalar or <p, A p> <= 0)";
        case STG_INVALID_ARG: return "invalid argument";
        case STG_HIP_ERROR: return "HIP runtime error";
        case STG_WORKSPACE_TOO_SMALL: return "workspace too small";
        default: return "unknown status";
    }
}

const char *stg_last_error(void) { return g_last_error.c_str(); }

int stg_set_tuning(int key, int value) {
    switch (key) {
        case STG_TUNE_XCD_REMAP:
            if (value != 0 && value != 1) return invalid("XCD remap takes 0 or 1");
            g_xcd_remap = value;
            return STG_OK;
        case STG_TUNE_SITES_PER_THREAD:
            if (value != 1 && value != 2 && value != 4 && value != 8)
                return invalid("sites per thread takes 1, 2, 4 or 8");
            g_sites_per_thread = value;
            return STG_OK;
        case STG_TUNE_STAGE_NEIGHBOURS:
            if (value != 0 && value != 1) return invalid("neighbour staging takes 0 or 1");
            g_stage_neighbours = value;
            return STG_OK;
        case STG_TUNE_THREADS_PER_SITE:
            if (value != 0 && value != 1 && value != 2 && value != 4)
                return invalid("threads per site takes 0 (automatic), 1, 2 or 4");
            g_threads_per_site = value;
            return STG_OK;
        case STG_TUNE_STAPLE_THREADS:
            if (value < 0 || value > 2)
                return invalid("staple threads per link takes 0 (automatic), 1 or 2");
            g_staple_threads = value;
            return STG_OK;
        case STG_TUNE_PENCIL_TILE:
            if (value < 0 || value >= kPencilShapes)
                return invalid("pencil tile takes 0 .. 5");
            g_pencil_tile = value;
            return STG_OK;
        case STG_TUNE_FIELDS_PER_LAUNCH:
            if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
                return invalid("fields per launch takes 0 (automatic), 1, 2, 4 or 8");
            g_fields_per_launch = value;
            return STG_OK;
        case STG_TUNE_LAYER_GROUP:
            if (value < 0 || value > 1024) return invalid("layer group takes 0 .. 1024");
            g_layer_group = value;
            return STG_OK;
        case STG_TUNE_SPREAD_EPILOGUE:
            if (value != 0 && value != 1) return invalid("spread epilogue takes 0 or 1");
            g_spread_epilogue = value;
            return STG_OK;
        case STG_TUNE_CG_FORM:
            if (value < 0 || value > 2)
                return invalid("CG form takes 0 (automatic), 1 (two reductions) or 2 (one)");
            g_cg_form = value;
            return STG_OK;
        case STG_TUNE_FIELD_SPLIT:
            if (value < -1 || value > 2)
                return invalid("field split takes -1 (off), 0 (automatic), 1 or 2 fields per wave");
            g_field_split = value;
            return STG_OK;
        default: return invalid("unknown tuning key");
    }
}

int stg_get_tuning(int key, int *value) {
    if (!value) return invalid("value is NULL");
    switch (key) {
        case STG_TUNE_XCD_REMAP: *value = g_xcd_remap; return STG_OK;
        case STG_TUNE_SITES_PER_THREAD: *value = g_sites_per_thread; return STG_OK;
        case STG_TUNE_STAGE_NEIGHBOURS: *value = g_stage_neighbours; return STG_OK;
        case STG_TUNE_THREADS_PER_SITE: *value = g_threads_per_site; return STG_OK;
        case STG_TUNE_STAPLE_THREADS: *value = g_staple_threads; return STG_OK;
        case STG_TUNE_PENCIL_TILE: *value = g_pencil_tile; return STG_OK;
        case STG_TUNE_FIELDS_PER_LAUNCH: *value = g_fields_per_launch; return STG_OK;
        case STG_TUNE_LAYER_GROUP: *value = g_layer_group; return STG_OK;
        case STG_TUNE_SPREAD_EPILOGUE: *value = g_spread_epilogue; return STG_OK;
        case STG_TUNE_FIELD_SPLIT: *value = g_field_split; return STG_OK;
        case STG_TUNE_CG_FORM: *value = g_cg_form; return STG_OK;
        default: return invalid("unknown tuning key");
    }
}

int stg_links_bytes(const stg_lattice *lat, stg_link_fmt fmt, size_t *bytes) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    if (!bytes) return invalid("bytes is NULL");
    size_t b = link_bytes(g, fmt);
    if (!b) return invalid("unknown link format");
    *bytes = b;
    return STG_OK;
}

int stg_pack_links(const stg_lattice *lat, const void *links_c128_18, stg_link_fmt dst_fmt,
                   void *dst, stg_stream_t stream) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    size_t nb = link_bytes(g, dst_fmt);
    if (!nb) return invalid("unknown link format");
    if (!aligned16(links_c128_18) || !aligned16(dst)) return invalid("NULL or misaligned links");
    if (overlap(links_c128_18, link_bytes(g, STG_LINK_C128_18), dst, nb))
        return invalid("source and destination overlap");
    launch_pack_links(g, links_c128_18, dst_fmt, dst, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

int stg_pack_phases(const stg_lattice *lat, const double *phases_f64, stg_field dst,
                    void *dst_ptr, stg_stream_t stream) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    if (!phases_f64 || !dst_ptr) return invalid("NULL phases");
    const size_t n = (size_t)8 * g.Vh;
    hipStream_t s = (hipStream_t)stream;
    if (dst == STG_C128) {
        if (overlap(phases_f64, n * 8, dst_ptr, n * 8)) return invalid("overlap");
        HIP_TRY(hipMemcpyAsync(dst_ptr, phases_f64, n * 8, hipMemcpyDeviceToDevice, s));
    } else if (dst == STG_C64) {
        if (overlap(phases_f64, n * 8, dst_ptr, n * 4)) return invalid("overlap");
        launch_pack_phases_f32(n, phases_f64, (float *)dst_ptr, s);
        HIP_TRY(hipGetLastError());
    } else {
        return invalid("unknown field type");
    }
    return STG_OK;
}

int gauge_staples(const stg_lattice *lat, const stg_gauge *gauge, double c0, double c1,
                  void *out, stg_stream_t stream) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    if (!gauge) return invalid("gauge is NULL");
    const size_t lb = link_bytes(g, gauge->fmt);
    if (!lb) return invalid("unknown link format");
    if (!aligned16(gauge->links) || !aligned16(out)) return invalid("NULL or misaligned pointer");
    if (!std::isfinite(c0) || !std::isfinite(c1)) return invalid("c0 and c1 must be finite");
    const bool fp64 = gauge->fmt == STG_LINK_C128_18 || gauge->fmt == STG_LINK_C128_12;
    const size_t ob = (size_t)8 * 9 * g.Vh * (fp64 ? 16 : 8);
    if (overlap(gauge->links, lb, out, ob)) return invalid("links and out overlap");
    StapleArgs a;
    std::memset(&a, 0, sizeof(a));
    a.geom = g;
    a.tile = pencil_tile(g, g_pencil_tile);
    a.links = gauge->links;
    a.out = out;
    a.c0 = c0;
    a.c1 = c1;
    a.xcd_remap = g_xcd_remap;
    const int threads = g_staple_threads ? g_staple_threads : staple_default_threads(gauge->fmt);
    if (launch_staples(a, gauge->fmt, threads, (hipStream_t)stream))
        return invalid("unknown link format");
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

int fermion_force(const stg_lattice *lat, const stg_gauge *gauge, int nshift,
                  const double *coeffs, const void *x_even, void *y_odd, void *out,
                  stg_stream_t stream) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    int rc = check_gauge(g, gauge, STG_C128);
    if (rc) return rc;
    if (nshift < 1 || !coeffs) return invalid("nshift >= 1 and coeffs non-NULL");
    for (int k = 0; k < nshift; ++k)
        if (!std::isfinite(coeffs[k])) return invalid("coefficients must be finite");
    if (!aligned16(x_even) || !aligned16(y_odd) || !aligned16(out))
        return invalid("x, y or out NULL or not 16-byte aligned");
    const size_t fb = (size_t)3 * g.Vh * 16;
    const size_t nb = (size_t)nshift * fb, ob = (size_t)8 * 9 * g.Vh * 16;
    const size_t lb = link_bytes(g, gauge->fmt);
    if (overlap(x_even, nb, y_odd, nb) || overlap(x_even, nb, out, ob) || overlap(y_odd, nb, out, ob) ||
        overlap(gauge->links, lb, y_odd, nb) || overlap(gauge->links, lb, out, ob))
        return invalid("x, y, out and the links must not overlap");
    hipStream_t s = (hipStream_t)stream;
    rc = hop_plain(g, gauge, STG_C128, nshift, x_even, y_odd, 1, s);
    if (rc) return rc;
    ForceArgs a;
    std::memset(&a, 0, sizeof(a));
    a.geom = g;
    a.tile = pencil_tile(g, g_pencil_tile);
    a.phases = reinterpret_cast<const double *>(gauge->phases);
    a.out = out;
    a.xcd_remap = g_xcd_remap;
    for (int k0 = 0; k0 < nshift; k0 += kForceChunk) {
        a.npoles = std::min(kForceChunk, nshift - k0);
        for (int k = 0; k < a.npoles; ++k) a.coeff[k] = coeffs[k0 + k];
        a.x = reinterpret_cast<const char *>(x_even) + (size_t)k0 * fb;
        a.y = reinterpret_cast<const char *>(y_odd) + (size_t)k0 * fb;
        a.accumulate = k0 > 0;
        launch_force(a, s);
    }
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

int stout_smear(const stg_lattice *lat, const stg_gauge *gauge, double rho, void *out,
                stg_stream_t stream) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    int rc = check_gauge(g, gauge, STG_C128);
    if (rc) return rc;
    if (!std::isfinite(rho)) return invalid("rho must be finite");
    if (!aligned16(out)) return invalid("out NULL or not 16-byte aligned");
    if (overlap(gauge->links, link_bytes(g, gauge->fmt), out, (size_t)8 * 9 * g.Vh * 16))
        return invalid("links and out overlap");
    StoutArgs a;
    std::memset(&a, 0, sizeof(a));
    a.geom = g;
    a.tile = pencil_tile(g, g_pencil_tile);
    a.links = gauge->links;
    a.out = out;
    a.rho = rho;
    a.xcd_remap = g_xcd_remap;
    if (launch_stout(a, gauge->fmt, (hipStream_t)stream)) return invalid("not an FP64 link format");
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

int gauge_momentum_update(const stg_lattice *lat, const stg_gauge *gauge, double beta, double c0,
                          double c1, double eps, void *mom, stg_stream_t stream) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    if (!gauge) return invalid("gauge is NULL");
    const bool fp32 = gauge->fmt == STG_LINK_C64_12;
    int rc = check_gauge(g, gauge, fp32 ? STG_C64 : STG_C128);
    if (rc) return rc;
    if (gauge->fmt == STG_LINK_BF16_12) return invalid("the momentum update takes no BF16 links");
    if (!std::isfinite(beta) || !std::isfinite(c0) || !std::isfinite(c1) || !std::isfinite(eps))
        return invalid("beta, c0, c1 and eps must be finite");
    if (!aligned16(mom)) return invalid("mom NULL or not 16-byte aligned");
    if (overlap(gauge->links, link_bytes(g, gauge->fmt), mom,
                (size_t)8 * 9 * g.Vh * (fp32 ? 8 : 16)))
        return invalid("links and mom overlap");
    StapleArgs a;
    std::memset(&a, 0, sizeof(a));
    a.geom = g;
    a.tile = pencil_tile(g, g_pencil_tile);
    a.links = gauge->links;
    a.out = mom;
    a.c0 = c0;
    a.c1 = c1;
    a.kmom = eps * beta / 3.0;
    a.xcd_remap = g_xcd_remap;
    const int threads = g_staple_threads ? g_staple_threads : staple_default_threads(gauge->fmt);
    if (launch_momentum(a, gauge->fmt, threads, (hipStream_t)stream))
        return invalid("unsupported link format for the momentum update");
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

int gauge_link_update(const stg_lattice *lat, stg_link_fmt fmt, void *links, double eps,
                      const void *mom, stg_stream_t stream) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    if (fmt != STG_LINK_C128_18 && fmt != STG_LINK_C128_12 && fmt != STG_LINK_C64_12)
        return invalid("the link update takes FP64 links or FP32-12 links");
    if (!std::isfinite(eps)) return invalid("eps must be finite");
    if (!aligned16(links) || !aligned16(mom)) return invalid("links or mom NULL or misaligned");
    if (overlap(links, link_bytes(g, fmt), mom,
                (size_t)8 * 9 * g.Vh * (fmt == STG_LINK_C64_12 ? 8 : 16)))
        return invalid("links and mom overlap");
    LinkUpdateArgs a;
    a.links = links;
    a.mom = mom;
    a.eps = eps;
    a.Vh = g.Vh;
    if (launch_link_update(a, fmt, (hipStream_t)stream)) return invalid("unknown link format");
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

int stout_force_backprop(const stg_lattice *lat, const stg_gauge *gauge, double rho,
                         const void *sigma_smeared, void *sigma_thin, void *ws,
                         stg_stream_t stream) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    int rc = check_gauge(g, gauge, STG_C128);
    if (rc) return rc;
    if (!std::isfinite(rho)) return invalid("rho must be finite");
    if (!aligned16(sigma_smeared) || !aligned16(sigma_thin) || !aligned16(ws))
        return invalid("sigma_smeared, sigma_thin or ws NULL or not 16-byte aligned");
    const size_t mb = (size_t)8 * 9 * g.Vh * 16, lb = link_bytes(g, gauge->fmt);
    const void *bufs[4] = {gauge->links, sigma_smeared, sigma_thin, ws};
    const size_t sizes[4] = {lb, mb, mb, mb};
    for (int i = 0; i < 4; ++i)
        for (int k = i + 1; k < 4; ++k)
            if (overlap(bufs[i], sizes[i], bufs[k], sizes[k]))
                return invalid("links, sigma_smeared, sigma_thin and ws must not overlap");
    StoutBackArgs a;
    std::memset(&a, 0, sizeof(a));
    a.geom = g;
    a.tile = pencil_tile(g, g_pencil_tile);
    a.links = gauge->links;
    a.sigp = sigma_smeared;
    a.out = sigma_thin;
    a.ws = ws;
    a.rho = rho;
    a.xcd_remap = g_xcd_remap;
    if (launch_stout_backprop(a, gauge->fmt, (hipStream_t)stream))
        return invalid("not an FP64 link format");
    HIP_TRY(hipGetLastError());
    return STG_OK;
}

int dirac_apply_eo(const stg_lattice *lat, const stg_gauge *gauge, stg_field field, int nrhs,
                   const void *in_odd, void *out_even, stg_stream_t stream) {
    return apply_dirac(lat, gauge, field, nrhs, in_odd, out_even, 0, stream);
}

int dirac_apply_oe(const stg_lattice *lat, const stg_gauge *gauge, stg_field field, int nrhs,
                   const void *in_even, void *out_odd, stg_stream_t stream) {
    return apply_dirac(lat, gauge, field, nrhs, in_even, out_odd, 1, stream);
}

int stg_apply_normal(const stg_lattice *lat, const stg_gauge *gauge, stg_field field, int nrhs,
                     double mass, double sigma, const void *in_even, void *out_even,
                     void *tmp_odd, stg_stream_t stream) {
    Geom g;
    int rc = check_normal(lat, gauge, field, nrhs, in_even, out_even, g);
    if (rc) return rc;
    if (!aligned16(tmp_odd)) return invalid("field NULL or not 16-byte aligned");
    const size_t fb = (size_t)nrhs * 3 * g.Vh * field_elem(field);
    if (overlap(in_even, fb, tmp_odd, fb) || overlap(out_even, fb, tmp_odd, fb))
        return invalid("fields overlap");
    return apply_normal(g, gauge, field, nrhs, mass, sigma, in_even, out_even, tmp_odd,
                        (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// allocation-free normal operator
// ---------------------------------------------------------------------------
namespace {

// The odd-site intermediate D_oe in of stg_apply_normal_noalloc lives in this
// array: every GPU the library runs on holds its own copy, from the loading of the
// library's code object on that device until the process ends.  On the host the
// name is only a stand-in for the device symbol; host code passes the address that
// hipGetSymbolAddress returned for the current device, never the name itself.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
__device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of scratch, per device ordinal

// Device address of scratch on the current device, looked up once per device.
int noalloc_scratch(void **ptr) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return internal("device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return internal("hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return STG_OK;
}

}  // namespace

size_t stg_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

int stg_apply_normal_noalloc(const stg_lattice *lat, const stg_gauge *gauge, stg_field field,
                             int nrhs, double mass, double sigma, const void *in_even,
                             void *out_even, stg_stream_t stream) {
    Geom g;
    int rc = check_normal(lat, gauge, field, nrhs, in_even, out_even, g);
    if (rc) return rc;
    const size_t fb = (size_t)nrhs * 3 * g.Vh * field_elem(field);
    if (fb > kNoAllocScratchBytes) {
        g_last_error = "stg_apply_normal_noalloc: the odd-site intermediate needs " +
                       std::to_string(fb) + " bytes, above the library's fixed scratch of " +
                       std::to_string(kNoAllocScratchBytes) + " bytes";
        return STG_WORKSPACE_TOO_SMALL;
    }
    void *tmp = nullptr;
    rc = noalloc_scratch(&tmp);
    if (rc) return rc;
    return apply_normal(g, gauge, field, nrhs, mass, sigma, in_even, out_even, tmp,
                        (hipStream_t)stream);
}

size_t stg_dot_workspace_bytes(void) {
    return align_up(sizeof(Ctl)) + align_up(sizeof(double) * 4 * 1024) + align_up(16);
}

int stg_dot(stg_field field, int nvec, size_t n, const void *x, const void *y, double *result,
            void *ws, size_t ws_bytes, stg_stream_t stream) {
    if (field != STG_C128 && field != STG_C64) return invalid("unknown field type");
    if (nvec < 1 || n < 1) return invalid("nvec and n must be >= 1");
    if (!aligned16(x) || !aligned16(y) || !result) return invalid("NULL or misaligned argument");
    if (!aligned16(ws)) return invalid("workspace NULL or misaligned");
    if (ws_bytes < stg_dot_workspace_bytes()) return STG_WORKSPACE_TOO_SMALL;
    Carver c{reinterpret_cast<char *>(ws)};
    Ctl *ctl = (Ctl *)c.take(sizeof(Ctl));
    double *partials = (double *)c.take(sizeof(double) * 4 * 1024);
    double *out = (double *)c.take(16);
    hipStream_t s = (hipStream_t)stream;
    launch_zero(ctl, sizeof(Ctl), s);  // a fill kernel, not a memset node
    for (int j = 0; j < nvec; ++j) {
        const size_t off = (size_t)j * n * field_elem(field);
        launch_dot(field == STG_C128, 1, n, (const char *)x + off, (const char *)y + off,
                   partials, ctl, OP_STORE, nullptr, out, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(result + 2 * j, out, 16, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    return STG_OK;
}

void stg_cg_default_params(stg_cg_params *p) {
    if (!p) return;
    p->tol = 1e-10;
    p->max_iter = 100000;
    p->mode = STG_CG_F64;
    p->delta = 0.1;
    p->poll_every = 0;
    p->restart = -1;
}

int stg_workspace_bytes(const stg_lattice *lat, int nrhs, int nshift, int mode, size_t *bytes) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    if (!bytes) return invalid("bytes is NULL");
    if (nrhs < 1 || nshift < 0) return invalid("nrhs >= 1, nshift >= 0");
    if (mode != STG_CG_F64 && mode != STG_CG_MIXED) return invalid("unknown solver mode");
    *bytes = nshift > 0 ? ms_workspace(g, nrhs, nshift, mode) : carve_cg(g, nrhs, mode, nullptr).bytes;
    return STG_OK;
}

int cg_solve(const stg_lattice *lat, const stg_gauge *hi, const stg_gauge *lo, double mass,
             int nrhs, const void *b_even, void *x_even, const stg_cg_params *params, void *ws,
             size_t ws_bytes, stg_cg_stats *stats, stg_stream_t stream) {
    Geom g;
    const int mode = params ? params->mode : -1;
    int rc = check_solver_common(lat, g, hi, lo, mode, nrhs, b_even, x_even, params);
    if (rc) return rc;
    if (!aligned16(ws)) return invalid("workspace NULL or misaligned");
    const size_t need = carve_cg(g, nrhs, mode, nullptr).bytes;
    if (ws_bytes < need) return STG_WORKSPACE_TOO_SMALL;
    const size_t fb = (size_t)nrhs * 3 * g.Vh * 16;
    if (overlap(b_even, fb, x_even, fb) || overlap(ws, ws_bytes, b_even, fb) ||
        overlap(ws, ws_bytes, x_even, fb))
        return invalid("b, x and workspace must not overlap");
    CgProblem P;
    P.g = g;
    P.hi = hi;
    P.lo = lo;
    P.mode = mode;
    P.nsys = nrhs;
    P.b = b_even;
    P.x = x_even;
    P.diag.assign(nrhs, mass * mass);
    P.cap = field_cap(g, mode == STG_CG_F64 ? hi->fmt : lo->fmt);
    P.cgcg = cg_single_reduction(P.nsys);
    P.prm = *params;
    CgWork w = carve_cg(g, nrhs, mode, ws);
    return run_cg(P, w, stats, (hipStream_t)stream);
}

int multishift_cg_solve(const stg_lattice *lat, const stg_gauge *hi, const stg_gauge *lo,
                        double mass, int nshift, const double *shifts, int nrhs,
                        const void *b_even, void *x_even, const stg_cg_params *params, void *ws,
                        size_t ws_bytes, stg_cg_stats *stats, stg_stream_t stream) {
    Geom g;
    const int mode = params ? params->mode : -1;
    int rc = check_solver_common(lat, g, hi, lo, mode, nrhs, b_even, x_even, params);
    if (rc) return rc;
    if (nshift < 1 || !shifts || !stats) return invalid("nshift >= 1, shifts and stats non-NULL");
    for (int k = 0; k < nshift; ++k)
        if (!(shifts[k] >= 0.0 && shifts[k] < 1e300)) return invalid("shifts must be >= 0");
    if (!aligned16(ws)) return invalid("workspace NULL or misaligned");
    const size_t need = ms_workspace(g, nrhs, nshift, mode);
    if (ws_bytes < need) return STG_WORKSPACE_TOO_SMALL;
    const size_t fbb = (size_t)nrhs * 3 * g.Vh * 16;
    const size_t fbx = fbb * nshift;
    if (overlap(b_even, fbb, x_even, fbx) || overlap(ws, ws_bytes, b_even, fbb) ||
        overlap(ws, ws_bytes, x_even, fbx))
        return invalid("b, x and workspace must not overlap");
    return run_mscg(g, hi, lo, mass, nshift, shifts, nrhs, b_even, x_even, *params, ws, stats,
                    (hipStream_t)stream);
}

// Rational function: the shifted solutions x_k (complex128 [nshift][nrhs][3][Vh])
// and the coefficients sit in front of the multi-shift workspace.
size_t rational_prefix(const Geom &g, int nrhs, int nshift) {
    return align_up((size_t)nshift * nrhs * 3 * g.Vh * 16) + align_up(sizeof(double) * nshift);
}

int stg_rational_workspace_bytes(const stg_lattice *lat, int nrhs, int nshift, int mode,
                                 size_t *bytes) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    if (!bytes) return invalid("bytes is NULL");
    if (nrhs < 1 || nshift < 1) return invalid("nrhs and nshift must be >= 1");
    if (mode != STG_CG_F64 && mode != STG_CG_MIXED) return invalid("unknown solver mode");
    *bytes = rational_prefix(g, nrhs, nshift) + ms_workspace(g, nrhs, nshift, mode);
    return STG_OK;
}

int rational_apply(const stg_lattice *lat, const stg_gauge *hi, const stg_gauge *lo, double mass,
                   int nshift, const double *shifts, const double *coeffs, double a0, int nrhs,
                   const void *b_even, void *y_even, const stg_cg_params *params, void *ws,
                   size_t ws_bytes, stg_cg_stats *stats, stg_stream_t stream) {
    Geom g;
    const int mode = params ? params->mode : -1;
    int rc = check_solver_common(lat, g, hi, lo, mode, nrhs, b_even, y_even, params);
    if (rc) return rc;
    if (nshift < 1 || !shifts || !coeffs || !stats)
        return invalid("nshift >= 1, shifts, coeffs and stats non-NULL");
    for (int k = 0; k < nshift; ++k) {
        if (!(shifts[k] >= 0.0 && shifts[k] < 1e300)) return invalid("shifts must be >= 0");
        if (!std::isfinite(coeffs[k])) return invalid("coefficients must be finite");
    }
    if (!std::isfinite(a0)) return invalid("a0 must be finite");
    if (!aligned16(ws)) return invalid("workspace NULL or misaligned");
    const size_t pre = rational_prefix(g, nrhs, nshift);
    const size_t need = pre + ms_workspace(g, nrhs, nshift, mode);
    if (ws_bytes < need) return STG_WORKSPACE_TOO_SMALL;
    const size_t fbb = (size_t)nrhs * 3 * g.Vh * 16;
    if (overlap(b_even, fbb, y_even, fbb) || overlap(ws, ws_bytes, b_even, fbb) ||
        overlap(ws, ws_bytes, y_even, fbb))
        return invalid("b, y and workspace must not overlap");
    hipStream_t s = (hipStream_t)stream;
    Carver c{reinterpret_cast<char *>(ws)};
    void *xs = c.take((size_t)nshift * nrhs * 3 * g.Vh * 16);
    double *dcoef = (double *)c.take(sizeof(double) * nshift);
    HIP_TRY(hipMemcpyAsync(dcoef, coeffs, sizeof(double) * nshift, hipMemcpyHostToDevice, s));
    rc = run_mscg(g, hi, lo, mass, nshift, shifts, nrhs, b_even, xs, *params,
                  (char *)ws + pre, stats, s);
    if (rc < 0) return rc;  // argument or HIP error: no result
    launch_rational_sum(fbb / 16, nshift, a0, dcoef, b_even, xs, y_even, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return rc;
}

int stg_batch_workspace_bytes(int nsolve, const stg_solve_desc *descs, int mode, size_t *bytes) {
    if (!bytes) return invalid("bytes is NULL");
    stg_cg_params prm;
    stg_cg_default_params(&prm);
    prm.mode = mode;
    int rc = check_batch(nsolve, descs, &prm);
    if (rc) return rc;
    BatchPlan B;
    rc = plan_batch(nsolve, descs, mode, nullptr, B);
    if (rc) return rc;
    *bytes = B.bytes;
    return STG_OK;
}

int cg_solve_batch(int nsolve, const stg_solve_desc *descs, const stg_cg_params *params, void *ws,
                   size_t ws_bytes, stg_cg_stats *stats, stg_stream_t stream) {
    int rc = check_batch(nsolve, descs, params);
    if (rc) return rc;
    if (!stats) return invalid("stats is NULL");
    if (!aligned16(ws)) return invalid("workspace NULL or misaligned");
    BatchPlan B;
    rc = plan_batch(nsolve, descs, params->mode, nullptr, B);
    if (rc) return rc;
    if (ws_bytes < B.bytes) return STG_WORKSPACE_TOO_SMALL;
    for (int i = 0; i < nsolve; ++i) {
        const Geom &g = B.solves[i].g;
        const size_t fb = (size_t)descs[i].nrhs * 3 * g.Vh * 16;
        if (overlap(ws, ws_bytes, descs[i].b, fb) || overlap(ws, ws_bytes, descs[i].x, fb))
            return invalid("batch: workspace overlaps b or x");
    }
    return run_cg_batch(nsolve, descs, *params, ws, stats, (hipStream_t)stream);
}

int stg_autotune(const stg_lattice *lat, const stg_gauge *gauge, stg_field field, int nrhs,
                 const void *in, void *out, const char *cache_path, stg_stream_t stream) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    if (field != STG_C128 && field != STG_C64) return invalid("unknown field type");
    int rc = check_gauge(g, gauge, field);
    if (rc) return rc;
    if (nrhs < 1) return invalid("nrhs < 1");
    if (!aligned16(in) || !aligned16(out)) return invalid("field NULL or not 16-byte aligned");
    const size_t fb = (size_t)nrhs * 3 * g.Vh * field_elem(field);
    if (overlap(in, fb, out, fb)) return invalid("input and output overlap");
    hipStream_t s = (hipStream_t)stream;
    const int nr = chunk_of(nrhs);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HopArgs a = base_hop(g, gauge);
    a.out_parity = 0;
    a.op = OP_NONE;
    a.in = in;
    a.out = out;
    // repetitions: about 20 ms of work per candidate, at least 5
    const double est_us = 1e-3 * (double)g.Vh * nr;  // ~1 ns per site and field
    const int reps = (int)std::max(5.0, std::min(200.0, 20000.0 / std::max(est_us, 1.0)));
    // the candidates, timed in two interleaved passes (each keeps its faster pass, so a
    // clock or power transient during one pass does not decide the choice)
    std::vector<TuneChoice> cand;
    const int spts[4] = {1, 2, 4, 8};
    const int nstage = stage_applies(nr, g.nh0) ? 2 : 1;
    const size_t elem = gauge->fmt == STG_LINK_C128_18 || gauge->fmt == STG_LINK_C128_12 ? 16 : 8;
    for (int xcd = 0; xcd < 2; ++xcd) {
        // one thread per site: chunks per block x LDS staging (where it applies)
        for (int stage = 0; stage < nstage; ++stage)
            for (int si = 0; si < 4; ++si) cand.push_back(TuneChoice{xcd, spts[si], stage, 1, 1e300});
        // several threads per site (one chunk, no staging)
        for (int tps = 2; tps <= 4; tps *= 2)
            if (split_lds_bytes(elem, nr, tps) <= kSplitLdsMax)
                cand.push_back(TuneChoice{xcd, 1, 0, tps, 1e300});
    }
    int rc2 = STG_OK;
    for (int pass = 0; pass < 2 && rc2 == STG_OK; ++pass)
        for (size_t k = 0; k < cand.size() && rc2 == STG_OK; ++k) {
            TuneChoice &c = cand[k];
            a.xcd_remap = c.xcd_remap;
            a.sites_per_thread = (uint32_t)c.sites_per_thread;
            a.stage_neighbours = (uint32_t)c.stage_neighbours;
            a.threads_per_site = (uint32_t)c.threads_per_site;
            for (int w = 0; w < 2; ++w) launch_hop(a, gauge->fmt, nr, EPI_PLAIN, s);
            hipError_t e = hipEventRecord(e0, s);
            for (int r = 0; r < reps && e == hipSuccess; ++r) launch_hop(a, gauge->fmt, nr, EPI_PLAIN, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc2 = hip_fail(e, "autotune timing");
                break;
            }
            c.us = std::min(c.us, 1e3 * ms / reps);
        }
    TuneChoice best{1, 1, 0, 1, 1e300};
    for (const TuneChoice &c : cand)
        if (c.us < best.us) best = c;
    if (rc2 == STG_OK) tune_store(g, gauge->fmt, nr, best);

    // fields per launch: with several fields, time D_eo of all nrhs of them chunked
    // at most 8, 4, 2 or 1 per launch (each chunk in its tuned or default shape) and
    // keep the chunking with the least time per field
    int best_cap = 0;
    double best_us = 1e300;
    if (rc2 == STG_OK && nrhs >= 2) {
        const size_t f1 = (size_t)3 * g.Vh * field_elem(field);
        HopArgs b = base_hop(g, gauge);
        b.out_parity = 0;
        b.op = OP_NONE;
        auto apply_all = [&](int cap) {
            for (int j0 = 0; j0 < nrhs;) {
                const int c = chunk_of(nrhs - j0, cap);
                b.in = (const char *)in + j0 * f1;
                b.out = (char *)out + j0 * f1;
                if (hop(b, gauge->fmt, c, EPI_PLAIN, s)) return false;
                j0 += c;
            }
            return true;
        };
        const int caps[4] = {8, 4, 2, 1};
        const int reps_all = std::max(3, reps * nr / nrhs);
        for (int pass = 0; pass < 2 && rc2 == STG_OK; ++pass)
            for (int ci = 0; ci < 4 && rc2 == STG_OK; ++ci) {
                const int cap = caps[ci];
                // a cap at or above the largest chunk of nrhs changes nothing
                if (cap != 8 && cap >= nr) continue;
                for (int w = 0; w < 2; ++w) apply_all(cap);
                hipError_t e = hipEventRecord(e0, s);
                for (int r = 0; r < reps_all && e == hipSuccess; ++r)
                    if (!apply_all(cap)) e = hipErrorInvalidValue;
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    rc2 = hip_fail(e, "autotune timing (fields per launch)");
                    break;
                }
                const double us = 1e3 * ms / reps_all / nrhs;
                if (us < best_us) {
                    best_us = us;
                    best_cap = cap;
                }
            }
        if (rc2 == STG_OK) fields_store(g, gauge->fmt, best_cap);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc2 != STG_OK) return rc2;
    HIP_TRY(hipGetLastError());
    if (cache_path && tune_append_file(cache_path, g, gauge->fmt, nr, best))
        return invalid("cannot append to the autotune cache file");
    if (cache_path && best_cap &&
        fields_append_file(cache_path, g, gauge->fmt, best_cap, best_us))
        return invalid("cannot append to the autotune cache file");
    return STG_OK;
}

int stg_autotune_load(const char *cache_path, int *loaded) {
    if (!cache_path) return invalid("cache_path is NULL");
    if (tune_load_file(cache_path, loaded)) return invalid("cannot read the autotune cache file");
    return STG_OK;
}

int stg_autotune_lookup(const stg_lattice *lat, stg_link_fmt fmt, int nr,
                        stg_tune_choice *choice) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    TuneChoice c;
    if (!tune_lookup(g, fmt, nr, c)) return STG_NOT_CONVERGED;
    if (choice) {
        choice->xcd_remap = c.xcd_remap;
        choice->sites_per_thread = c.sites_per_thread;
        choice->stage_neighbours = c.stage_neighbours;
        choice->threads_per_site = c.threads_per_site;
        choice->us = c.us;
    }
    return STG_OK;
}

int stg_autotune_fields_lookup(const stg_lattice *lat, stg_link_fmt fmt, int *fields_per_launch) {
    Geom g;
    if (!make_geom(lat, g)) return invalid("lattice extents must be even, >= 2, Vh < 2^30");
    if (!fields_per_launch) return invalid("fields_per_launch is NULL");
    int cap;
    if (!fields_lookup(g, fmt, cap)) return STG_NOT_CONVERGED;
    *fields_per_launch = cap;
    return STG_OK;
}

void stg_autotune_clear(void) { tune_clear(); }

}  // extern "C"
