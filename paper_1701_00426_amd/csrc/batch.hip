// batch.hip -- CG on many independent lattices at once (uneven batch).
//
// Paper: arXiv:1701.00426, Sec. 2.2 (CG on Eq. lineqeo), Sec. 4.3 (deo/doe); the
// paper fixes the lattice extents at compile time (Sec. 4.1 LNH_N0..), so one
// launch serves one lattice.  Here every kernel of a CG step walks a table of
// tiles that spans all lattices of the batch: a tile is kBlock consecutive sites of
// one lattice for a chunk of 1 to 4 right-hand sides.  One launch per step (per tile
// class for the hop) therefore serves every solve, small lattices ride along with
// large ones, and the launch count does not grow with the number of solves.  Each
// tile (each pass of a tile, for the hop) has a block of its own, in XCD-aware
// order, so no block carries a second tile's latency; a block whose tile holds no
// system in the state its kernel acts on (running, parked or resumed) exits.

#include <algorithm>

#include "batch.hpp"
#include "device_common.hpp"
#include "hop_core.hpp"
#include "kernels.hpp"
#include "solver_state.hpp"

namespace stg {

// A tile is worked on when one of its systems has a flag of a.tile_mask (0: always).
__device__ __forceinline__ bool tile_active(const BArgs &a, const BSolve &S, const BTile &t) {
    if (!a.tile_mask) return true;
    for (int j = 0; j < t.nr; ++j)
        if (a.state[S.sys0 + t.j0 + j].flags & a.tile_mask) return true;
    return false;
}

// Thread 0 stores the block's (sum, error) pair of system js in slot `slot` of tile
// t; the writer of slot 0 also clears the slots used .. kTileSlots - 1 that no block
// of its launch writes.
__device__ __forceinline__ void put_tile_partial(double *partials, const BSolve &S, const BTile &t,
                                                 int js, int slot, int used, double sum,
                                                 double err) {
    double *pj = partials + 2 * (((size_t)S.part0 + (size_t)js * S.nblk + t.blk) * kTileSlots);
    pj[2 * slot] = sum;
    pj[2 * slot + 1] = err;
    if (slot == 0)
        for (int k = used; k < kTileSlots; ++k) pj[2 * k] = pj[2 * k + 1] = 0.0;
}

// Tile ti of the vector kernels is block ti: these kernels reuse nothing between
// tiles, and the hardware deals consecutive blocks to the XCDs in turn, so every
// XCD gets its share of each solve's tiles however few solves still run.  The
// launches give every tile a block of its own; the loop only guards a grid smaller
// than the range.
#define FOR_EACH_TILE(a, ti) \
    for (uint32_t ti = (a).tile0 + blockIdx.x; ti < (a).ntiles; ti += gridDim.x)

// Epilogue of a tile's fields at site h (acc = twice the hop): plain, normal
// operator with Re<p, q> partials, or true residual with |r|^2 partials.
template <typename T, int NR, int EPI>
__device__ __forceinline__ void bhop_epilogue(const BArgs &a, const BSolve &S, const BTile &t,
                                              uint32_t h, const vec3<T> (&acc)[NR],
                                              double (&ps)[NR], double (&pc)[NR]) {
    const Geom &g = S.g;
    const size_t fs = (size_t)3 * g.Vh;
    const size_t e = sizeof(T) * 2;
    char *out = (char *)a.field(S, a.f_out) + t.j0 * fs * e;
    const char *aux0 = (const char *)a.field(S, a.f_aux0) + t.j0 * fs * e;
    const char *aux1 = EPI == EPI_RESID ? (const char *)S.b + t.j0 * fs * 16 : nullptr;
    const T half = T(0.5);
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const SysState &st = a.state[S.sys0 + t.j0 + j];
        vec3<T> o;
        if (EPI == EPI_PLAIN) {
#pragma unroll
            for (int c = 0; c < 3; ++c) o.c[c] = cscale(half, acc[j].c[c]);
        } else if (EPI == EPI_NORMAL) {
            const T d = (T)st.diag;
            vec3<T> p = ld_v<T>(aux0, fs, g.Vh, j, h);
            double site = 0.0;  // the site's terms in FP64, then one compensated add
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                o.c[c].re = d * p.c[c].re - half * acc[j].c[c].re;
                o.c[c].im = d * p.c[c].im - half * acc[j].c[c].im;
                site = fmat((double)p.c[c].re, (double)o.c[c].re, site);
                site = fmat((double)p.c[c].im, (double)o.c[c].im, site);
            }
            pair_add(ps[j], pc[j], site, 0.0);
        } else {  // EPI_RESID: FP64 only (aux1 = b, complex128)
            if (!(st.flags & SYS_RU_PENDING)) continue;
            const T d = (T)st.diag;
            vec3<T> x = ld_v<T>(aux0, fs, g.Vh, j, h);
            vec3<T> b = ld_v<T>(aux1, fs, g.Vh, j, h);
            double site = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                o.c[c].re = b.c[c].re - (d * x.c[c].re - half * acc[j].c[c].re);
                o.c[c].im = b.c[c].im - (d * x.c[c].im - half * acc[j].c[c].im);
                site = fmat((double)o.c[c].re, (double)o.c[c].re, site);
                site = fmat((double)o.c[c].im, (double)o.c[c].im, site);
            }
            pair_add(ps[j], pc[j], site, 0.0);
        }
        st_v<T>(out, fs, g.Vh, j, h, o);
    }
}

template <typename T, int FMT, bool STDPH, int NR, int EPI>
__device__ void bhop_tile(const BArgs &a, const BSolve &S, const BTile &t) {
    const Geom &g = S.g;
    const size_t fs = (size_t)3 * g.Vh;
    const size_t e = sizeof(T) * 2;
    const bool hi = a.use_hi;
    const void *links = hi ? S.hi_links : S.lo_links;
    const void *phases = hi ? S.hi_phases : S.lo_phases;
    const char *in = (const char *)a.field(S, a.f_in) + t.j0 * fs * e;
    const uint32_t h = t.blk * kBlock + threadIdx.x;
    double ps[NR], pc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) ps[j] = pc[j] = 0.0;
    if (h < g.Vh) {
        // one direction at a time: the loads of one direction in flight per thread
        // (76 to 105 VGPRs for the FP32 one-thread-per-site classes of 1 to 4 fields)
        vec3<T> acc[NR];
        const Site s = site_coords(g, a.out_parity, h);
        zero_acc<T, NR>(acc);
        hop_dirs<T, FMT, STDPH, NR, 0, 4, 1>(g, a.out_parity, h, s, links, phases,
                                             GlobalNb<T>{in, fs, g.Vh}, acc);
        bhop_epilogue<T, NR, EPI>(a, S, t, h, acc, ps, pc);
    }
    if (EPI != EPI_PLAIN) {
        __shared__ double sh_red[2 * kWaves];
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            block_sum_pair(ps[j], pc[j], sh_red);
            if (threadIdx.x == 0) put_tile_partial(a.partials, S, t, t.j0 + j, 0, 1, ps[j], pc[j]);
        }
    }
}

// Pass `sub` of the tile with TPS threads per site: the block covers the SPB =
// kBlock / TPS sites sub * SPB .. of the tile, thread group q (whole waves) sums
// directions q * 4/TPS .. (q + 1) * 4/TPS - 1 of every site, the groups' partial
// sums meet in LDS (lds: [TPS - 1][NR][3][SPB] entries) and group 0 adds them in the
// order q = 1, 2, 3 and runs the epilogue.
template <typename T, int FMT, bool STDPH, int NR, int EPI, int TPS, int Q>
__device__ __forceinline__ void bgroup_dirs(const Geom &g, int P, uint32_t h, const Site &s,
                                            const void *links, const void *phases,
                                            const GlobalNb<T> &nb, vec3<T> (&acc)[NR]) {
    constexpr int DPT = 4 / TPS;
    hop_dirs<T, FMT, STDPH, NR, Q * DPT, DPT, 1>(g, P, h, s, links, phases, nb, acc);
}

template <typename T, int FMT, bool STDPH, int NR, int EPI, int TPS>
__device__ void bhop_tile_split(const BArgs &a, const BSolve &S, const BTile &t, int sub,
                                void *lds) {
    constexpr int SPB = kBlock / TPS;
    auto part = reinterpret_cast<cpx<T>(*)[NR][3][SPB]>(lds);
    const Geom &g = S.g;
    const int P = a.out_parity;
    const size_t fs = (size_t)3 * g.Vh;
    const size_t e = sizeof(T) * 2;
    const bool hi = a.use_hi;
    const void *links = hi ? S.hi_links : S.lo_links;
    const void *phases = hi ? S.hi_phases : S.lo_phases;
    const char *in = (const char *)a.field(S, a.f_in) + t.j0 * fs * e;
    const GlobalNb<T> nb{in, fs, g.Vh};
    const int q = threadIdx.x / SPB;  // the same in a whole wave
    const int l = threadIdx.x % SPB;
    double ps[NR], pc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) ps[j] = pc[j] = 0.0;
    {
        const uint32_t h = t.blk * kBlock + sub * SPB + l;
        const bool live = h < g.Vh;
        vec3<T> acc[NR];
        zero_acc<T, NR>(acc);
        if (live) {
            const Site s = site_coords(g, P, h);
            if (q == 0)
                bgroup_dirs<T, FMT, STDPH, NR, EPI, TPS, 0>(g, P, h, s, links, phases, nb, acc);
            else if (q == 1)
                bgroup_dirs<T, FMT, STDPH, NR, EPI, TPS, 1>(g, P, h, s, links, phases, nb, acc);
            else if (TPS == 4 && q == 2)
                bgroup_dirs<T, FMT, STDPH, NR, EPI, TPS, (TPS == 4 ? 2 : 0)>(g, P, h, s, links,
                                                                              phases, nb, acc);
            else if (TPS == 4)
                bgroup_dirs<T, FMT, STDPH, NR, EPI, TPS, (TPS == 4 ? 3 : 0)>(g, P, h, s, links,
                                                                              phases, nb, acc);
        }
        if (q > 0) {
#pragma unroll
            for (int j = 0; j < NR; ++j)
#pragma unroll
                for (int c = 0; c < 3; ++c) part[q - 1][j][c][l] = acc[j].c[c];
        }
        __syncthreads();
        if (q == 0 && live) {
#pragma unroll
            for (int r = 0; r < TPS - 1; ++r)
#pragma unroll
                for (int j = 0; j < NR; ++j)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const cpx<T> v = part[r][j][c][l];
                        acc[j].c[c].re += v.re;
                        acc[j].c[c].im += v.im;
                    }
            bhop_epilogue<T, NR, EPI>(a, S, t, h, acc, ps, pc);
        }
    }
    if (EPI != EPI_PLAIN) {
        __shared__ double sh_red[2 * kWaves];
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            block_sum_pair(ps[j], pc[j], sh_red);
            if (threadIdx.x == 0) put_tile_partial(a.partials, S, t, t.j0 + j, sub, TPS, ps[j], pc[j]);
        }
    }
}

// One launch per tile class: every tile of the range has NR fields, TPS threads per
// site and standard (STDPH) or stored phases on the gauge field of the launch, so the
// kernel carries only that shape.  Block L
// of the XCD order takes pass L % TPS of tile tile0 + L / TPS: the grid is TPS
// blocks per tile, and a block whose tile has no system in the masked state exits.
template <typename T, int FMT, int EPI, int NR, int TPS, bool STDPH>
__global__ __launch_bounds__(kBlock) void bhop_class_kernel(BArgs a) {
    if (a.gate_running && a.ctl->n_running == 0) return;
    constexpr int NP = TPS > 1 ? TPS - 1 : 1;
    __shared__ cpx<T> part[NP][NR][3][kBlock / TPS];
    const uint32_t L = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t ti = a.tile0 + L / TPS;
    if (ti >= a.ntiles) return;
    const BTile t = a.tiles[ti];
    const BSolve &S = a.solves[t.solve];
    if (!tile_active(a, S, t)) return;
    if constexpr (TPS == 1)
        bhop_tile<T, FMT, STDPH, NR, EPI>(a, S, t);
    else
        bhop_tile_split<T, FMT, STDPH, NR, EPI, TPS>(a, S, t, (int)(L % TPS), part);
}

// ---------------------------------------------------------------------------
// vector kernels over tiles
// ---------------------------------------------------------------------------

// x += alpha p; r -= alpha q; partials of |r|^2  (running systems).  Compiled per
// field count so that the loads of all fields of a tile are issued together and
// the block reductions follow them.
template <typename T, int NR>
__device__ void bcg_update_tile(const BArgs &a, const BSolve &S, const BTile &t,
                                double *sh_red) {
    const size_t fs = (size_t)3 * S.g.Vh;
    const uint32_t h = t.blk * kBlock + threadIdx.x;
    double ps[NR], pc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        ps[j] = pc[j] = 0.0;
        const int js = t.j0 + j;
        const SysState &st = a.state[S.sys0 + js];
        if (!(st.flags & SYS_RUNNING) || h >= S.g.Vh) continue;
        const T al = (T)st.alpha;
        // the site's twelve loads first (the stores may alias them as far as the
        // compiler knows, so loads issued per colour would wait for the stores)
        vec3<T> x = ld_v<T>(S.xin, fs, S.g.Vh, js, h);
        const vec3<T> p = ld_v<T>(S.p, fs, S.g.Vh, js, h);
        vec3<T> r = ld_v<T>(S.r, fs, S.g.Vh, js, h);
        const vec3<T> q = ld_v<T>(S.q, fs, S.g.Vh, js, h);
        double site = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x.c[c].re += al * p.c[c].re;
            x.c[c].im += al * p.c[c].im;
            r.c[c].re -= al * q.c[c].re;
            r.c[c].im -= al * q.c[c].im;
            site = fmat((double)r.c[c].re, (double)r.c[c].re, site);
            site = fmat((double)r.c[c].im, (double)r.c[c].im, site);
        }
        st_v<T>(S.xin, fs, S.g.Vh, js, h, x);
        st_v<T>(S.r, fs, S.g.Vh, js, h, r);
        pair_add(ps[j], pc[j], site, 0.0);
    }
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        block_sum_pair(ps[j], pc[j], sh_red);
        if (threadIdx.x == 0) put_tile_partial(a.partials, S, t, t.j0 + j, 0, 1, ps[j], pc[j]);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void bcg_update_kernel(BArgs a) {
    if (block_gate_closed(a.ctl, a.gate_running)) return;
    __shared__ double sh_red[2 * kWaves];
    FOR_EACH_TILE(a, ti) {
        const BTile t = a.tiles[ti];
        const BSolve &S = a.solves[t.solve];
        if (!tile_active(a, S, t)) continue;
        switch (t.nr) {
            case 1: bcg_update_tile<T, 1>(a, S, t, sh_red); break;
            case 2: bcg_update_tile<T, 2>(a, S, t, sh_red); break;
            case 3: bcg_update_tile<T, 3>(a, S, t, sh_red); break;
            default: bcg_update_tile<T, 4>(a, S, t, sh_red); break;
        }
    }
}

// p = r + beta p  (running systems)
template <typename T, int NR>
__device__ __forceinline__ void bp_update_tile(const BArgs &a, const BSolve &S, const BTile &t) {
    const size_t fs = (size_t)3 * S.g.Vh;
    const uint32_t h = t.blk * kBlock + threadIdx.x;
    if (h >= S.g.Vh) return;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int js = t.j0 + j;
        const SysState &st = a.state[S.sys0 + js];
        if (!(st.flags & SYS_RUNNING)) continue;
        const T be = (T)st.beta;
        vec3<T> p = ld_v<T>(S.p, fs, S.g.Vh, js, h);  // loads first, as above
        const vec3<T> r = ld_v<T>(S.r, fs, S.g.Vh, js, h);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            p.c[c].re = r.c[c].re + be * p.c[c].re;
            p.c[c].im = r.c[c].im + be * p.c[c].im;
        }
        st_v<T>(S.p, fs, S.g.Vh, js, h, p);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void bp_update_kernel(BArgs a) {
    if (a.gate_running && a.ctl->n_running == 0) return;
    FOR_EACH_TILE(a, ti) {
        const BTile t = a.tiles[ti];
        const BSolve &S = a.solves[t.solve];
        if (!tile_active(a, S, t)) continue;
        switch (t.nr) {
            case 1: bp_update_tile<T, 1>(a, S, t); break;
            case 2: bp_update_tile<T, 2>(a, S, t); break;
            case 3: bp_update_tile<T, 3>(a, S, t); break;
            default: bp_update_tile<T, 4>(a, S, t); break;
        }
    }
}

// Single-reduction form (Chronopoulos and Gear, solver_state.hpp cgcg_step), running
// systems: p = r + beta p, s = w + beta s (s = A p by recurrence; w = A r is in q),
// x += alpha p, r -= alpha s, and the new |r|^2 partials into partials2 for the next
// step's finalize.
template <typename T, int NR>
__device__ void bcgcg_update_tile(const BArgs &a, const BSolve &S, const BTile &t,
                                  double *sh_red) {
    const size_t fs = (size_t)3 * S.g.Vh;
    const uint32_t h = t.blk * kBlock + threadIdx.x;
    double ps[NR], pc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        ps[j] = pc[j] = 0.0;
        const int js = t.j0 + j;
        const SysState &st = a.state[S.sys0 + js];
        if (!(st.flags & SYS_RUNNING) || h >= S.g.Vh) continue;
        const T al = (T)st.alpha, be = (T)st.beta;
        // the site's fifteen loads first, as in the x/r update
        vec3<T> r = ld_v<T>(S.r, fs, S.g.Vh, js, h);
        const vec3<T> w = ld_v<T>(S.q, fs, S.g.Vh, js, h);
        vec3<T> p = ld_v<T>(S.p, fs, S.g.Vh, js, h);
        vec3<T> sv = ld_v<T>(S.s, fs, S.g.Vh, js, h);
        vec3<T> x = ld_v<T>(S.xin, fs, S.g.Vh, js, h);
        double site = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            p.c[c].re = r.c[c].re + be * p.c[c].re;
            p.c[c].im = r.c[c].im + be * p.c[c].im;
            sv.c[c].re = w.c[c].re + be * sv.c[c].re;
            sv.c[c].im = w.c[c].im + be * sv.c[c].im;
            x.c[c].re += al * p.c[c].re;
            x.c[c].im += al * p.c[c].im;
            r.c[c].re -= al * sv.c[c].re;
            r.c[c].im -= al * sv.c[c].im;
            site = fmat((double)r.c[c].re, (double)r.c[c].re, site);
            site = fmat((double)r.c[c].im, (double)r.c[c].im, site);
        }
        st_v<T>(S.p, fs, S.g.Vh, js, h, p);
        st_v<T>(S.s, fs, S.g.Vh, js, h, sv);
        st_v<T>(S.xin, fs, S.g.Vh, js, h, x);
        st_v<T>(S.r, fs, S.g.Vh, js, h, r);
        pair_add(ps[j], pc[j], site, 0.0);
    }
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        block_sum_pair(ps[j], pc[j], sh_red);
        if (threadIdx.x == 0) put_tile_partial(a.partials2, S, t, t.j0 + j, 0, 1, ps[j], pc[j]);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void bcgcg_update_kernel(BArgs a) {
    if (block_gate_closed(a.ctl, a.gate_running)) return;
    __shared__ double sh_red[2 * kWaves];
    FOR_EACH_TILE(a, ti) {
        const BTile t = a.tiles[ti];
        const BSolve &S = a.solves[t.solve];
        if (!tile_active(a, S, t)) continue;
        switch (t.nr) {
            case 1: bcgcg_update_tile<T, 1>(a, S, t, sh_red); break;
            case 2: bcgcg_update_tile<T, 2>(a, S, t, sh_red); break;
            case 3: bcgcg_update_tile<T, 3>(a, S, t, sh_red); break;
            default: bcgcg_update_tile<T, 4>(a, S, t, sh_red); break;
        }
    }
}

// parked systems: x64 += x32, x32 = 0 (mixed mode)
__global__ __launch_bounds__(kBlock) void bru_accumulate_kernel(BArgs a) {
    FOR_EACH_TILE(a, ti) {
        const BTile t = a.tiles[ti];
        const BSolve &S = a.solves[t.solve];
        const size_t fs = (size_t)3 * S.g.Vh;
        const uint32_t h = t.blk * kBlock + threadIdx.x;
        if (h >= S.g.Vh || !tile_active(a, S, t)) continue;
        for (int j = 0; j < t.nr; ++j) {
            const int js = t.j0 + j;
            if (!(a.state[S.sys0 + js].flags & SYS_RU_PENDING)) continue;
            for (int c = 0; c < 3; ++c) {
                const size_t i = js * fs + (size_t)c * S.g.Vh + h;
                cpx<float> xs = ld_c<float>(S.xin, i);
                cpx<double> xd = ld_c<double>(S.x64, i);
                xd.re += (double)xs.re;
                xd.im += (double)xs.im;
                st_c<double>(S.x64, i, xd);
                st_c<float>(S.xin, i, cpx<float>{0.0f, 0.0f});
            }
        }
    }
}

// resumed systems: r_inner = r64 (rounded); p = r_inner + beta p
template <typename T>
__global__ __launch_bounds__(kBlock) void bru_resume_kernel(BArgs a) {
    FOR_EACH_TILE(a, ti) {
        const BTile t = a.tiles[ti];
        const BSolve &S = a.solves[t.solve];
        const size_t fs = (size_t)3 * S.g.Vh;
        const uint32_t h = t.blk * kBlock + threadIdx.x;
        if (h >= S.g.Vh || !tile_active(a, S, t)) continue;
        for (int j = 0; j < t.nr; ++j) {
            const int js = t.j0 + j;
            const SysState &st = a.state[S.sys0 + js];
            if (!(st.flags & SYS_RESUME)) continue;
            const T be = (T)st.beta;
            for (int c = 0; c < 3; ++c) {
                const size_t i = js * fs + (size_t)c * S.g.Vh + h;
                cpx<double> rd = ld_c<double>(S.r64, i);
                cpx<T> r{(T)rd.re, (T)rd.im};
                if (S.r != S.r64) st_c<T>(S.r, i, r);
                if (a.skip_p) continue;
                cpx<T> p = ld_c<T>(S.p, i);
                p.re = r.re + be * p.re;
                p.im = r.im + be * p.im;
                st_c<T>(S.p, i, p);
            }
        }
    }
}

// |b|^2 partials of every system (complex128 b)
__global__ __launch_bounds__(kBlock) void bnorm_b_kernel(BArgs a) {
    __shared__ double sh_red[2 * kWaves];
    FOR_EACH_TILE(a, ti) {
        const BTile t = a.tiles[ti];
        const BSolve &S = a.solves[t.solve];
        const size_t fs = (size_t)3 * S.g.Vh;
        const uint32_t h = t.blk * kBlock + threadIdx.x;
        for (int j = 0; j < t.nr; ++j) {
            const int js = t.j0 + j;
            double ps = 0.0, pc = 0.0;
            if (h < S.g.Vh)
                for (int c = 0; c < 3; ++c) {
                    cpx<double> v = ld_c<double>(S.b, js * fs + (size_t)c * S.g.Vh + h);
                    pair_add(ps, pc, v.re * v.re, 0.0);
                    pair_add(ps, pc, v.im * v.im, 0.0);
                }
            block_sum_pair(ps, pc, sh_red);
            if (threadIdx.x == 0) put_tile_partial(a.partials, S, t, js, 0, 1, ps, pc);
        }
    }
}

// One block per system: fixed-order compensated sum of its partials, then op.
__global__ __launch_bounds__(kBlock) void bfinalize_kernel(BArgs a, int op) {
    __shared__ double sh_red[2 * kWaves];
    if (block_gate_closed(a.ctl, a.gate_running)) return;
    const uint32_t sys = blockIdx.x;
    const BSysRef ref = a.sysref[sys];
    const BSolve &S = a.solves[ref.solve];
    const size_t first = ((size_t)S.part0 + (size_t)ref.j * S.nblk) * kTileSlots;
    double tot = block_sum2_pairs(a.partials + 2 * first, (int)(S.nblk * kTileSlots), sh_red);
    double tot2 = 0.0;
    if (op == OP_CGCG)
        tot2 = block_sum2_pairs(a.partials2 + 2 * first, (int)(S.nblk * kTileSlots), sh_red);
    if (threadIdx.x == 0) finalize_one(op, a.ctl, a.state, nullptr, (int)sys, tot, tot2);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int FMT, int EPI, int NR, bool STDPH>
static void bhop_launch_ph(const BArgs &a, int tps, hipStream_t s) {
    const dim3 grid(a.grid);
    if (tps == 4)
        bhop_class_kernel<T, FMT, EPI, NR, 4, STDPH><<<grid, kBlock, 0, s>>>(a);
    else if (tps == 2)
        bhop_class_kernel<T, FMT, EPI, NR, 2, STDPH><<<grid, kBlock, 0, s>>>(a);
    else
        bhop_class_kernel<T, FMT, EPI, NR, 1, STDPH><<<grid, kBlock, 0, s>>>(a);
}

template <typename T, int FMT, int EPI, int NR>
static void bhop_launch_nr(const BArgs &a, int tps, bool stdph, hipStream_t s) {
    if (stdph)
        bhop_launch_ph<T, FMT, EPI, NR, true>(a, tps, s);
    else
        bhop_launch_ph<T, FMT, EPI, NR, false>(a, tps, s);
}

template <typename T, int FMT, int EPI>
static void bhop_launch(const BArgs &a, int nr, int tps, bool stdph, hipStream_t s) {
    switch (nr) {
        case 1: bhop_launch_nr<T, FMT, EPI, 1>(a, tps, stdph, s); return;
        case 2: bhop_launch_nr<T, FMT, EPI, 2>(a, tps, stdph, s); return;
        case 3: bhop_launch_nr<T, FMT, EPI, 3>(a, tps, stdph, s); return;
        default: bhop_launch_nr<T, FMT, EPI, 4>(a, tps, stdph, s); return;
    }
}

template <typename T, int FMT>
static void bhop_launch_epi(const BArgs &a, int epi, int nr, int tps, bool stdph, hipStream_t s) {
    if (epi == EPI_PLAIN)
        bhop_launch<T, FMT, EPI_PLAIN>(a, nr, tps, stdph, s);
    else if (epi == EPI_NORMAL)
        bhop_launch<T, FMT, EPI_NORMAL>(a, nr, tps, stdph, s);
    else
        bhop_launch<T, FMT, EPI_RESID>(a, nr, tps, stdph, s);
}

// Kernel boundary stays the synchronisation point: the classes' launches follow one
// another on the stream, and the finalize kernel after them sees every tile's partials.
int launch_bhop(const BArgs &a, const BClass *cls, int ncls, int fmt, int epi, hipStream_t s) {
    if ((fmt == FMT_C64_12 || fmt == FMT_BF16_12) && epi == EPI_RESID) return -1;
    if (fmt < FMT_C128_18 || fmt > FMT_BF16_12) return -1;
    for (int c = 0; c < ncls; ++c) {
        BArgs b = a;
        b.tile0 = cls[c].begin;
        b.ntiles = cls[c].end;
        b.grid = (cls[c].end - cls[c].begin) * (uint32_t)cls[c].tps;
        if (b.grid == 0) continue;
        const int nr = cls[c].nr, tps = cls[c].tps;
        const bool ph = a.use_hi ? cls[c].std_hi : cls[c].std_lo;
        switch (fmt) {
            case FMT_C128_18: bhop_launch_epi<double, FMT_C128_18>(b, epi, nr, tps, ph, s); break;
            case FMT_C128_12: bhop_launch_epi<double, FMT_C128_12>(b, epi, nr, tps, ph, s); break;
            case FMT_C64_12: bhop_launch_epi<float, FMT_C64_12>(b, epi, nr, tps, ph, s); break;
            default: bhop_launch_epi<float, FMT_BF16_12>(b, epi, nr, tps, ph, s); break;
        }
    }
    return 0;
}

int launch_bfinalize(const BArgs &a, int op, hipStream_t s) {
    bfinalize_kernel<<<dim3(a.nsys), kBlock, 0, s>>>(a, op);
    return 0;
}

int launch_bcg_update(const BArgs &a, int fp64, hipStream_t s) {
    if (fp64)
        bcg_update_kernel<double><<<dim3(a.grid), kBlock, 0, s>>>(a);
    else
        bcg_update_kernel<float><<<dim3(a.grid), kBlock, 0, s>>>(a);
    return 0;
}

int launch_bcgcg_update(const BArgs &a, int fp64, hipStream_t s) {
    if (fp64)
        bcgcg_update_kernel<double><<<dim3(a.grid), kBlock, 0, s>>>(a);
    else
        bcgcg_update_kernel<float><<<dim3(a.grid), kBlock, 0, s>>>(a);
    return 0;
}

int launch_bp_update(const BArgs &a, int fp64, hipStream_t s) {
    if (fp64)
        bp_update_kernel<double><<<dim3(a.grid), kBlock, 0, s>>>(a);
    else
        bp_update_kernel<float><<<dim3(a.grid), kBlock, 0, s>>>(a);
    return 0;
}

int launch_bru_accumulate(const BArgs &a, hipStream_t s) {
    bru_accumulate_kernel<<<dim3(a.grid), kBlock, 0, s>>>(a);
    return 0;
}

int launch_bru_resume(const BArgs &a, int fp64, hipStream_t s) {
    if (fp64)
        bru_resume_kernel<double><<<dim3(a.grid), kBlock, 0, s>>>(a);
    else
        bru_resume_kernel<float><<<dim3(a.grid), kBlock, 0, s>>>(a);
    return 0;
}

int launch_bnorm_b(const BArgs &a, hipStream_t s) {
    bnorm_b_kernel<<<dim3(a.grid), kBlock, 0, s>>>(a);
    return 0;
}

}  // namespace stg
