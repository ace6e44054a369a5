// kernels.hpp -- argument blocks and host launchers of the library's kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device_common.hpp"
#include "solver_state.hpp"

namespace stg {

enum Epilogue { EPI_PLAIN = 0, EPI_NORMAL = 1, EPI_RESID = 2 };

struct HopArgs {
    Geom geom;
    const void *links;
    const void *phases;   // nullptr: standard phases computed in the kernel
    const void *in;       // field on the input parity, [NR][3][Vh]
    void *out;            // field on the output parity, [NR][3][Vh]
    const void *aux0;     // EPI_NORMAL: p;  EPI_RESID: x
    const void *aux1;     // EPI_RESID: b
    size_t fstride;       // complex elements between consecutive fields
    int out_parity;       // 0: D_eo (even outputs), 1: D_oe (odd outputs)
    int op;               // FinOp of the reduction (OP_NONE: no reduction)
    int gate_running;     // exit at once when ctl->n_running == 0
    int xcd_remap;        // 1: blocks of one XCD take one contiguous range of sites
    uint32_t sites_per_thread;  // each block covers this many consecutive kBlock-site chunks
    uint32_t stage_neighbours;  // 1: x0/x1 neighbour fields read from an LDS copy
    uint32_t threads_per_site;  // 0: by format and fields (default_threads_per_site),
                                // 1, or 2 / 4 threads sharing the directions of a site
    uint32_t layer_group;       // 0: sites in half-index order; G (divides N3): layer
                                // order with G planes per group (layer_site)
    uint32_t spread_epilogue;   // 2 / 4 threads per site, fields a multiple of them:
                                // each thread group finishes and stores its share of
                                // the fields (0: group 0 finishes every field)
    uint32_t layer_group_auto;  // layer order of automatic field-split launches when
                                // the caller leaves layer_group at 0 (0: none)
    int32_t fields_per_wave;    // several fields per launch on the field-split hop
                                // (hop_fsplit.hip): 1 or 2 fields per wave, 0: by
                                // format and fields (default_fields_per_wave), -1: off
    double diag;          // m^2 + sigma when state == nullptr
    SysState *state;      // per-field solver state, or nullptr
    Ctl *ctl;
    double *partials;     // [NR][grid] block partials
    size_t partial_pairs; // (sum, error) pairs that fit in partials; a launch with a
                          // reduction that needs more is refused
    double *out_sums;     // OP_STORE destination [NR]
    int defer_finish;     // 1: leave the block partials to the next kernel (no finalize)
    uint32_t *grid_out;   // host: receives the launch's block count (partials per field)

    __device__ __forceinline__ double st_diag(int j) const {
        return state ? state[j].diag : diag;
    }
    __device__ __forceinline__ bool st_pending(int j) const {
        return state ? (state[j].flags & SYS_RU_PENDING) != 0 : true;
    }
};

// Tail of every reduction kernel: per-thread compensated partials (s[j], c[j]) of
// NR sums -> one (sum, error) pair per block in `partials` ([NR][grid][2]).  The
// sums are finished by finalize_kernel, launched right after on the same stream:
// the kernel boundary makes the partials of every XCD visible without a
// device-scope fence in each block (which costs an L2 write-back per block).
template <int NR>
__device__ __forceinline__ void block_partials(double (&s)[NR], double (&c)[NR],
                                               double *partials) {
    __shared__ double sh_red[2 * kWaves];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        block_sum_pair(s[j], c[j], sh_red);
        if (threadIdx.x == 0) {
            double *pj = partials + 2 * ((size_t)j * gridDim.x + blockIdx.x);
            pj[0] = s[j];
            pj[1] = c[j];
        }
    }
}

// One block per system j < nr: adds the nblocks pairs of its sum in a fixed order
// and runs the scalar step `op` (solver_state.hpp) for it.
struct FinArgs {
    const double *partials;
    uint32_t nblocks;
    int nr;
    int op;
    int gate_running;
    Ctl *ctl;
    SysState *state;
    double *out;
    const double *partials2;  // OP_CGCG: the |r|^2 partials, [nr][nblocks2][2]
    uint32_t nblocks2;
};
int launch_finalize(const FinArgs &f, hipStream_t stream);

// LDS staging of the x0/x1 neighbours: the block's kBlock sites plus one x1 row
// (nh0 half-sites) on either side, for one or two fields per launch.
constexpr uint32_t kStageMax = 384;  // staged sites per block: kBlock + 2 * nh0, nh0 <= 64

__host__ __device__ __forceinline__ bool stage_applies(int nr, uint32_t nh0) {
    return nr <= 2 && nh0 <= (kStageMax - kBlock) / 2;
}

// Workgroups are dispatched to the 8 XCDs of the chip round-robin by block index,
// and each XCD has its own L2.  This maps the launch's block b to a logical block
// so that the blocks running on one XCD cover one contiguous range of sites: the
// neighbour field lines that nearby sites share (x1, x2 and most x3 neighbours)
// then meet in the same L2.  A bijection of [0, nb) for any nb.
constexpr uint32_t kXcds = 8;

__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
    const uint32_t x = b % kXcds, i = b / kXcds;
    const uint32_t q = nb / kXcds, r = nb % kXcds;
    return x * q + (x < r ? x : r) + i;
}

// Layer order of the output sites.  A layer is one (x2, x3) plane of nh0 * N1
// consecutive half indices.  The layers are visited in groups of G consecutive x3
// planes (G divides N3): x3 fastest within a group, then x2, then the group.  Sites
// at position pos of this order form each block, so a block's accesses stay
// contiguous runs, while a site's x3 neighbours are visited one layer (not one
// whole x3 plane) before or after it: with several fields per launch one x3 plane
// of the input fields outgrows an XCD's L2 (8 FP32 fields at 32^4: 3.1 MB), and
// in half-index order every input line came back from memory for each of the three
// x3 planes that read it.  A bijection of [0, Vh).
__device__ __forceinline__ uint32_t layer_site(const Geom &g, uint32_t G, uint32_t pos) {
    const uint32_t L = g.stride[2];               // nh0 * N1 sites per layer
    const uint32_t lp = pos / L, off = pos - lp * L;
    const uint32_t gs = G * g.N[2];               // layers per group
    const uint32_t grp = lp / gs, r = lp - grp * gs;
    const uint32_t x2 = r / G, x3 = grp * G + (r - x2 * G);
    return (x2 + g.N[2] * x3) * L + off;
}

// Blocks of kBlock threads needed to cover Vh sites.
inline uint32_t site_blocks(uint32_t Vh) { return (Vh + kBlock - 1) / kBlock; }

// Most blocks any hop launch uses: 4 threads per site leave kBlock / 4 sites per block.
inline uint32_t hop_max_blocks(uint32_t Vh) { return (Vh + kBlock / 4 - 1) / (kBlock / 4); }

int launch_hop(const HopArgs &a, int fmt, int nr, int epi, hipStream_t stream);

// The hop with 2 or 4 threads per site (hop_split.hip): LDS for the partial sums
// of the helper threads, elem_bytes per complex entry.  Returns -1 when the
// combination is not built (more LDS than kSplitLdsMax).
constexpr size_t kSplitLdsMax = 48 * 1024;
constexpr size_t split_lds_bytes(size_t elem_bytes, int nr, int tps) {
    return (size_t)(tps - 1) * nr * 3 * elem_bytes * (kBlock / tps);
}
int launch_hop_split(const HopArgs &a, int fmt, int nr, int epi, hipStream_t stream);  // -1: not built, -2: partials too small

// The hop with the fields of a launch split over the waves of a block and the
// block's links shared through LDS (hop_fsplit.hip): a.fields_per_wave fields per
// wave, 64 sites per block.  -1: not built for (format, fields, fields per wave),
// -2: partials too small.
int launch_hop_fsplit(const HopArgs &a, int fmt, int nr, int epi, hipStream_t stream);

// Fields per wave of the field-split hop when the caller leaves both it and the
// threads per site open, from 32^4 timings on MI355X with 8 fields (rotating copies):
// FP64-12 one field per wave (D_eo 206.6 us, normal operator 441.5 us, against 251.1
// and 537.9 with 2 threads per site), FP32-12 and BF16-12 two (113.8 / 227.7 against
// 121.9 / 273.8, and 101.7 / 205.8 against 104.1 / 263.9 with 4 threads per site).
// Other field counts keep the direction-split hop (0).  Such automatic launches also
// take the layer order with 4 x3 planes per group unless the caller set an order
// (HopArgs::layer_group_auto): at 32^4 it cut their reads from 1.7 to 1.2 times the
// algorithmic bytes (FP64-12 D_eo 206.6 -> 192.7 us; FP32-12 about 1 % faster).
inline int default_fields_per_wave(int fmt, int nr) {
    if (nr != 8) return 0;
    if (fmt == FMT_C128_12) return 1;
    return (fmt == FMT_C64_12 || fmt == FMT_BF16_12) ? 2 : 0;
}

// Threads per site when the caller leaves the choice open, from hop timings at 32^4
// on MI355X: one field: one thread per site (the same speed or faster inside CG,
// and the profiled FP64-12 configuration), except the plain BF16-12 hop (4: 5 %
// faster); two to four fields: 4; eight fields: 4 for the plain FP32 / BF16 hop,
// else 2 (group 0 runs the whole epilogue, which for 8 fields costs more than the
// extra waves gain, and FP64 at 4 would need 72 KB of LDS per block).  Small
// lattices (Vh below kSmallSites: a one-thread launch fills under a quarter of the
// chip's CUs) take 4 threads per site for one field too: the launch is latency-bound
// there and the shorter per-thread chains win (8^4 FP64 CG: 26.4 -> 21.9 us per
// iteration).
constexpr uint32_t kSmallSites = 16384;

inline int default_threads_per_site(int fmt, int nr, int epi, uint32_t Vh) {
    const bool fp64 = fmt == FMT_C128_18 || fmt == FMT_C128_12;
    if (nr == 1) {
        if (Vh < kSmallSites) return 4;
        return (epi == EPI_PLAIN && fmt == FMT_BF16_12) ? 4 : 1;
    }
    if (nr <= 4) return 4;
    return (epi == EPI_PLAIN && !fp64) ? 4 : 2;
}

// BLAS-1 style site kernels; fields are [NR][3][Vh] with stride fstride.
struct VecArgs {
    uint32_t Vh;
    int pad_;
    size_t fstride;
    void *x;              // solution (inner precision)
    void *p;
    void *r;
    const void *q;
    void *x64;            // FP64 solution (reliable updates)
    const void *r64;      // FP64 true residual (reliable updates)
    SysState *state;
    Ctl *ctl;
    double *partials;
    int gate_running;
    int op;
    // multi-shift: shifted solutions and directions, [nshift][nrhs][3][Vh]
    void *xs;
    void *ps;
    size_t kstride;       // complex elements between shifts (nrhs * 3 * Vh)
    int nshift;
    int pad2_;
    // single-field CG with the reductions finished in the consumers: the block
    // partials of the previous kernel, and the state buffer the next iteration reads
    const double *fin_partials;
    uint32_t fin_blocks;
    int pad3_;
    SysState *state_out;
    // single-reduction CG: w = A r (from the hop), s = A p (kept by recurrence), and
    // the |r|^2 partials of the previous update (read by the fused update)
    const void *w;
    void *s;
    const double *fin_partials2;
    uint32_t fin_blocks2;
    int skip_p;           // ru_resume: rebuild r only (the update kernel applies beta)
};

// x += alpha p; r -= alpha q; |r|^2 -> OP_BETA  (running systems)
int launch_cg_update(const VecArgs &a, int fp64, int nr, hipStream_t stream);
// p = r + beta p  (running systems)
int launch_p_update(const VecArgs &a, int fp64, int nr, hipStream_t stream);
// One field: alpha = rr / <p, q> finished from a.fin_partials in every block, then
// x += alpha p, r -= alpha q and the block partials of |r|^2 (no state written).
int launch_cg_update_fused(const VecArgs &a, int fp64, hipStream_t stream);
// One field: |r|^2 finished from a.fin_partials in every block, the beta step on a
// copy of a.state, p = r + beta p while the system runs; block 0 writes the new
// state to a.state_out (never a.state, which other blocks are reading).
int launch_p_update_fused(const VecArgs &a, int fp64, hipStream_t stream);
// Single-reduction CG (solver_state.hpp cgcg_step), after the scalar step of the
// finalize kernel: p = r + beta p; s = w + beta s; x += alpha p; r -= alpha s;
// block partials of |r|^2  (running systems)
int launch_cgcg_update(const VecArgs &a, int fp64, int nr, hipStream_t stream);
// One field, the reductions finished in every block: delta from a.fin_partials (the
// hop's), gamma from a.fin_partials2 (the previous update's), the scalar step on a
// copy of a.state, the update, |r|^2 partials into a.partials; block 0 writes the new
// state to a.state_out.
int launch_cgcg_update_fused(const VecArgs &a, int fp64, hipStream_t stream);
// x64 += x32; x32 = 0  (parked systems)
int launch_ru_accumulate(const VecArgs &a, int nr, hipStream_t stream);
// r_inner = r64 (rounded); p = r_inner + beta p  (systems just resumed)
int launch_ru_resume(const VecArgs &a, int fp64, int nr, hipStream_t stream);

// multi-shift: r -= alpha q; |r|^2 -> OP_MS_BETA
int launch_ms_r_update(const VecArgs &a, int fp64, int nr, hipStream_t stream);
// multi-shift: x_k += alpha_k p_k; p = r + beta p; p_k = zeta_k r + beta_k p_k
int launch_ms_p_update(const VecArgs &a, int fp64, int nr, hipStream_t stream);
// dst (complex128) = src (complex64), n complex entries
int launch_c64_to_c128(size_t n, const void *src, void *dst, hipStream_t stream);

// sum_i conj(x_i) y_i over n complex entries of nvec vectors; the finalize kernel
// applies op (OP_STORE into out as (re, im) pairs, or OP_INIT_BB on state).
int launch_dot(int fp64, int nvec, size_t n, const void *x, const void *y, double *partials,
               Ctl *ctl, int op, SysState *state, double *out, hipStream_t stream);
size_t dot_blocks(size_t n);

// full complex128 links -> packed format
int launch_pack_links(const Geom &g, const void *src, int fmt, void *dst, hipStream_t stream);
// double phases -> float phases (n entries)
int launch_pack_phases_f32(size_t n, const double *src, float *dst, hipStream_t stream);
// zero n bytes (multiple of 4) with a kernel
int launch_zero(void *dst, size_t bytes, hipStream_t stream);
// y[i] = a0 b[i] + sum_k coeffs[k] xs[k * n + i] over n complex128 entries;
// coeffs (device) has nshift entries.
int launch_rational_sum(size_t n, int nshift, double a0, const double *coeffs, const void *b,
                        const void *xs, void *y, hipStream_t stream);
// dst (complex64) = src (complex128), n complex entries
int launch_c128_to_c64(size_t n, const void *src, void *dst, hipStream_t stream);

}  // namespace stg
