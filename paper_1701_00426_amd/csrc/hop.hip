// hop.hip -- the even/odd staggered hop D_eo / D_oe on gfx950, with fused epilogues.
//
// Paper: arXiv:1701.00426, Sec. 2.2 Eq. diracblock (D connects only even and odd
// sites; D_oe^dag = -D_eo), Sec. 4.3 deo listing (links, in, out and a real
// per-link factor array), Sec. 2.3 (12-real links, third row rebuilt on the fly).
//
// For every output site x of parity P the kernel forms
//   (D psi)(x) = 1/2 sum_mu [ phi_mu(x) U_mu(x) psi(x+mu)
//                            - phi_mu(x-mu) U_mu(x-mu)^dag psi(x-mu) ]
// for NR fields at once, so that each link read from memory serves NR mat-vecs.
// One thread owns one output site; consecutive threads own consecutive half
// indices (in half-index or in layer order, kernels.hpp), so every link, phase and
// field access of a wave is one coalesced run (forward links at h, backward links
// at h - stride_mu, neighbours likewise).
// Links are read with non-temporal loads: they are streamed once per hop and must
// not evict the neighbour field lines that the surrounding sites re-read from L2.
//
// Epilogues (all on the output site):
//   EPI_PLAIN   out = D in
//   EPI_NORMAL  out = diag_j * p - D in           with p on the output parity;
//               block partials of Re<p, out>      (normal operator, CG's <p, A p>)
//   EPI_RESID   out = b - (diag_j * x - D in)      true residual; block partials of |out|^2
// Reductions leave one compensated (sum, error) pair per block; a finalize kernel
// (one block per system) adds them in a fixed order and runs the scalar step of
// solver_state.hpp.

#include "device_common.hpp"
#include "hop_core.hpp"
#include "kernels.hpp"
#include "solver_state.hpp"

namespace stg {

template <typename T, int FMT, bool STDPH, int NR, int EPI, bool STAGE, bool MULTI>
__global__ __launch_bounds__(kBlock) void hop_kernel(HopArgs a) {
    if (a.gate_running && a.ctl->n_running == 0) return;

    const Geom &g = a.geom;
    const uint32_t blk = a.xcd_remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int P = a.out_parity;

    double ps[NR], pc[NR];  // compensated per-thread partials of the epilogue sums
#pragma unroll
    for (int j = 0; j < NR; ++j) ps[j] = pc[j] = 0.0;

    // the block owns sites_per_thread consecutive chunks of kBlock sites; with one
    // chunk (MULTI false) the loop disappears, which saves registers
    const uint32_t nchunk = MULTI ? a.sites_per_thread : 1u;
#pragma unroll 1
    for (uint32_t k = 0; k < nchunk; ++k) {
    const uint32_t chunk0 = (blk * a.sites_per_thread + k) * kBlock;
    const uint32_t pos = chunk0 + threadIdx.x;
    // the layer order does not apply with LDS staging (a chunk's neighbours there are
    // the half-index range around it)
    const uint32_t h = (!STAGE && a.layer_group && pos < g.Vh)
                           ? layer_site(g, a.layer_group, pos) : pos;
    vec3<T> acc[NR];
    if constexpr (STAGE) {
        // the block's sites and one x1 row on either side, staged in LDS
        __shared__ cpx<T> tile[NR][3][kStageMax];
        const int64_t s0 = (int64_t)chunk0 - (int64_t)g.nh0;
        const uint32_t len = kBlock + 2 * g.nh0;
        if (k > 0) __syncthreads();  // the previous chunk's reads are done
        stage_fill<T, NR>(tile, a.in, a.fstride, g.Vh, s0, len);
        if (h < g.Vh) {
            StagedNb<T, NR> nb{tile, s0, len, GlobalNb<T>{a.in, a.fstride, g.Vh}};
            hop_site_nb<T, FMT, STDPH, NR>(g, P, h, a.links, a.phases, nb, acc);
        }
    } else if (h < g.Vh) {
        hop_site<T, FMT, STDPH, NR>(g, P, h, a.links, a.phases, a.in, a.fstride, acc);
    }
    // FP64: the epilogue's loads (p, or x and b) stay after the eight directions;
    // hoisted above them they held registers through the whole site (the FP64-12
    // normal hop then needed 256 VGPRs + 57 AGPRs, one wave per SIMD; with the barrier
    // 244, two; 87.1 -> 85.0 us at 32^4).  The FP32 hops ran 1 % slower with it.
    if constexpr (EPI != EPI_PLAIN && sizeof(T) == 8) __builtin_amdgcn_sched_barrier(0);
    if (h < g.Vh) hop_epilogue<T, NR, EPI>(a, h, acc, ps, pc);
    }

    if (EPI == EPI_PLAIN || a.op == OP_NONE) return;

    block_partials<NR>(ps, pc, a.partials);
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <typename T, int FMT, bool STDPH, int NR, bool STAGE, bool MULTI>
static void launch_epi(const HopArgs &a, int epi, dim3 grid, hipStream_t stream) {
    switch (epi) {
        case EPI_PLAIN:
            hop_kernel<T, FMT, STDPH, NR, EPI_PLAIN, STAGE, MULTI><<<grid, kBlock, 0, stream>>>(a);
            return;
        case EPI_NORMAL:
            hop_kernel<T, FMT, STDPH, NR, EPI_NORMAL, STAGE, MULTI><<<grid, kBlock, 0, stream>>>(a);
            return;
        default:
            hop_kernel<T, FMT, STDPH, NR, EPI_RESID, STAGE, MULTI><<<grid, kBlock, 0, stream>>>(a);
            return;
    }
}

template <typename T, int FMT, bool STDPH, int NR, bool STAGE>
static void launch_multi(const HopArgs &a, int epi, dim3 grid, hipStream_t stream) {
    if (a.sites_per_thread > 1)
        launch_epi<T, FMT, STDPH, NR, STAGE, true>(a, epi, grid, stream);
    else
        launch_epi<T, FMT, STDPH, NR, STAGE, false>(a, epi, grid, stream);
}

template <typename T, int FMT, bool STDPH, int NR>
static int launch_nr(const HopArgs &a, int epi, hipStream_t stream) {
    const uint32_t chunk = kBlock * a.sites_per_thread;
    dim3 grid((a.geom.Vh + chunk - 1) / chunk);
    const bool reduce = epi != EPI_PLAIN && a.op != OP_NONE;
    if (reduce && (size_t)NR * grid.x > a.partial_pairs) return -1;
    // LDS staging of the x0/x1 neighbours: one or two fields, rows of <= 64 half-sites
    if (a.stage_neighbours && stage_applies(NR, a.geom.nh0))
        launch_multi<T, FMT, STDPH, NR, (NR <= 2)>(a, epi, grid, stream);
    else
        launch_multi<T, FMT, STDPH, NR, false>(a, epi, grid, stream);
    if (a.grid_out) *a.grid_out = grid.x;
    if (reduce && !a.defer_finish) {
        FinArgs f{a.partials, grid.x, NR, a.op, a.gate_running, a.ctl, a.state, a.out_sums};
        launch_finalize(f, stream);
    }
    return 0;
}

template <typename T, int FMT, bool STDPH>
static int launch_fmt(const HopArgs &a, int nr, int epi, hipStream_t stream) {
    switch (nr) {
        case 1: return launch_nr<T, FMT, STDPH, 1>(a, epi, stream);
        case 2: return launch_nr<T, FMT, STDPH, 2>(a, epi, stream);
        case 3: return launch_nr<T, FMT, STDPH, 3>(a, epi, stream);
        case 4: return launch_nr<T, FMT, STDPH, 4>(a, epi, stream);
        case 8: return launch_nr<T, FMT, STDPH, 8>(a, epi, stream);
        default: return -1;
    }
}

template <typename T, int FMT>
static int launch_ph(const HopArgs &a, int nr, int epi, hipStream_t stream) {
    return a.phases ? launch_fmt<T, FMT, false>(a, nr, epi, stream)
                    : launch_fmt<T, FMT, true>(a, nr, epi, stream);
}

// Launches one hop over NR in {1, 2, 3, 4, 8} fields.  Returns 0, or nonzero without
// launching for an unsupported combination (checked by the caller beforehand) or
// when a reduction needs more (sum, error) pairs than a.partial_pairs.
int launch_hop(const HopArgs &a, int fmt, int nr, int epi, hipStream_t stream) {
    // fields split over the waves where asked for (or by default, when the threads
    // per site are left open too) and built
    int fpw = a.fields_per_wave;
    const bool automatic = fpw == 0;
    if (automatic) fpw = a.threads_per_site ? 0 : default_fields_per_wave(fmt, nr);
    if (fpw > 0 && nr >= 2) {
        HopArgs b = a;
        b.fields_per_wave = fpw;
        if (automatic && b.layer_group == 0) b.layer_group = a.layer_group_auto;
        const int rc = launch_hop_fsplit(b, fmt, nr, epi, stream);
        if (rc != -1) return rc;  // launched, or refused for lack of partials
    }
    // several threads per site where that variant is built, else one
    const uint32_t tps = a.threads_per_site ? a.threads_per_site
                                            : (uint32_t)default_threads_per_site(fmt, nr, epi,
                                                                                 a.geom.Vh);
    if (tps > 1) {
        HopArgs b = a;
        b.threads_per_site = tps;
        const int rc = launch_hop_split(b, fmt, nr, epi, stream);
        if (rc != -1) return rc;  // launched, or refused for lack of partials
    }
    switch (fmt) {
        case FMT_C128_18: return launch_ph<double, FMT_C128_18>(a, nr, epi, stream);
        case FMT_C128_12: return launch_ph<double, FMT_C128_12>(a, nr, epi, stream);
        case FMT_C64_12: return launch_ph<float, FMT_C64_12>(a, nr, epi, stream);
        case FMT_BF16_12: return launch_ph<float, FMT_BF16_12>(a, nr, epi, stream);
        default: return -1;
    }
}

}  // namespace stg
