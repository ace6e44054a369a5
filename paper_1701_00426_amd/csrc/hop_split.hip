// hop_split.hip -- the staggered hop with the four directions of a site shared by
// 2 or 4 threads.
//
// Paper: arXiv:1701.00426, Sec. 2.2 Eq. diracblock and the deo listing of Sec. 4.3
// (the same operator and epilogues as hop.hip).
//
// A block of kBlock threads covers kBlock / TPS consecutive output sites (in
// half-index or in layer order, kernels.hpp).  Thread group q (threads
// q * SPB .. (q + 1) * SPB - 1, whole waves) takes directions
// q * 4/TPS .. (q + 1) * 4/TPS - 1 of every site of the block, so each wave's link
// and field loads stay single coalesced runs.  The partial sums of the groups meet
// in LDS: either group 0 adds them in the order q = 1, 2, 3 and runs the epilogue
// of every field, or (fields a multiple of TPS, the spread epilogue) each group
// adds and finishes its own share of the fields, so the epilogue's loads and
// stores are spread over all the block's waves.  Each thread holds the loads of
// one or two directions instead of four: fewer registers, more waves in flight per
// SIMD, and the same bytes from HBM.

#include "device_common.hpp"
#include "hop_core.hpp"
#include "kernels.hpp"
#include "solver_state.hpp"

namespace stg {

template <typename T, int FMT, bool STDPH, int NR, int DPT, int Q>
__device__ __forceinline__ void group_dirs(const Geom &g, int P, uint32_t h, const Site &s,
                                           const void *links, const void *phases,
                                           const GlobalNb<T> &nb, vec3<T> (&acc)[NR]) {
    hop_dirs<T, FMT, STDPH, NR, Q * DPT, DPT>(g, P, h, s, links, phases, nb, acc);
}

// Owner of field j when the epilogue is spread: group j / (NR / TPS).  The other
// groups leave their partial sums of field j in LDS slot r = q' (q' below the
// owner) or q' - 1 (above it), and the owner adds the TPS partials in the order
// q' = 0, 1, ..., TPS - 1, its own from registers: the same additions, in the same
// order, as when group 0 finishes every field.
template <int NR, int TPS>
__host__ __device__ constexpr int spread_owner(int j) { return j / (NR / TPS); }

template <typename T, int FMT, bool STDPH, int NR, int EPI, int TPS, bool SPREAD>
__global__ __launch_bounds__(kBlock) void hop_split_kernel(HopArgs a) {
    if (a.gate_running && a.ctl->n_running == 0) return;
    constexpr int SPB = kBlock / TPS;  // sites per block, a multiple of the wave size
    constexpr int DPT = 4 / TPS;       // directions per thread
    static_assert(split_lds_bytes(sizeof(cpx<T>), NR, TPS) <= kSplitLdsMax,
                  "partial sums exceed the LDS budget of one block");
    static_assert(!SPREAD || NR % TPS == 0, "a spread epilogue needs NR a multiple of TPS");
    __shared__ cpx<T> part[TPS - 1][NR][3][SPB];

    const Geom &g = a.geom;
    const int P = a.out_parity;
    const uint32_t blk = a.xcd_remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int q = threadIdx.x / SPB;  // the same in a whole wave
    const int l = threadIdx.x % SPB;
    const uint32_t pos = blk * SPB + l;
    const bool live = pos < g.Vh;
    const uint32_t h = (live && a.layer_group) ? layer_site(g, a.layer_group, pos) : pos;

    vec3<T> acc[NR];
    zero_acc<T, NR>(acc);
    if (live) {
        const Site s = site_coords(g, P, h);
        const GlobalNb<T> nb{a.in, a.fstride, g.Vh};
        if (q == 0)
            group_dirs<T, FMT, STDPH, NR, DPT, 0>(g, P, h, s, a.links, a.phases, nb, acc);
        else if (q == 1)
            group_dirs<T, FMT, STDPH, NR, DPT, 1>(g, P, h, s, a.links, a.phases, nb, acc);
        else if (TPS == 4 && q == 2)
            group_dirs<T, FMT, STDPH, NR, DPT, (TPS == 4 ? 2 : 0)>(g, P, h, s, a.links,
                                                                  a.phases, nb, acc);
        else if (TPS == 4)
            group_dirs<T, FMT, STDPH, NR, DPT, (TPS == 4 ? 3 : 0)>(g, P, h, s, a.links,
                                                                  a.phases, nb, acc);
    }

    double ps[NR], pc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) ps[j] = pc[j] = 0.0;

    if constexpr (SPREAD) {
        constexpr int K = NR / TPS;  // fields per group
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const int o = spread_owner<NR, TPS>(j);
            if (o == q) continue;
            const int r = q < o ? q : q - 1;
#pragma unroll
            for (int c = 0; c < 3; ++c) part[r][j][c][l] = acc[j].c[c];
        }
        __syncthreads();
        if (live) {
            // group q owns fields q * K .. q * K + K - 1; the partials are added in
            // the order of the groups, own partial included in its place
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int j = q * K + k;
                vec3<T> sum;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    cpx<T> t = (q == 0) ? acc[j].c[c] : part[0][j][c][l];
#pragma unroll
                    for (int src = 1; src < TPS; ++src) {
                        const cpx<T> v = (src == q) ? acc[j].c[c]
                                                    : part[src < q ? src : src - 1][j][c][l];
                        t.re += v.re;
                        t.im += v.im;
                    }
                    sum.c[c] = t;
                }
                hop_epilogue_field<T, EPI>(a, h, j, sum, ps[j], pc[j]);
            }
        }
    } else {
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
            hop_epilogue<T, NR, EPI>(a, h, acc, ps, pc);
        }
    }
    if (EPI == EPI_PLAIN || a.op == OP_NONE) return;
    block_partials<NR>(ps, pc, a.partials);
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <typename T, int FMT, bool STDPH, int NR, int TPS>
static int launch_tps(const HopArgs &a, int epi, hipStream_t stream) {
    constexpr int SPB = kBlock / TPS;
    dim3 grid((a.geom.Vh + SPB - 1) / SPB);
    const bool reduce = epi != EPI_PLAIN && a.op != OP_NONE;
    if (reduce && (size_t)NR * grid.x > a.partial_pairs) return -2;
    constexpr bool kCanSpread = NR % TPS == 0;
    const bool spread = kCanSpread && a.spread_epilogue;
    switch (epi) {
        case EPI_PLAIN:
            if (spread)
                hop_split_kernel<T, FMT, STDPH, NR, EPI_PLAIN, TPS, kCanSpread>
                    <<<grid, kBlock, 0, stream>>>(a);
            else
                hop_split_kernel<T, FMT, STDPH, NR, EPI_PLAIN, TPS, false>
                    <<<grid, kBlock, 0, stream>>>(a);
            break;
        case EPI_NORMAL:
            if (spread)
                hop_split_kernel<T, FMT, STDPH, NR, EPI_NORMAL, TPS, kCanSpread>
                    <<<grid, kBlock, 0, stream>>>(a);
            else
                hop_split_kernel<T, FMT, STDPH, NR, EPI_NORMAL, TPS, false>
                    <<<grid, kBlock, 0, stream>>>(a);
            break;
        default:
            if (spread)
                hop_split_kernel<T, FMT, STDPH, NR, EPI_RESID, TPS, kCanSpread>
                    <<<grid, kBlock, 0, stream>>>(a);
            else
                hop_split_kernel<T, FMT, STDPH, NR, EPI_RESID, TPS, false>
                    <<<grid, kBlock, 0, stream>>>(a);
            break;
    }
    if (a.grid_out) *a.grid_out = grid.x;
    if (reduce && !a.defer_finish) {
        FinArgs f{a.partials, grid.x, NR, a.op, a.gate_running, a.ctl, a.state, a.out_sums};
        launch_finalize(f, stream);
    }
    return 0;
}

template <typename T, int FMT, bool STDPH, int NR>
static int launch_nr_split(const HopArgs &a, int epi, hipStream_t stream) {
    if (a.threads_per_site == 2) return launch_tps<T, FMT, STDPH, NR, 2>(a, epi, stream);
    if constexpr (split_lds_bytes(sizeof(cpx<T>), NR, 4) <= kSplitLdsMax) {
        if (a.threads_per_site == 4) return launch_tps<T, FMT, STDPH, NR, 4>(a, epi, stream);
    }
    return -1;
}

template <typename T, int FMT, bool STDPH>
static int launch_fmt_split(const HopArgs &a, int nr, int epi, hipStream_t stream) {
    switch (nr) {
        case 1: return launch_nr_split<T, FMT, STDPH, 1>(a, epi, stream);
        case 2: return launch_nr_split<T, FMT, STDPH, 2>(a, epi, stream);
        case 3: return launch_nr_split<T, FMT, STDPH, 3>(a, epi, stream);
        case 4: return launch_nr_split<T, FMT, STDPH, 4>(a, epi, stream);
        case 8: return launch_nr_split<T, FMT, STDPH, 8>(a, epi, stream);
        default: return -1;
    }
}

template <typename T, int FMT>
static int launch_ph_split(const HopArgs &a, int nr, int epi, hipStream_t stream) {
    return a.phases ? launch_fmt_split<T, FMT, false>(a, nr, epi, stream)
                    : launch_fmt_split<T, FMT, true>(a, nr, epi, stream);
}

// 0: launched; -1: this (format, fields, threads per site) is not built; -2: the
// partials buffer is too small for the reduction (nothing launched).
int launch_hop_split(const HopArgs &a, int fmt, int nr, int epi, hipStream_t stream) {
    switch (fmt) {
        case FMT_C128_18: return launch_ph_split<double, FMT_C128_18>(a, nr, epi, stream);
        case FMT_C128_12: return launch_ph_split<double, FMT_C128_12>(a, nr, epi, stream);
        case FMT_C64_12: return launch_ph_split<float, FMT_C64_12>(a, nr, epi, stream);
        case FMT_BF16_12: return launch_ph_split<float, FMT_BF16_12>(a, nr, epi, stream);
        default: return -1;
    }
}

}  // namespace stg
