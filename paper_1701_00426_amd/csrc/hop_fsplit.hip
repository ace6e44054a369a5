// hop_fsplit.hip -- the staggered hop for several fields per launch with the fields
// split over the waves of a block and the block's links shared through LDS.
//
// Paper: arXiv:1701.00426, Sec. 2.2 Eq. diracblock and the deo listing of Sec. 4.3
// (the same operator and epilogues as hop.hip); Sec. 4.3 on reusing each link read
// for several mat-vecs.
//
// A block covers kFsSites = 64 consecutive output sites (half-index or layer order)
// with G = NR / FPG waves: wave f owns fields f * FPG .. f * FPG + FPG - 1 of all 64
// sites over all four directions, so it finishes its own fields (no partial sums
// cross waves) and its neighbour and output accesses are single coalesced runs.
// The eight links of the block's sites are read from memory once: wave f fetches the
// forward and backward link of directions f, f + G, ... into LDS, and after one
// barrier every wave reads all eight from there.  Reductions of the epilogue are
// finished per wave (each field lives in one wave) into one (sum, error) pair per
// block and field, the layout of the other hop kernels.

#include "device_common.hpp"
#include "hop_core.hpp"
#include "kernels.hpp"
#include "solver_state.hpp"

namespace stg {

// A stored link as 16-byte words, in the order of its storage format, and its
// decoding (with the third row rebuilt for the 12-real formats).
template <typename T, int FMT>
struct LinkWords;

template <>
struct LinkWords<double, FMT_C128_12> {
    static constexpr int W = 6;
    __device__ __forceinline__ static void fetch(const void *L, uint32_t Vh, int s, uint32_t h,
                                                 nu4 (&w)[W]) {
        const size_t base = (size_t)s * 6 * Vh + h;
#pragma unroll
        for (int k = 0; k < 6; ++k) w[k] = nt_load<nu4>(L, base + (size_t)k * Vh);
    }
    __device__ __forceinline__ static su3<double> decode(const nu4 (&w)[W]) {
        su3<double> u;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const nd2 v = __builtin_bit_cast(nd2, w[k]);
            u.e[k / 3][k % 3] = {v.x, v.y};
        }
        rebuild_row2(u);
        return u;
    }
};

template <>
struct LinkWords<float, FMT_C64_12> {
    static constexpr int W = 3;
    __device__ __forceinline__ static void fetch(const void *L, uint32_t Vh, int s, uint32_t h,
                                                 nu4 (&w)[W]) {
        const size_t base = (size_t)s * 3 * Vh + h;
#pragma unroll
        for (int k = 0; k < 3; ++k) w[k] = nt_load<nu4>(L, base + (size_t)k * Vh);
    }
    __device__ __forceinline__ static su3<float> decode(const nu4 (&w)[W]) {
        su3<float> u;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const nf4 v = __builtin_bit_cast(nf4, w[k]);
            u.e[(2 * k) / 3][(2 * k) % 3] = {v.x, v.y};
            u.e[(2 * k + 1) / 3][(2 * k + 1) % 3] = {v.z, v.w};
        }
        rebuild_row2(u);
        return u;
    }
};

template <>
struct LinkWords<float, FMT_BF16_12> {
    static constexpr int W = 2;  // 16 + 8 bytes, the second word half used
    __device__ __forceinline__ static void fetch(const void *L, uint32_t Vh, int s, uint32_t h,
                                                 nu4 (&w)[W]) {
        const void *Lb = reinterpret_cast<const nu4 *>(L) + (size_t)8 * Vh;
        w[0] = nt_load<nu4>(L, (size_t)s * Vh + h);
        const nu2 b = nt_load<nu2>(Lb, (size_t)s * Vh + h);
        w[1] = nu4{b.x, b.y, 0u, 0u};
    }
    __device__ __forceinline__ static su3<float> decode(const nu4 (&w)[W]) {
        su3<float> u;
        u.e[0][0] = {bf16_lo(w[0].x), bf16_hi(w[0].x)};
        u.e[0][1] = {bf16_lo(w[0].y), bf16_hi(w[0].y)};
        u.e[0][2] = {bf16_lo(w[0].z), bf16_hi(w[0].z)};
        u.e[1][0] = {bf16_lo(w[0].w), bf16_hi(w[0].w)};
        u.e[1][1] = {bf16_lo(w[1].x), bf16_hi(w[1].x)};
        u.e[1][2] = {bf16_lo(w[1].y), bf16_hi(w[1].y)};
        rebuild_row2(u);
        return u;
    }
};

constexpr int kFsSites = 64;  // output sites per block: one per lane of each wave

template <typename T, int FMT>
constexpr size_t fsplit_lds_bytes() {
    return (size_t)8 * LinkWords<T, FMT>::W * kFsSites * 16;
}

// Compensated sum of the wave's per-lane (s, c) pairs in a fixed shuffle order;
// valid in lane 0.
__device__ __forceinline__ void wave_sum_pair(double &s, double &c) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double s2 = __shfl_down(s, off, 64);
        const double c2 = __shfl_down(c, off, 64);
        pair_add(s, c, s2, c2);
    }
}

template <typename T, int FMT, bool STDPH, int NR, int FPG, int EPI>
__global__ __launch_bounds__(64 * (NR / FPG)) void hop_fsplit_kernel(HopArgs a) {
    constexpr int G = NR / FPG;
    constexpr int W = LinkWords<T, FMT>::W;
    static_assert(NR % FPG == 0, "fields per wave must divide the fields of the launch");
    static_assert(fsplit_lds_bytes<T, FMT>() <= kSplitLdsMax, "link tile exceeds the LDS budget");
    if (a.gate_running && a.ctl->n_running == 0) return;
    // [slot 2 d + (0 forward, 1 backward)][word][site]: lanes read consecutive words
    __shared__ nu4 tile[8][W][kFsSites];

    const Geom &g = a.geom;
    const int P = a.out_parity;
    const uint32_t blk = a.xcd_remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int f = threadIdx.x >> 6;  // field group = wave
    const int l = threadIdx.x & 63;
    const uint32_t pos = blk * kFsSites + l;
    const bool live = pos < g.Vh;
    const uint32_t h = (live && a.layer_group) ? layer_site(g, a.layer_group, pos) : pos;
    Site s;
    if (live) {
        s = site_coords(g, P, h);
        // this wave's share of the block's links into LDS
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            if (d % G != f) continue;  // wave f takes directions f, f + G, ... (none when f >= 4)
            nu4 wf[W], wb[W];
            LinkWords<T, FMT>::fetch(a.links, g.Vh, 2 * d + P, h, wf);
            LinkWords<T, FMT>::fetch(a.links, g.Vh, 2 * d + (1 - P), nb_bwd(g, s, h, d), wb);
#pragma unroll
            for (int k = 0; k < W; ++k) {
                tile[2 * d][k][l] = wf[k];
                tile[2 * d + 1][k][l] = wb[k];
            }
        }
    }
    __syncthreads();

    vec3<T> acc[FPG];
    zero_acc<T, FPG>(acc);
    if (live) {
        // neighbour loads on the wave's scalar field bases with 32-bit byte offsets, as
        // in the decoded-tile kernel below
        const int j0 = __builtin_amdgcn_readfirstlane(f) * FPG;
        const char *fb[FPG][3];
#pragma unroll
        for (int jj = 0; jj < FPG; ++jj)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                fb[jj][c] = reinterpret_cast<const char *>(a.in) +
                            ((size_t)(j0 + jj) * a.fstride + (size_t)c * g.Vh) * sizeof(cpx<T>);
        // one direction at a time (the loads of one direction in flight per wave keep
        // the registers low enough for many waves); the direction's neighbour indices
        // and phases come from compile-time arms, so no per-thread array is indexed
        // at run time
#pragma unroll 1
        for (int d = 0; d < 4; ++d) {
            uint32_t hf, hb;
            T pf, pb;
            dir_sites_rt<T, STDPH>(d, g, s, h, P, a.phases, hf, hb, pf, pb);
            nu4 w[W];
#pragma unroll
            for (int k = 0; k < W; ++k) w[k] = tile[2 * d][k][l];
            const su3<T> uf = LinkWords<T, FMT>::decode(w);
            const uint32_t of = hf * (uint32_t)sizeof(cpx<T>);
#pragma unroll
            for (int jj = 0; jj < FPG; ++jj) {
                vec3<T> v;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    using Pr = typename field_traits<T>::pair;
                    const Pr w = *reinterpret_cast<const Pr *>(fb[jj][c] + of);
                    v.c[c] = {w.x, w.y};
                }
                acc_mv(acc[jj], pf, uf, v);
            }
#pragma unroll
            for (int k = 0; k < W; ++k) w[k] = tile[2 * d + 1][k][l];
            const su3<T> ub = LinkWords<T, FMT>::decode(w);
            const uint32_t ob = hb * (uint32_t)sizeof(cpx<T>);
#pragma unroll
            for (int jj = 0; jj < FPG; ++jj) {
                vec3<T> v;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    using Pr = typename field_traits<T>::pair;
                    const Pr w = *reinterpret_cast<const Pr *>(fb[jj][c] + ob);
                    v.c[c] = {w.x, w.y};
                }
                acc_mdv(acc[jj], -pb, ub, v);
            }
        }
    }
    double ps[FPG], pc[FPG];
#pragma unroll
    for (int jj = 0; jj < FPG; ++jj) {
        ps[jj] = pc[jj] = 0.0;
        if (live) hop_epilogue_field<T, EPI>(a, h, f * FPG + jj, acc[jj], ps[jj], pc[jj]);
    }
    if (EPI == EPI_PLAIN || a.op == OP_NONE) return;
#pragma unroll
    for (int jj = 0; jj < FPG; ++jj) {
        wave_sum_pair(ps[jj], pc[jj]);
        if (l == 0) {
            double *pj = a.partials + 2 * ((size_t)(f * FPG + jj) * gridDim.x + blockIdx.x);
            pj[0] = ps[jj];
            pj[1] = pc[jj];
        }
    }
}

// The single-precision variant keeps the block's links in LDS decoded: the wave that
// fetches a link rebuilds its third row and folds in its phase (and the minus sign
// of the backward term) once, and stores the nine complex entries with the
// neighbour's half index, so the other waves of the block only read them; for FP32
// arithmetic the rebuild, the phase and the index arithmetic repeated in every wave
// cost about as many instructions as the mat-vecs of one field.
constexpr size_t kFsDecLdsBytes = (size_t)8 * 9 * kFsSites * 8 + (size_t)8 * kFsSites * 4;

// y += U v and y += U^dag v with the phase already in U (three fused complex
// multiply-adds per row into the accumulator)
__device__ __forceinline__ void acc_mv_folded(vec3<float> &y, const su3<float> &u,
                                              const vec3<float> &v) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) cfma(y.c[a], u.e[a][b], v.c[b]);
}

__device__ __forceinline__ void acc_mdv_folded(vec3<float> &y, const su3<float> &u,
                                               const vec3<float> &v) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) cfmac(y.c[a], u.e[b][a], v.c[b]);
}

// Direction D of lane l's site into the decoded tile: the forward link at x and the
// backward link at x - D, each with its phase folded in (the backward one negated),
// and the two neighbours' half indices.
template <int FMT, bool STDPH, int D>
__device__ __forceinline__ void dec_fill(const HopArgs &a, const Geom &g, const Site &s,
                                         uint32_t h, int P, int l,
                                         cpx<float> (*ltile)[9][kFsSites],
                                         uint32_t (*ntile)[kFsSites]) {
    uint32_t hf, hb;
    float pf, pb;
    dir_sites<float, STDPH, D>(g, s, h, P, a.phases, hf, hb, pf, pb);
    const su3<float> uf = link_loader<float, FMT>::load(a.links, g.Vh, 2 * D + P, h);
    const su3<float> ub = link_loader<float, FMT>::load(a.links, g.Vh, 2 * D + 1 - P, hb);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        ltile[2 * D][e][l] = cscale(pf, uf.e[e / 3][e % 3]);
        ltile[2 * D + 1][e][l] = cscale(-pb, ub.e[e / 3][e % 3]);
    }
    ntile[2 * D][l] = hf;
    ntile[2 * D + 1][l] = hb;
}

template <int FMT, bool STDPH, int NR, int FPG, int EPI>
__global__ __launch_bounds__(64 * (NR / FPG)) void hop_fsplit_dec_kernel(HopArgs a) {
    constexpr int G = NR / FPG;
    static_assert(NR % FPG == 0, "fields per wave must divide the fields of the launch");
    static_assert(kFsDecLdsBytes <= kSplitLdsMax, "link tile exceeds the LDS budget");
    if (a.gate_running && a.ctl->n_running == 0) return;
    // [slot 2 d + (0 forward, 1 backward)][entry 3 row + column][site]
    __shared__ cpx<float> ltile[8][9][kFsSites];
    __shared__ uint32_t ntile[8][kFsSites];

    const Geom &g = a.geom;
    const int P = a.out_parity;
    const uint32_t blk = a.xcd_remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int f = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const uint32_t pos = blk * kFsSites + l;
    const bool live = pos < g.Vh;
    const uint32_t h = (live && a.layer_group) ? layer_site(g, a.layer_group, pos) : pos;
    if (live) {
        // wave f takes directions f, f + G, ...
        const Site s = site_coords(g, P, h);
        if (0 % G == f) dec_fill<FMT, STDPH, 0>(a, g, s, h, P, l, ltile, ntile);
        if (1 % G == f) dec_fill<FMT, STDPH, 1>(a, g, s, h, P, l, ltile, ntile);
        if (2 % G == f) dec_fill<FMT, STDPH, 2>(a, g, s, h, P, l, ltile, ntile);
        if (3 % G == f) dec_fill<FMT, STDPH, 3>(a, g, s, h, P, l, ltile, ntile);
    }
    __syncthreads();

    vec3<float> acc[FPG];
    zero_acc<float, FPG>(acc);
    if (live) {
        // The wave's field bases are uniform (scalar registers) and a neighbour's byte
        // offset fits in 32 bits (Vh < 2^29), so each neighbour load is a scalar base
        // plus one 32-bit offset: no 64-bit address arithmetic per load in this
        // issue-bound loop (1-1.5 % faster at 32^4 with 8 fields).
        const int j0 = __builtin_amdgcn_readfirstlane(f) * FPG;
        const char *fb[FPG][3];
#pragma unroll
        for (int jj = 0; jj < FPG; ++jj)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                fb[jj][c] = reinterpret_cast<const char *>(
                    reinterpret_cast<const float2 *>(a.in) + (size_t)(j0 + jj) * a.fstride +
                    (size_t)c * g.Vh);
#pragma unroll 1
        for (int k = 0; k < 8; k += 2) {
            su3<float> u;
#pragma unroll
            for (int e = 0; e < 9; ++e) u.e[e / 3][e % 3] = ltile[k][e][l];
            const uint32_t of = ntile[k][l] << 3;
#pragma unroll
            for (int jj = 0; jj < FPG; ++jj) {
                vec3<float> v;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float2 w = *reinterpret_cast<const float2 *>(fb[jj][c] + of);
                    v.c[c] = {w.x, w.y};
                }
                acc_mv_folded(acc[jj], u, v);
            }
#pragma unroll
            for (int e = 0; e < 9; ++e) u.e[e / 3][e % 3] = ltile[k + 1][e][l];
            const uint32_t ob = ntile[k + 1][l] << 3;
#pragma unroll
            for (int jj = 0; jj < FPG; ++jj) {
                vec3<float> v;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float2 w = *reinterpret_cast<const float2 *>(fb[jj][c] + ob);
                    v.c[c] = {w.x, w.y};
                }
                acc_mdv_folded(acc[jj], u, v);
            }
        }
    }
    double ps[FPG], pc[FPG];
#pragma unroll
    for (int jj = 0; jj < FPG; ++jj) {
        ps[jj] = pc[jj] = 0.0;
        if (live) hop_epilogue_field<float, EPI>(a, h, f * FPG + jj, acc[jj], ps[jj], pc[jj]);
    }
    if (EPI == EPI_PLAIN || a.op == OP_NONE) return;
#pragma unroll
    for (int jj = 0; jj < FPG; ++jj) {
        wave_sum_pair(ps[jj], pc[jj]);
        if (l == 0) {
            double *pj = a.partials + 2 * ((size_t)(f * FPG + jj) * gridDim.x + blockIdx.x);
            pj[0] = ps[jj];
            pj[1] = pc[jj];
        }
    }
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <typename T, int FMT, bool STDPH, int NR, int FPG>
static int launch_fpg(const HopArgs &a, int epi, hipStream_t stream) {
    if constexpr (NR % FPG != 0 || fsplit_lds_bytes<T, FMT>() > kSplitLdsMax) {
        return -1;
    } else {
        // both kernels address neighbours by 32-bit byte offsets (8 or 16 B per entry)
        if ((size_t)a.geom.Vh * sizeof(cpx<T>) >= ((size_t)1 << 32)) return -1;
        dim3 grid((a.geom.Vh + kFsSites - 1) / kFsSites);
        const dim3 block(64 * (NR / FPG));
        const bool reduce = epi != EPI_PLAIN && a.op != OP_NONE;
        if (reduce && (size_t)NR * grid.x > a.partial_pairs) return -2;
        if constexpr (sizeof(T) == 4) {
            switch (epi) {
                case EPI_PLAIN:
                    hop_fsplit_dec_kernel<FMT, STDPH, NR, FPG, EPI_PLAIN><<<grid, block, 0, stream>>>(a);
                    break;
                case EPI_NORMAL:
                    hop_fsplit_dec_kernel<FMT, STDPH, NR, FPG, EPI_NORMAL><<<grid, block, 0, stream>>>(a);
                    break;
                default:
                    hop_fsplit_dec_kernel<FMT, STDPH, NR, FPG, EPI_RESID><<<grid, block, 0, stream>>>(a);
                    break;
            }
        } else {
            switch (epi) {
                case EPI_PLAIN:
                    hop_fsplit_kernel<T, FMT, STDPH, NR, FPG, EPI_PLAIN><<<grid, block, 0, stream>>>(a);
                    break;
                case EPI_NORMAL:
                    hop_fsplit_kernel<T, FMT, STDPH, NR, FPG, EPI_NORMAL><<<grid, block, 0, stream>>>(a);
                    break;
                default:
                    hop_fsplit_kernel<T, FMT, STDPH, NR, FPG, EPI_RESID><<<grid, block, 0, stream>>>(a);
                    break;
            }
        }
        if (a.grid_out) *a.grid_out = grid.x;
        if (reduce && !a.defer_finish) {
            FinArgs f{a.partials, grid.x, NR, a.op, a.gate_running, a.ctl, a.state, a.out_sums};
            launch_finalize(f, stream);
        }
        return 0;
    }
}

template <typename T, int FMT, bool STDPH, int NR>
static int launch_nr_fsplit(const HopArgs &a, int epi, hipStream_t stream) {
    if (a.fields_per_wave == 1) return launch_fpg<T, FMT, STDPH, NR, 1>(a, epi, stream);
    if (a.fields_per_wave == 2) return launch_fpg<T, FMT, STDPH, NR, 2>(a, epi, stream);
    return -1;
}

template <typename T, int FMT, bool STDPH>
static int launch_fmt_fsplit(const HopArgs &a, int nr, int epi, hipStream_t stream) {
    switch (nr) {
        case 2: return launch_nr_fsplit<T, FMT, STDPH, 2>(a, epi, stream);
        case 3: return launch_nr_fsplit<T, FMT, STDPH, 3>(a, epi, stream);
        case 4: return launch_nr_fsplit<T, FMT, STDPH, 4>(a, epi, stream);
        case 8: return launch_nr_fsplit<T, FMT, STDPH, 8>(a, epi, stream);
        default: return -1;
    }
}

template <typename T, int FMT>
static int launch_ph_fsplit(const HopArgs &a, int nr, int epi, hipStream_t stream) {
    return a.phases ? launch_fmt_fsplit<T, FMT, false>(a, nr, epi, stream)
                    : launch_fmt_fsplit<T, FMT, true>(a, nr, epi, stream);
}

// 0: launched; -1: this (format, fields, fields per wave) is not built; -2: the
// partials buffer is too small for the reduction (nothing launched).
int launch_hop_fsplit(const HopArgs &a, int fmt, int nr, int epi, hipStream_t stream) {
    switch (fmt) {
        case FMT_C128_12: return launch_ph_fsplit<double, FMT_C128_12>(a, nr, epi, stream);
        case FMT_C64_12: return launch_ph_fsplit<float, FMT_C64_12>(a, nr, epi, stream);
        case FMT_BF16_12: return launch_ph_fsplit<float, FMT_BF16_12>(a, nr, epi, stream);
        default: return -1;
    }
}

}  // namespace stg
