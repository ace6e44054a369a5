// hop_core.hpp -- the staggered hop at one output site, shared by the single-lattice
// and the batched (many-lattice) kernels.
//
// Paper: arXiv:1701.00426, Sec. 2.2 Eq. diracblock (D connects only even and odd
// sites), Sec. 4.3 deo listing (links, in, out and a real per-link factor array),
// Sec. 2.3 (12-real links, third row rebuilt on the fly).
#pragma once

#include "device_common.hpp"

namespace stg {

// Directions unrolled in the hop: with all four unrolled the compiler issues the
// sixteen link loads (and the eight neighbour loads) of a site together, which
// hides HBM latency far better than more waves with one direction in flight
// (measured at 32^4: FP64-12 D_eo 89.6 -> 80.7 us, FP32-12 50.9 -> 41.5 us).
// Several fields per launch multiply the accumulators and neighbour loads, so
// larger NR keeps one direction at a time to stay clear of register spills.
template <typename T, int NR>
struct HopUnroll {
    static constexpr int value = (NR == 1 || (NR == 2 && sizeof(T) == 4)) ? 4 : 1;
};

// acc[j] = sum_mu [ phi_mu(x) U_mu(x) in_j(x+mu) - phi_mu(x-mu) U_mu(x-mu)^dag in_j(x-mu) ]
// for the output site x of parity P with half index h, and NR fields in_j stored
// [NR][3][Vh] with stride fstride (the factor 1/2 is left to the caller).
// Neighbour-field reads straight from global memory (L1/L2 serve the re-reads).
template <typename T>
struct GlobalNb {
    const void *in;
    size_t fstride;
    uint32_t Vh;
    __device__ __forceinline__ vec3<T> operator()(int j, uint32_t n) const {
        return ld_v<T>(in, fstride, Vh, j, n);
    }
};

// Neighbour-field reads from an LDS copy of the global index range [s0, s0 + len)
// (the block's own sites and one x1 row on each side: every x0 and most x1
// neighbours), from global memory outside it.
constexpr uint32_t kStageMax = 384;  // staged sites per block: kBlock + 2 * nh0, nh0 <= 64

template <typename T, int NR>
struct StagedNb {
    const cpx<T> (*tile)[3][kStageMax];
    int64_t s0;
    uint32_t len;
    GlobalNb<T> glob;
    __device__ __forceinline__ vec3<T> operator()(int j, uint32_t n) const {
        const int64_t i = (int64_t)n - s0;
        if (i >= 0 && i < (int64_t)len) {
            vec3<T> v;
#pragma unroll
            for (int c = 0; c < 3; ++c) v.c[c] = tile[j][c][i];
            return v;
        }
        return glob(j, n);
    }
};

// Cooperative fill of the LDS copy by the whole block (followed by a barrier).
template <typename T, int NR>
__device__ __forceinline__ void stage_fill(cpx<T> (*tile)[3][kStageMax], const void *in,
                                           size_t fstride, uint32_t Vh, int64_t s0,
                                           uint32_t len) {
    for (uint32_t i = threadIdx.x; i < len; i += kBlock) {
        const int64_t n = s0 + (int64_t)i;
        if (n < 0 || n >= (int64_t)Vh) continue;
#pragma unroll
        for (int j = 0; j < NR; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                tile[j][c][i] = ld_c<T>(in, (size_t)j * fstride + (size_t)c * Vh + (uint32_t)n);
    }
    __syncthreads();
}

template <typename T, int FMT, bool STDPH, int NR, typename NB>
__device__ __forceinline__ void hop_site_nb(const Geom &g, int P, uint32_t h, const void *links,
                                            const void *phases, const NB &nb,
                                            vec3<T> (&acc)[NR]) {
    Site s = site_coords(g, P, h);
#pragma unroll
    for (int j = 0; j < NR; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[j].c[c] = {T(0), T(0)};

    constexpr int kUnroll = HopUnroll<T, NR>::value;
#pragma unroll kUnroll
    for (int mu = 0; mu < 4; ++mu) {
        const uint32_t hf = nb_fwd(g, s, h, mu);
        const uint32_t hb = nb_bwd(g, s, h, mu);
        const int sf = 2 * mu + P;        // U_mu(x) starts at x
        const int sb = 2 * mu + (1 - P);  // U_mu(x - mu) starts at x - mu
        T pf, pb;
        if (STDPH) {
            pf = (T)std_phase(g, s, mu, false);
            pb = (T)std_phase(g, s, mu, true);
        } else {
            const T *ph = reinterpret_cast<const T *>(phases);
            pf = ph[(size_t)sf * g.Vh + h];
            pb = ph[(size_t)sb * g.Vh + hb];
        }
        su3<T> uf = link_loader<T, FMT>::load(links, g.Vh, sf, h);
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            vec3<T> v = nb(j, hf);
            acc_mv(acc[j], pf, uf, v);
        }
        su3<T> ub = link_loader<T, FMT>::load(links, g.Vh, sb, hb);
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            vec3<T> v = nb(j, hb);
            acc_mdv(acc[j], -pb, ub, v);
        }
    }
}

template <typename T, int FMT, bool STDPH, int NR>
__device__ __forceinline__ void hop_site(const Geom &g, int P, uint32_t h, const void *links,
                                         const void *phases, const void *in, size_t fstride,
                                         vec3<T> (&acc)[NR]) {
    hop_site_nb<T, FMT, STDPH, NR>(g, P, h, links, phases, GlobalNb<T>{in, fstride, g.Vh}, acc);
}

}  // namespace stg
