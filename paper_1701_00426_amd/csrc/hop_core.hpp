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
template <typename T, int FMT, bool STDPH, int NR>
__device__ __forceinline__ void hop_site(const Geom &g, int P, uint32_t h, const void *links,
                                         const void *phases, const void *in, size_t fstride,
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
            vec3<T> v = ld_v<T>(in, fstride, g.Vh, j, hf);
            acc_mv(acc[j], pf, uf, v);
        }
        su3<T> ub = link_loader<T, FMT>::load(links, g.Vh, sb, hb);
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            vec3<T> v = ld_v<T>(in, fstride, g.Vh, j, hb);
            acc_mdv(acc[j], -pb, ub, v);
        }
    }
}

}  // namespace stg
