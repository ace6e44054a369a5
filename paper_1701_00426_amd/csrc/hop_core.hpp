// hop_core.hpp -- the staggered hop at one output site, shared by the single-lattice
// and the batched (many-lattice) kernels.
//
// Paper: arXiv:1701.00426, Sec. 2.2 Eq. diracblock (D connects only even and odd
// sites), Sec. 4.3 deo listing (links, in, out and a real per-link factor array),
// Sec. 2.3 (12-real links, third row rebuilt on the fly).
#pragma once

#include "device_common.hpp"
#include "kernels.hpp"

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

// Neighbour half indices of site h along direction MU and the phases of its forward
// and backward link.
template <typename T, bool STDPH, int MU>
__device__ __forceinline__ void dir_sites(const Geom &g, const Site &s, uint32_t h, int P,
                                          const void *phases, uint32_t &hf, uint32_t &hb,
                                          T &pf, T &pb) {
    hf = nb_fwd(g, s, h, MU);
    hb = nb_bwd(g, s, h, MU);
    if (STDPH) {
        pf = (T)std_phase(g, s, MU, false);
        pb = (T)std_phase(g, s, MU, true);
    } else {
        const T *ph = reinterpret_cast<const T *>(phases);
        pf = ph[(size_t)(2 * MU + P) * g.Vh + h];
        pb = ph[(size_t)(2 * MU + 1 - P) * g.Vh + hb];
    }
}

// The same for a direction known only at run time: compile-time arms, so that a loop
// over directions that is not unrolled indexes no per-thread array (the site's
// coordinates would otherwise go to scratch memory).
template <typename T, bool STDPH>
__device__ __forceinline__ void dir_sites_rt(int mu, const Geom &g, const Site &s, uint32_t h,
                                             int P, const void *phases, uint32_t &hf,
                                             uint32_t &hb, T &pf, T &pb) {
    switch (mu) {
        case 0: dir_sites<T, STDPH, 0>(g, s, h, P, phases, hf, hb, pf, pb); break;
        case 1: dir_sites<T, STDPH, 1>(g, s, h, P, phases, hf, hb, pf, pb); break;
        case 2: dir_sites<T, STDPH, 2>(g, s, h, P, phases, hf, hb, pf, pb); break;
        default: dir_sites<T, STDPH, 3>(g, s, h, P, phases, hf, hb, pf, pb); break;
    }
}

// Adds the terms of directions MU0 .. MU0 + ND - 1 at output site h (parity P) to
// acc[j] for the NR fields: forward link U_mu(x) and neighbour x + mu, backward
// link U_mu(x - mu)^dag and neighbour x - mu, each times its phase.  UNR directions
// are unrolled (0: HopUnroll's choice).
template <typename T, int FMT, bool STDPH, int NR, int MU0, int ND, int UNR = 0, typename NB>
__device__ __forceinline__ void hop_dirs(const Geom &g, int P, uint32_t h, const Site &s,
                                         const void *links, const void *phases, const NB &nb,
                                         vec3<T> (&acc)[NR]) {
    constexpr int kU = UNR > 0 ? UNR : HopUnroll<T, NR>::value;
    constexpr int kUnroll = kU < ND ? kU : ND;
#pragma unroll kUnroll
    for (int d = 0; d < ND; ++d) {
        const int mu = MU0 + d;
        const int sf = 2 * mu + P;        // U_mu(x) starts at x
        const int sb = 2 * mu + (1 - P);  // U_mu(x - mu) starts at x - mu
        uint32_t hf, hb;
        T pf, pb;
        if constexpr (kUnroll >= ND) {
            // fully unrolled: mu is a constant in every copy, and the loads of all the
            // directions are scheduled together
            hf = nb_fwd(g, s, h, mu);
            hb = nb_bwd(g, s, h, mu);
            if (STDPH) {
                pf = (T)std_phase(g, s, mu, false);
                pb = (T)std_phase(g, s, mu, true);
            } else {
                const T *ph = reinterpret_cast<const T *>(phases);
                pf = ph[(size_t)sf * g.Vh + h];
                pb = ph[(size_t)sb * g.Vh + hb];
            }
        } else {
            dir_sites_rt<T, STDPH>(mu, g, s, h, P, phases, hf, hb, pf, pb);
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

template <typename T, int NR>
__device__ __forceinline__ void zero_acc(vec3<T> (&acc)[NR]) {
#pragma unroll
    for (int j = 0; j < NR; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[j].c[c] = {T(0), T(0)};
}

template <typename T, int FMT, bool STDPH, int NR, typename NB>
__device__ __forceinline__ void hop_site_nb(const Geom &g, int P, uint32_t h, const void *links,
                                            const void *phases, const NB &nb,
                                            vec3<T> (&acc)[NR]) {
    Site s = site_coords(g, P, h);
    zero_acc<T, NR>(acc);
    hop_dirs<T, FMT, STDPH, NR, 0, 4>(g, P, h, s, links, phases, nb, acc);
}

template <typename T, int FMT, bool STDPH, int NR>
__device__ __forceinline__ void hop_site(const Geom &g, int P, uint32_t h, const void *links,
                                         const void *phases, const void *in, size_t fstride,
                                         vec3<T> (&acc)[NR]) {
    hop_site_nb<T, FMT, STDPH, NR>(g, P, h, links, phases, GlobalNb<T>{in, fstride, g.Vh}, acc);
}

// Epilogue at output site h from acc = sum_mu [...] (twice the hop):
//   EPI_PLAIN   out = acc / 2
//   EPI_NORMAL  out = diag_j p - acc / 2, and Re<p, out> into the partials (ps, pc)
//   EPI_RESID   out = b - (diag_j x - acc / 2), and |out|^2 into the partials, for
//               the fields whose system waits for a true residual
template <typename T, int EPI>
__device__ __forceinline__ void hop_epilogue_field(const HopArgs &a, uint32_t h, int j,
                                                   const vec3<T> &acc, double &ps, double &pc) {
    const Geom &g = a.geom;
    const T half = T(0.5);
    vec3<T> o;
    if (EPI == EPI_PLAIN) {
#pragma unroll
        for (int c = 0; c < 3; ++c) o.c[c] = cscale(half, acc.c[c]);
    } else if (EPI == EPI_NORMAL) {
        const T d = (T)a.st_diag(j);
        vec3<T> p = ld_v<T>(a.aux0, a.fstride, g.Vh, j, h);
        double site = 0.0;  // this site's six terms in FP64, then one compensated add
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            o.c[c].re = d * p.c[c].re - half * acc.c[c].re;
            o.c[c].im = d * p.c[c].im - half * acc.c[c].im;
            site = fmat((double)p.c[c].re, (double)o.c[c].re, site);
            site = fmat((double)p.c[c].im, (double)o.c[c].im, site);
        }
        pair_add(ps, pc, site, 0.0);
    } else {  // EPI_RESID
        if (!a.st_pending(j)) return;
        const T d = (T)a.st_diag(j);
        vec3<T> x = ld_v<T>(a.aux0, a.fstride, g.Vh, j, h);
        vec3<T> b = ld_v<T>(a.aux1, a.fstride, g.Vh, j, h);
        double site = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            o.c[c].re = b.c[c].re - (d * x.c[c].re - half * acc.c[c].re);
            o.c[c].im = b.c[c].im - (d * x.c[c].im - half * acc.c[c].im);
            site = fmat((double)o.c[c].re, (double)o.c[c].re, site);
            site = fmat((double)o.c[c].im, (double)o.c[c].im, site);
        }
        pair_add(ps, pc, site, 0.0);
    }
    // FP64 plain output streams past the caches (measured 2 % faster at 32^4; the
    // FP32 hop gains nothing)
    if constexpr (EPI == EPI_PLAIN && sizeof(T) == 8)
        st_v_nt(a.out, a.fstride, g.Vh, j, h, o);
    else
        st_v<T>(a.out, a.fstride, g.Vh, j, h, o);
}

template <typename T, int NR, int EPI>
__device__ __forceinline__ void hop_epilogue(const HopArgs &a, uint32_t h,
                                             const vec3<T> (&acc)[NR], double (&ps)[NR],
                                             double (&pc)[NR]) {
#pragma unroll
    for (int j = 0; j < NR; ++j) hop_epilogue_field<T, EPI>(a, h, j, acc[j], ps[j], pc[j]);
}

}  // namespace stg
