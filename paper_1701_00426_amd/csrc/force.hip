// force.hip -- derivative of the rational pseudofermion action with respect to
// every link, from the multi-shift solutions.
//
// Paper: arXiv:1701.00426, Sec. 2.2 (the forces of the molecular dynamics come
// from the solutions of the shifted systems, Eq. shlineq, of the rational
// approximation, Eq. rooting; the operator is Eq. diracblock).
//
// With X_k = (A + sigma_k)^{-1} phi on the even sites and Y_k = D_oe X_k on the odd
// ones, S = Re phi^dag sum_k a_k X_k changes by Re Tr(E G_mu(z)) when the link
// U_mu(z) becomes U_mu(z) + E, where
//   z even:  G_mu(z) =  phi_mu(z) sum_k a_k Y_k(z+mu) X_k(z)^dag
//   z odd:   G_mu(z) = -phi_mu(z) sum_k a_k X_k(z+mu) Y_k(z)^dag
// (dS = sum_k a_k 2 Re X_k^dag dD_eo Y_k; a link enters D_eo through the forward
// term at an even site and the backward term at z + mu for an odd one).
//
// One thread per site: it reads its own vector once per pole and the forward
// neighbours' in the four directions, and sums the weighted outer products of its
// four links in FP64 (the own vector serves all four).  Sites are visited in pencil
// order (pencil.hpp), even and odd ones in adjacent blocks, each XCD on one
// contiguous range, so a site's forward neighbours are mostly read by blocks in
// flight at the same time.

#include "device_common.hpp"
#include "force.hpp"
#include "kernels.hpp"

namespace stg {

namespace {

__global__ __launch_bounds__(kForceBlock) void force_kernel(ForceArgs a) {
    const Geom &g = a.geom;
    const uint32_t blk = a.xcd_remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int P = (int)(blk % 2);
    const uint32_t j = (blk / 2) * kForceBlock + threadIdx.x;
    if (j >= g.Vh) return;
    const uint32_t h = pencil_site(g, a.tile, j);
    const Site s = site_coords(g, P, h);
    uint32_t hf[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) hf[mu] = nb_fwd(g, s, h, mu);
    const void *own = P == 0 ? a.x : a.y;  // the field at z
    const void *nbf = P == 0 ? a.y : a.x;  // the field at z + mu
    const size_t fs = (size_t)3 * g.Vh;

    cpx<double> acc[4][3][3];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) acc[mu][i][j] = {0.0, 0.0};

    for (int k = 0; k < a.npoles; ++k) {
        const double c = a.coeff[k];
        const vec3<double> o = ld_v<double>(own, fs, g.Vh, k, h);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const vec3<double> n = ld_v<double>(nbf, fs, g.Vh, k, hf[mu]);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const cpx<double> t = cscale(c, n.c[i]);
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    // acc += t * conj(o_j)
                    acc[mu][i][j].re = fmat(t.re, o.c[j].re, acc[mu][i][j].re);
                    acc[mu][i][j].re = fmat(t.im, o.c[j].im, acc[mu][i][j].re);
                    acc[mu][i][j].im = fmat(t.im, o.c[j].re, acc[mu][i][j].im);
                    acc[mu][i][j].im = fmat(-t.re, o.c[j].im, acc[mu][i][j].im);
                }
            }
        }
    }

#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int slot = 2 * mu + P;
        const double ph = a.phases ? a.phases[(size_t)slot * g.Vh + h]
                                   : (double)std_phase(g, s, mu, false);
        const double sg = P == 0 ? ph : -ph;
        const size_t base = (size_t)slot * 9 * g.Vh + h;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const size_t idx = base + (size_t)(i * 3 + j) * g.Vh;
                cpx<double> v = cscale(sg, acc[mu][i][j]);
                if (a.accumulate) v = cadd(v, ld_c<double>(a.out, idx));
                st_c<double>(a.out, idx, v);
            }
    }
}

}  // namespace

void launch_force(const ForceArgs &a, hipStream_t stream) {
    force_kernel<<<dim3(force_blocks(a.geom.Vh)), kForceBlock, 0, stream>>>(a);
}

}  // namespace stg
