// staple.hip -- staples of the tree-level Symanzik gauge force.
//
// Paper: arXiv:1701.00426, Sec. 2.1 (tree-level Symanzik improved gauge action:
// 1x1 and 1x2 Wilson loops) and Sec. 4.3 (the gauge cycle's most expensive step:
// staples, products of 3 and 5 SU(3) links along C-shaped paths, computed per
// link with second-neighbour addressing).
//
// For the link U_mu(x) the kernel forms
//   Sigma_mu(x) = sum_{nu != mu} [ c0 (2 three-link paths) + c1 (6 five-link paths) ],
// each path a product of links leading from x + mu back to x, so U_mu(x) Sigma_mu(x)
// is the weighted sum of the closed loops through the link.
//
// One or two threads per link (with two, the paths above and below the link run
// on separate waves of the block and meet in LDS); the link's (mu, parity) is
// uniform in a block, the 8 slots of a group of sites run in adjacent blocks, and
// the sites are visited in pencil order (pencil.hpp) so that a link's radius-2
// neighbourhood is mostly in the XCD's L2.  Neighbour half indices come from
// coordinate arithmetic (no index tables).  The 8 paths of each side (above /
// below the link) share their factors:
//   above:  A = U_nu(x+mu), W = U_mu(x+nu)^dag U_nu(x)^dag,
//           D = U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu),
//           T = U_nu(x+mu+nu) U_mu(x+2nu)^dag U_nu(x+nu)^dag,
//           E = U_mu(x+mu) U_nu(x+2mu) U_mu(x+mu+nu)^dag,
//   1x1: A W;  1x2: E W (long side forward), A U_mu(x+nu)^dag D (long side
//   backward), A T U_nu(x)^dag (long side along nu), so the side contributes
//           A [c0 W + c1 (U_mu(x+nu)^dag D + T U_nu(x)^dag)] + c1 E W,
// 11 SU(3) products instead of 14 taken path by path; below the link likewise
// with nu -> -nu.  Products accumulate in the arithmetic type of the format
// (FP64 for complex128 links, FP32 for the 12-real FP32 / BF16 ones).
//
// The same file holds one stout-smearing step (Sec. 2.1: the fermion action is
// built on stout-smeared links; Sec. 2.3: the configurations of the stout levels
// are kept): with C_mu(x) = rho * (the six 3-link paths from x to x + mu),
// Omega = C U^dag and Q = (i/2)(Omega^dag - Omega) - (i/6) Tr(Omega^dag - Omega),
// every link becomes exp(iQ) U (Morningstar and Peardon's definition).

#include "device_common.hpp"
#include "kernels.hpp"
#include "staple.hpp"

namespace stg {

namespace {

// acc += a * conj(b)
template <typename T>
__device__ __forceinline__ void cfma_cb(cpx<T> &acc, cpx<T> a, cpx<T> b) {
    acc.re = fmat(a.re, b.re, acc.re);
    acc.re = fmat(a.im, b.im, acc.re);
    acc.im = fmat(a.im, b.re, acc.im);
    acc.im = fmat(-a.re, b.im, acc.im);
}

// C = A B
template <typename T>
__device__ __forceinline__ su3<T> mm(const su3<T> &a, const su3<T> &b) {
    su3<T> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cpx<T> t = cmul(a.e[i][0], b.e[0][j]);
            cfma(t, a.e[i][1], b.e[1][j]);
            cfma(t, a.e[i][2], b.e[2][j]);
            c.e[i][j] = t;
        }
    return c;
}

// C += A B
template <typename T>
__device__ __forceinline__ void mm_acc(su3<T> &c, const su3<T> &a, const su3<T> &b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) cfma(c.e[i][j], a.e[i][k], b.e[k][j]);
}

// C = A B^dag
template <typename T>
__device__ __forceinline__ su3<T> mmd(const su3<T> &a, const su3<T> &b) {
    su3<T> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cpx<T> t = {T(0), T(0)};
#pragma unroll
            for (int k = 0; k < 3; ++k) cfma_cb(t, a.e[i][k], b.e[j][k]);
            c.e[i][j] = t;
        }
    return c;
}

// C += A B^dag
template <typename T>
__device__ __forceinline__ void mmd_acc(su3<T> &c, const su3<T> &a, const su3<T> &b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) cfma_cb(c.e[i][j], a.e[i][k], b.e[j][k]);
}

// C = A^dag B
template <typename T>
__device__ __forceinline__ su3<T> mdm(const su3<T> &a, const su3<T> &b) {
    su3<T> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cpx<T> t = cmulc(a.e[0][i], b.e[0][j]);
            cfmac(t, a.e[1][i], b.e[1][j]);
            cfmac(t, a.e[2][i], b.e[2][j]);
            c.e[i][j] = t;
        }
    return c;
}

// C += A^dag B
template <typename T>
__device__ __forceinline__ void mdm_acc(su3<T> &c, const su3<T> &a, const su3<T> &b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) cfmac(c.e[i][j], a.e[k][i], b.e[k][j]);
}

// C = A^dag B^dag = (B A)^dag
template <typename T>
__device__ __forceinline__ su3<T> mdmd(const su3<T> &a, const su3<T> &b) {
    su3<T> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cpx<T> t = cmul(b.e[j][0], a.e[0][i]);
            cfma(t, b.e[j][1], a.e[1][i]);
            cfma(t, b.e[j][2], a.e[2][i]);
            c.e[i][j] = cconj(t);
        }
    return c;
}

// C = s C + r B
template <typename T>
__device__ __forceinline__ void axpby(su3<T> &c, T s, T r, const su3<T> &b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            c.e[i][j].re = fmat(s, c.e[i][j].re, r * b.e[i][j].re);
            c.e[i][j].im = fmat(s, c.e[i][j].im, r * b.e[i][j].im);
        }
}

template <typename T>
__device__ __forceinline__ void scale(su3<T> &c, T s) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            c.e[i][j].re *= s;
            c.e[i][j].im *= s;
        }
}

__device__ __forceinline__ uint32_t pick4(uint32_t v0, uint32_t v1, uint32_t v2, uint32_t v3,
                                          int i) {
    return i == 0 ? v0 : i == 1 ? v1 : i == 2 ? v2 : v3;
}

// x_d + s with periodic wrap, |s| <= 2 <= N
__device__ __forceinline__ int wrap_step(int x, int s, int n) {
    int y = x + s;
    y += (y < 0) ? n : 0;
    y -= (y >= n) ? n : 0;
    return y;
}

// Lexicographic displacement of the site x when its coordinate x_d (extent n,
// lexicographic stride st) moves by s.
__device__ __forceinline__ int lex_step(int x, int s, int n, int st) {
    return (wrap_step(x, s, n) - x) * st;
}

// Link loads through the caches: every link is read by about sixty staple
// computations of nearby links, so these loads must stay cached (the hop's loader
// streams its links past the caches instead).
template <typename T, int FMT>
struct cached_link;

template <>
struct cached_link<double, FMT_C128_18> {
    __device__ __forceinline__ static su3<double> load(const void *L, uint32_t Vh, int s,
                                                        uint32_t h) {
        const double2 *p = reinterpret_cast<const double2 *>(L) + (size_t)s * 9 * Vh + h;
        su3<double> u;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const double2 v = p[(size_t)(a * 3 + b) * Vh];
                u.e[a][b] = {v.x, v.y};
            }
        return u;
    }
};

template <>
struct cached_link<double, FMT_C128_12> {
    __device__ __forceinline__ static su3<double> load(const void *L, uint32_t Vh, int s,
                                                        uint32_t h) {
        const double2 *p = reinterpret_cast<const double2 *>(L) + (size_t)s * 6 * Vh + h;
        su3<double> u;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const double2 v = p[(size_t)(a * 3 + b) * Vh];
                u.e[a][b] = {v.x, v.y};
            }
        rebuild_row2(u);
        return u;
    }
};

template <>
struct cached_link<float, FMT_C64_12> {
    __device__ __forceinline__ static su3<float> load(const void *L, uint32_t Vh, int s,
                                                       uint32_t h) {
        const float4 *p = reinterpret_cast<const float4 *>(L) + (size_t)s * 3 * Vh + h;
        const float4 c0 = p[0], c1 = p[Vh], c2 = p[2 * (size_t)Vh];
        su3<float> u;
        u.e[0][0] = {c0.x, c0.y};
        u.e[0][1] = {c0.z, c0.w};
        u.e[0][2] = {c1.x, c1.y};
        u.e[1][0] = {c1.z, c1.w};
        u.e[1][1] = {c2.x, c2.y};
        u.e[1][2] = {c2.z, c2.w};
        rebuild_row2(u);
        return u;
    }
};

template <>
struct cached_link<float, FMT_BF16_12> {
    __device__ __forceinline__ static su3<float> load(const void *L, uint32_t Vh, int s,
                                                       uint32_t h) {
        const uint4 a = reinterpret_cast<const uint4 *>(L)[(size_t)s * Vh + h];
        const uint2 b = reinterpret_cast<const uint2 *>(
            reinterpret_cast<const uint4 *>(L) + (size_t)8 * Vh)[(size_t)s * Vh + h];
        su3<float> u;
        u.e[0][0] = {bf16_lo(a.x), bf16_hi(a.x)};
        u.e[0][1] = {bf16_lo(a.y), bf16_hi(a.y)};
        u.e[0][2] = {bf16_lo(a.z), bf16_hi(a.z)};
        u.e[1][0] = {bf16_lo(a.w), bf16_hi(a.w)};
        u.e[1][1] = {bf16_lo(b.x), bf16_hi(b.x)};
        u.e[1][2] = {bf16_lo(b.y), bf16_hi(b.y)};
        rebuild_row2(u);
        return u;
    }
};

// The links around one site x: lexicographic index L of x, parity P of x.
template <typename T, int FMT>
struct LinkAt {
    const void *links;
    uint32_t Vh;
    int L, P;
    // U_d(y) for y = x + (displacement dl in lexicographic units, odd-even flip par)
    __device__ __forceinline__ su3<T> operator()(int d, int dl, int flip) const {
        const int par = (P + flip) & 1;
        const uint32_t h = (uint32_t)(L + dl) >> 1;
        return cached_link<T, FMT>::load(links, Vh, 2 * d + par, h);
    }
};

// The 1x1 and 1x2 paths on the +nu side of the link: A [c0 W + c1 (U_mu(x+nu)^dag D +
// T U_nu(x)^dag)] + c1 E W.  mp1 .. np2: lexicographic displacements of x +- mu, x + 2mu,
// x +- nu, x + 2nu (periodic).
template <typename T, int FMT>
__device__ __forceinline__ void side_above(su3<T> &acc, const LinkAt<T, FMT> &U, int mu, int nu,
                                           int mp1, int mm1, int mp2, int np1, int np2, T c0,
                                           T c1) {
    su3<T> y = mm(mdmd(U(mu, mm1 + np1, 0), U(nu, mm1, 1)), U(mu, mm1, 1));  // D
    su3<T> x = mdm(U(mu, np1, 1), y);
    y = mmd(mmd(U(nu, mp1 + np1, 0), U(mu, np2, 0)), U(nu, np1, 1));          // T
    mmd_acc(x, y, U(nu, 0, 0));
    su3<T> w = mdmd(U(mu, np1, 1), U(nu, 0, 0));  // W = U_mu(x+nu)^dag U_nu(x)^dag
    axpby(x, c1, c0, w);                           // c0 W + c1 (...)
    mm_acc(acc, U(nu, mp1, 1), x);                 // A = U_nu(x+mu)
    y = mmd(mm(U(mu, mp1, 1), U(nu, mp2, 0)), U(mu, mp1 + np1, 0));          // E
    scale(w, c1);
    mm_acc(acc, y, w);
}

// The same on the -nu side: A' = U_nu(x+mu-nu)^dag, W' = U_mu(x-nu)^dag U_nu(x-nu),
// D' = U_mu(x-mu-nu)^dag U_nu(x-mu-nu) U_mu(x-mu), T' = U_nu(x+mu-2nu)^dag
// U_mu(x-2nu)^dag U_nu(x-2nu), E' = U_mu(x+mu) U_nu(x+2mu-nu)^dag U_mu(x+mu-nu)^dag.
template <typename T, int FMT>
__device__ __forceinline__ void side_below(su3<T> &acc, const LinkAt<T, FMT> &U, int mu, int nu,
                                           int mp1, int mm1, int mp2, int nm1, int nm2, T c0,
                                           T c1) {
    su3<T> y = mm(mdm(U(mu, mm1 + nm1, 0), U(nu, mm1 + nm1, 0)), U(mu, mm1, 1));  // D'
    su3<T> x = mdm(U(mu, nm1, 1), y);
    y = mm(mdmd(U(nu, mp1 + nm2, 1), U(mu, nm2, 0)), U(nu, nm2, 0));             // T'
    mm_acc(x, y, U(nu, nm1, 1));
    su3<T> w = mdm(U(mu, nm1, 1), U(nu, nm1, 1));
    axpby(x, c1, c0, w);
    mdm_acc(acc, U(nu, mp1 + nm1, 0), x);
    y = mmd(mmd(U(mu, mp1, 1), U(nu, mp2 + nm1, 1)), U(mu, mp1 + nm1, 0));     // E'
    scale(w, c1);
    mm_acc(acc, y, w);
}

// TPL threads per link (1 or 2): a block is TPL waves over the same kStapleLinks
// links; with 2, wave 0 sums the +nu sides and wave 1 the -nu sides, and wave 0
// adds wave 1's sums from LDS.  Two waves per SIMD are asked of the FP64 split
// kernel (it then fits in 256 registers).
// EPI 0 writes Sigma; EPI 1 (FP64 or FP32-12 links) instead adds (eps beta / 3) times the
// traceless Hermitian part of i U Sigma to the link's momentum: P -> P - eps F with the
// Symanzik gauge force F = -(beta/3) [i U Sigma]_TH, the staples never leaving the
// kernel.
template <typename T, int FMT, int TPL, int EPI>
__global__ __launch_bounds__(kStapleLinks * TPL)
__attribute__((amdgpu_waves_per_eu((TPL == 2 && sizeof(T) == 8) ? 2 : 1)))
void staple_kernel(StapleArgs a) {
    __shared__ cpx<T> part[9][kStapleLinks];
    const Geom &g = a.geom;
    const uint32_t blk = a.xcd_remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int slot = (int)(blk % 8);
    const int q = (int)threadIdx.x / kStapleLinks;  // the same in a whole wave
    const int l = (int)threadIdx.x % kStapleLinks;
    const uint32_t j = (blk / 8) * kStapleLinks + l;
    const bool valid = j < g.Vh;
    const uint32_t h = valid ? pencil_site(g, a.tile, j) : 0;
    const int mu = slot >> 1, P = slot & 1;

    su3<T> acc;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) acc.e[i][k] = {T(0), T(0)};

    if (valid) {
        const Site s = site_coords(g, P, h);
        const int st[4] = {1, (int)g.N[0], (int)(g.N[0] * g.N[1]),
                           (int)(g.N[0] * g.N[1] * g.N[2])};
        const int L = (int)s.x[0] + st[1] * (int)s.x[1] + st[2] * (int)s.x[2] +
                      st[3] * (int)s.x[3];
        const LinkAt<T, FMT> U{a.links, g.Vh, L, P};
        const int xm = (int)pick4(s.x[0], s.x[1], s.x[2], s.x[3], mu);
        const int nm = (int)pick4(g.N[0], g.N[1], g.N[2], g.N[3], mu);
        const int sm = (int)pick4(st[0], st[1], st[2], st[3], mu);
        const int mp1 = lex_step(xm, 1, nm, sm), mm1 = lex_step(xm, -1, nm, sm);
        const int mp2 = lex_step(xm, 2, nm, sm);
        const T c0 = (T)a.c0, c1 = (T)a.c1;
#pragma unroll 1
        for (int k = 1; k < 4; ++k) {
            const int nu = (mu + k) & 3;
            const int xn = (int)pick4(s.x[0], s.x[1], s.x[2], s.x[3], nu);
            const int nn = (int)pick4(g.N[0], g.N[1], g.N[2], g.N[3], nu);
            const int sn = (int)pick4(st[0], st[1], st[2], st[3], nu);
            if (TPL == 1 || q == 0)
                side_above(acc, U, mu, nu, mp1, mm1, mp2, lex_step(xn, 1, nn, sn),
                           lex_step(xn, 2, nn, sn), c0, c1);
            if (TPL == 1 || q == 1)
                side_below(acc, U, mu, nu, mp1, mm1, mp2, lex_step(xn, -1, nn, sn),
                           lex_step(xn, -2, nn, sn), c0, c1);
        }
    }
    if (TPL == 2) {
        if (q == 1) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int k = 0; k < 3; ++k) part[i * 3 + k][l] = acc.e[i][k];
        }
        __syncthreads();
        if (q == 1) return;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const cpx<T> v = part[i * 3 + k][l];
                acc.e[i][k].re += v.re;
                acc.e[i][k].im += v.im;
            }
    }
    if (!valid) return;
    const size_t base = (size_t)slot * 9 * g.Vh + h;
    if constexpr (EPI == 0) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                st_c<T>(a.out, base + (size_t)(i * 3 + k) * g.Vh, acc.e[i][k]);
    } else {
        // M = U Sigma; [iM]_TH = i (M - M^dag) / 2 + (sum_j Im M_jj / 3) I
        const su3<T> u = cached_link<T, FMT>::load(a.links, g.Vh, slot, h);
        const su3<T> m = mm(u, acc);
        const T tr = (m.e[0][0].im + m.e[1][1].im + m.e[2][2].im) / T(3);
        const T kf = (T)a.kmom;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const cpx<T> d = csub(m.e[i][k], cconj(m.e[k][i]));
                cpx<T> th = {T(-0.5) * d.im, T(0.5) * d.re};
                if (i == k) th.re += tr;
                const size_t idx = base + (size_t)(i * 3 + k) * g.Vh;
                cpx<T> pm = ld_c<T>(a.out, idx);
                pm.re = fmat(kf, th.re, pm.re);
                pm.im = fmat(kf, th.im, pm.im);
                st_c<T>(a.out, idx, pm);
            }
    }
}

// exp(iQ) for a traceless Hermitian 3x3 matrix Q.  Cayley-Hamilton gives
// Q^3 = c1 Q + c0 with c0 = det Q = Tr(Q^3)/3 and c1 = Tr(Q^2)/2, so
// exp(iQ) = f0 + f1 Q + f2 Q^2.  For c1 >= 1e-3 the f_j come in closed form from the
// eigenvalues of Q, parametrised by u and w (Morningstar and Peardon, Phys. Rev. D 69,
// 054501 (2004), Sec. III), computed for |c0| and mapped back by
// f_j(-c0) = (-1)^j conj(f_j(c0)).  Below that, the power series of exp, reduced by the
// same recurrence (Q^n = a_n + b_n Q + d_n Q^2), to 16 terms.
__device__ __forceinline__ su3<double> exp_iq(const su3<double> &q) {
    const su3<double> q2 = mm(q, q);
    const double c1 = 0.5 * (q2.e[0][0].re + q2.e[1][1].re + q2.e[2][2].re);
    double tr3 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) tr3 += cmul(q.e[i][k], q2.e[k][i]).re;
    const double c0 = tr3 / 3.0;
    cpx<double> f0, f1, f2;
    if (c1 < 1e-3) {
        double an = 1.0, bn = 0.0, dn = 0.0, fact = 1.0;
        cpx<double> ip = {1.0, 0.0};  // i^n
        f0 = f1 = f2 = {0.0, 0.0};
        for (int n = 0; n < 16; ++n) {
            f0 = cadd(f0, cscale(an / fact, ip));
            f1 = cadd(f1, cscale(bn / fact, ip));
            f2 = cadd(f2, cscale(dn / fact, ip));
            const double a1 = dn * c0, b1 = an + dn * c1, d1 = bn;
            an = a1;
            bn = b1;
            dn = d1;
            fact *= (double)(n + 1);
            ip = {-ip.im, ip.re};
        }
    } else {
        const double c0a = fabs(c0);
        const double s3 = sqrt(c1 / 3.0);
        const double c0max = 2.0 * s3 * s3 * s3;
        const double th = acos(fmin(c0a / c0max, 1.0));
        double st3, ct3, sw, cw, su, cu;
        sincos(th / 3.0, &st3, &ct3);
        const double u = s3 * ct3, w = sqrt(c1) * st3;
        const double uu = u * u, ww = w * w;
        sincos(w, &sw, &cw);
        sincos(u, &su, &cu);
        const double xi0 = fabs(w) < 0.05 ? 1.0 - ww / 6.0 * (1.0 - ww / 20.0 * (1.0 - ww / 42.0))
                                          : sw / w;
        const cpx<double> e2iu = {cu * cu - su * su, 2.0 * su * cu};  // exp(2iu)
        const cpx<double> emiu = {cu, -su};                          // exp(-iu)
        const cpx<double> h0 = cadd(cscale(uu - ww, e2iu),
                                    cmul(emiu, cpx<double>{8.0 * uu * cw,
                                                           2.0 * u * (3.0 * uu + ww) * xi0}));
        const cpx<double> h1 = csub(cscale(2.0 * u, e2iu),
                                    cmul(emiu, cpx<double>{2.0 * u * cw,
                                                           -(3.0 * uu - ww) * xi0}));
        const cpx<double> h2 = csub(e2iu, cmul(emiu, cpx<double>{cw, 3.0 * u * xi0}));
        const double inv = 1.0 / (9.0 * uu - ww);
        f0 = cscale(inv, h0);
        f1 = cscale(inv, h1);
        f2 = cscale(inv, h2);
        if (c0 < 0.0) {
            f0 = cconj(f0);
            f1 = cscale(-1.0, cconj(f1));
            f2 = cconj(f2);
        }
    }
    su3<double> e;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cpx<double> v = cadd(cmul(f1, q.e[i][k]), cmul(f2, q2.e[i][k]));
            if (i == k) v = cadd(v, f0);
            e.e[i][k] = v;
        }
    return e;
}

// exp(B) and the Frechet derivative L(B, M) = d/dt exp(B + t M) at t = 0 for a general
// 3x3 complex B, M: exp of the block matrix [[B, M], [0, B]] is [[e^B, L], [0, e^B]].  With
// T_n = B^n / n! and X_n the top-right block of the n-th term, X_n = (B X_{n-1} + M T_{n-1})/n;
// B and M are first scaled by 2^-s so that |B|_F <= 1/4, the series taken to 14 terms
// (remainder below 1e-20), and the pair squared back s times: (E, L) -> (E E, E L + L E).
__device__ __forceinline__ void exp_frechet(const su3<double> &b, const su3<double> &m,
                                            su3<double> &e, su3<double> &l) {
    double nb = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) nb += b.e[i][k].re * b.e[i][k].re + b.e[i][k].im * b.e[i][k].im;
    nb = sqrt(nb);
    int sq = 0;
    while (nb > 0.25 && sq < 40) {
        nb *= 0.5;
        ++sq;
    }
    const double sc = ldexp(1.0, -sq);
    su3<double> bs, ms, t, x;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            bs.e[i][k] = cscale(sc, b.e[i][k]);
            ms.e[i][k] = cscale(sc, m.e[i][k]);
            t.e[i][k] = {i == k ? 1.0 : 0.0, 0.0};
            x.e[i][k] = {0.0, 0.0};
        }
    e = t;
    l = x;
#pragma unroll 1
    for (int n = 1; n <= 14; ++n) {
        su3<double> xn = mm(bs, x);
        mm_acc(xn, ms, t);
        t = mm(bs, t);
        const double inv = 1.0 / (double)n;
        scale(xn, inv);
        scale(t, inv);
        x = xn;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                e.e[i][k] = cadd(e.e[i][k], t.e[i][k]);
                l.e[i][k] = cadd(l.e[i][k], x.e[i][k]);
            }
    }
#pragma unroll 1
    for (int r = 0; r < sq; ++r) {
        su3<double> ln = mm(e, l);
        mm_acc(ln, l, e);
        l = ln;
        e = mm(e, e);
    }
}

// Pass 1 of the force through a stout step, one thread per link l = (mu, x):
// C = rho (3-link paths from x to x+mu), Omega = C U^dag, Q, M = U Sigma'_l,
// Gamma = L(iQ, M); G = (Gamma - Gamma^dag)/2 + (conj(Tr Gamma) - Tr Gamma)/6;
// out_l = Sigma'_l exp(iQ) + C^dag G^dag, ws_l = U^dag G.
template <int FMT>
__global__ __launch_bounds__(kStoutBlock) void stout_back1_kernel(StoutBackArgs a) {
    const Geom &g = a.geom;
    const uint32_t blk = a.xcd_remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int slot = (int)(blk % 8);
    const uint32_t j = (blk / 8) * kStoutBlock + threadIdx.x;
    if (j >= g.Vh) return;
    const uint32_t h = pencil_site(g, a.tile, j);
    const int mu = slot >> 1, P = slot & 1;
    const Site s = site_coords(g, P, h);
    const int st[4] = {1, (int)g.N[0], (int)(g.N[0] * g.N[1]), (int)(g.N[0] * g.N[1] * g.N[2])};
    const int L = (int)s.x[0] + st[1] * (int)s.x[1] + st[2] * (int)s.x[2] + st[3] * (int)s.x[3];
    const LinkAt<double, FMT> U{a.links, g.Vh, L, P};
    const int xm = (int)pick4(s.x[0], s.x[1], s.x[2], s.x[3], mu);
    const int nm = (int)pick4(g.N[0], g.N[1], g.N[2], g.N[3], mu);
    const int sm = (int)pick4(st[0], st[1], st[2], st[3], mu);
    const int mp1 = lex_step(xm, 1, nm, sm);
    su3<double> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) c.e[i][k] = {0.0, 0.0};
#pragma unroll 1
    for (int k = 1; k < 4; ++k) {
        const int nu = (mu + k) & 3;
        const int xn = (int)pick4(s.x[0], s.x[1], s.x[2], s.x[3], nu);
        const int nn = (int)pick4(g.N[0], g.N[1], g.N[2], g.N[3], nu);
        const int sn = (int)pick4(st[0], st[1], st[2], st[3], nu);
        const int np1 = lex_step(xn, 1, nn, sn), nm1 = lex_step(xn, -1, nn, sn);
        mmd_acc(c, mm(U(nu, 0, 0), U(mu, np1, 1)), U(nu, mp1, 1));
        mm_acc(c, mdm(U(nu, nm1, 1), U(mu, nm1, 1)), U(nu, mp1 + nm1, 0));
    }
    scale(c, a.rho);
    const su3<double> u = U(mu, 0, 0);
    const su3<double> om = mmd(c, u);
    const double tq = (om.e[0][0].im + om.e[1][1].im + om.e[2][2].im) / 3.0;
    su3<double> iq;  // i Q
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const cpx<double> z = csub(cconj(om.e[k][i]), om.e[i][k]);
            cpx<double> qv = {-0.5 * z.im, 0.5 * z.re};
            if (i == k) qv.re -= tq;
            iq.e[i][k] = {-qv.im, qv.re};
        }
    const su3<double> sp = cached_link<double, FMT_C128_18>::load(a.sigp, g.Vh, slot, h);
    su3<double> e, gam;
    exp_frechet(iq, mm(u, sp), e, gam);
    const cpx<double> tg = cadd(cadd(gam.e[0][0], gam.e[1][1]), gam.e[2][2]);
    const cpx<double> dtr = cscale(1.0 / 6.0, csub(cconj(tg), tg));
    su3<double> gg;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cpx<double> v = cscale(0.5, csub(gam.e[i][k], cconj(gam.e[k][i])));
            if (i == k) v = cadd(v, dtr);
            gg.e[i][k] = v;
        }
    su3<double> loc = mm(sp, e);
    // + C^dag G^dag = (G C)^dag
    const su3<double> gcm = mm(gg, c);
    const su3<double> ug = mdm(u, gg);  // U^dag G
    const size_t base = (size_t)slot * 9 * g.Vh + h;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const size_t idx = base + (size_t)(i * 3 + k) * g.Vh;
            st_c<double>(a.out, idx, cadd(loc.e[i][k], cconj(gcm.e[k][i])));
            st_c<double>(a.ws, idx, ug.e[i][k]);
        }
}

// Pass 2, two threads per link l = (nu, y): add rho times every product in which l
// stands in a 3-link path of C at a neighbouring link (gc = U^dag G from pass 1):
// for each direction b != nu,
//   l as the middle link:  U_b(y-b+nu)^dag gc(nu, y-b) U_b(y-b),
//                          U_b(y+nu) gc(nu, y+b) U_b(y)^dag;
//   l as a side link:      U_b(y+nu) U_nu(y+b)^dag gc(b, y),
//                          [gc(b, y-b) U_nu(y-b) U_b(y-b+nu)]^dag,
//                          [U_b(y) U_nu(y+b) gc(b, y+nu)]^dag,
//                          gc(b, y+nu-b) U_nu(y-b)^dag U_b(y-b).
template <int FMT>
__global__ __launch_bounds__(2 * kStapleLinks) void stout_back2_kernel(StoutBackArgs a) {
    // two waves over the same kStapleLinks links: wave 0 sums the first three products
    // of each direction, wave 1 the last three; wave 1's sums meet wave 0's in LDS
    __shared__ cpx<double> part[9][kStapleLinks];
    const Geom &g = a.geom;
    const uint32_t blk = a.xcd_remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int slot = (int)(blk % 8);
    const int q = (int)threadIdx.x / kStapleLinks;  // the same in a whole wave
    const int l = (int)threadIdx.x % kStapleLinks;
    const uint32_t j = (blk / 8) * kStapleLinks + l;
    const bool valid = j < g.Vh;
    const uint32_t h = valid ? pencil_site(g, a.tile, j) : 0;
    const int nu = slot >> 1, P = slot & 1;
    su3<double> acc;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) acc.e[i][k] = {0.0, 0.0};
    if (valid) {
        const Site s = site_coords(g, P, h);
        const int st[4] = {1, (int)g.N[0], (int)(g.N[0] * g.N[1]),
                           (int)(g.N[0] * g.N[1] * g.N[2])};
        const int L = (int)s.x[0] + st[1] * (int)s.x[1] + st[2] * (int)s.x[2] +
                      st[3] * (int)s.x[3];
        const LinkAt<double, FMT> U{a.links, g.Vh, L, P};
        const LinkAt<double, FMT_C128_18> W{a.ws, g.Vh, L, P};
        const int xv = (int)pick4(s.x[0], s.x[1], s.x[2], s.x[3], nu);
        const int nv = (int)pick4(g.N[0], g.N[1], g.N[2], g.N[3], nu);
        const int sv = (int)pick4(st[0], st[1], st[2], st[3], nu);
        const int vp1 = lex_step(xv, 1, nv, sv);
#pragma unroll 1
        for (int k = 1; k < 4; ++k) {
            const int b = (nu + k) & 3;
            const int xb = (int)pick4(s.x[0], s.x[1], s.x[2], s.x[3], b);
            const int nb = (int)pick4(g.N[0], g.N[1], g.N[2], g.N[3], b);
            const int sb = (int)pick4(st[0], st[1], st[2], st[3], b);
            const int bp1 = lex_step(xb, 1, nb, sb), bm1 = lex_step(xb, -1, nb, sb);
            if (q == 0) {
                // middle link
                mm_acc(acc, mdm(U(b, bm1 + vp1, 0), W(nu, bm1, 1)), U(b, bm1, 1));
                mmd_acc(acc, mm(U(b, vp1, 1), W(nu, bp1, 1)), U(b, 0, 0));
                // side link, forward: U_b(y+nu) U_nu(y+b)^dag gc(b, y)
                mm_acc(acc, mmd(U(b, vp1, 1), U(nu, bp1, 1)), W(b, 0, 0));
            } else {
                // side link, forward: gc(b, y+nu-b) U_nu(y-b)^dag U_b(y-b)
                mm_acc(acc, mmd(W(b, vp1 + bm1, 0), U(nu, bm1, 1)), U(b, bm1, 1));
                // side links walked backwards: add the daggers, one product at a time
                {
                    const su3<double> t4 =
                        mm(mm(W(b, bm1, 1), U(nu, bm1, 1)), U(b, bm1 + vp1, 0));
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            acc.e[i][c] = cadd(acc.e[i][c], cconj(t4.e[c][i]));
                }
                {
                    const su3<double> t5 = mm(mm(U(b, 0, 0), U(nu, bp1, 1)), W(b, vp1, 1));
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            acc.e[i][c] = cadd(acc.e[i][c], cconj(t5.e[c][i]));
                }
            }
        }
    }
    if (q == 1) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) part[i * 3 + k][l] = acc.e[i][k];
    }
    __syncthreads();
    if (q == 1 || !valid) return;
    const size_t base = (size_t)slot * 9 * g.Vh + h;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const size_t idx = base + (size_t)(i * 3 + k) * g.Vh;
            const cpx<double> w1 = part[i * 3 + k][l];
            cpx<double> v = ld_c<double>(a.out, idx);
            v.re = fmat(a.rho, acc.e[i][k].re + w1.re, v.re);
            v.im = fmat(a.rho, acc.e[i][k].im + w1.im, v.im);
            st_c<double>(a.out, idx, v);
        }
}

template <int FMT>
__global__ __launch_bounds__(kStoutBlock) void stout_kernel(StoutArgs a) {
    const Geom &g = a.geom;
    const uint32_t blk = a.xcd_remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int slot = (int)(blk % 8);
    const uint32_t j = (blk / 8) * kStoutBlock + threadIdx.x;
    if (j >= g.Vh) return;
    const uint32_t h = pencil_site(g, a.tile, j);
    const int mu = slot >> 1, P = slot & 1;
    const Site s = site_coords(g, P, h);
    const int st[4] = {1, (int)g.N[0], (int)(g.N[0] * g.N[1]), (int)(g.N[0] * g.N[1] * g.N[2])};
    const int L = (int)s.x[0] + st[1] * (int)s.x[1] + st[2] * (int)s.x[2] + st[3] * (int)s.x[3];
    const LinkAt<double, FMT> U{a.links, g.Vh, L, P};
    const int xm = (int)pick4(s.x[0], s.x[1], s.x[2], s.x[3], mu);
    const int nm = (int)pick4(g.N[0], g.N[1], g.N[2], g.N[3], mu);
    const int sm = (int)pick4(st[0], st[1], st[2], st[3], mu);
    const int mp1 = lex_step(xm, 1, nm, sm);

    // C / rho: the 3-link paths from x to x + mu, above and below in each plane
    su3<double> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) c.e[i][k] = {0.0, 0.0};
#pragma unroll 1
    for (int k = 1; k < 4; ++k) {
        const int nu = (mu + k) & 3;
        const int xn = (int)pick4(s.x[0], s.x[1], s.x[2], s.x[3], nu);
        const int nn = (int)pick4(g.N[0], g.N[1], g.N[2], g.N[3], nu);
        const int sn = (int)pick4(st[0], st[1], st[2], st[3], nu);
        const int np1 = lex_step(xn, 1, nn, sn), nm1 = lex_step(xn, -1, nn, sn);
        // U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
        mmd_acc(c, mm(U(nu, 0, 0), U(mu, np1, 1)), U(nu, mp1, 1));
        // U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu)
        mm_acc(c, mdm(U(nu, nm1, 1), U(mu, nm1, 1)), U(nu, mp1 + nm1, 0));
    }
    scale(c, a.rho);
    const su3<double> u = U(mu, 0, 0);
    const su3<double> om = mmd(c, u);  // Omega = C U^dag
    // Q = (i/2)(Omega^dag - Omega) - (1/3) sum_i Im(Omega_ii) I
    const double tq = (om.e[0][0].im + om.e[1][1].im + om.e[2][2].im) / 3.0;
    su3<double> q;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const cpx<double> z = csub(cconj(om.e[k][i]), om.e[i][k]);
            q.e[i][k] = {-0.5 * z.im, 0.5 * z.re};
            if (i == k) q.e[i][k].re -= tq;
        }
    const su3<double> up = mm(exp_iq(q), u);
    const size_t base = (size_t)slot * 9 * g.Vh + h;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) st_c<double>(a.out, base + (size_t)(i * 3 + k) * g.Vh, up.e[i][k]);
}

template <typename T, int FMT>
int launch_tpl(const StapleArgs &a, int threads, hipStream_t stream) {
    const dim3 grid(staple_blocks(a.geom.Vh));
    if (threads == 1) {
        staple_kernel<T, FMT, 1, 0><<<grid, kStapleLinks, 0, stream>>>(a);
        return 0;
    }
    if (threads == 2) {
        staple_kernel<T, FMT, 2, 0><<<grid, 2 * kStapleLinks, 0, stream>>>(a);
        return 0;
    }
    return -1;
}

template <typename T, int FMT>
int launch_mom(const StapleArgs &a, int threads, hipStream_t stream) {
    const dim3 grid(staple_blocks(a.geom.Vh));
    if (threads == 1) {
        staple_kernel<T, FMT, 1, 1><<<grid, kStapleLinks, 0, stream>>>(a);
        return 0;
    }
    if (threads == 2) {
        staple_kernel<T, FMT, 2, 1><<<grid, 2 * kStapleLinks, 0, stream>>>(a);
        return 0;
    }
    return -1;
}

// U -> exp(i eps P) U in place, one thread per link, in the link's own format.  The
// exponential is formed in FP64 also for FP32 links and momenta (its cost is small
// next to the link and momentum traffic), the product with U in the format's type.
template <typename T, int FMT>
__global__ __launch_bounds__(kStoutBlock) void link_update_kernel(LinkUpdateArgs a) {
    const uint32_t Vh = a.Vh;
    const size_t n = (size_t)8 * Vh;
    const size_t t = (size_t)blockIdx.x * kStoutBlock + threadIdx.x;
    if (t >= n) return;
    const int slot = (int)(t / Vh);
    const uint32_t h = (uint32_t)(t % Vh);
    const su3<T> u = cached_link<T, FMT>::load(a.links, Vh, slot, h);
    su3<double> q;
    const size_t base = (size_t)slot * 9 * Vh + h;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const cpx<T> p = ld_c<T>(a.mom, base + (size_t)(i * 3 + k) * Vh);
            q.e[i][k] = {a.eps * (double)p.re, a.eps * (double)p.im};
        }
    const su3<double> e64 = exp_iq(q);
    su3<T> e;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) e.e[i][k] = {(T)e64.e[i][k].re, (T)e64.e[i][k].im};
    const su3<T> up = mm(e, u);
    if constexpr (FMT == FMT_C64_12) {
        // float4 chunks: (U00, U01), (U02, U10), (U11, U12)
        float4 *p = reinterpret_cast<float4 *>(a.links) + (size_t)slot * 3 * Vh + h;
        p[0] = make_float4(up.e[0][0].re, up.e[0][0].im, up.e[0][1].re, up.e[0][1].im);
        p[Vh] = make_float4(up.e[0][2].re, up.e[0][2].im, up.e[1][0].re, up.e[1][0].im);
        p[2 * (size_t)Vh] = make_float4(up.e[1][1].re, up.e[1][1].im, up.e[1][2].re, up.e[1][2].im);
    } else {
        constexpr int rows = FMT == FMT_C128_18 ? 3 : 2;
        const size_t lbase = (size_t)slot * rows * 3 * Vh + h;
#pragma unroll
        for (int i = 0; i < rows; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                st_c<T>(a.links, lbase + (size_t)(i * 3 + k) * Vh, up.e[i][k]);
    }
}

}  // namespace

int launch_stout_backprop(const StoutBackArgs &a, int fmt, hipStream_t stream) {
    const dim3 grid(stout_blocks(a.geom.Vh));
    const dim3 grid2(staple_blocks(a.geom.Vh));  // kStapleLinks links per block, two waves
    switch (fmt) {
        case FMT_C128_18:
            stout_back1_kernel<FMT_C128_18><<<grid, kStoutBlock, 0, stream>>>(a);
            stout_back2_kernel<FMT_C128_18><<<grid2, 2 * kStapleLinks, 0, stream>>>(a);
            return 0;
        case FMT_C128_12:
            stout_back1_kernel<FMT_C128_12><<<grid, kStoutBlock, 0, stream>>>(a);
            stout_back2_kernel<FMT_C128_12><<<grid2, 2 * kStapleLinks, 0, stream>>>(a);
            return 0;
        default: return -1;
    }
}

int launch_stout(const StoutArgs &a, int fmt, hipStream_t stream) {
    const dim3 grid(stout_blocks(a.geom.Vh));
    switch (fmt) {
        case FMT_C128_18: stout_kernel<FMT_C128_18><<<grid, kStoutBlock, 0, stream>>>(a); return 0;
        case FMT_C128_12: stout_kernel<FMT_C128_12><<<grid, kStoutBlock, 0, stream>>>(a); return 0;
        default: return -1;
    }
}

int launch_momentum(const StapleArgs &a, int fmt, int threads, hipStream_t stream) {
    switch (fmt) {
        case FMT_C128_18: return launch_mom<double, FMT_C128_18>(a, threads, stream);
        case FMT_C128_12: return launch_mom<double, FMT_C128_12>(a, threads, stream);
        case FMT_C64_12: return launch_mom<float, FMT_C64_12>(a, threads, stream);
        default: return -1;
    }
}

int launch_link_update(const LinkUpdateArgs &a, int fmt, hipStream_t stream) {
    const dim3 grid((unsigned)(((size_t)8 * a.Vh + kStoutBlock - 1) / kStoutBlock));
    switch (fmt) {
        case FMT_C128_18:
            link_update_kernel<double, FMT_C128_18><<<grid, kStoutBlock, 0, stream>>>(a);
            return 0;
        case FMT_C128_12:
            link_update_kernel<double, FMT_C128_12><<<grid, kStoutBlock, 0, stream>>>(a);
            return 0;
        case FMT_C64_12:
            link_update_kernel<float, FMT_C64_12><<<grid, kStoutBlock, 0, stream>>>(a);
            return 0;
        default: return -1;
    }
}

int launch_staples(const StapleArgs &a, int fmt, int threads, hipStream_t stream) {
    switch (fmt) {
        case FMT_C128_18: return launch_tpl<double, FMT_C128_18>(a, threads, stream);
        case FMT_C128_12: return launch_tpl<double, FMT_C128_12>(a, threads, stream);
        case FMT_C64_12: return launch_tpl<float, FMT_C64_12>(a, threads, stream);
        case FMT_BF16_12: return launch_tpl<float, FMT_BF16_12>(a, threads, stream);
        default: return -1;
    }
}

}  // namespace stg
