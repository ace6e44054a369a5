// device_common.hpp -- device-side building blocks shared by the library's kernels:
// complex arithmetic, gauge-link loads in every storage format (with the SU(3)
// third-row rebuild), lattice site geometry, and deterministic block reductions.
//
// Paper: arXiv:1701.00426.  Sec. 2.3 (store two rows of each SU(3) link and rebuild
// the third as the conjugate of their cross product), Sec. 4.1 (structure of arrays,
// half-lattice index of Eq. lexicographic_eo, gauge field as 8 su3_soa slots).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stg {

constexpr int kBlock = 256;            // threads per block of every site kernel
constexpr int kWaves = kBlock / 64;    // wave64

// ---------------------------------------------------------------------------
// complex arithmetic on (re, im) pairs
// ---------------------------------------------------------------------------
template <typename T>
struct cpx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> cmake(T r, T i) { return cpx<T>{r, i}; }

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }

template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }

template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// conj(a) * b
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

template <typename T>
__device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return {a.re, -a.im}; }

template <typename T>
__device__ __forceinline__ cpx<T> cscale(T s, cpx<T> a) { return {s * a.re, s * a.im}; }

// fused multiply-add a * b + c with one rounding
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// acc += a * b as four fused multiply-adds into the accumulator (written out: the
// compiler would otherwise form the product first and add it, six operations)
template <typename T>
__device__ __forceinline__ void cfma(cpx<T> &acc, cpx<T> a, cpx<T> b) {
    acc.re = fmat(a.re, b.re, acc.re);
    acc.re = fmat(-a.im, b.im, acc.re);
    acc.im = fmat(a.re, b.im, acc.im);
    acc.im = fmat(a.im, b.re, acc.im);
}

// acc += conj(a) * b
template <typename T>
__device__ __forceinline__ void cfmac(cpx<T> &acc, cpx<T> a, cpx<T> b) {
    acc.re = fmat(a.re, b.re, acc.re);
    acc.re = fmat(a.im, b.im, acc.re);
    acc.im = fmat(a.re, b.im, acc.im);
    acc.im = fmat(-a.im, b.re, acc.im);
}

template <typename T>
struct vec3 {
    cpx<T> c[3];
};

template <typename T>
struct su3 {
    cpx<T> e[3][3];
};

// ---------------------------------------------------------------------------
// field element access: interleaved complex, layout [nrhs][3][Vh]
// ---------------------------------------------------------------------------
template <typename T>
struct field_traits;

template <>
struct field_traits<double> {
    using pair = double2;
};

template <>
struct field_traits<float> {
    using pair = float2;
};

template <typename T>
__device__ __forceinline__ cpx<T> ld_c(const void *base, size_t idx) {
    using P = typename field_traits<T>::pair;
    P v = reinterpret_cast<const P *>(base)[idx];
    return {v.x, v.y};
}

template <typename T>
__device__ __forceinline__ void st_c(void *base, size_t idx, cpx<T> v) {
    using P = typename field_traits<T>::pair;
    P p;
    p.x = v.re;
    p.y = v.im;
    reinterpret_cast<P *>(base)[idx] = p;
}

// colour vector at site h of field j: entries (j*3 + c)*Vh + h
template <typename T>
__device__ __forceinline__ vec3<T> ld_v(const void *base, size_t fstride, uint32_t Vh, int j,
                                        uint32_t h) {
    vec3<T> v;
    size_t o = (size_t)j * fstride + h;
#pragma unroll
    for (int c = 0; c < 3; ++c) v.c[c] = ld_c<T>(base, o + (size_t)c * Vh);
    return v;
}

template <typename T>
__device__ __forceinline__ void st_v(void *base, size_t fstride, uint32_t Vh, int j, uint32_t h,
                                     const vec3<T> &v) {
    size_t o = (size_t)j * fstride + h;
#pragma unroll
    for (int c = 0; c < 3; ++c) st_c<T>(base, o + (size_t)c * Vh, v.c[c]);
}

// FP64 colour vector stored with non-temporal stores (streamed past the caches):
// the hop's plain output is not re-read by the same launch.
__device__ __forceinline__ void st_v_nt(void *base, size_t fstride, uint32_t Vh, int j,
                                        uint32_t h, const vec3<double> &v) {
    typedef double sd2 __attribute__((ext_vector_type(2)));
    sd2 *p = reinterpret_cast<sd2 *>(base) + (size_t)j * fstride + h;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        sd2 w = {v.c[c].re, v.c[c].im};
        __builtin_nontemporal_store(w, p + (size_t)c * Vh);
    }
}

// ---------------------------------------------------------------------------
// gauge links: formats of the C ABI, slot s = 2*mu + parity
// ---------------------------------------------------------------------------
enum LinkFmt { FMT_C128_18 = 0, FMT_C128_12 = 1, FMT_C64_12 = 2, FMT_BF16_12 = 3 };

// row 2 of an SU(3) matrix from rows 0 and 1: conj(row0 x row1)
template <typename T>
__device__ __forceinline__ void rebuild_row2(su3<T> &u) {
    const cpx<T> *a = u.e[0];
    const cpx<T> *b = u.e[1];
    u.e[2][0] = cconj(csub(cmul(a[1], b[2]), cmul(a[2], b[1])));
    u.e[2][1] = cconj(csub(cmul(a[2], b[0]), cmul(a[0], b[2])));
    u.e[2][2] = cconj(csub(cmul(a[0], b[1]), cmul(a[1], b[0])));
}

// native clang vectors (the nontemporal builtin does not take HIP's vector structs)
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf4 __attribute__((ext_vector_type(4)));
typedef uint32_t nu4 __attribute__((ext_vector_type(4)));
typedef uint32_t nu2 __attribute__((ext_vector_type(2)));

template <typename V>
__device__ __forceinline__ V nt_load(const void *p, size_t idx) {
    return __builtin_nontemporal_load(reinterpret_cast<const V *>(p) + idx);
}

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

template <typename T, int FMT>
struct link_loader;

template <>
struct link_loader<double, FMT_C128_18> {
    __device__ __forceinline__ static su3<double> load(const void *L, uint32_t Vh, int s,
                                                        uint32_t h) {
        su3<double> u;
        const size_t base = (size_t)s * 9 * Vh + h;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                nd2 v = nt_load<nd2>(L, base + (size_t)(a * 3 + b) * Vh);
                u.e[a][b] = {v.x, v.y};
            }
        return u;
    }
};

template <>
struct link_loader<double, FMT_C128_12> {
    __device__ __forceinline__ static su3<double> load(const void *L, uint32_t Vh, int s,
                                                        uint32_t h) {
        su3<double> u;
        const size_t base = (size_t)s * 6 * Vh + h;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                nd2 v = nt_load<nd2>(L, base + (size_t)(a * 3 + b) * Vh);
                u.e[a][b] = {v.x, v.y};
            }
        rebuild_row2(u);
        return u;
    }
};

template <>
struct link_loader<float, FMT_C64_12> {
    __device__ __forceinline__ static su3<float> load(const void *L, uint32_t Vh, int s,
                                                       uint32_t h) {
        su3<float> u;
        const size_t base = (size_t)s * 3 * Vh + h;
        nf4 c0 = nt_load<nf4>(L, base);
        nf4 c1 = nt_load<nf4>(L, base + Vh);
        nf4 c2 = nt_load<nf4>(L, base + 2 * (size_t)Vh);
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
struct link_loader<float, FMT_BF16_12> {
    __device__ __forceinline__ static su3<float> load(const void *L, uint32_t Vh, int s,
                                                       uint32_t h) {
        su3<float> u;
        const void *Lb = reinterpret_cast<const nu4 *>(L) + (size_t)8 * Vh;
        nu4 a = nt_load<nu4>(L, (size_t)s * Vh + h);
        nu2 b = nt_load<nu2>(Lb, (size_t)s * Vh + h);
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

// y += s * U v
template <typename T>
__device__ __forceinline__ void acc_mv(vec3<T> &y, T s, const su3<T> &u, const vec3<T> &v) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cpx<T> t = cmul(u.e[a][0], v.c[0]);
        cfma(t, u.e[a][1], v.c[1]);
        cfma(t, u.e[a][2], v.c[2]);
        y.c[a].re = fmat(s, t.re, y.c[a].re);
        y.c[a].im = fmat(s, t.im, y.c[a].im);
    }
}

// y += s * U^dag v
template <typename T>
__device__ __forceinline__ void acc_mdv(vec3<T> &y, T s, const su3<T> &u, const vec3<T> &v) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cpx<T> t = cmulc(u.e[0][a], v.c[0]);
        cfmac(t, u.e[1][a], v.c[1]);
        cfmac(t, u.e[2][a], v.c[2]);
        y.c[a].re = fmat(s, t.re, y.c[a].re);
        y.c[a].im = fmat(s, t.im, y.c[a].im);
    }
}

// ---------------------------------------------------------------------------
// lattice geometry (Sec. 4.1, Eq. lexicographic_eo)
// ---------------------------------------------------------------------------
struct Geom {
    uint32_t N[4];
    uint32_t nh0;       // N0 / 2
    uint32_t Vh;        // V / 2
    uint32_t stride[4]; // half-index step of x_mu -> x_mu + 1 for mu >= 1 (stride[0] unused)
};

struct Site {
    uint32_t x[4];
};

__device__ __forceinline__ Site site_coords(const Geom &g, int parity, uint32_t h) {
    Site s;
    uint32_t x0h = h % g.nh0;
    uint32_t t = h / g.nh0;
    s.x[1] = t % g.N[1];
    t /= g.N[1];
    s.x[2] = t % g.N[2];
    s.x[3] = t / g.N[2];
    s.x[0] = 2 * x0h + ((parity + s.x[1] + s.x[2] + s.x[3]) & 1);
    return s;
}

// half index of x + mu (fwd) or x - mu, for the site x with half index h
__device__ __forceinline__ uint32_t nb_fwd(const Geom &g, const Site &s, uint32_t h, int mu) {
    if (mu == 0) {
        uint32_t base = h - (s.x[0] >> 1);
        uint32_t xn = s.x[0] + 1;
        return base + ((xn == g.N[0]) ? 0u : (xn >> 1));
    }
    return (s.x[mu] + 1 == g.N[mu]) ? h - (g.N[mu] - 1) * g.stride[mu] : h + g.stride[mu];
}

__device__ __forceinline__ uint32_t nb_bwd(const Geom &g, const Site &s, uint32_t h, int mu) {
    if (mu == 0) {
        uint32_t base = h - (s.x[0] >> 1);
        return base + ((s.x[0] == 0) ? (g.N[0] - 1) >> 1 : (s.x[0] - 1) >> 1);
    }
    return (s.x[mu] == 0) ? h + (g.N[mu] - 1) * g.stride[mu] : h - g.stride[mu];
}

// standard staggered phase of the link U_mu(x): eta_mu(x), times -1 when mu = 3
// and x3 = N3 - 1 (antiperiodic in time)
__device__ __forceinline__ float std_phase(const Geom &g, const Site &s, int mu, bool backward) {
    uint32_t e = 0;
    if (mu >= 1) e += s.x[0];
    if (mu >= 2) e += s.x[1];
    if (mu >= 3) e += s.x[2];
    bool neg = (e & 1u) != 0;
    if (mu == 3) {
        // forward link leaves x; backward link leaves x - 3 (x3 - 1, wrapped)
        bool edge = backward ? (s.x[3] == 0) : (s.x[3] == g.N[3] - 1);
        neg ^= edge;
    }
    return neg ? -1.0f : 1.0f;
}

// ---------------------------------------------------------------------------
// deterministic reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// error-free transformation: a + b = s + e exactly (Knuth TwoSum)
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// (s, c) += (s2, c2) for compensated (sum, error) pairs
__device__ __forceinline__ void pair_add(double &s, double &c, double s2, double c2) {
    double e;
    two_sum(s, s2, s, e);
    c += c2 + e;
}

// Compensated block sum of per-thread (s, c) pairs in a fixed order (wave64
// shuffle tree, then the four waves in order); the pair is valid in thread 0.
// scratch: 2 * kWaves doubles of shared memory.
__device__ __forceinline__ void block_sum_pair(double &s, double &c, double *scratch) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double s2 = __shfl_down(s, off, 64);
        double c2 = __shfl_down(c, off, 64);
        pair_add(s, c, s2, c2);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        scratch[2 * wave] = s;
        scratch[2 * wave + 1] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s = scratch[0];
        c = scratch[1];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) pair_add(s, c, scratch[2 * w], scratch[2 * w + 1]);
    }
    __syncthreads();
}

// Compensated sum (Ogita-Rump-Oishi Sum2 order) of n (sum, error) pairs stored
// interleaved at x, by the whole block; result valid in thread 0.  Fixed order:
// thread t takes pairs t, t+B, ... (loads unrolled so several are in flight),
// then the fixed tree of block_sum_pair.  scratch: 2 * kWaves doubles of LDS.
__device__ __forceinline__ double block_sum2_pairs(const double *x, int n, double *scratch) {
    double s = 0.0, c = 0.0;
#pragma unroll 8
    for (int i = threadIdx.x; i < n; i += kBlock) pair_add(s, c, x[2 * i], x[2 * i + 1]);
    block_sum_pair(s, c, scratch);
    return s + c;
}

}  // namespace stg
