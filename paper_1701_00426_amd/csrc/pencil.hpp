// pencil.hpp -- a visiting order of the sites of one parity that keeps neighbours
// in the same XCD's L2: tiles of T0 x T1 x T2 sites in (x0, x1, x2), each swept
// along x3 ("pencils"), the pencils in x0, x1, x2 order.  Kernels whose threads
// read radius-1 or radius-2 neighbourhoods walk their sites in this order, with
// each XCD on a contiguous range of it (xcd_block).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace stg {

struct PencilTile {
    uint32_t t0h, t1, t2;  // tile extents; t0h = T0 / 2 (half sites along x0)
    uint32_t nsl;          // sites of one parity in a tile layer: t0h * t1 * t2
    uint32_t np0, np1;     // tiles along x0 and x1
};

// Largest divisor of n that is at most cap and a multiple of step.
inline uint32_t pencil_extent(uint32_t n, uint32_t cap, uint32_t step) {
    for (uint32_t d = cap - cap % step; d > step; d -= step)
        if (n % d == 0) return d;
    return step;
}

// Tile shapes (caps on T0 x T1 x T2) selectable by the STG_TUNE_PENCIL_TILE knob;
// 0 is the default, 32 x 2 x 4 (the fastest of these for the staple and stout
// kernels at 32^4; 8 x 8 x 8 is much slower: 64-byte runs along x0).
constexpr int kPencilShapes = 6;
constexpr uint32_t kPencilCaps[kPencilShapes][3] = {
    {32, 2, 4}, {32, 4, 2}, {16, 4, 4}, {16, 8, 4}, {8, 8, 8}, {32, 8, 2}};

// T0 the largest even divisor of N0 up to cap 0, T1 and T2 the largest divisors of
// N1 and N2 up to caps 1 and 2 (shape: an index into kPencilCaps).
inline PencilTile pencil_tile(const Geom &g, int shape = 0) {
    PencilTile t;
    const uint32_t *cap = kPencilCaps[(shape >= 0 && shape < kPencilShapes) ? shape : 0];
    const uint32_t T0 = pencil_extent(g.N[0], cap[0], 2), T1 = pencil_extent(g.N[1], cap[1], 1);
    const uint32_t T2 = pencil_extent(g.N[2], cap[2], 1);
    t.t0h = T0 / 2;
    t.t1 = T1;
    t.t2 = T2;
    t.nsl = t.t0h * T1 * T2;
    t.np0 = g.N[0] / T0;
    t.np1 = g.N[1] / T1;
    return t;
}

// Half index of the j-th site (0 <= j < Vh) of one parity in pencil order.
__device__ __forceinline__ uint32_t pencil_site(const Geom &g, const PencilTile &t, uint32_t j) {
    const uint32_t i = j % t.nsl;
    uint32_t r = j / t.nsl;
    const uint32_t x3 = r % g.N[3];
    r /= g.N[3];
    const uint32_t p0 = r % t.np0;
    r /= t.np0;
    const uint32_t p1 = r % t.np1;
    const uint32_t p2 = r / t.np1;
    const uint32_t x0h = p0 * t.t0h + i % t.t0h;
    const uint32_t x1 = p1 * t.t1 + (i / t.t0h) % t.t1;
    const uint32_t x2 = p2 * t.t2 + i / (t.t0h * t.t1);
    return x0h + g.nh0 * (x1 + g.N[1] * (x2 + g.N[2] * x3));
}

}  // namespace stg
