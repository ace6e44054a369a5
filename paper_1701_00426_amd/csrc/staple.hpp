// staple.hpp -- launch interface of the staple kernel (staple.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace stg {

// Links per block of the staple kernel (one wave's worth); a block has one wave
// per thread of a link.
constexpr int kStapleLinks = 64;

// Order in which the links of one slot are visited: tiles of t0h half-sites (x0)
// x t1 (x1) x t2 (x2), each swept along x3 ("pencils"), the pencils in x0, x1, x2
// order.  Consecutive blocks cover consecutive links of this order.
struct StapleTile {
    uint32_t t0h, t1, t2;  // tile extents; t0h = T0 / 2
    uint32_t nsl;          // sites of one parity in a tile layer: t0h * t1 * t2
    uint32_t np0, np1;     // tiles along x0 and x1
};

struct StapleArgs {
    Geom geom;
    StapleTile tile;
    const void *links;  // gauge field in its format, slot 2*mu + parity
    void *out;          // complex T [8][3][3][Vh], T = double or float by format
    double c0, c1;      // weights of the 3-link and 5-link paths
    int xcd_remap;      // give each XCD a contiguous range of blocks
};

// The tile of a lattice: T0 the largest even divisor of N0 up to 32, T1 and T2 the
// largest divisors of N1 and N2 up to 4 and 2.
StapleTile staple_tile(const Geom &g);

// Blocks of one staple launch: 8 link slots of Vh links, kStapleLinks per block.
inline uint32_t staple_blocks(uint32_t Vh) {
    return 8u * ((Vh + kStapleLinks - 1) / kStapleLinks);
}

// Threads per link the format gets by default: 2 (the two sides of the link on
// separate waves) for FP64 links, 1 for FP32 ones.
inline int staple_default_threads(int fmt) { return (fmt == FMT_C128_18 || fmt == FMT_C128_12) ? 2 : 1; }

// 0: launched; -1: unknown format or thread count (nothing launched).
int launch_staples(const StapleArgs &a, int fmt, int threads, hipStream_t stream);

}  // namespace stg
