// staple.hpp -- launch interface of the staple kernel (staple.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace stg {

// Threads per block of the staple kernel: one link per thread.
constexpr int kStapleBlock = 128;

struct StapleArgs {
    Geom geom;
    const void *links;  // gauge field in its format, slot 2*mu + parity
    void *out;          // complex T [8][3][3][Vh], T = double or float by format
    double c0, c1;      // weights of the 3-link and 5-link paths
    int xcd_remap;      // give each XCD a contiguous range of blocks
};

// Blocks of one staple launch: 8 link slots of Vh links, kStapleBlock per block.
inline uint32_t staple_blocks(uint32_t Vh) {
    return 8u * ((Vh + kStapleBlock - 1) / kStapleBlock);
}

// 0: launched; -1: unknown format (nothing launched).
int launch_staples(const StapleArgs &a, int fmt, hipStream_t stream);

}  // namespace stg
