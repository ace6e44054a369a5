// force.hpp -- launch interface of the fermion-force kernel (force.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"
#include "pencil.hpp"

namespace stg {

constexpr int kForceBlock = 256;  // sites per block (one parity)
constexpr int kForceChunk = 32;   // poles per launch (their weights travel in the arguments)

struct ForceArgs {
    Geom geom;
    PencilTile tile;        // visiting order of the sites of a parity (pencil.hpp)
    const void *x;          // complex128 [npoles][3][Vh], even sites
    const void *y;          // complex128 [npoles][3][Vh], odd sites
    const double *phases;   // real [8][Vh], or NULL for the standard phases
    void *out;              // complex128 [8][3][3][Vh]
    double coeff[kForceChunk];
    int npoles;             // 1 .. kForceChunk
    int accumulate;         // add to out instead of overwriting it
    int xcd_remap;
};

inline uint32_t force_blocks(uint32_t Vh) { return 2u * ((Vh + kForceBlock - 1) / kForceBlock); }

void launch_force(const ForceArgs &a, hipStream_t stream);

}  // namespace stg
