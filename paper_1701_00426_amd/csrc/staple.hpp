// staple.hpp -- launch interface of the staple kernel (staple.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"
#include "pencil.hpp"

namespace stg {

// Links per block of the staple kernel (one wave's worth); a block has one wave
// per thread of a link.
constexpr int kStapleLinks = 64;

struct StapleArgs {
    Geom geom;
    PencilTile tile;    // visiting order of the links of a slot (pencil.hpp)
    const void *links;  // gauge field in its format, slot 2*mu + parity
    void *out;          // complex T [8][3][3][Vh], T = double or float by format
    double c0, c1;      // weights of the 3-link and 5-link paths
    double kmom;        // momentum update only: eps * beta / 3
    int xcd_remap;      // give each XCD a contiguous range of blocks
};

// Blocks of one staple launch: 8 link slots of Vh links, kStapleLinks per block.
inline uint32_t staple_blocks(uint32_t Vh) {
    return 8u * ((Vh + kStapleLinks - 1) / kStapleLinks);
}

// Threads per link the format gets by default: 2 (the two sides of the link on
// separate waves) for FP64 links, 1 for FP32 ones.
inline int staple_default_threads(int fmt) { return (fmt == FMT_C128_18 || fmt == FMT_C128_12) ? 2 : 1; }

// 0: launched; -1: unknown format or thread count (nothing launched).
int launch_staples(const StapleArgs &a, int fmt, int threads, hipStream_t stream);

// The momentum update of the pure-gauge molecular dynamics (staple.hip): the same
// staples, then P -> P + kmom [i U Sigma]_TH for every link, out = the momenta
// (complex T [8][3][3][Vh], read and written).  FP64 formats and FP32-12.
int launch_momentum(const StapleArgs &a, int fmt, int threads, hipStream_t stream);

struct LinkUpdateArgs {
    void *links;        // FP64 or FP32-12 gauge field, updated in place
    const void *mom;    // complex T [8][3][3][Vh] (complex64 for FP32-12)
    double eps;
    uint32_t Vh;
};

// U -> exp(i eps P) U for every link, in place (FP64 formats and FP32-12).
int launch_link_update(const LinkUpdateArgs &a, int fmt, hipStream_t stream);

// The force through one stout step (staple.hip), in two passes over the links:
// pass 1 writes Sigma' exp(iQ) + C^dag G^dag to out and U^dag G to ws; pass 2 adds
// rho times the gathered products of ws with the links of the 3-link paths.
struct StoutBackArgs {
    Geom geom;
    PencilTile tile;
    const void *links;  // thin FP64 gauge field
    const void *sigp;   // complex128 [8][3][3][Vh]: dS/dU' of the smeared links
    void *out;          // complex128 [8][3][3][Vh]: dS/dU of the thin links
    void *ws;           // complex128 [8][3][3][Vh]: U^dag G per link
    double rho;
    int xcd_remap;
};

// 0: both passes launched; -1: not an FP64 format (nothing launched).
int launch_stout_backprop(const StoutBackArgs &a, int fmt, hipStream_t stream);

// One stout-smearing step of every link (staple.hip): U' = exp(iQ) U.
constexpr int kStoutBlock = 128;

struct StoutArgs {
    Geom geom;
    PencilTile tile;    // visiting order of the links of a slot (pencil.hpp)
    const void *links;  // FP64 gauge field (FMT_C128_18 or FMT_C128_12)
    void *out;          // complex128 [8][3][3][Vh]
    double rho;         // weight of the six 3-link paths
    int xcd_remap;
};

inline uint32_t stout_blocks(uint32_t Vh) { return 8u * ((Vh + kStoutBlock - 1) / kStoutBlock); }

// 0: launched; -1: not an FP64 format (nothing launched).
int launch_stout(const StoutArgs &a, int fmt, hipStream_t stream);

}  // namespace stg
