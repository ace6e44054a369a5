// batch.hpp -- tables of the uneven-batch CG (many lattices per launch).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"
#include "solver_state.hpp"

namespace stg {

// One solve of the batch: its lattice, gauge fields and Krylov fields.
struct BSolve {
    Geom g;
    const void *hi_links;
    const void *hi_phases;
    const void *lo_links;
    const void *lo_phases;
    const void *b;   // complex128 [nrhs][3][Vh]
    void *x64;       // complex128 [nrhs][3][Vh]: the caller's x
    void *xin;       // inner-precision solution (the caller's x in FP64 mode)
    void *p, *r, *q, *t;  // inner precision (q holds w = A r in the single-reduction form)
    void *s;              // inner precision: s = A p of the single-reduction form
    void *r64, *t64;      // FP64 residual and odd temporary (aliases in FP64 mode)
    uint32_t sys0;   // global index of its first system
    uint32_t nblk;   // blocks of kBlock sites
    uint32_t part0;  // first partial slot group of this solve (see kTileSlots)
    uint32_t nrhs;
};

// Partial sums: every tile holds kTileSlots (sum, error) pairs per system, pair
// ((part0 + j * nblk + blk) * kTileSlots + slot).  The hop launches a tile as tps
// blocks, one per pass of kBlock / tps sites, and pass k writes slot k; the vector
// kernels write slot 0.  The writer of slot 0 also zeroes the slots no block of its
// launch owns, so the finalize sums all kTileSlots * nblk pairs of a system.
constexpr int kTileSlots = 4;

// kBlock consecutive sites (block blk) of one solve for systems j0 .. j0+nr-1.  The
// hop kernel works on a tile with tps threads per site (1, 2 or 4; the directions of
// a site shared as in hop_split.hip), as tps blocks of kBlock / tps sites each.
struct BTile {
    uint32_t solve;
    uint32_t blk;
    uint16_t j0;
    uint8_t nr;   // 1 to 4
    uint8_t tps;  // threads per site of the hop
};

struct BSysRef {
    uint32_t solve;
    uint32_t j;
};

enum BField { BF_X64 = 0, BF_XIN, BF_P, BF_R, BF_Q, BF_T, BF_R64, BF_T64, BF_B };

struct BArgs {
    const BSolve *solves;
    const BTile *tiles;
    const BSysRef *sysref;
    SysState *state;  // [nsys]
    Ctl *ctl;
    double *partials;
    double *partials2;  // single-reduction form: the update's |r|^2, same slot layout
    uint32_t ntiles;  // end of the tile range the kernel walks
    uint32_t tile0;   // its first tile (the hop launches one range per tile class)
    uint32_t nsys;
    uint32_t grid;    // blocks of the launch (at most one per tile, or per tile pass)
    int out_parity;
    int use_hi;       // hop on the FP64 gauge field (true residual) or the inner one
    int gate_running;     // exit at once when ctl->n_running == 0
    int tile_mask;        // work on a tile only when one of its systems has one of these flags
    int f_in, f_out, f_aux0;  // BField selectors of the hop operands
    int skip_p;           // resume kernel: rebuild r only (the single-reduction update applies
                          // beta to p and s itself)

    __device__ __forceinline__ const void *field(const BSolve &S, int f) const {
        switch (f) {
            case BF_X64: return S.x64;
            case BF_XIN: return S.xin;
            case BF_P: return S.p;
            case BF_R: return S.r;
            case BF_Q: return S.q;
            case BF_T: return S.t;
            case BF_R64: return S.r64;
            case BF_T64: return S.t64;
            default: return S.b;
        }
    }
};

// Tiles of one class (fields per tile, threads per site, standard or stored phases
// on the inner and on the FP64 gauge field) sit in one contiguous range of the tile
// table; the hop runs one launch per class, so each launch holds only the registers
// its own tile shape needs.
struct BClass {
    uint32_t begin, end;
    int nr, tps;
    int std_lo, std_hi;  // 1: the class's solves have standard phases (no phase array)
};
int launch_bhop(const BArgs &a, const BClass *cls, int ncls, int fmt, int epi, hipStream_t s);
int launch_bfinalize(const BArgs &a, int op, hipStream_t s);
int launch_bcg_update(const BArgs &a, int fp64, hipStream_t s);
int launch_bp_update(const BArgs &a, int fp64, hipStream_t s);
// single-reduction form: p = r + beta p, s = w + beta s, x += alpha p, r -= alpha s and
// the |r|^2 partials (into partials2) of every running system
int launch_bcgcg_update(const BArgs &a, int fp64, hipStream_t s);
int launch_bru_accumulate(const BArgs &a, hipStream_t s);
int launch_bru_resume(const BArgs &a, int fp64, hipStream_t s);
int launch_bnorm_b(const BArgs &a, hipStream_t s);

}  // namespace stg
