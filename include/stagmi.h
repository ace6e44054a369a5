/*
 * stagmi.h -- C ABI of the MI355X (gfx950) staggered-fermion library.
 *
 * The library applies the even/odd staggered Dirac operator and solves the
 * even/odd normal equations with it, on one GPU, in hand-written HIP kernels; it
 * also computes the gauge-force staples and the fermion force from the solutions.
 *
 * Paper: C. Bonati et al., "Design and optimization of a portable LQCD Monte
 * Carlo code using OpenACC", arXiv:1701.00426.
 *   - Sec. 2.2, Eq. diracblock: M = m + [[0, D_oe], [D_eo, 0]], D_oe^dag = -D_eo;
 *     the blocks connect only even and odd sites.
 *   - Sec. 2.2, Eq. lineqeo: (m^2 - D_eo D_oe) phi_e = b_e on even sites, Hermitian
 *     positive definite, solved by conjugate gradient.
 *   - Sec. 2.2, Eq. shlineq: shifted systems (M + sigma_i) phi_i = b for the poles
 *     of the rational approximation, all solved with one operator application
 *     per iteration (multi-shift CG).
 *   - Sec. 2.3: SU(3) links stored as their first two rows, the third rebuilt
 *     as the complex conjugate of the cross product of the first two.
 *   - Sec. 4.1: structure-of-arrays layouts (vec3_soa fields, gauge field as an
 *     array of 8 su3_soa), half-lattice site index of Eq. lexicographic_eo.
 *   - Sec. 4.3, deo listing: the operator reads links, an input field, a real
 *     per-link factor array ("backfield") and writes an output field.
 *   - Sec. 2.1 and Sec. 4.3 (gauge cycle): staples of the tree-level Symanzik
 *     gauge action, products of 3 and 5 links along C-shaped paths.
 *   - Sec. 2.2: molecular-dynamics forces from the multi-shift solutions (the
 *     derivative of the rational pseudofermion action with respect to the links).
 *   - Sec. 2.1 and Sec. 2.3: stout-smeared links (one smearing step per call).
 *   - Sec. 4.3 and Table 4: the pure-gauge molecular-dynamics step (gauge force
 *     from the staples, momentum and link updates).
 *
 * Conventions used by every call
 * ------------------------------
 *  Lattice: extents N0..N3, each even and >= 2; x0 runs fastest; the time
 *    direction is x3.  V = N0 N1 N2 N3, Vh = V / 2.  A site x has parity
 *    (x0+x1+x2+x3) mod 2 (0 = even) and half-lattice index
 *    h(x) = floor((x0 + N0 (x1 + N1 (x2 + N2 x3))) / 2), a bijection onto
 *    [0, Vh) for each parity.
 *  Operator: (D psi)(x) = 1/2 sum_mu [ phi_mu(x) U_mu(x) psi(x+mu)
 *                                     - phi_mu(x-mu) U_mu(x-mu)^dag psi(x-mu) ]
 *    with periodic index wrap.  D_eo maps a field on odd sites to even sites,
 *    D_oe maps even to odd.  The normal operator is
 *    A_sigma = (m^2 + sigma) - D_eo D_oe on even sites.
 *  Phases phi_mu(x): real.  With a NULL phase pointer the library uses the
 *    standard staggered phases eta_mu(x) = (-1)^(x0+...+x_{mu-1}) times -1 on the
 *    links leaving x3 = N3-1 (antiperiodic time boundary), computed in the
 *    kernel without reading memory.  Otherwise phases point to a real array
 *    [8][Vh], entry (2*mu + parity(x))*Vh + h(x) = phi_mu(x); its element type
 *    is double for STG_LINK_C128_* gauge fields and float for the others.
 *  Fields: interleaved complex (re, im), layout [nrhs][3][Vh] (colour, then
 *    site), element complex128 (STG_C128) or complex64 (STG_C64).
 *  Gauge field formats (slot s = 2*mu + parity of the link's start site x):
 *    STG_LINK_C128_18  complex128 [8][3][3][Vh]  row, column, site (full matrix)
 *    STG_LINK_C128_12  complex128 [8][2][3][Vh]  rows 0 and 1 only
 *    STG_LINK_C64_12   float4     [8][3][Vh]     chunk k of a link holds the
 *                      complex64 entries 2k and 2k+1 of (U00 U01 U02 U10 U11 U12)
 *    STG_LINK_BF16_12  [8][Vh] x 16 bytes, then [8][Vh] x 8 bytes: bfloat16
 *                      (re, im) of U00 U01 U02 U10 in the first array and of
 *                      U11 U12 in the second
 *    The 12-real formats rebuild row 2 as conj(row0 x row1): links must be SU(3).
 *    Only STG_LINK_C128_* may be used with STG_C128 fields and only
 *    STG_LINK_C64_12 / STG_LINK_BF16_12 with STG_C64 fields (compute in FP32).
 *
 * Memory ownership: every buffer argument marked "device" is a device pointer
 * owned by the caller; the library allocates no device memory (apart from the
 * fixed scratch array of stg_apply_normal_noalloc, loaded with its code object)
 * and keeps no pointer after a call returns.  Solvers take a caller-owned device workspace
 * whose size comes from stg_workspace_bytes.  Arguments marked "host" are host
 * memory.  Device buffers must be 16-byte aligned; an input and an output
 * buffer of one call must not overlap.
 *
 * Streams: stg_stream_t is a hipStream_t (NULL = the default stream).  The
 * operator and packing calls only enqueue work and return; the solvers enqueue
 * on the stream and return after it has drained, because they report
 * convergence in host memory.
 *
 * Errors: every call returns an int status (below).  No call aborts the process
 * or lets an exception cross the ABI; stg_status_string gives the text.
 */
#ifndef STAGMI_H
#define STAGMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *stg_stream_t; /* a hipStream_t */

enum {
    STG_OK = 0,
    STG_NOT_CONVERGED = 1,      /* iteration cap reached; x holds the last iterate */
    STG_BREAKDOWN = 2,          /* non-finite scalar or <p, A p> <= 0 */
    STG_INVALID_ARG = -1,       /* bad extent, null or misaligned pointer, overlap, bad count */
    STG_HIP_ERROR = -2,         /* a HIP runtime call failed */
    STG_WORKSPACE_TOO_SMALL = -3
};

typedef struct { int32_t dims[4]; } stg_lattice;

typedef enum {
    STG_LINK_C128_18 = 0,
    STG_LINK_C128_12 = 1,
    STG_LINK_C64_12 = 2,
    STG_LINK_BF16_12 = 3
} stg_link_fmt;

typedef enum { STG_C128 = 0, STG_C64 = 1 } stg_field;

typedef struct {
    const void *links;   /* device, layout given by fmt */
    stg_link_fmt fmt;
    const void *phases;  /* device real [8][Vh], or NULL for the standard phases */
} stg_gauge;

/* Library version, (major << 16) | minor. */
int stg_version(void);

/* Text of a status code; never NULL. */
const char *stg_status_string(int status);

/* Last HIP error text seen by the library on this thread (empty if none). */
const char *stg_last_error(void);

/*
 * Launch-shape choices of the hop and staple kernels, process-wide (results do not depend
 * on them, only the speed).  Set them before launching work; calls that are in
 * flight keep the choice they were launched with.
 *   STG_TUNE_XCD_REMAP: 1 (default) maps the blocks that run on one XCD of the
 *     chip to one contiguous range of sites, so neighbour field lines meet in
 *     that XCD's L2; 0 keeps the plain block order.
 *   STG_TUNE_SITES_PER_THREAD: 1 (default), 2, 4 or 8 output sites per thread
 *     (a block covers that many consecutive 256-site chunks): fewer, longer
 *     blocks, to balance the last wave of blocks against the chip's capacity.
 *   STG_TUNE_STAGE_NEIGHBOURS: 0 (default) or 1: each block first copies the input
 *     field over its sites and one x1 row on either side into LDS and reads the x0
 *     and x1 neighbours from there (one or two fields per launch, N0 <= 128).
 *   STG_TUNE_THREADS_PER_SITE: 0 (default: automatic), 1, 2 or 4: the four
 *     directions of a site are shared by that many threads, whose partial sums
 *     meet in LDS (with 2 or 4, sites per thread and staging do not apply; 4 is
 *     not built for FP64 links with 8 fields per launch, which then take one
 *     thread per site).  Automatic: by link format, fields per launch, epilogue
 *     and size (one field: 4 when Vh < 16384, else 1, or 4 for the plain BF16-12
 *     hop; two to four fields: 4; eight fields: 4 for the plain FP32 / BF16 hop,
 *     else 2).  An
 *     autotuned shape sets it for the plain hop only.  The choice changes the
 *     order of floating-point additions, so results may differ in the last bits
 *     between choices (each choice is deterministic).
 *   STG_TUNE_STAPLE_THREADS: 0 (default: automatic), 1 or 2 threads per link in
 *     gauge_staples; with 2 the paths above and below the link run on separate
 *     waves and meet in LDS.  Automatic: 2 for FP64 links, 1 for FP32 / BF16
 *     ones.  Like the threads per site, it changes the order of additions.
 *     STG_TUNE_XCD_REMAP applies to gauge_staples too.
 *   STG_TUNE_PENCIL_TILE: 0 (default) .. 5: the tile of the order in which
 *     gauge_staples, stout_smear and fermion_force visit the sites: tiles of
 *     T0 x T1 x T2 sites in (x0, x1, x2), each swept along x3; the caps on
 *     (T0, T1, T2) are 0: 32x2x4, 1: 32x4x2, 2: 16x4x4, 3: 16x8x4, 4: 8x8x8,
 *     5: 32x8x2 (each extent the largest divisor of the lattice's within its cap).
 *     Only the speed depends on it.
 *   STG_TUNE_FIELDS_PER_LAUNCH: 0 (default: the autotuner's choice for the lattice
 *     and link format, else 8), 1, 2, 4 or 8: the most fields one hop launch takes
 *     when a call works on several (dirac_apply_*, stg_apply_normal, fermion_force,
 *     cg_solve, multishift_cg_solve, rational_apply; cg_solve_batch keeps its own
 *     tiles of at most 4 fields); more fields share each link read, fewer keep fewer
 *     registers and partial sums per thread.  Only the speed depends on it.
 *   STG_TUNE_LAYER_GROUP: 0 (default) or G in 1 .. 1024: the order in which the hop
 *     kernels hand output sites to blocks.  0: half-index order.  G: layer order,
 *     a layer being one (x2, x3) plane of N0/2 * N1 sites, visited in groups of G'
 *     consecutive x3 planes (G' the largest divisor of N3 not above G; none above 1
 *     keeps half-index order), x3 fastest within a group, then x2: a site's x3
 *     neighbours are read one layer, not one x3 plane, apart, so the input fields
 *     of several fields per launch stay in L2 between their reads.  Not applied
 *     with LDS neighbour staging.  It changes which sites share a block, so the
 *     order of additions in the reductions (not the operator) may change.  With 0,
 *     launches that take the field split automatically (STG_TUNE_FIELD_SPLIT) use
 *     G = 4.
 *   STG_TUNE_SPREAD_EPILOGUE: 0 (default) or 1: with 2 or 4 threads per site and a
 *     number of fields per launch that is a multiple of it, every thread group adds
 *     the partial sums of its share of the fields and runs their epilogue (the
 *     same additions in the same order as when group 0 finishes every field, so
 *     the results are identical).  Only the speed depends on it.
 *   STG_TUNE_FIELD_SPLIT: 0 (default: automatic), -1 (off) or F in 1, 2: a hop
 *     launch with 2, 3, 4 or 8 fields and 12-real links runs with the fields split
 *     over the waves of a block, F fields per wave (F must divide the fields of the
 *     launch), 64 sites per block: each wave sums all four directions of its fields,
 *     and the block reads its sites' links from memory once into LDS, where every
 *     wave reads them.  F takes precedence over STG_TUNE_THREADS_PER_SITE for such
 *     launches.  Automatic, when STG_TUNE_THREADS_PER_SITE is automatic too: launches
 *     of 8 fields take F = 1 with FP64-12 links and F = 2 with FP32-12 / BF16-12
 *     links; other launches keep the threads per site.  It changes the order of
 *     additions, so results may differ in the last bits.
 *   STG_TUNE_CG_FORM: 0 (default: automatic: form 2 for a solve of one field, else
 *     form 1), 1 or 2: the form of
 *     the CG iteration of cg_solve, cg_solve_batch and of the refinement stage of
 *     multishift_cg_solve / rational_apply.  1: the classic iteration of Sec. 2.2
 *     (<p, A p> -> alpha, then |r|^2 -> beta: two global reductions per iteration).
 *     2: the single-reduction form of Chronopoulos and Gear (w = A r; |r|^2 and
 *     <r, w> -> alpha and beta together; s = A p kept by recurrence), the same
 *     iterates in exact arithmetic with one reduction and fewer launches per
 *     iteration; the convergence test of an update runs one iteration later.
 *     Results differ from form 1 by rounding; both reach the requested true residual.
 * Returns STG_INVALID_ARG for an unknown key or value.
 */
enum {
    STG_TUNE_XCD_REMAP = 0,
    STG_TUNE_SITES_PER_THREAD = 1,
    STG_TUNE_STAGE_NEIGHBOURS = 2,
    STG_TUNE_THREADS_PER_SITE = 3,
    STG_TUNE_STAPLE_THREADS = 4,
    STG_TUNE_PENCIL_TILE = 5,
    STG_TUNE_FIELDS_PER_LAUNCH = 6,
    STG_TUNE_LAYER_GROUP = 7,
    STG_TUNE_SPREAD_EPILOGUE = 8,
    STG_TUNE_FIELD_SPLIT = 9,
    STG_TUNE_CG_FORM = 10
};
int stg_set_tuning(int key, int value);
int stg_get_tuning(int key, int *value);

/*
 * Autotuner of the hop launch shape (the run-time counterpart of the paper's
 * per-architecture compile-time tile sizes, Sec. 4.3 TILE0..2 and Sec. 5).
 * stg_autotune times every candidate shape (XCD remap on/off x [one thread per
 * site with 1, 2, 4, 8 chunks per block and LDS neighbour staging off/on where it
 * applies, or 2 / 4 threads per site]) of D_eo on the caller's gauge field and
 * fields (in: device
 * [nrhs][3][Vh] on odd sites; out: device, overwritten), keeps the fastest for
 * the key (lattice extents, gauge format, fields per launch = the largest chunk
 * of nrhs among 8, 4, 3, 2, 1) in a process-wide table that every later hop launch
 * with that key uses, and, when cache_path is not NULL, appends it to that file as
 * one JSON object per line.  With nrhs >= 2 it then times D_eo of all nrhs fields
 * chunked at most 8, 4, 2 or 1 fields per launch (the RHS per block; each chunk in
 * its stored or default shape) and keeps, per (lattice extents, gauge format), the
 * cap with the least time per field: every later multi-field hop, normal-operator
 * apply and solver on that lattice and format (cg_solve_batch aside) chunks its
 * fields by it (unless STG_TUNE_FIELDS_PER_LAUNCH is set), and it is appended to the
 * cache file too.
 * Synchronous.  stg_autotune_load reads such a file into the tables (later lines
 * win) and reports the entries read in *loaded.  stg_autotune_lookup returns STG_OK
 * and the stored shape, stg_autotune_fields_lookup the stored fields per launch, or
 * STG_NOT_CONVERGED when the key has no entry.  stg_autotune_clear empties both
 * tables.
 */
int stg_autotune(const stg_lattice *lat, const stg_gauge *gauge, stg_field field, int nrhs,
                 const void *in, void *out, const char *cache_path, stg_stream_t stream);
int stg_autotune_load(const char *cache_path, int *loaded);
typedef struct {
    int xcd_remap;
    int sites_per_thread;
    int stage_neighbours;
    int threads_per_site;
    double us;          /* measured duration of one D_eo with this shape */
} stg_tune_choice;
int stg_autotune_lookup(const stg_lattice *lat, stg_link_fmt fmt, int nr,
                        stg_tune_choice *choice);
int stg_autotune_fields_lookup(const stg_lattice *lat, stg_link_fmt fmt, int *fields_per_launch);
void stg_autotune_clear(void);

/* Bytes of a gauge field of format fmt on lattice lat, written to *bytes (host). */
int stg_links_bytes(const stg_lattice *lat, stg_link_fmt fmt, size_t *bytes);

/*
 * Converts a full complex128 gauge field [8][3][3][Vh] (device) into format
 * dst_fmt at dst (device, stg_links_bytes bytes).  Conversions round to
 * nearest even.  Sec. 2.3 / Sec. 4.1: only rows 0 and 1 are kept by the 12-real
 * formats.  Asynchronous on stream.
 */
int stg_pack_links(const stg_lattice *lat, const void *links_c128_18, stg_link_fmt dst_fmt,
                   void *dst, stg_stream_t stream);

/*
 * Converts real phases [8][Vh] double (device) to element type dst (STG_C128:
 * double copy, STG_C64: float) at dst (device).  Asynchronous on stream.
 */
int stg_pack_phases(const stg_lattice *lat, const double *phases_f64, stg_field dst, void *dst_ptr,
                    stg_stream_t stream);

/*
 * out_even = D_eo in_odd for nrhs fields (Sec. 2.2 Eq. diracblock; Sec. 4.3 deo).
 * in_odd, out_even: device [nrhs][3][Vh] of element type field.  Asynchronous.
 */
int dirac_apply_eo(const stg_lattice *lat, const stg_gauge *gauge, stg_field field, int nrhs,
                   const void *in_odd, void *out_even, stg_stream_t stream);

/* out_odd = D_oe in_even for nrhs fields (Sec. 2.2 Eq. diracblock).  Asynchronous. */
int dirac_apply_oe(const stg_lattice *lat, const stg_gauge *gauge, stg_field field, int nrhs,
                   const void *in_even, void *out_odd, stg_stream_t stream);

/*
 * out_even = (mass^2 + sigma) in_even - D_eo D_oe in_even (Sec. 2.2 Eq. lineqeo,
 * shifted as in Eq. shlineq).  tmp_odd: device scratch field of the same shape
 * as in_even, overwritten with D_oe in_even.  Asynchronous.
 */
int stg_apply_normal(const stg_lattice *lat, const stg_gauge *gauge, stg_field field, int nrhs,
                     double mass, double sigma, const void *in_even, void *out_even,
                     void *tmp_odd, stg_stream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops that forbid allocation): stg_apply_normal without the tmp_odd
 * argument.  out_even = (mass^2 + sigma) in_even - D_eo D_oe in_even as in
 * stg_apply_normal (the same kernels, bitwise the same result); the odd-site
 * intermediate D_oe in_even goes to a device array of fixed size that the library
 * holds on each GPU it runs on, from its first call there until the process ends
 * (stg_noalloc_scratch_bytes: 64 MiB).  The call makes no hipMalloc, hipFree or
 * other allocating call; its first call on a device looks up that device's copy of
 * the array.  The array keeps the last call's contents (each call overwrites what it
 * reads), and it is shared by every call on one GPU: calls that overlap in time on
 * one GPU (other streams, other host threads) race on it and must be serialised by
 * the caller.  Errors: as stg_apply_normal; STG_WORKSPACE_TOO_SMALL (nothing
 * launched) when nrhs * 3 * Vh * element size exceeds the array.  Asynchronous.
 */
size_t stg_noalloc_scratch_bytes(void);
int stg_apply_normal_noalloc(const stg_lattice *lat, const stg_gauge *gauge, stg_field field,
                             int nrhs, double mass, double sigma, const void *in_even,
                             void *out_even, stg_stream_t stream);

/* Device workspace bytes needed by stg_dot. */
size_t stg_dot_workspace_bytes(void);

/*
 * Compensated complex inner products <x_j, y_j> = sum conj(x) y over n complex
 * entries for j < nvec (x, y device [nvec][n], element type field), accumulated
 * in FP64 with error-free transformations (TwoSum) and a fixed summation order,
 * so the result is bitwise reproducible.  These are the dot products of the
 * Krylov solvers (Sec. 2.3).  result (host) receives nvec (re, im) pairs.
 * ws (device) has ws_bytes >= stg_dot_workspace_bytes().  Synchronous.
 */
int stg_dot(stg_field field, int nvec, size_t n, const void *x, const void *y, double *result,
            void *ws, size_t ws_bytes, stg_stream_t stream);

/* Solver modes */
enum {
    STG_CG_F64 = 0,         /* FP64 operator and vectors on the hi gauge field */
    STG_CG_MIXED = 1        /* FP32 operator and vectors on the lo gauge field, FP64
                               reliable updates and true residual on the hi one */
};

typedef struct {
    double tol;        /* stop when the FP64 true |b - A x| / |b| <= tol */
    int max_iter;      /* cap on operator applications of the inner iteration */
    int mode;          /* STG_CG_F64 or STG_CG_MIXED */
    double delta;      /* reliable update when |r| < delta * max|r| since the last one (0.1) */
    int poll_every;    /* iterations enqueued between host convergence checks (0: auto) */
    int restart;       /* 1: restart p = r at each reliable update, 0: keep p, -1: auto
                          (restart when the lo gauge field is BF16-12, else keep p) */
} stg_cg_params;

typedef struct {
    int iters;              /* iterations of the solve (shared by a batch) */
    int reliable_updates;   /* FP64 true-residual recomputations */
    int status;             /* STG_OK / STG_NOT_CONVERGED / STG_BREAKDOWN */
    int converged_iter;     /* iteration at which this system met its stopping test */
    double true_rel_resid;  /* FP64 |b - A x| / |b| at return */
    double seconds;         /* wall time of the call */
    int ms_iters;           /* multishift_cg_solve / rational_apply: iterations of the shared
                               multi-shift stage this (shift, RHS) system took part in (the
                               rest of iters refined it alone); 0 for the other solvers */
    int pad_;
} stg_cg_stats;

/* Fills p with the defaults: tol 1e-10, max_iter 100000, mode F64, delta 0.1,
   poll_every 0 (auto), restart -1 (auto). */
void stg_cg_default_params(stg_cg_params *p);

/* Device workspace bytes needed by cg_solve (nshift = 0) or multishift_cg_solve. */
int stg_workspace_bytes(const stg_lattice *lat, int nrhs, int nshift, int mode, size_t *bytes);

/*
 * Solves (mass^2 - D_eo D_oe) x_j = b_j for j < nrhs by CG (Sec. 2.2 Eq. lineqeo).
 * hi: FP64 gauge field (STG_LINK_C128_*) used for the operator in mode F64 and
 * for the true residual and reliable updates in mode MIXED.  lo: FP32 gauge field
 * (STG_LINK_C64_12 or STG_LINK_BF16_12) for the inner iteration in mode MIXED,
 * ignored in mode F64.  b_even (device) and x_even (device, initial guess on
 * entry, solution on exit) are complex128 [nrhs][3][Vh].  ws (device) has
 * ws_bytes >= stg_workspace_bytes.  stats (host) gets nrhs entries.  Returns
 * STG_OK when every system converged, else the worst status.
 */
int cg_solve(const stg_lattice *lat, const stg_gauge *hi, const stg_gauge *lo, double mass,
             int nrhs, const void *b_even, void *x_even, const stg_cg_params *params, void *ws,
             size_t ws_bytes, stg_cg_stats *stats, stg_stream_t stream);

/*
 * Solves (mass^2 + shifts[k] - D_eo D_oe) x_{k,j} = b_j for k < nshift, j < nrhs
 * (Sec. 2.2 Eq. shlineq) with one operator application per iteration on the
 * smallest shift, then refines every (k, j) to the FP64 tolerance.  shifts
 * (host) >= 0.  x_even (device, output) is complex128 [nshift][nrhs][3][Vh];
 * stats (host) gets nshift*nrhs entries in the same order.
 */
int multishift_cg_solve(const stg_lattice *lat, const stg_gauge *hi, const stg_gauge *lo,
                        double mass, int nshift, const double *shifts, int nrhs,
                        const void *b_even, void *x_even, const stg_cg_params *params, void *ws,
                        size_t ws_bytes, stg_cg_stats *stats, stg_stream_t stream);

/*
 * Rational function of the normal operator applied to each RHS (the RHMC use of
 * Eq. shlineq: the fractional power of Eq. rooting is replaced by a rational
 * approximation whose poles are the shifts, Sec. 2.2):
 *   y_j = a0 b_j + sum_k coeffs[k] (mass^2 + shifts[k] - D_eo D_oe)^{-1} b_j,  j < nrhs.
 * The coefficients and poles are the caller's (the library does not compute
 * rational approximations).  Solves every shifted system as multishift_cg_solve
 * does (same params, modes and stopping test) into the workspace, then forms y in
 * one fused pass.  shifts, coeffs (host) have nshift entries, shifts >= 0.
 * b_even, y_even (device) are complex128 [nrhs][3][Vh].  ws (device) has
 * ws_bytes >= stg_rational_workspace_bytes.  stats (host) gets nshift*nrhs entries
 * ordered as for multishift_cg_solve.  Returns STG_OK when every system converged,
 * else the worst status (y is then formed from the last iterates).
 */
int stg_rational_workspace_bytes(const stg_lattice *lat, int nrhs, int nshift, int mode,
                                 size_t *bytes);
int rational_apply(const stg_lattice *lat, const stg_gauge *hi, const stg_gauge *lo, double mass,
                   int nshift, const double *shifts, const double *coeffs, double a0, int nrhs,
                   const void *b_even, void *y_even, const stg_cg_params *params, void *ws,
                   size_t ws_bytes, stg_cg_stats *stats, stg_stream_t stream);

/*
 * Uneven batch: independent CG solves on lattices of different sizes, each
 * (mass^2 - D_eo D_oe) x_j = b_j as in cg_solve (Sec. 2.2 Eq. lineqeo), advanced
 * together.  Every kernel of a CG step walks one table of tiles spanning all the
 * lattices (the paper fixes one lattice per compiled kernel, Sec. 4.1), so one
 * launch serves every solve; the iterations are captured once in a hipGraph and
 * replayed, with one host flag read per replay.
 *   lat, hi, lo, mass, nrhs, b, x: as in cg_solve for this solve (b and x device
 *   complex128 [nrhs][3][Vh]; x holds the guess on entry).  Every hi field must
 *   have one format, and in mode MIXED every lo field one format.
 */
/*
 * Staples of the tree-level Symanzik gauge force (Sec. 2.1: the tree-level
 * Symanzik improved gauge action, built from 1x1 and 1x2 Wilson loops; Sec. 4.3:
 * the staples, products of 3 and 5 links along C-shaped paths, are the most
 * expensive step of the gauge cycle).  For every link U_mu(x), out receives
 *   Sigma_mu(x) = sum_{nu != mu} ( c0 [2 three-link paths] + c1 [6 five-link paths] ),
 * each path the ordered product of the links met going from x+mu back to x (a
 * step from y to y-nu contributes U_nu(y-nu)^dag), so that U_mu(x) Sigma_mu(x) is
 * the c0/c1-weighted sum of the 1x1 and 1x2 loops through the link.  The
 * tree-level weights are c1 = -1/12, c0 = 1 - 8 c1 = 5/3.
 *  gauge: links in any format; its phases are ignored (staples use the bare
 *    links).  The 12-real formats rebuild row 2, so their links must be SU(3).
 *  out: device, [8][3][3][Vh] (slot 2*mu + parity of x, row, column, site),
 *    complex128 for STG_LINK_C128_* (FP64 arithmetic) and complex64 for
 *    STG_LINK_C64_12 / STG_LINK_BF16_12 (FP32 arithmetic); 16-byte aligned and
 *    not overlapping the links.  Written entirely.
 * Errors: STG_INVALID_ARG (bad extents, NULL or misaligned pointer, overlap,
 * unknown format, non-finite c0 or c1), and nothing is launched.  Asynchronous.
 */
int gauge_staples(const stg_lattice *lat, const stg_gauge *gauge, double c0, double c1,
                  void *out, stg_stream_t stream);

/*
 * Derivative of the rational pseudofermion action with respect to every link, from
 * the multi-shift solutions (Sec. 2.2: the molecular-dynamics forces come from the
 * solutions of the shifted systems of Eq. shlineq for the rational approximation of
 * Eq. rooting; most of that step is the operator, Sec. 4.3).  For
 *   S = Re phi^dag sum_k a_k X_k,  X_k = (A + sigma_k)^{-1} phi  (even sites),
 * with Y_k = D_oe X_k the call writes, for every link U_mu(z),
 *   z even:  G_mu(z) =  phi_mu(z) sum_k a_k Y_k(z+mu) X_k(z)^dag
 *   z odd:   G_mu(z) = -phi_mu(z) sum_k a_k X_k(z+mu) Y_k(z)^dag
 * so that S changes by Re Tr(E G_mu(z)) to first order when U_mu(z) becomes
 * U_mu(z) + E (phi_mu: the gauge field's phases).  The rest of the force (the
 * projection U G -> its traceless anti-Hermitian part, smearing) is the caller's.
 *  gauge: an FP64 format (STG_LINK_C128_18 / _12), the one the solutions belong to.
 *  coeffs: host, nshift weights a_k (any real values; a_0 of the rational
 *    function does not depend on the links and takes no part).
 *  x_even: device complex128 [nshift][3][Vh], the solutions X_k (e.g. from
 *    multishift_cg_solve with one right-hand side).
 *  y_odd: device complex128 [nshift][3][Vh], overwritten with D_oe X_k.
 *  out: device complex128 [8][3][3][Vh] (the link layout), written entirely.
 * Buffers 16-byte aligned and pairwise disjoint.  Errors: STG_INVALID_ARG (nothing
 * launched).  Asynchronous.
 */
int fermion_force(const stg_lattice *lat, const stg_gauge *gauge, int nshift,
                  const double *coeffs, const void *x_even, void *y_odd, void *out,
                  stg_stream_t stream);

/*
 * One stout-smearing step of every link (Sec. 2.1: the staggered fermion action is
 * built on stout-smeared links; Sec. 2.3: the configurations of the stout levels
 * U^(k) are kept), by the definition of Morningstar and Peardon:
 *   C_mu(x)  = rho * sum_{nu != mu} [ U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
 *                                    + U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) ],
 *   Omega    = C_mu(x) U_mu(x)^dag,
 *   Q        = (i/2)(Omega^dag - Omega) - (i/6) Tr(Omega^dag - Omega),
 *   U'_mu(x) = exp(i Q) U_mu(x).
 * exp(iQ) is evaluated in closed form through the Cayley-Hamilton theorem (FP64).
 *  gauge: STG_LINK_C128_18 or STG_LINK_C128_12 (links in SU(3)); phases ignored.
 *  rho: isotropic weight, finite.
 *  out: device complex128 [8][3][3][Vh] (the STG_LINK_C128_18 layout), 16-byte
 *    aligned, not overlapping the links; written entirely.  Several levels: call
 *    again with out as an STG_LINK_C128_18 gauge field (into a second buffer).
 * Errors: STG_INVALID_ARG (nothing launched).  Asynchronous.
 */
int stout_smear(const stg_lattice *lat, const stg_gauge *gauge, double rho, void *out,
                stg_stream_t stream);

/*
 * Momentum update of the pure-gauge molecular dynamics (Sec. 4.3: the gauge cycle,
 * whose most expensive step is the staples; Table 4 times it per site).  With the
 * tree-level Symanzik action S = -(beta/3) (c0 sum Re Tr(1x1 loops) +
 * c1 sum Re Tr(1x2 loops)) and the staple sum Sigma_mu(x) of gauge_staples, the
 * force is F_mu(x) = -(beta/3) [i U_mu(x) Sigma_mu(x)]_TH ([A]_TH: the traceless
 * Hermitian part of A), i.e. dS/dt = Tr(F X) when the link moves as
 * U -> exp(i t X) U; the call sets P_mu(x) <- P_mu(x) - eps F_mu(x) for every link.
 *  gauge: STG_LINK_C128_18 or STG_LINK_C128_12 (FP64 arithmetic, complex128
 *    momenta), or STG_LINK_C64_12 (the single-precision molecular dynamics: FP32
 *    arithmetic, complex64 momenta); SU(3) links; phases ignored.
 *  mom: device [8][3][3][Vh] (the link layout) of that element type, traceless
 *    Hermitian momenta, read and written; not overlapping the links.
 *  beta, c0, c1, eps: finite.  STG_TUNE_STAPLE_THREADS and the pencil tile apply.
 * Errors: STG_INVALID_ARG (nothing launched).  Asynchronous.
 */
int gauge_momentum_update(const stg_lattice *lat, const stg_gauge *gauge, double beta, double c0,
                          double c1, double eps, void *mom, stg_stream_t stream);

/*
 * Link update of the molecular dynamics: U_mu(x) <- exp(i eps P_mu(x)) U_mu(x) for every
 * link, in place, with exp(iQ) in the Cayley-Hamilton closed form (as in stout_smear).
 *  fmt: STG_LINK_C128_18, STG_LINK_C128_12 or STG_LINK_C64_12 (the 12-real formats
 *    keep rows 0 and 1 of the updated link; exp(i eps P) is formed in FP64 in every
 *    case, the product with U in the format's precision).  links: device, that
 *    format, read and written.
 *  mom: device [8][3][3][Vh], complex128 (complex64 with STG_LINK_C64_12), traceless
 *    Hermitian; not overlapping links.
 *  eps: finite.
 * Errors: STG_INVALID_ARG (nothing launched).  Asynchronous.
 */
int gauge_link_update(const stg_lattice *lat, stg_link_fmt fmt, void *links, double eps,
                      const void *mom, stg_stream_t stream);

/*
 * The force through one stout-smearing step (Sec. 2.2: the fermion force follows
 * Morningstar and Peardon through the stout levels of Sec. 2.1 / Sec. 2.3): given
 * Sigma'_l = dS/dU'_l for every link of U' = stout_smear(U, rho) (convention:
 * dS = Re Tr(dU' Sigma'), as for fermion_force and gauge_staples), writes
 * Sigma_l = dS/dU_l for the thin links U (same convention), the chain rule through
 * exp(iQ) U, Q(Omega), Omega = C U^dag and the six 3-link paths of C.  Repeated calls
 * carry a force down several levels (each with that level's thin links).
 *  gauge: STG_LINK_C128_18 or STG_LINK_C128_12, the thin links of the level.
 *  sigma_smeared: device complex128 [8][3][3][Vh].
 *  sigma_thin: device complex128 [8][3][3][Vh], written entirely.
 *  ws: device scratch, complex128 [8][3][3][Vh] (8*9*Vh*16 bytes), overwritten.
 * The four buffers and the links are pairwise disjoint and 16-byte aligned; rho finite.
 * Errors: STG_INVALID_ARG (nothing launched).  Asynchronous.
 */
int stout_force_backprop(const stg_lattice *lat, const stg_gauge *gauge, double rho,
                         const void *sigma_smeared, void *sigma_thin, void *ws,
                         stg_stream_t stream);

typedef struct {
    stg_lattice lat;
    stg_gauge hi;
    stg_gauge lo;
    double mass;
    int nrhs;
    const void *b;
    void *x;
} stg_solve_desc;

/* Device workspace bytes needed by cg_solve_batch for these solves and mode. */
int stg_batch_workspace_bytes(int nsolve, const stg_solve_desc *descs, int mode, size_t *bytes);

/*
 * Solves every system of every descriptor.  params->poll_every is the number of
 * iterations per graph replay (0: 16).  stats (host) receives one entry per
 * system, descriptors in order and RHS in order within each.  Returns STG_OK when
 * every system converged, else the worst status.
 */
int cg_solve_batch(int nsolve, const stg_solve_desc *descs, const stg_cg_params *params, void *ws,
                   size_t ws_bytes, stg_cg_stats *stats, stg_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* STAGMI_H */
