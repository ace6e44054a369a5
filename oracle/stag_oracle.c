/*
 * stag_oracle.c -- FP64 CPU oracle for the even/odd staggered Dirac operator and
 * the (multi-shift) conjugate-gradient solves built on it.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * helper with the GPU library and must never be linked into it.
 *
 * Paper: Bonati et al., "Design and optimization of a portable LQCD Monte Carlo
 * code using OpenACC" (arXiv:1701.00426).
 *
 * What is computed, written out from its definition (no blocking, no fusion):
 *
 *  - Site indexing (Sec. 4.1, Eq. lexicographic_eo): lex(x) = x0 + N0(x1 + N1(x2
 *    + N2 x3)) with x0 fastest, every extent even, half-index h = floor(lex/2).
 *    The paper writes this for even sites; the same map is used for odd sites
 *    (it is a bijection per parity because N0 is even).
 *  - Links (Sec. 4.1, "array of 8 su3_soa"): U_mu(x) stored as a full 3x3 complex
 *    matrix at slot 2*mu + parity(x), position h(x); layout [8][3][3][Vh] with
 *    row, column, then site (structure of arrays).
 *  - Fields (Sec. 4.1, vec3_soa): one colour 3-vector per site of one parity,
 *    layout [3][Vh].
 *  - Staggered operator (Sec. 2.2, Eq. diracblock; the explicit form is the
 *    textbook one, which the paper does not print):
 *      (D psi)(x) = 1/2 sum_mu [ phi_mu(x) U_mu(x) psi(x+mu)
 *                               - phi_mu(x-mu) U_mu(x-mu)^dagger psi(x-mu) ]
 *    with real per-link phases phi (the "backfield" argument of the paper's deo
 *    listing, Sec. 4.3).  D_oe is D restricted to odd outputs and even inputs,
 *    D_eo to even outputs and odd inputs.
 *  - Standard phases: phi_mu(x) = eta_mu(x) s_mu(x), eta_mu(x) =
 *    (-1)^(x0+...+x_{mu-1}), s_3(x) = -1 on the links leaving x3 = N3-1
 *    (antiperiodic time boundary, time = x3), s_mu = +1 otherwise.
 *  - Even/odd normal operator (Sec. 2.2, Eq. lineqeo): A = m^2 - D_eo D_oe on even
 *    sites, shifted by sigma for the rational-approximation poles (Eq. shlineq).
 *  - CG (Sec. 2.2, the Krylov solver the paper uses for the normal equations):
 *    textbook Hestenes-Stiefel iteration.
 *  - Multi-shift CG (Sec. 2.2, Eq. shlineq: all shifted systems with one
 *    matrix-vector product per iteration): the shifted residuals stay collinear
 *    with the base residual, r_k = zeta_k r; zeta, alpha_k and beta_k follow from
 *    matching the three-term residual recurrence of CG on A+sigma_0 and on
 *    A+sigma_k (derivation in the design notes).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC stag_oracle.c -o libstag_oracle.so -lm
 * (the CPU baseline builds its own copy with -O3 -march=native on the host it runs on)
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Geometry (Sec. 4.1, Eq. lexicographic_eo)                                 */
/* ------------------------------------------------------------------------ */

/* threads the OpenMP loops of this library use */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* sets the threads of the OpenMP loops (the CPU baseline times 1 and all cores) */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

long orc_half_volume(const int *N) { return (long)N[0] * N[1] * N[2] * N[3] / 2; }

static long lex_of(const int *N, const int *x) {
    return x[0] + (long)N[0] * (x[1] + (long)N[1] * (x[2] + (long)N[2] * x[3]));
}

/* half-lattice index of site x: floor(lex / 2) */
long orc_half_index(const int *N, const int *x) { return lex_of(N, x) / 2; }

int orc_parity(const int *x) { return (x[0] + x[1] + x[2] + x[3]) & 1; }

/* inverse of orc_half_index for a site of the given parity */
void orc_coords(const int *N, int parity, long h, int *x) {
    long nh0 = N[0] / 2;
    long rest = h / nh0;
    int x0half = (int)(h % nh0);
    x[1] = (int)(rest % N[1]);
    rest /= N[1];
    x[2] = (int)(rest % N[2]);
    x[3] = (int)(rest / N[2]);
    /* x0 is 2*x0half or 2*x0half+1, whichever gives the requested parity */
    x[0] = 2 * x0half + ((parity + x[1] + x[2] + x[3]) & 1);
}

/* ------------------------------------------------------------------------ */
/* Phases                                                                    */
/* ------------------------------------------------------------------------ */

/* phases[(2*mu+parity)*Vh + h] = eta_mu(x) * s_mu(x) for the site x = (parity,h) */
void orc_standard_phases(const int *N, double *phases) {
    long Vh = orc_half_volume(N);
    for (int mu = 0; mu < 4; ++mu)
        for (int par = 0; par < 2; ++par)
            for (long h = 0; h < Vh; ++h) {
                int x[4];
                orc_coords(N, par, h, x);
                int s = 0;
                for (int nu = 0; nu < mu; ++nu) s += x[nu];
                double eta = (s & 1) ? -1.0 : 1.0;
                double bc = (mu == 3 && x[3] == N[3] - 1) ? -1.0 : 1.0;
                phases[(long)(2 * mu + par) * Vh + h] = eta * bc;
            }
}

/* ------------------------------------------------------------------------ */
/* Staggered hop D restricted to one output parity (Sec. 2.2)                */
/* ------------------------------------------------------------------------ */

static inline cplx link_at(const cplx *U, long Vh, int slot, int row, int col, long h) {
    return U[((long)(slot * 3 + row) * 3 + col) * Vh + h];
}

/*
 * out[c][h] for every site of parity out_parity:
 *   1/2 sum_mu [ phi_mu(x) U_mu(x) in(x+mu) - phi_mu(x-mu) U_mu(x-mu)^dag in(x-mu) ]
 * in is a field on the other parity.  out_parity = 0 gives D_eo, 1 gives D_oe.
 */
void orc_dslash(const int *N, const double *links, const double *phases, int out_parity,
                const double *in, double *out) {
    const cplx *U = (const cplx *)links;
    const cplx *vin = (const cplx *)in;
    cplx *vout = (cplx *)out;
    long Vh = orc_half_volume(N);
    int in_parity = 1 - out_parity;
#pragma omp parallel for schedule(static)
    for (long h = 0; h < Vh; ++h) {
        int x[4];
        orc_coords(N, out_parity, h, x);
        cplx acc[3] = {0, 0, 0};
        for (int mu = 0; mu < 4; ++mu) {
            int xf[4] = {x[0], x[1], x[2], x[3]};
            int xb[4] = {x[0], x[1], x[2], x[3]};
            xf[mu] = (x[mu] + 1) % N[mu];
            xb[mu] = (x[mu] - 1 + N[mu]) % N[mu];
            long hf = orc_half_index(N, xf);
            long hb = orc_half_index(N, xb);
            /* forward: link U_mu(x) starts at x (parity out_parity) */
            int sf = 2 * mu + out_parity;
            double pf = phases[(long)sf * Vh + h];
            /* backward: link U_mu(x-mu) starts at x-mu (parity in_parity) */
            int sb = 2 * mu + in_parity;
            double pb = phases[(long)sb * Vh + hb];
            for (int a = 0; a < 3; ++a) {
                cplx fwd = 0, bwd = 0;
                for (int b = 0; b < 3; ++b) {
                    fwd += link_at(U, Vh, sf, a, b, h) * vin[(long)b * Vh + hf];
                    /* (U^dag)_{ab} = conj(U_{ba}) */
                    bwd += conj(link_at(U, Vh, sb, b, a, hb)) * vin[(long)b * Vh + hb];
                }
                acc[a] += pf * fwd - pb * bwd;
            }
        }
        for (int a = 0; a < 3; ++a) vout[(long)a * Vh + h] = 0.5 * acc[a];
    }
}

/* ------------------------------------------------------------------------ */
/* Normal operator (Sec. 2.2, Eq. lineqeo, shifted as in Eq. shlineq)         */
/* ------------------------------------------------------------------------ */

/* out_e = (m^2 + sigma) in_e - D_eo D_oe in_e ; tmp_o holds D_oe in_e */
void orc_apply_normal(const int *N, const double *links, const double *phases, double mass,
                      double sigma, const double *in_e, double *out_e, double *tmp_o) {
    long Vh = orc_half_volume(N);
    orc_dslash(N, links, phases, 1, in_e, tmp_o);
    orc_dslash(N, links, phases, 0, tmp_o, out_e);
    const cplx *vi = (const cplx *)in_e;
    cplx *vo = (cplx *)out_e;
    double diag = mass * mass + sigma;
    for (long i = 0; i < 3 * Vh; ++i) vo[i] = diag * vi[i] - vo[i];
}

/* ------------------------------------------------------------------------ */
/* Plain BLAS-1 over complex fields                                         */
/* ------------------------------------------------------------------------ */

static double re_dot(const cplx *a, const cplx *b, long n) {
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += creal(conj(a[i]) * b[i]);
    return s;
}

static double norm2(const cplx *a, long n) { return re_dot(a, a, n); }

/* ------------------------------------------------------------------------ */
/* Conjugate gradient (Sec. 2.2): textbook Hestenes-Stiefel on A + sigma      */
/* ------------------------------------------------------------------------ */

/*
 * Solves (m^2 + sigma - D_eo D_oe) x = b.  x holds the initial guess on entry
 * and the iterate on exit.  Stops when |r| <= tol |b| on the recurrence residual
 * or after max_iter iterations.  Reports the iterations and the true relative
 * residual |b - A x| / |b|.  Returns 0 when converged, 1 otherwise.
 */
int orc_cg(const int *N, const double *links, const double *phases, double mass, double sigma,
           const double *b_in, double *x_io, double tol, int max_iter, int *iters_out,
           double *true_rel_out) {
    long Vh = orc_half_volume(N);
    long n = 3 * Vh;
    const cplx *b = (const cplx *)b_in;
    cplx *x = (cplx *)x_io;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);

    orc_apply_normal(N, links, phases, mass, sigma, (double *)x, (double *)q, (double *)t);
    for (long i = 0; i < n; ++i) { r[i] = b[i] - q[i]; p[i] = r[i]; }
    double bb = norm2(b, n);
    double rr = norm2(r, n);
    int it = 0, status = 1;
    if (rr <= tol * tol * bb) status = 0;
    while (status && it < max_iter) {
        orc_apply_normal(N, links, phases, mass, sigma, (double *)p, (double *)q, (double *)t);
        double alpha = rr / re_dot(p, q, n);
        for (long i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        double rr_new = norm2(r, n);
        ++it;
        if (rr_new <= tol * tol * bb) { status = 0; break; }
        double beta = rr_new / rr;
        for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
    }
    /* true residual */
    orc_apply_normal(N, links, phases, mass, sigma, (double *)x, (double *)q, (double *)t);
    for (long i = 0; i < n; ++i) r[i] = b[i] - q[i];
    if (iters_out) *iters_out = it;
    if (true_rel_out) *true_rel_out = sqrt(norm2(r, n) / bb);
    free(r); free(p); free(q); free(t);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Multi-shift CG (Sec. 2.2, Eq. shlineq)                                    */
/* ------------------------------------------------------------------------ */

/*
 * Solves (m^2 + sigma_k - D_eo D_oe) x_k = b for all k with one operator
 * application per iteration.  The base system is the smallest shift sigma_0.
 * With alpha_i, beta_i the base CG scalars and delta_k = sigma_k - sigma_0:
 *
 *   zeta_k(i+1) = zeta_k(i) zeta_k(i-1) alpha(i-1) /
 *                 [ alpha(i) beta(i-1) (zeta_k(i-1) - zeta_k(i))
 *                   + zeta_k(i-1) alpha(i-1) (1 + delta_k alpha(i)) ]
 *   alpha_k(i) = alpha(i) zeta_k(i+1) / zeta_k(i);  x_k += alpha_k(i) p_k
 *   beta_k(i)  = beta(i) (zeta_k(i+1) / zeta_k(i))^2
 *   p_k        = zeta_k(i+1) r(i+1) + beta_k(i) p_k
 *
 * starting from zeta(-1) = zeta(0) = 1, alpha(-1) = 1, beta(-1) = 0, p_k = b,
 * x_k = 0.  Shift k stops (its scalars are frozen) once
 * |zeta_k| |r| <= tol |b|; the iteration ends when every shift has stopped.
 * x is [nshift][3][Vh]; iters_out[k] gets the iteration at which shift k
 * stopped; true_rel_out[k] its true relative residual.  Returns 0 when all
 * shifts converged.
 */
int orc_mscg(const int *N, const double *links, const double *phases, double mass, int nshift,
             const double *shifts, const double *b_in, double *x_out, double tol, int max_iter,
             int *iters_out, double *true_rel_out) {
    long Vh = orc_half_volume(N);
    long n = 3 * Vh;
    const cplx *b = (const cplx *)b_in;
    cplx *x = (cplx *)x_out;
    /* base shift = smallest sigma */
    int k0 = 0;
    for (int k = 1; k < nshift; ++k)
        if (shifts[k] < shifts[k0]) k0 = k;
    double sigma0 = shifts[k0];

    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    cplx *pk = malloc(sizeof(cplx) * n * nshift);
    double *zeta = malloc(sizeof(double) * nshift), *zeta_prev = malloc(sizeof(double) * nshift);
    int *active = malloc(sizeof(int) * nshift);

    for (long i = 0; i < n; ++i) { r[i] = b[i]; p[i] = b[i]; }
    for (int k = 0; k < nshift; ++k) {
        for (long i = 0; i < n; ++i) { x[k * n + i] = 0; pk[k * n + i] = b[i]; }
        zeta[k] = 1.0;
        zeta_prev[k] = 1.0;
        active[k] = 1;
        iters_out[k] = 0;
    }
    double bb = norm2(b, n);
    double rr = bb;
    double alpha_prev = 1.0, beta_prev = 0.0;
    int it = 0, n_active = nshift;
    while (n_active > 0 && it < max_iter) {
        orc_apply_normal(N, links, phases, mass, sigma0, (double *)p, (double *)q, (double *)t);
        double alpha = rr / re_dot(p, q, n);
        /* shifted scalars and solution updates, using the pre-update p_k */
        double zeta_next[64];
        double *zn = nshift <= 64 ? zeta_next : malloc(sizeof(double) * nshift);
        for (int k = 0; k < nshift; ++k) {
            if (!active[k]) continue;
            double dk = shifts[k] - sigma0;
            double z = zeta[k], zp = zeta_prev[k];
            double den = alpha * beta_prev * (zp - z) + zp * alpha_prev * (1.0 + dk * alpha);
            zn[k] = z * zp * alpha_prev / den;
            double ak = alpha * zn[k] / z;
            for (long i = 0; i < n; ++i) x[k * n + i] += ak * pk[k * n + i];
        }
        for (long i = 0; i < n; ++i) r[i] -= alpha * q[i];
        double rr_new = norm2(r, n);
        double beta = rr_new / rr;
        ++it;
        for (int k = 0; k < nshift; ++k) {
            if (!active[k]) continue;
            double bk = beta * (zn[k] / zeta[k]) * (zn[k] / zeta[k]);
            for (long i = 0; i < n; ++i) pk[k * n + i] = zn[k] * r[i] + bk * pk[k * n + i];
            zeta_prev[k] = zeta[k];
            zeta[k] = zn[k];
            if (zn[k] * zn[k] * rr_new <= tol * tol * bb) {
                active[k] = 0;
                --n_active;
                iters_out[k] = it;
            }
        }
        if (zn != zeta_next) free(zn);
        for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        alpha_prev = alpha;
        beta_prev = beta;
        rr = rr_new;
    }
    for (int k = 0; k < nshift; ++k) {
        if (active[k]) iters_out[k] = it;
        orc_apply_normal(N, links, phases, mass, shifts[k], (double *)(x + k * n), (double *)q,
                         (double *)t);
        for (long i = 0; i < n; ++i) q[i] = b[i] - q[i];
        true_rel_out[k] = sqrt(norm2(q, n) / bb);
    }
    free(r); free(p); free(q); free(t); free(pk); free(zeta); free(zeta_prev); free(active);
    return n_active == 0 ? 0 : 1;
}
