// solver_state.hpp -- per-system solver scalars kept on the device, and the scalar
// step that the finalize kernel of a reduction performs on them.
//
// The CG scalars alpha = |r|^2 / <p, A p> and beta = |r_new|^2 / |r|^2 (Sec. 2.2,
// conjugate gradient on Eq. lineqeo) never leave the GPU during the iteration: the
// finalize kernel that completes a reduction computes them and the next kernel
// reads them.  The host only polls the flags every few iterations.
//
// Reliable updates (mixed precision): the inner recurrence runs until its
// residual norm has dropped by delta relative to the largest one since the last
// update, or below the target; the system is then parked (RU_PENDING) until the
// host has the FP64 true residual b - A x recomputed, which either finishes the
// system or resumes it from the true residual.
#pragma once

#include <hip/hip_runtime.h>

namespace stg {

enum SysFlags : int {
    SYS_RUNNING = 1,     // takes part in the inner iteration
    SYS_RU_PENDING = 2,  // parked, waiting for a true-residual update
    SYS_DONE = 4,        // true residual met the target
    SYS_BREAKDOWN = 8,   // non-finite scalar or <p, A p> <= 0
    SYS_RESUME = 16,     // just updated: the resume kernel rebuilds r_inner and p
    SYS_CAPPED = 32,     // stopped by the iteration cap (not converged)
    SYS_FINISHING = 64   // multi-shift base: stopped this iteration, the shifted solutions
                         // still take this iteration's step; final_flags follows
};

struct SysState {
    double diag;     // m^2 + sigma of this system
    double bb;       // |b|^2
    double tol2bb;   // tol^2 |b|^2
    double delta2;   // delta^2; 0 disables the delta-triggered updates
    double rr;       // |r|^2 of the current inner residual
    double rr_old;   // |r|^2 before the iteration that parked the system
    double maxrr;    // largest |r|^2 since the last true-residual update
    double alpha;
    double beta;
    double rr_true;  // last FP64 true |b - A x|^2
    int iter;        // inner iterations done by this system
    int n_ru;        // true-residual updates done
    int flags;
    int conv_iter;   // iteration at which the system finished
    int restart;     // 1: p = r after each update
    int gid;         // index of this system in the solve (multi-shift: the RHS index)
    int max_iter;    // iteration cap: the system stops (SYS_CAPPED) when iter reaches it
    int final_flags; // multi-shift: flags a finishing base system takes next
    double alpha_prev;  // multi-shift base scalars of the previous iteration
    double beta_prev;
};

// One shifted system of the multi-shift iteration (Sec. 2.2, Eq. shlineq): its
// residual stays collinear with the base residual, r_k = zeta r.
struct ShiftState {
    double delta;      // sigma_k - sigma_0
    double zeta;       // zeta at the current iteration
    double zeta_prev;  // zeta one iteration back
    double zeta_next;  // zeta of the next iteration (set after alpha is known)
    double alpha;      // alpha_k of the current iteration
    double beta;       // beta_k of the current iteration
    int active;        // 1 running, 2 retired this iteration (its x_k still takes the
                       // step), 0 retired
    int conv_iter;     // base iteration at which it retired
};

struct Ctl {
    int n_running;   // systems with SYS_RUNNING set; kernels of the inner loop exit when 0
    int pad0_;
    int nshift;      // multi-shift: shifts per RHS
    int nrhs;        // multi-shift: right-hand sides
    ShiftState *ms;  // multi-shift: [nshift][nrhs]
    int pad_[10];
};

enum FinOp {
    OP_NONE = 0,     // no reduction at all
    OP_STORE = 1,    // sums -> out[j]
    OP_INIT_BB = 2,  // sums -> bb, tol2bb = tol^2 bb  (tol^2 passed in delta2 slot)
    OP_ALPHA = 3,    // sums = <p, A p> -> alpha
    OP_BETA = 4,     // sums = |r_new|^2 -> beta, convergence / park test
    OP_RU = 5,       // sums = |b - A x|^2 of parked systems -> done or resume
    OP_MS_ALPHA = 6, // multi-shift: base alpha, then zeta_next and alpha_k of every shift
    OP_MS_BETA = 7,  // multi-shift: base beta, then beta_k, zeta shift and retirement
    OP_CGCG = 8      // single-reduction CG: sums = <r, A r>, sums2 = |r|^2 -> alpha, beta
};

// Gate of the kernels that finish reductions: other blocks of the same launch may
// change the running count meanwhile, so one thread reads it and the whole block
// takes the same branch (every wave then reaches the same barriers).  A block whose
// system is still counted as running always finds the count above zero.
__device__ __forceinline__ bool block_gate_closed(const Ctl *ctl, int gate) {
    __shared__ int closed;
    if (threadIdx.x == 0) closed = (gate && ctl->n_running == 0) ? 1 : 0;
    __syncthreads();
    return closed != 0;
}

__device__ __forceinline__ bool finite_pos(double v) { return v > 0.0 && v < 1.0e300; }

// The CG step after |r_new|^2 = sum on a running system: beta = sum / |r|^2, or the
// system parks for a true-residual update (sum below the target, or dropped by
// delta since the largest |r|^2 since the last update), stops at the iteration cap,
// or breaks down (sum not finite).  Returns true when the system leaves the
// running state.
__device__ __forceinline__ bool beta_step(SysState &s, double sum) {
    s.iter += 1;
    if (!(sum >= 0.0 && sum < 1.0e300)) {
        s.flags = SYS_BREAKDOWN;
        return true;
    }
    if (sum > s.maxrr) s.maxrr = sum;
    if (sum <= s.tol2bb || sum < s.delta2 * s.maxrr) {
        s.rr_old = s.rr;
        s.rr = sum;
        s.flags = SYS_RU_PENDING;
        return true;
    }
    s.beta = sum / s.rr;
    s.rr = sum;
    if (s.iter >= s.max_iter) {
        s.flags = SYS_CAPPED;
        return true;
    }
    return false;
}

// The scalar step of the single-reduction form of CG (Chronopoulos and Gear): with
// w = A r, gamma = |r|^2 and delta = <r, w> from one pass,
//   beta = gamma / gamma_prev,  alpha = gamma / (delta - beta gamma / alpha_prev),
// then p = r + beta p, s = w + beta s (s = A p by recurrence), x += alpha p,
// r -= alpha s: the iterates of CG (Sec. 2.2) in exact arithmetic, with one global
// reduction per iteration instead of two.  gamma is the |r|^2 of the update of the
// previous iteration, so the convergence and reliable-update tests of that update
// happen here; just after a true-residual update (SYS_RESUME) gamma and beta come
// from the update (rr, beta) instead.  Returns true when the system leaves the
// running state (parked, capped or broken down); alpha and beta are then unused.
__device__ __forceinline__ bool cgcg_step(SysState &s, double delta, double gamma) {
    double beta;
    if (s.flags & SYS_RESUME) {
        s.flags &= ~SYS_RESUME;
        gamma = s.rr;
        beta = s.beta;
    } else {
        s.iter += 1;
        if (!(gamma >= 0.0 && gamma < 1.0e300)) {
            s.flags = SYS_BREAKDOWN;
            return true;
        }
        if (gamma > s.maxrr) s.maxrr = gamma;
        if (gamma <= s.tol2bb || gamma < s.delta2 * s.maxrr) {
            s.rr_old = s.rr;
            s.rr = gamma;
            s.flags = SYS_RU_PENDING;
            return true;
        }
        beta = gamma / s.rr;
        s.rr = gamma;
        if (s.iter >= s.max_iter) {
            s.flags = SYS_CAPPED;
            return true;
        }
    }
    const double den = beta == 0.0 ? delta : delta - beta * gamma / s.alpha;
    if (!finite_pos(den) || !finite_pos(gamma)) {
        s.flags = SYS_BREAKDOWN;
        return true;
    }
    s.alpha = gamma / den;
    s.beta = beta;
    return false;
}

// Scalar step for system j after a reduction (one thread).  Several blocks may run
// it at once for different systems (the batched finalize), so the running count is
// changed with atomics only.
__device__ __forceinline__ void finalize_one(int op, Ctl *ctl, SysState *st, double *out, int j,
                                             double sum, double sum2 = 0.0) {
    if (op == OP_STORE) {
        out[j] = sum;
        return;
    }
    SysState &s = st[j];
    if (op == OP_INIT_BB) {
        s.bb = sum;
        s.rr = sum;
        s.tol2bb = s.tol2bb * sum;  // tol^2 was stored there by the host
        return;
    }
    if (op == OP_ALPHA) {
        s.flags &= ~SYS_RESUME;
        if (!(s.flags & SYS_RUNNING)) return;
        if (!finite_pos(sum) || !(s.rr >= 0.0 && s.rr < 1.0e300)) {
            s.flags = SYS_BREAKDOWN;
            atomicAdd(&ctl->n_running, -1);
            return;
        }
        s.alpha = s.rr / sum;
        return;
    }
    if (op == OP_BETA) {
        if (!(s.flags & SYS_RUNNING)) return;
        if (beta_step(s, sum)) atomicAdd(&ctl->n_running, -1);
        return;
    }
    if (op == OP_CGCG) {
        if (!(s.flags & SYS_RUNNING)) return;
        if (cgcg_step(s, sum, sum2)) atomicAdd(&ctl->n_running, -1);
        return;
    }
    if (op == OP_RU) {
        if (!(s.flags & SYS_RU_PENDING)) return;
        s.n_ru += 1;
        s.rr_true = sum;
        if (!(sum >= 0.0 && sum < 1.0e300)) {
            s.flags = SYS_BREAKDOWN;
            return;
        }
        if (sum <= s.tol2bb) {
            s.flags = SYS_DONE;
            s.conv_iter = s.iter;
            return;
        }
        if (s.iter >= s.max_iter) {
            s.flags = SYS_CAPPED;
            return;
        }
        s.beta = (s.restart || !(s.rr_old > 0.0)) ? 0.0 : sum / s.rr_old;
        s.rr = sum;
        s.maxrr = sum;
        s.flags = SYS_RUNNING | SYS_RESUME;
        atomicAdd(&ctl->n_running, 1);
        return;
    }
}

// Multi-shift scalar steps for system j, by the whole block: thread 0 takes the
// base system's step, then thread k < nshift that of shift k (the recurrences of
// different shifts are independent).  Every thread of the block must call it;
// sum is read in thread 0 only.
enum MsMode { MS_SKIP = 0, MS_RUN = 1, MS_FINISH = 2 };

__device__ __forceinline__ void finalize_ms_block(int op, Ctl *ctl, SysState *st, int j,
                                                  double sum) {
    __shared__ int mode;
    __shared__ double sh_sum;
    SysState &s = st[j];
    if (threadIdx.x == 0) {
        sh_sum = sum;
        mode = MS_SKIP;
        if (op == OP_MS_ALPHA) {
            if (s.flags & SYS_FINISHING) {
                // the base stopped last iteration and every x_k took its last step
                s.flags = s.final_flags;
                atomicAdd(&ctl->n_running, -1);
                mode = MS_FINISH;
            } else if (s.flags & SYS_RUNNING) {
                if (!finite_pos(sum)) {
                    s.flags = SYS_BREAKDOWN;
                    atomicAdd(&ctl->n_running, -1);
                } else {
                    s.alpha = s.rr / sum;
                    mode = MS_RUN;
                }
            }
        } else if (s.flags & SYS_RUNNING) {  // OP_MS_BETA
            s.iter += 1;
            if (!(sum >= 0.0 && sum < 1.0e300)) {
                s.flags = SYS_BREAKDOWN;
                atomicAdd(&ctl->n_running, -1);
            } else {
                const double b = sum / s.rr;
                s.beta = b;
                s.alpha_prev = s.alpha;
                s.beta_prev = b;
                s.rr = sum;
                if (sum <= s.tol2bb || s.iter >= s.max_iter) {
                    s.final_flags = sum <= s.tol2bb ? SYS_DONE : SYS_CAPPED;
                    if (sum <= s.tol2bb) s.conv_iter = s.iter;
                    s.flags = SYS_FINISHING;  // still counted as running until the next alpha
                }
                mode = MS_RUN;
            }
        }
    }
    __syncthreads();  // also makes thread 0's state writes visible to the block
    const int m = mode;
    sum = sh_sum;
    for (int k = threadIdx.x; k < ctl->nshift && m != MS_SKIP; k += blockDim.x) {
        ShiftState &z = ctl->ms[k * ctl->nrhs + s.gid];
        if (op == OP_MS_ALPHA) {
            if (z.active == 2) z.active = 0;
            if (m != MS_RUN || z.active != 1) continue;
            // three-term recurrence of CG on A + sigma_0 matched on A + sigma_k
            const double a = s.alpha;
            const double den = a * s.beta_prev * (z.zeta_prev - z.zeta) +
                               z.zeta_prev * s.alpha_prev * (1.0 + z.delta * a);
            z.zeta_next = z.zeta * z.zeta_prev * s.alpha_prev / den;
            z.alpha = a * z.zeta_next / z.zeta;
        } else {
            if (z.active != 1) continue;
            const double ratio = z.zeta_next / z.zeta;
            z.beta = s.beta * ratio * ratio;
            z.zeta_prev = z.zeta;
            z.zeta = z.zeta_next;
            // |r_k| = |zeta| |r|: solved; x_k still takes this iteration's step
            if (z.zeta * z.zeta * sum <= s.tol2bb) {
                z.active = 2;
                z.conv_iter = s.iter;
            }
        }
    }
}

}  // namespace stg
