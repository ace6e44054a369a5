// blas.hip -- site-local kernels of the Krylov solvers (the paper's "zaxpy-like"
// functions, Sec. 2.3 and Sec. 4.2), compensated dot products, and the packing of
// gauge links into the 12-real formats (Sec. 2.3, Sec. 4.1).
//
// Every vector kernel fuses the axpy updates with the reduction that follows
// them (|r|^2 after x += alpha p, r -= alpha q), so a CG iteration reads each
// vector the minimum number of times.  Reductions: TwoSum per thread, wave64
// shuffle and LDS pair tree, one (sum, error) pair per block, and a finalize
// kernel (one block per system) that adds the pairs in a fixed order and runs the
// scalar step.

#include "device_common.hpp"
#include "kernels.hpp"
#include "solver_state.hpp"

namespace stg {

// x += alpha p; r -= alpha q; block partials of |r|^2 (OP_BETA in the finalize kernel)
template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void cg_update_kernel(VecArgs a) {
    if (a.gate_running && a.ctl->n_running == 0) return;
    const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
    double ps[NR], pc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        ps[j] = 0.0;
        pc[j] = 0.0;
        const SysState &s = a.state[j];
        if (!(s.flags & SYS_RUNNING) || h >= a.Vh) continue;
        const T al = (T)s.alpha;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t i = (size_t)j * a.fstride + (size_t)c * a.Vh + h;
            cpx<T> x = ld_c<T>(a.x, i), p = ld_c<T>(a.p, i), r = ld_c<T>(a.r, i),
                   q = ld_c<T>(a.q, i);
            x.re += al * p.re;
            x.im += al * p.im;
            r.re -= al * q.re;
            r.im -= al * q.im;
            st_c<T>(a.x, i, x);
            st_c<T>(a.r, i, r);
            pair_add(ps[j], pc[j], (double)r.re * (double)r.re + (double)r.im * (double)r.im,
                     0.0);
        }
    }
    block_partials<NR>(ps, pc, a.partials);
}

// p = r + beta p
template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void p_update_kernel(VecArgs a) {
    if (a.gate_running && a.ctl->n_running == 0) return;
    const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
    if (h >= a.Vh) return;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const SysState &s = a.state[j];
        if (!(s.flags & SYS_RUNNING)) continue;
        const T be = (T)s.beta;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t i = (size_t)j * a.fstride + (size_t)c * a.Vh + h;
            cpx<T> p = ld_c<T>(a.p, i), r = ld_c<T>(a.r, i);
            p.re = r.re + be * p.re;
            p.im = r.im + be * p.im;
            st_c<T>(a.p, i, p);
        }
    }
}

// ---------------------------------------------------------------------------
// single-field CG iteration with the reductions finished by their consumers
// ---------------------------------------------------------------------------
// Sum of the n (sum, error) pairs at x by the whole block, in the fixed order of
// block_sum2_pairs, returned to every thread: every block of a launch obtains the
// bitwise same total, so each can take the scalar step itself and no finalize
// kernel runs between the producer and the consumer.
__device__ __forceinline__ double block_total(const double *x, uint32_t n) {
    __shared__ double sh_red[2 * kWaves];
    __shared__ double sh_tot;
    const double t = block_sum2_pairs(x, (int)n, sh_red);
    if (threadIdx.x == 0) sh_tot = t;
    __syncthreads();
    return sh_tot;
}

// alpha = rr / <p, q> (the hop's partials), x += alpha p, r -= alpha q, partials of
// |r|^2.  Writes no solver state.  A breakdown (<p, q> not a finite positive
// number) leaves x and r alone and writes NaN partials, which the beta step of the
// next kernel turns into SYS_BREAKDOWN.
template <typename T>
__global__ __launch_bounds__(kBlock) void cg_update_fused_kernel(VecArgs a) {
    if (block_gate_closed(a.ctl, a.gate_running)) return;
    const double pq = block_total(a.fin_partials, a.fin_blocks);
    const SysState &s = a.state[0];
    const bool running = (s.flags & SYS_RUNNING) != 0;
    const bool ok = finite_pos(pq) && (s.rr >= 0.0 && s.rr < 1.0e300);
    const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
    double ps[1] = {0.0}, pc[1] = {0.0};
    if (running && !ok) {
        ps[0] = __builtin_nan("");
    } else if (running && h < a.Vh) {
        const T al = (T)(s.rr / pq);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t i = (size_t)c * a.Vh + h;
            cpx<T> x = ld_c<T>(a.x, i), p = ld_c<T>(a.p, i), r = ld_c<T>(a.r, i),
                   q = ld_c<T>(a.q, i);
            x.re += al * p.re;
            x.im += al * p.im;
            r.re -= al * q.re;
            r.im -= al * q.im;
            st_c<T>(a.x, i, x);
            st_c<T>(a.r, i, r);
            pair_add(ps[0], pc[0], (double)r.re * (double)r.re + (double)r.im * (double)r.im,
                     0.0);
        }
    }
    block_partials<1>(ps, pc, a.partials);
}

// |r_new|^2 from the partials of cg_update_fused, the beta step (solver_state.hpp)
// on a copy of the state, p = r + beta p while the system still runs.  Block 0
// stores the new state in a.state_out: the next iteration reads that buffer, so
// no block reads a state that another block of this launch is writing.  Block 0
// always runs (also when no system runs), so that a.state_out is always current.
template <typename T>
__global__ __launch_bounds__(kBlock) void p_update_fused_kernel(VecArgs a) {
    const bool closed = block_gate_closed(a.ctl, a.gate_running);
    if (closed && blockIdx.x != 0) return;
    SysState ns = a.state[0];
    ns.flags &= ~SYS_RESUME;
    bool left = false;
    if (!closed && (ns.flags & SYS_RUNNING)) {
        const double rr = block_total(a.fin_partials, a.fin_blocks);
        left = beta_step(ns, rr);
        const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
        if (!left && h < a.Vh) {
            const T be = (T)ns.beta;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const size_t i = (size_t)c * a.Vh + h;
                cpx<T> p = ld_c<T>(a.p, i), r = ld_c<T>(a.r, i);
                p.re = r.re + be * p.re;
                p.im = r.im + be * p.im;
                st_c<T>(a.p, i, p);
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.state_out[0] = ns;
        if (left) atomicAdd(&a.ctl->n_running, -1);
    }
}

int launch_cg_update_fused(const VecArgs &a, int fp64, hipStream_t stream) {
    dim3 grid(site_blocks(a.Vh));
    if (fp64)
        cg_update_fused_kernel<double><<<grid, kBlock, 0, stream>>>(a);
    else
        cg_update_fused_kernel<float><<<grid, kBlock, 0, stream>>>(a);
    return 0;
}

int launch_p_update_fused(const VecArgs &a, int fp64, hipStream_t stream) {
    dim3 grid(site_blocks(a.Vh));
    if (fp64)
        p_update_fused_kernel<double><<<grid, kBlock, 0, stream>>>(a);
    else
        p_update_fused_kernel<float><<<grid, kBlock, 0, stream>>>(a);
    return 0;
}

// ---------------------------------------------------------------------------
// single-reduction CG (Chronopoulos and Gear; solver_state.hpp cgcg_step)
// ---------------------------------------------------------------------------
// One site's update of one system: p = r + beta p; s = w + beta s; x += alpha p;
// r -= alpha s; returns the site's |r_new|^2 in FP64.
template <typename T>
__device__ __forceinline__ double cgcg_site(const VecArgs &a, size_t o, uint32_t h, T al, T be) {
    double rr = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const size_t i = o + (size_t)c * a.Vh + h;
        cpx<T> r = ld_c<T>(a.r, i), w = ld_c<T>(a.w, i), p = ld_c<T>(a.p, i),
               sv = ld_c<T>(a.s, i), x = ld_c<T>(a.x, i);
        p.re = r.re + be * p.re;
        p.im = r.im + be * p.im;
        sv.re = w.re + be * sv.re;
        sv.im = w.im + be * sv.im;
        x.re += al * p.re;
        x.im += al * p.im;
        r.re -= al * sv.re;
        r.im -= al * sv.im;
        st_c<T>(a.p, i, p);
        st_c<T>(a.s, i, sv);
        st_c<T>(a.x, i, x);
        st_c<T>(a.r, i, r);
        rr = fmat((double)r.re, (double)r.re, rr);
        rr = fmat((double)r.im, (double)r.im, rr);
    }
    return rr;
}

template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void cgcg_update_kernel(VecArgs a) {
    if (a.gate_running && a.ctl->n_running == 0) return;
    const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
    double ps[NR], pc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        ps[j] = 0.0;
        pc[j] = 0.0;
        const SysState &st = a.state[j];
        if (!(st.flags & SYS_RUNNING) || h >= a.Vh) continue;
        pair_add(ps[j], pc[j], cgcg_site<T>(a, (size_t)j * a.fstride, h, (T)st.alpha, (T)st.beta),
                 0.0);
    }
    block_partials<NR>(ps, pc, a.partials);
}

// One field, no finalize kernel: every block sums the hop's <r, w> partials and the
// previous update's |r|^2 partials in the same fixed order (bitwise the same totals),
// takes the scalar step on a copy of the state, and updates its sites; block 0 stores
// the new state in a.state_out (the next iteration's buffer, never a.state, which the
// other blocks are reading).  Block 0 always runs, so that a.state_out stays current.
// A breakdown or a system that parks leaves the vectors alone.
template <typename T>
__global__ __launch_bounds__(kBlock) void cgcg_update_fused_kernel(VecArgs a) {
    const bool closed = block_gate_closed(a.ctl, a.gate_running);
    if (closed && blockIdx.x != 0) return;
    SysState ns = a.state[0];
    bool left = false, step = false;
    double ps[1] = {0.0}, pc[1] = {0.0};
    if (!closed && (ns.flags & SYS_RUNNING)) {
        const double delta = block_total(a.fin_partials, a.fin_blocks);
        // just resumed: gamma comes from the state, the partials are stale
        const double gamma = (ns.flags & SYS_RESUME) ? 0.0
                                                     : block_total(a.fin_partials2, a.fin_blocks2);
        left = cgcg_step(ns, delta, gamma);
        step = !left;
        const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
        if (step && h < a.Vh)
            pair_add(ps[0], pc[0], cgcg_site<T>(a, 0, h, (T)ns.alpha, (T)ns.beta), 0.0);
    }
    if (!closed) block_partials<1>(ps, pc, a.partials);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.state_out[0] = ns;
        if (left) atomicAdd(&a.ctl->n_running, -1);
    }
}

int launch_cgcg_update(const VecArgs &a, int fp64, int nr, hipStream_t stream);
int launch_cgcg_update_fused(const VecArgs &a, int fp64, hipStream_t stream) {
    dim3 grid(site_blocks(a.Vh));
    if (fp64)
        cgcg_update_fused_kernel<double><<<grid, kBlock, 0, stream>>>(a);
    else
        cgcg_update_fused_kernel<float><<<grid, kBlock, 0, stream>>>(a);
    return 0;
}

// x64 += x32; x32 = 0 for parked systems
template <int NR>
__global__ __launch_bounds__(kBlock) void ru_accumulate_kernel(VecArgs a) {
    const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
    if (h >= a.Vh) return;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (!(a.state[j].flags & SYS_RU_PENDING)) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t i = (size_t)j * a.fstride + (size_t)c * a.Vh + h;
            cpx<float> xs = ld_c<float>(a.x, i);
            cpx<double> xd = ld_c<double>(a.x64, i);
            xd.re += (double)xs.re;
            xd.im += (double)xs.im;
            st_c<double>(a.x64, i, xd);
            st_c<float>(a.x, i, cpx<float>{0.0f, 0.0f});
        }
    }
}

// resumed systems: r_inner = r64 (rounded to T); p = r_inner + beta p
template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void ru_resume_kernel(VecArgs a) {
    const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
    if (h >= a.Vh) return;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const SysState &s = a.state[j];
        if (!(s.flags & SYS_RESUME)) continue;
        const T be = (T)s.beta;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t i = (size_t)j * a.fstride + (size_t)c * a.Vh + h;
            cpx<double> rd = ld_c<double>(a.r64, i);
            cpx<T> r{(T)rd.re, (T)rd.im};
            if (a.r != a.r64) st_c<T>(a.r, i, r);
            if (a.skip_p) continue;
            cpx<T> p = ld_c<T>(a.p, i);
            p.re = r.re + be * p.re;
            p.im = r.im + be * p.im;
            st_c<T>(a.p, i, p);
        }
    }
}

// multi-shift (Sec. 2.2, Eq. shlineq): base residual r -= alpha q; |r|^2 -> OP_MS_BETA
template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void ms_r_update_kernel(VecArgs a) {
    if (a.gate_running && a.ctl->n_running == 0) return;
    const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
    double ps[NR], pc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        ps[j] = 0.0;
        pc[j] = 0.0;
        const SysState &s = a.state[j];
        if (!(s.flags & SYS_RUNNING) || h >= a.Vh) continue;
        const T al = (T)s.alpha;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t i = (size_t)j * a.fstride + (size_t)c * a.Vh + h;
            cpx<T> r = ld_c<T>(a.r, i), q = ld_c<T>(a.q, i);
            r.re -= al * q.re;
            r.im -= al * q.im;
            st_c<T>(a.r, i, r);
            pair_add(ps[j], pc[j], (double)r.re * (double)r.re + (double)r.im * (double)r.im,
                     0.0);
        }
    }
    block_partials<NR>(ps, pc, a.partials);
}

// multi-shift, after beta: every shift that took part in this iteration steps
// x_k += alpha_k p_k with its old p_k, then the still active ones p_k = zeta_k r +
// beta_k p_k (one read of p_k for both); the base p = r + beta p.
//
// One block works on one chunk of kBlock sites for one shift (or, for the last
// index, the base directions), so every (shift, RHS) pair is its own streamed pass
// over its two fields and a retired shift costs one scalar test per block.  The
// shift blocks of a site chunk sit next to each other in the XCD-ordered block
// sequence: they run on the same XCD, where the base residual r they all read
// stays in L2.
template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void ms_p_update_kernel(VecArgs a) {
    if (a.gate_running && a.ctl->n_running == 0) return;
    const uint32_t nk = (uint32_t)a.nshift + 1;
    const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t k = lb % nk;
    const uint32_t h = (lb / nk) * kBlock + threadIdx.x;
    const Ctl &ctl = *a.ctl;
    if (k == (uint32_t)a.nshift) {  // base directions of the running systems
        if (h >= a.Vh) return;
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const SysState &s = a.state[j];
            if (!(s.flags & SYS_RUNNING)) continue;
            const T be = (T)s.beta;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const size_t i = (size_t)j * a.fstride + (size_t)c * a.Vh + h;
                cpx<T> p = ld_c<T>(a.p, i), r = ld_c<T>(a.r, i);
                p.re = r.re + be * p.re;
                p.im = r.im + be * p.im;
                st_c<T>(a.p, i, p);
            }
        }
        return;
    }
    // this shift for every RHS: wave-uniform tests, the loads of all its active
    // systems issued together
    bool any = false;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const SysState &s = a.state[j];
        const bool part = (s.flags & (SYS_RUNNING | SYS_FINISHING)) != 0;
        any = any || (part && ctl.ms[k * ctl.nrhs + s.gid].active != 0);
    }
    if (!any || h >= a.Vh) return;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const SysState &s = a.state[j];
        const bool running = (s.flags & SYS_RUNNING) != 0;
        if (!running && !(s.flags & SYS_FINISHING)) continue;
        const ShiftState &z = ctl.ms[k * ctl.nrhs + s.gid];
        if (!z.active) continue;
        const bool more = running && z.active == 1;
        const T ak = (T)z.alpha, zk = (T)z.zeta, bk = (T)z.beta;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t ir = (size_t)j * a.fstride + (size_t)c * a.Vh + h;
            const size_t i = (size_t)k * a.kstride + ir;
            cpx<T> p = ld_c<T>(a.ps, i), x = ld_c<T>(a.xs, i);
            x.re += ak * p.re;
            x.im += ak * p.im;
            st_c<T>(a.xs, i, x);
            if (more) {
                const cpx<T> r = ld_c<T>(a.r, ir);
                p.re = zk * r.re + bk * p.re;
                p.im = zk * r.im + bk * p.im;
                st_c<T>(a.ps, i, p);
            }
        }
    }
}

// one launcher per kernel template: precision and chunk size are compile-time
#define STG_VEC_LAUNCHER(NAME, KERNEL)                                                   \
    int NAME(const VecArgs &a, int fp64, int nr, hipStream_t stream) {                  \
        dim3 grid(site_blocks(a.Vh));                                                    \
        switch (nr * 2 + (fp64 ? 1 : 0)) {                                               \
            case 3: KERNEL<double, 1><<<grid, kBlock, 0, stream>>>(a); return 0;        \
            case 2: KERNEL<float, 1><<<grid, kBlock, 0, stream>>>(a); return 0;         \
            case 5: KERNEL<double, 2><<<grid, kBlock, 0, stream>>>(a); return 0;        \
            case 4: KERNEL<float, 2><<<grid, kBlock, 0, stream>>>(a); return 0;         \
            case 7: KERNEL<double, 3><<<grid, kBlock, 0, stream>>>(a); return 0;        \
            case 6: KERNEL<float, 3><<<grid, kBlock, 0, stream>>>(a); return 0;         \
            case 9: KERNEL<double, 4><<<grid, kBlock, 0, stream>>>(a); return 0;        \
            case 8: KERNEL<float, 4><<<grid, kBlock, 0, stream>>>(a); return 0;         \
            case 17: KERNEL<double, 8><<<grid, kBlock, 0, stream>>>(a); return 0;       \
            case 16: KERNEL<float, 8><<<grid, kBlock, 0, stream>>>(a); return 0;        \
            default: return -1;                                                          \
        }                                                                                \
    }

STG_VEC_LAUNCHER(launch_cg_update_only, cg_update_kernel)
STG_VEC_LAUNCHER(launch_p_update, p_update_kernel)
STG_VEC_LAUNCHER(launch_ru_resume, ru_resume_kernel)
STG_VEC_LAUNCHER(launch_ms_r_update_only, ms_r_update_kernel)
STG_VEC_LAUNCHER(launch_cgcg_update, cgcg_update_kernel)

int launch_cg_update(const VecArgs &a, int fp64, int nr, hipStream_t stream) {
    if (launch_cg_update_only(a, fp64, nr, stream)) return -1;
    FinArgs f{a.partials, site_blocks(a.Vh), nr, OP_BETA, a.gate_running, a.ctl, a.state, nullptr};
    return launch_finalize(f, stream);
}

// grid: (nshift + 1) blocks per chunk of kBlock sites
int launch_ms_p_update(const VecArgs &a, int fp64, int nr, hipStream_t stream) {
    dim3 grid(site_blocks(a.Vh) * (uint32_t)(a.nshift + 1));
    switch (nr * 2 + (fp64 ? 1 : 0)) {
        case 3: ms_p_update_kernel<double, 1><<<grid, kBlock, 0, stream>>>(a); return 0;
        case 2: ms_p_update_kernel<float, 1><<<grid, kBlock, 0, stream>>>(a); return 0;
        case 5: ms_p_update_kernel<double, 2><<<grid, kBlock, 0, stream>>>(a); return 0;
        case 4: ms_p_update_kernel<float, 2><<<grid, kBlock, 0, stream>>>(a); return 0;
        case 7: ms_p_update_kernel<double, 3><<<grid, kBlock, 0, stream>>>(a); return 0;
        case 6: ms_p_update_kernel<float, 3><<<grid, kBlock, 0, stream>>>(a); return 0;
        case 9: ms_p_update_kernel<double, 4><<<grid, kBlock, 0, stream>>>(a); return 0;
        case 8: ms_p_update_kernel<float, 4><<<grid, kBlock, 0, stream>>>(a); return 0;
        case 17: ms_p_update_kernel<double, 8><<<grid, kBlock, 0, stream>>>(a); return 0;
        case 16: ms_p_update_kernel<float, 8><<<grid, kBlock, 0, stream>>>(a); return 0;
        default: return -1;
    }
}

int launch_ms_r_update(const VecArgs &a, int fp64, int nr, hipStream_t stream) {
    if (launch_ms_r_update_only(a, fp64, nr, stream)) return -1;
    FinArgs f{a.partials, site_blocks(a.Vh), nr, OP_MS_BETA, a.gate_running, a.ctl, a.state,
              nullptr};
    return launch_finalize(f, stream);
}

// ---------------------------------------------------------------------------
// finishing the reductions: one block per system, fixed order, compensated
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void finalize_kernel(FinArgs f) {
    __shared__ double sh_red[2 * kWaves];
    if (block_gate_closed(f.ctl, f.gate_running)) return;
    const int j = blockIdx.x;
    double tot = block_sum2_pairs(f.partials + 2 * (size_t)j * f.nblocks, (int)f.nblocks, sh_red);
    double tot2 = 0.0;
    if (f.op == OP_CGCG)
        tot2 = block_sum2_pairs(f.partials2 + 2 * (size_t)j * f.nblocks2, (int)f.nblocks2, sh_red);
    if (f.op == OP_MS_ALPHA || f.op == OP_MS_BETA)
        finalize_ms_block(f.op, f.ctl, f.state, j, tot);
    else if (threadIdx.x == 0)
        finalize_one(f.op, f.ctl, f.state, f.out, j, tot, tot2);
}

int launch_finalize(const FinArgs &f, hipStream_t stream) {
    finalize_kernel<<<f.nr, kBlock, 0, stream>>>(f);
    return 0;
}

int launch_ru_accumulate(const VecArgs &a, int nr, hipStream_t stream) {
    dim3 grid(site_blocks(a.Vh));
    switch (nr) {
        case 1: ru_accumulate_kernel<1><<<grid, kBlock, 0, stream>>>(a); return 0;
        case 2: ru_accumulate_kernel<2><<<grid, kBlock, 0, stream>>>(a); return 0;
        case 3: ru_accumulate_kernel<3><<<grid, kBlock, 0, stream>>>(a); return 0;
        case 4: ru_accumulate_kernel<4><<<grid, kBlock, 0, stream>>>(a); return 0;
        case 8: ru_accumulate_kernel<8><<<grid, kBlock, 0, stream>>>(a); return 0;
        default: return -1;
    }
}

// ---------------------------------------------------------------------------
// compensated complex dot product of one vector pair
// ---------------------------------------------------------------------------
constexpr uint32_t kDotMaxBlocks = 1024;

size_t dot_blocks(size_t n) {
    size_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return b > kDotMaxBlocks ? kDotMaxBlocks : b;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void dot_kernel(size_t n, const void *x, const void *y,
                                                     double *partials) {
    // per-thread compensated accumulation of the real and imaginary parts
    double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kBlock) {
        cpx<T> a = ld_c<T>(x, i), b = ld_c<T>(y, i);
        // conj(a) b; products of two floats are exact in double
        double pr1 = (double)a.re * (double)b.re, pr2 = (double)a.im * (double)b.im;
        double pi1 = (double)a.re * (double)b.im, pi2 = -(double)a.im * (double)b.re;
        double e;
        two_sum(sr, pr1, sr, e);
        cr += e;
        two_sum(sr, pr2, sr, e);
        cr += e;
        two_sum(si, pi1, si, e);
        ci += e;
        two_sum(si, pi2, si, e);
        ci += e;
    }
    double ps[2] = {sr, si}, pc[2] = {cr, ci};
    block_partials<2>(ps, pc, partials);
}

int launch_dot(int fp64, int nvec, size_t n, const void *x, const void *y, double *partials,
               Ctl *ctl, int op, SysState *state, double *out, hipStream_t stream) {
    const size_t esz = fp64 ? 16 : 8;
    dim3 grid((uint32_t)dot_blocks(n));
    for (int j = 0; j < nvec; ++j) {
        const char *xj = reinterpret_cast<const char *>(x) + (size_t)j * n * esz;
        const char *yj = reinterpret_cast<const char *>(y) + (size_t)j * n * esz;
        SysState *sj = state ? state + j : nullptr;
        double *oj = out ? out + 2 * j : nullptr;
        if (fp64)
            dot_kernel<double><<<grid, kBlock, 0, stream>>>(n, xj, yj, partials);
        else
            dot_kernel<float><<<grid, kBlock, 0, stream>>>(n, xj, yj, partials);
        // OP_STORE finishes both parts (re, im); the solver ops use the real part
        FinArgs f{partials, grid.x, op == OP_STORE ? 2 : 1, op, 0, ctl, sj, oj};
        launch_finalize(f, stream);
    }
    return 0;
}

// ---------------------------------------------------------------------------
// packing (Sec. 2.3: keep rows 0 and 1; Sec. 4.1 layouts)
// ---------------------------------------------------------------------------

// double -> bfloat16, round to nearest even, via round-to-odd float: the float
// keeps 16 more bits than bfloat16, so the second rounding is the correct one.
__device__ __forceinline__ uint32_t bf16_rne(double x) {
    float f = __double2float_rz(x);
    uint32_t u = __float_as_uint(f);
    if ((double)f != x) u |= 1u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

__global__ __launch_bounds__(kBlock) void pack_links_kernel(uint32_t Vh, const double2 *src,
                                                            int fmt, void *dst) {
    const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
    const int s = blockIdx.y;
    if (h >= Vh) return;
    double2 e[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) e[a][b] = src[((size_t)(s * 3 + a) * 3 + b) * Vh + h];
    if (fmt == FMT_C128_18) {
        double2 *d = reinterpret_cast<double2 *>(dst);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) d[((size_t)(s * 3 + a) * 3 + b) * Vh + h] = e[a][b];
    } else if (fmt == FMT_C128_12) {
        double2 *d = reinterpret_cast<double2 *>(dst);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) d[((size_t)(s * 2 + a) * 3 + b) * Vh + h] = e[a][b];
    } else if (fmt == FMT_C64_12) {
        float4 *d = reinterpret_cast<float4 *>(dst);
        const double2 *flat = &e[0][0];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double2 u = flat[2 * k], v = flat[2 * k + 1];
            d[(size_t)(s * 3 + k) * Vh + h] =
                make_float4((float)u.x, (float)u.y, (float)v.x, (float)v.y);
        }
    } else {  // FMT_BF16_12
        const double2 *flat = &e[0][0];
        uint32_t w[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) w[k] = bf16_rne(flat[k].x) | (bf16_rne(flat[k].y) << 16);
        uint4 *da = reinterpret_cast<uint4 *>(dst);
        uint2 *db = reinterpret_cast<uint2 *>(da + (size_t)8 * Vh);
        da[(size_t)s * Vh + h] = make_uint4(w[0], w[1], w[2], w[3]);
        db[(size_t)s * Vh + h] = make_uint2(w[4], w[5]);
    }
}

int launch_pack_links(const Geom &g, const void *src, int fmt, void *dst, hipStream_t stream) {
    dim3 grid(site_blocks(g.Vh), 8);
    pack_links_kernel<<<grid, kBlock, 0, stream>>>(g.Vh, reinterpret_cast<const double2 *>(src),
                                                   fmt, dst);
    return 0;
}

__global__ __launch_bounds__(kBlock) void f64_to_f32_kernel(size_t n, const double *src,
                                                            float *dst) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kBlock)
        dst[i] = (float)src[i];
}

int launch_pack_phases_f32(size_t n, const double *src, float *dst, hipStream_t stream) {
    size_t b = (n + kBlock - 1) / kBlock;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    f64_to_f32_kernel<<<dim3((uint32_t)b), kBlock, 0, stream>>>(n, src, dst);
    return 0;
}

int launch_c128_to_c64(size_t n, const void *src, void *dst, hipStream_t stream) {
    return launch_pack_phases_f32(2 * n, reinterpret_cast<const double *>(src),
                                  reinterpret_cast<float *>(dst), stream);
}

__global__ __launch_bounds__(kBlock) void f32_to_f64_kernel(size_t n, const float *src,
                                                            double *dst) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kBlock)
        dst[i] = (double)src[i];
}

int launch_c64_to_c128(size_t n, const void *src, void *dst, hipStream_t stream) {
    size_t b = (2 * n + kBlock - 1) / kBlock;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    f32_to_f64_kernel<<<dim3((uint32_t)b), kBlock, 0, stream>>>(
        2 * n, reinterpret_cast<const float *>(src), reinterpret_cast<double *>(dst));
    return 0;
}

__global__ __launch_bounds__(kBlock) void zero_kernel(size_t n4, uint32_t *dst) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n4;
         i += (size_t)gridDim.x * kBlock)
        dst[i] = 0u;
}

int launch_zero(void *dst, size_t bytes, hipStream_t stream) {
    size_t n4 = bytes / 4;
    if (n4 == 0) return 0;
    size_t b = (n4 + kBlock - 1) / kBlock;
    if (b > 65536) b = 65536;
    zero_kernel<<<dim3((uint32_t)b), kBlock, 0, stream>>>(n4, reinterpret_cast<uint32_t *>(dst));
    return 0;
}

// ---------------------------------------------------------------------------
// rational function: y = a0 b + sum_k a_k x_k (FP64), one pass over the x_k
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void rational_sum_kernel(size_t n, int nshift, double a0,
                                                              const double *coeffs, const void *b,
                                                              const void *xs, void *y) {
    const size_t stride = (size_t)gridDim.x * kBlock;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const cpx<double> bi = ld_c<double>(b, i);
        cpx<double> acc{a0 * bi.re, a0 * bi.im};
        for (int k = 0; k < nshift; ++k) {
            const double a = coeffs[k];
            const cpx<double> x = ld_c<double>(xs, (size_t)k * n + i);
            acc.re = fmat(a, x.re, acc.re);
            acc.im = fmat(a, x.im, acc.im);
        }
        st_c<double>(y, i, acc);
    }
}

int launch_rational_sum(size_t n, int nshift, double a0, const double *coeffs, const void *b,
                        const void *xs, void *y, hipStream_t stream) {
    size_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) return 0;
    rational_sum_kernel<<<dim3((uint32_t)blocks), kBlock, 0, stream>>>(n, nshift, a0, coeffs, b,
                                                                      xs, y);
    return 0;
}

}  // namespace stg
