// Hermite predictor / corrector, block scheduler, time steps, energy and
// the device-resident block-step driver (Section 2).  All float64; the
// predictor and corrector are compiled without contraction so that their
// results follow the printed formulas operation by operation.
#include <cmath>

#include "common.hpp"
#include "integ.hpp"

namespace nb {

static inline unsigned grid_for(int64_t n, int threads, int64_t cap) {
    int64_t g = (n + threads - 1) / threads;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

__device__ __forceinline__ void latch(StepInfo *info, int32_t bits) {
    if (info) atomicOr(&info->status, bits);
}

// ---------------------------------------------------------------- predictor
__global__ void predict_kernel(int64_t n, double t_target, const StepInfo *__restrict__ info,
                               const double *__restrict__ t_target_dev,
                               const double *__restrict__ t, const double *__restrict__ x,
                               const double *__restrict__ v, const double *__restrict__ a,
                               const double *__restrict__ k, double *__restrict__ xp,
                               double *__restrict__ vp, const double *__restrict__ mass,
                               JRec *__restrict__ jrec, int rep) {
#pragma clang fp contract(off)
    if (info && info->done) return;
    const double tt = info ? info->t_next : (t_target_dev ? *t_target_dev : t_target);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double px[3], pv[3];
        predict_one(tt - t[i], x, v, a, k, i, n, px, pv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xp[c * n + i] = px[c];
            vp[c * n + i] = pv[c];
        }
        if (jrec) store_rec(rep, jrec + i, px[0], px[1], px[2], pv[0], pv[1], pv[2], mass[i]);
    }
}

// ---------------------------------------------------------------- scheduler
// t_next = min(t + dt) by a grid-wide reduction whose last-arriving block
// finishes it; then a count / scan / compaction pass that writes the active
// indices in ascending order.  min is exact, and the scan works on integer
// counts in block order, so the result is independent of timing.
__global__ __launch_bounds__(256) void sched_min_kernel(int64_t n, const double *__restrict__ t,
                                                        const double *__restrict__ dt,
                                                        double *__restrict__ partial,
                                                        StepInfo *__restrict__ info) {
    __shared__ double red[256];
    __shared__ bool last;
    double m = INFINITY;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = fmin(m, t[i] + dt[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = red[0];
        __threadfence();
        unsigned tk = __hip_atomic_fetch_add(&info->ticket0, 1u, __ATOMIC_ACQ_REL,
                                             __HIP_MEMORY_SCOPE_AGENT);
        last = (tk == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    m = INFINITY;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x)
        m = fmin(m, __builtin_nontemporal_load(&partial[b]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double tn = red[0];
        info->t_next = tn;
        const bool done = !(tn <= info->t_end);
        info->done = done ? 1 : 0;
        if (done) info->n_i = 0;
        __hip_atomic_store(&info->ticket0, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ __forceinline__ bool is_active(const double *t, const double *dt, int64_t i,
                                          double tn) {
    return t[i] + dt[i] == tn;
}

// Exclusive scan, in block order, of the per-block counts of a grid of at
// most 1024 blocks of 256 threads, in place; returns the total.  Run by all
// threads of the one (last) block: each thread scans 4 consecutive counts,
// then a block scan of the 256 thread totals.
__device__ int64_t block_order_scan(int64_t *counts) {
    __shared__ int64_t tsum[256];
    int64_t cb[4], run = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const unsigned b = threadIdx.x * 4 + q;
        cb[q] = b < gridDim.x ? __builtin_nontemporal_load(&counts[b]) : 0;
        run += cb[q];
    }
    tsum[threadIdx.x] = run;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int64_t v = (int)threadIdx.x >= o ? tsum[threadIdx.x - o] : 0;
        __syncthreads();
        tsum[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t off = tsum[threadIdx.x] - run;  // exclusive prefix of this thread
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const unsigned b = threadIdx.x * 4 + q;
        if (b < gridDim.x) counts[b] = off;
        off += cb[q];
    }
    return tsum[255];
}

// Minimum over the 256 threads of a block (every thread gets it).
__device__ double block_min(double m) {
    __shared__ double wm[4];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    return fmin(fmin(wm[0], wm[1]), fmin(wm[2], wm[3]));
}

__global__ __launch_bounds__(256) void sched_count_kernel(
    int64_t n, const double *__restrict__ t, const double *__restrict__ dt,
    int64_t *__restrict__ counts, StepInfo *__restrict__ info, int count_steps,
    int64_t *__restrict__ n_i_out, double *__restrict__ t_next_out) {
    __shared__ int64_t red[256];
    __shared__ bool last;
    if (info->done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (n_i_out) *n_i_out = 0;
            if (t_next_out) *t_next_out = info->t_next;
        }
        return;
    }
    const double tn = info->t_next;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    int64_t c = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) c += is_active(t, dt, i, tn);
    red[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        counts[blockIdx.x] = red[0];
        __threadfence();
        unsigned tk = __hip_atomic_fetch_add(&info->ticket1, 1u, __ATOMIC_ACQ_REL,
                                             __HIP_MEMORY_SCOPE_AGENT);
        last = (tk == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    const int64_t total = block_order_scan(counts);
    if (threadIdx.x == 255) {
        info->n_i = total;
        if (count_steps) {
            info->steps += 1;
            info->interactions += total * n;
        }
        if (n_i_out) *n_i_out = total;
        if (t_next_out) *t_next_out = tn;
        __hip_atomic_store(&info->ticket1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Writes the indices i in [lo, hi) with t + dt == tn to active[base...] in
// ascending order (all threads of a block of 256).
__device__ void compact_chunk(int64_t lo, int64_t hi, int64_t base, double tn,
                              const double *__restrict__ t, const double *__restrict__ dt,
                              int32_t *__restrict__ active) {
    __shared__ int wsum[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t p = lo; p < hi; p += blockDim.x) {
        const int64_t i = p + threadIdx.x;
        const bool f = i < hi && is_active(t, dt, i, tn);
        const unsigned long long bal = __ballot(f);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wave] = __popcll(bal);
        __syncthreads();
        int woff = 0, tot = 0;
        for (int w = 0; w < 4; ++w) {
            if (w < wave) woff += wsum[w];
            tot += wsum[w];
        }
        if (f) active[base + woff + before] = (int32_t)i;
        base += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void sched_compact_kernel(int64_t n,
                                                            const double *__restrict__ t,
                                                            const double *__restrict__ dt,
                                                            const int64_t *__restrict__ offsets,
                                                            const StepInfo *__restrict__ info,
                                                            int32_t *__restrict__ active) {
    if (info->done) return;
    const double tn = info->t_next;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    compact_chunk(lo, hi, offsets[blockIdx.x], tn, t, dt, active);
}

// Block step of the driver for n > kSmallStep, without grid-wide fences:
// each kernel leaves per-block partial results that the next kernel folds
// (every block of it redundantly where all need the value), so the launch
// boundaries order the passes.
//   step_scan_kernel    t_next (see below); per chunk of particles the
//                       number in the block (t + dt == t_next), the minimum
//                       of t + dt over the others, and the prediction of
//                       every particle to t_next (state and j records);
//   step_compact_kernel each chunk's offset = the counts of the chunks
//                       before it, then the chunk's block indices in
//                       ascending order; chunk 0 also writes n_i and folds
//                       the minima outside the block into rest_min;
//   pair sums, corrector (correct_kernel with `mins`: per corrector block
//                       the minimum of the new t + dt of its particles).
// The next step's t_next is the minimum of rest_min and the corrector's
// minima; at the first step of a call it comes from sched_min_kernel.  The
// block, its order, the predicted values and t_next are those of the
// separate sched_min / sched_count / sched_compact / predict passes.
__global__ __launch_bounds__(256) void step_scan_kernel(
    int64_t n, StepInfo *__restrict__ info, int fold, const double *__restrict__ cmin,
    int ncmin, const double *__restrict__ t, const double *__restrict__ dt,
    const double *__restrict__ x, const double *__restrict__ v, const double *__restrict__ a,
    const double *__restrict__ k, double *__restrict__ xp, double *__restrict__ vp,
    const double *__restrict__ mass, JRec *__restrict__ jrec, int rep,
    int64_t *__restrict__ counts, double *__restrict__ rmin) {
    __shared__ int64_t red[256];
    if (info->done) return;
    double tn;
    if (fold) {
        double m = INFINITY;
        for (int b = threadIdx.x; b < ncmin; b += blockDim.x) m = fmin(m, cmin[b]);
        tn = fmin(block_min(m), info->rest_min);
        const bool done = !(tn <= info->t_end);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            info->t_next = tn;
            if (done) {
                info->n_i = 0;
                info->done = 1;
            }
        }
        if (done) return;
    } else {
        tn = info->t_next;
    }
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    int64_t c = 0;
    double m = INFINITY;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const double ti = t[i];
        const double e = ti + dt[i];
        if (e == tn)
            ++c;
        else
            m = fmin(m, e);
        double px[3], pv[3];
        predict_one(tn - ti, x, v, a, k, i, n, px, pv);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            xp[q * n + i] = px[q];
            vp[q * n + i] = pv[q];
        }
        store_rec(rep, jrec + i, px[0], px[1], px[2], pv[0], pv[1], pv[2], mass[i]);
    }
    m = block_min(m);
    red[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        counts[blockIdx.x] = red[0];
        rmin[blockIdx.x] = m;
    }
}

// Sum over the 256 threads of a block (every thread gets it).
__device__ int64_t block_sum(int64_t c) {
    __shared__ int64_t ws[4];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
    __syncthreads();
    return (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

__global__ __launch_bounds__(256) void step_compact_kernel(int64_t n, StepInfo *__restrict__ info,
                                                           const double *__restrict__ t,
                                                           const double *__restrict__ dt,
                                                           const int64_t *__restrict__ counts,
                                                           const double *__restrict__ rmin,
                                                           int32_t *__restrict__ active) {
    if (info->done) return;
    const double tn = info->t_next;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    // chunk 0 (offset 0) totals the counts and folds the minima; the
    // others sum the counts of the chunks before them
    const unsigned upto = blockIdx.x == 0 ? gridDim.x : blockIdx.x;
    int64_t c = 0;
    double m = INFINITY;
    for (unsigned b = threadIdx.x; b < upto; b += blockDim.x) {
        c += counts[b];
        if (blockIdx.x == 0) m = fmin(m, rmin[b]);
    }
    c = block_sum(c);
    if (blockIdx.x == 0) {
        m = block_min(m);
        if (threadIdx.x == 0) {
            info->n_i = c;
            info->rest_min = m;
            info->steps += 1;
            info->interactions += c * n;
        }
        c = 0;
    }
    compact_chunk(lo, hi, c, tn, t, dt, active);
}

// Small systems (n <= kSmallStep): the whole scheduling part of a block step
// -- t_next = min(t + dt), the block in ascending order, and the prediction
// of every particle -- in one workgroup of 1024 threads, i.e. one launch
// instead of four (each of which costs a few microseconds at this size).
// Same arithmetic as sched_* and predict_kernel: exact minimum, block-order
// compaction, the Section 2 predictor.
constexpr int64_t kSmallStep = 2048;
constexpr int kSmallThreads = 1024;

__global__ __launch_bounds__(kSmallThreads) void small_step_kernel(
    int64_t n, StepInfo *__restrict__ info, const double *__restrict__ t,
    const double *__restrict__ dt, const double *__restrict__ x, const double *__restrict__ v,
    const double *__restrict__ a, const double *__restrict__ k, double *__restrict__ xp,
    double *__restrict__ vp, const double *__restrict__ mass, JRec *__restrict__ jrec, int rep,
    int32_t *__restrict__ active, int count_steps) {
    constexpr int NW = kSmallThreads / 64;
    __shared__ double wmin[NW];
    __shared__ int wcnt[NW];
    __shared__ double s_tn;
    __shared__ int s_done;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double mn = INFINITY;
    for (int64_t i = tid; i < n; i += kSmallThreads) mn = fmin(mn, t[i] + dt[i]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));
    if (lane == 0) wmin[wave] = mn;
    __syncthreads();
    if (tid == 0) {
        double tn = wmin[0];
        for (int w = 1; w < NW; ++w) tn = fmin(tn, wmin[w]);
        const int done = !(tn <= info->t_end);
        info->t_next = tn;
        info->done = done;
        if (done) info->n_i = 0;
        s_tn = tn;
        s_done = done;
    }
    __syncthreads();
    if (s_done) return;
    const double tn = s_tn;
    // the block, ascending
    int64_t base = 0;
    for (int64_t p = 0; p < n; p += kSmallThreads) {
        const int64_t i = p + tid;
        const bool f = i < n && t[i] + dt[i] == tn;
        const unsigned long long bal = __ballot(f);
        if (lane == 0) wcnt[wave] = __popcll(bal);
        __syncthreads();
        int woff = 0, tot = 0;
        for (int w = 0; w < NW; ++w) {
            woff += (w < wave) ? wcnt[w] : 0;
            tot += wcnt[w];
        }
        if (f) active[base + woff + __popcll(bal & ((1ull << lane) - 1ull))] = (int32_t)i;
        base += tot;
        __syncthreads();
    }
    // every particle predicted to t_next
    for (int64_t i = tid; i < n; i += kSmallThreads) {
        double px[3], pv[3];
        predict_one(tn - t[i], x, v, a, k, i, n, px, pv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xp[c * n + i] = px[c];
            vp[c * n + i] = pv[c];
        }
        if (jrec) store_rec(rep, jrec + i, px[0], px[1], px[2], pv[0], pv[1], pv[2], mass[i]);
    }
    if (tid == 0) {
        info->n_i = base;
        if (count_steps) {
            info->steps += 1;
            info->interactions += base * n;
        }
    }
}

static int sched_grids(int64_t n, unsigned *g1, unsigned *g2) {
    *g1 = grid_for(n, 256 * 8, 1024);
    *g2 = grid_for(n, 1024, 1024);
    return NBODY_OK;
}

static int launch_schedule(nbody_ctx *ctx, int64_t n, const double *t, const double *dt,
                           int32_t *active, int count_steps, int64_t *n_i_out,
                           double *t_next_out) {
    unsigned g1, g2;
    sched_grids(n, &g1, &g2);
    NB_TRY(ensure(ctx, &ctx->work, &ctx->work_bytes, 2048 * sizeof(double)));
    double *partial = (double *)ctx->work;
    int64_t *counts = (int64_t *)ctx->work + 1024;
    sched_min_kernel<<<g1, 256, 0, ctx->stream>>>(n, t, dt, partial, ctx->info);
    sched_count_kernel<<<g2, 256, 0, ctx->stream>>>(n, t, dt, counts, ctx->info, count_steps,
                                                    n_i_out, t_next_out);
    sched_compact_kernel<<<g2, 256, 0, ctx->stream>>>(n, t, dt, counts, ctx->info, active);
    return hip_check(ctx, hipGetLastError(), "scheduler");
}

__global__ void set_info_kernel(StepInfo *info, double t_end, int reset_counters) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        info->t_end = t_end;
        info->done = 0;
        if (reset_counters) {
            info->steps = 0;
            info->interactions = 0;
        }
    }
}

// ---------------------------------------------------------------- corrector
__global__ void correct_kernel(int64_t n, int64_t n_i_arg, const int64_t *__restrict__ n_i_dev,
                               const StepInfo *__restrict__ cinfo,
                               StepInfo *__restrict__ sinfo, const int32_t *__restrict__ active,
                               const double *__restrict__ xp, const double *__restrict__ vp,
                               const double *__restrict__ acc_new,
                               const double *__restrict__ jerk_new, int64_t stride_new,
                               double eta, double dt_max, double dt_min, int fixed_dt,
                               double *__restrict__ t, double *__restrict__ dtv,
                               double *__restrict__ x, double *__restrict__ v,
                               double *__restrict__ a, double *__restrict__ k,
                               double *__restrict__ mins) {
#pragma clang fp contract(off)
    // with `mins` (the block-step driver, blocks of 256 threads): also the
    // minimum of the new t + dt of the block's particles, per corrector
    // block (infinity for blocks without one), for the next step's t_next;
    // nothing once the run is done (no block was scheduled)
    if (mins && cinfo->done) return;
    int64_t n_i = cinfo ? cinfo->n_i : n_i_arg;
    if (n_i_dev) {
        // device-counted block of at most n_i_arg slots
        n_i = *n_i_dev;
        if (n_i > n_i_arg) {
            if (blockIdx.x == 0 && threadIdx.x == 0) latch(sinfo, ST_INDEX);
            n_i = n_i_arg;
        }
    }
    const int64_t sn = stride_new > 0 ? stride_new : n_i;
    double m = INFINITY;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n_i;
         s += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = active ? (int64_t)active[s] : s;
        if (i < 0 || i >= n) {
            latch(sinfo, ST_INDEX);
            continue;
        }
        double a1v[3], k1v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a1v[c] = acc_new[c * sn + s];
            k1v[c] = jerk_new[c * sn + s];
        }
        const int32_t st = correct_one(i, n, xp, vp, a1v, k1v, eta, dt_max, dt_min, fixed_dt, t,
                                       dtv, x, v, a, k);
        if (st) latch(sinfo, st);
        if (mins) m = fmin(m, t[i] + dtv[i]);
    }
    if (!mins) return;
    m = block_min(m);
    if (threadIdx.x == 0) mins[blockIdx.x] = m;
}

// ------------------------------------------------------------ initial steps
__global__ void initial_dt_kernel(int64_t n, double t0, const double *__restrict__ a,
                                  const double *__restrict__ k, double eta_s, double dt_max,
                                  double dt_min, double *__restrict__ dt, StepInfo *info) {
#pragma clang fp contract(off)
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t st = 0;
        dt[i] = initial_dt_one(i, n, t0, a, k, eta_s, dt_max, dt_min, &st);
        if (st) latch(info, st);
    }
}

__global__ void fill_kernel(int64_t n, double v, double *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = v;
}

// ------------------------------------------------------------------ energy
// phi_i = -sum_{j != i} m_j / sqrt(|x_j - x_i|^2 + eps2) in float64, one
// lane per i, j wave-uniform; K and W are reduced per block in a fixed tree
// and across blocks in block order by the last block to finish.
__global__ __launch_bounds__(256) void energy_kernel(int64_t n, const double *__restrict__ pos,
                                                     const double *__restrict__ vel,
                                                     const double *__restrict__ mass,
                                                     double eps2, double *__restrict__ partial,
                                                     StepInfo *__restrict__ info,
                                                     double *__restrict__ out) {
    __shared__ double rk[256], rw[256];
    __shared__ bool last;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double kin = 0.0, wpot = 0.0;
    // j-side reads through the constant address space: wave-uniform scalar loads
    typedef const __attribute__((address_space(4))) double *CD;
    const CD pk = (CD)pos;
    const CD mk = (CD)mass;
    if (i < n) {
        const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
        double ph = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double rx = pk[j] - xi, ry = pk[n + j] - yi, rz = pk[2 * n + j] - zi;
            const double term = mk[j] / sqrt(rx * rx + ry * ry + rz * rz + eps2);
            ph -= (j == i) ? 0.0 : term;
        }
        const double u = vel[i], w = vel[n + i], z = vel[2 * n + i];
        kin = 0.5 * mass[i] * (u * u + w * w + z * z);
        wpot = mass[i] * ph;
    }
    rk[threadIdx.x] = kin;
    rw[threadIdx.x] = wpot;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            rk[threadIdx.x] += rk[threadIdx.x + o];
            rw[threadIdx.x] += rw[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = rk[0];
        partial[2 * blockIdx.x + 1] = rw[0];
        __threadfence();
        unsigned tk = __hip_atomic_fetch_add(&info->ticket2, 1u, __ATOMIC_ACQ_REL,
                                             __HIP_MEMORY_SCOPE_AGENT);
        last = (tk == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (threadIdx.x == 0) {
        double K = 0.0, W = 0.0;
        for (unsigned b = 0; b < gridDim.x; ++b) {
            K += __builtin_nontemporal_load(&partial[2 * b]);
            W += __builtin_nontemporal_load(&partial[2 * b + 1]);
        }
        out[0] = K;
        out[1] = 0.5 * W;
        __hip_atomic_store(&info->ticket2, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

static bool pow2(double d) {
    int e;
    return d > 0 && std::isfinite(d) && std::frexp(d, &e) == 0.5;
}

}  // namespace nb

using namespace nb;

extern "C" {

int nbody_predict(nbody_ctx *ctx, int64_t n, double t_target, const double *t, const double *x,
                  const double *v, const double *a, const double *k, double *xp, double *vp) {
    if (!ctx) return NBODY_E_INVAL;
    if (n < 0 || !std::isfinite(t_target)) return fail(ctx, NBODY_E_INVAL, "nbody_predict: bad args");
    if (n == 0) return NBODY_OK;
    if (!t || !x || !v || !a || !k || !xp || !vp)
        return fail(ctx, NBODY_E_INVAL, "nbody_predict: null array");
    NB_TRY(activate(ctx));
    predict_kernel<<<grid_for(n, 256, 16 * ctx->cus), 256, 0, ctx->stream>>>(
        n, t_target, nullptr, nullptr, t, x, v, a, k, xp, vp, nullptr, nullptr, 0);
    return hip_check(ctx, hipGetLastError(), "predict_kernel");
}

int nbody_schedule(nbody_ctx *ctx, int64_t n, const double *t, const double *dt,
                   int32_t *active_idx, int64_t *n_i_out, double *t_next_out) {
    if (!ctx) return NBODY_E_INVAL;
    if (n < 1 || n > 0x7fffffffLL || !t || !dt || !active_idx || !n_i_out || !t_next_out)
        return fail(ctx, NBODY_E_INVAL, "nbody_schedule: bad args");
    NB_TRY(activate(ctx));
    set_info_kernel<<<1, 64, 0, ctx->stream>>>(ctx->info, INFINITY, 0);
    return launch_schedule(ctx, n, t, dt, active_idx, 0, n_i_out, t_next_out);
}

int nbody_correct(nbody_ctx *ctx, int64_t n, int64_t n_i, const int32_t *active_idx,
                  const double *xp, const double *vp, const double *acc_new,
                  const double *jerk_new, double eta, double dt_max, double dt_min,
                  int fixed_dt, double *t, double *dt, double *x, double *v, double *a,
                  double *k) {
    if (!ctx) return NBODY_E_INVAL;
    if (n < 1 || n_i < 0 || (active_idx == nullptr && n_i > n) || !(dt_min > 0) ||
        !(dt_max >= dt_min) || !(eta > 0 || fixed_dt))
        return fail(ctx, NBODY_E_INVAL, "nbody_correct: bad args");
    if (n_i == 0) return NBODY_OK;
    if (!xp || !vp || !acc_new || !jerk_new || !t || !dt || !x || !v || !a || !k)
        return fail(ctx, NBODY_E_INVAL, "nbody_correct: null array");
    NB_TRY(activate(ctx));
    correct_kernel<<<grid_for(n_i, 256, 16 * ctx->cus), 256, 0, ctx->stream>>>(
        n, n_i, nullptr, nullptr, ctx->info, active_idx, xp, vp, acc_new, jerk_new, n_i, eta, dt_max,
        dt_min, fixed_dt, t, dt, x, v, a, k, nullptr);
    return hip_check(ctx, hipGetLastError(), "correct_kernel");
}

int nbody_predict_dev(nbody_ctx *ctx, int64_t n, const double *t_target_dev, const double *t,
                      const double *x, const double *v, const double *a, const double *k,
                      double *xp, double *vp) {
    if (!ctx) return NBODY_E_INVAL;
    if (n < 0) return fail(ctx, NBODY_E_INVAL, "nbody_predict_dev: bad args");
    if (n == 0) return NBODY_OK;
    if (!t_target_dev || !t || !x || !v || !a || !k || !xp || !vp)
        return fail(ctx, NBODY_E_INVAL, "nbody_predict_dev: null array");
    NB_TRY(activate(ctx));
    predict_kernel<<<grid_for(n, 256, 16 * ctx->cus), 256, 0, ctx->stream>>>(
        n, 0.0, nullptr, t_target_dev, t, x, v, a, k, xp, vp, nullptr, nullptr, 0);
    return hip_check(ctx, hipGetLastError(), "predict_kernel");
}

int nbody_correct_dev(nbody_ctx *ctx, int64_t n, const int64_t *n_i_dev, int64_t n_i_cap,
                      const int32_t *active_idx, const double *xp, const double *vp,
                      const double *acc_new, const double *jerk_new, double eta, double dt_max,
                      double dt_min, int fixed_dt, double *t, double *dt, double *x, double *v,
                      double *a, double *k) {
    if (!ctx) return NBODY_E_INVAL;
    if (n < 1 || n_i_cap < 0 || (active_idx == nullptr && n_i_cap > n) || !(dt_min > 0) ||
        !(dt_max >= dt_min) || !(eta > 0 || fixed_dt))
        return fail(ctx, NBODY_E_INVAL, "nbody_correct_dev: bad args");
    if (n_i_cap == 0) return NBODY_OK;
    if (!n_i_dev || !xp || !vp || !acc_new || !jerk_new || !t || !dt || !x || !v || !a || !k)
        return fail(ctx, NBODY_E_INVAL, "nbody_correct_dev: null array");
    NB_TRY(activate(ctx));
    correct_kernel<<<grid_for(n_i_cap, 256, 16 * ctx->cus), 256, 0, ctx->stream>>>(
        n, n_i_cap, n_i_dev, nullptr, ctx->info, active_idx, xp, vp, acc_new, jerk_new, n_i_cap,
        eta, dt_max, dt_min, fixed_dt, t, dt, x, v, a, k, nullptr);
    return hip_check(ctx, hipGetLastError(), "correct_kernel");
}

int nbody_initial_dt(nbody_ctx *ctx, int64_t n, double t0, const double *a, const double *k,
                     double eta_s, double dt_max, double dt_min, double *dt) {
    if (!ctx) return NBODY_E_INVAL;
    if (n < 0 || !pow2(dt_max) || !(dt_min > 0) || !(dt_max >= dt_min) || !(eta_s > 0) ||
        !std::isfinite(t0))
        return fail(ctx, NBODY_E_INVAL, "nbody_initial_dt: bad args");
    if (n == 0) return NBODY_OK;
    if (!a || !k || !dt) return fail(ctx, NBODY_E_INVAL, "nbody_initial_dt: null array");
    NB_TRY(activate(ctx));
    initial_dt_kernel<<<grid_for(n, 256, 16 * ctx->cus), 256, 0, ctx->stream>>>(
        n, t0, a, k, eta_s, dt_max, dt_min, dt, ctx->info);
    return hip_check(ctx, hipGetLastError(), "initial_dt_kernel");
}

int nbody_energy(nbody_ctx *ctx, int64_t n, const double *pos, const double *vel,
                 const double *mass, double eps2, double *out) {
    if (!ctx) return NBODY_E_INVAL;
    if (n < 1 || n > 0x7fffffffLL || !(eps2 >= 0) || std::isinf(eps2) || !pos || !vel ||
        !mass || !out)
        return fail(ctx, NBODY_E_INVAL, "nbody_energy: bad args");
    NB_TRY(activate(ctx));
    const unsigned g = grid_for(n, 256, 1 << 30);
    NB_TRY(ensure(ctx, &ctx->part, &ctx->part_bytes, (size_t)g * 2 * sizeof(double)));
    energy_kernel<<<g, 256, 0, ctx->stream>>>(n, pos, vel, mass, eps2, (double *)ctx->part,
                                              ctx->info, out);
    return hip_check(ctx, hipGetLastError(), "energy_kernel");
}

static int check_system(nbody_ctx *ctx, const nbody_system *s) {
    if (!s || s->n < 1 || s->n > 0x7fffffffLL)
        return fail(ctx, NBODY_E_INVAL, "system: bad size");
    if (!s->t || !s->dt || !s->x || !s->v || !s->a || !s->k || !s->m)
        return fail(ctx, NBODY_E_INVAL, "system: null array");
    if (!(s->eps2 >= 0) || std::isinf(s->eps2) || !(s->eta > 0) || !(s->eta_s > 0) ||
        !pow2(s->dt_max) || !(s->dt_min > 0) || !(s->dt_max >= s->dt_min))
        return fail(ctx, NBODY_E_INVAL, "system: bad parameters");
    if (s->flags & ~(NBODY_ACC_DS | NBODY_FIXED_DT))
        return fail(ctx, NBODY_E_INVAL, "system: unknown flags");
    return NBODY_OK;
}

int nbody_init(nbody_ctx *ctx, const nbody_system *s, double t0) {
    if (!ctx) return NBODY_E_INVAL;
    NB_TRY(check_system(ctx, s));
    if (!std::isfinite(t0)) return fail(ctx, NBODY_E_INVAL, "nbody_init: bad t0");
    NB_TRY(activate(ctx));
    const int64_t n = s->n;
    fill_kernel<<<grid_for(n, 256, 4 * ctx->cus), 256, 0, ctx->stream>>>(n, t0, s->t);
    NB_TRY(hip_check(ctx, hipGetLastError(), "fill_kernel"));
    NB_TRY(ensure(ctx, &ctx->jrec, &ctx->jrec_bytes, (size_t)n * sizeof(JRec)));
    ForceCall c;
    c.mode = acc_mode(s->flags);
    c.shape = shape_for(pick_shape(ctx, n, n), c.mode);
    NB_TRY(launch_pack(ctx, c.shape.rep, n, s->x, s->v, s->m, (JRec *)ctx->jrec));
    c.jrec = (const JRec *)ctx->jrec;
    c.n_j = n;
    c.pos = s->x;
    c.vel = s->v;
    c.n_i = n;
    c.eps2 = s->eps2;
    c.acc = s->a;
    c.jerk = s->k;
    c.out_stride = n;
    NB_TRY(launch_force(ctx, c));
    if (s->flags & NBODY_FIXED_DT) {
        fill_kernel<<<grid_for(n, 256, 4 * ctx->cus), 256, 0, ctx->stream>>>(n, s->dt_max, s->dt);
        return hip_check(ctx, hipGetLastError(), "fill_kernel");
    }
    initial_dt_kernel<<<grid_for(n, 256, 16 * ctx->cus), 256, 0, ctx->stream>>>(
        n, t0, s->a, s->k, s->eta_s, s->dt_max, s->dt_min, s->dt, ctx->info);
    return hip_check(ctx, hipGetLastError(), "initial_dt_kernel");
}

int nbody_blockstep(nbody_ctx *ctx, const nbody_system *s, int64_t max_steps, double t_end,
                    int64_t *steps_done, int64_t *interactions) {
    if (!ctx) return NBODY_E_INVAL;
    NB_TRY(check_system(ctx, s));
    if (max_steps < 0 || std::isnan(t_end)) return fail(ctx, NBODY_E_INVAL, "nbody_blockstep: bad args");
    if (steps_done) *steps_done = 0;
    if (interactions) *interactions = 0;
    NB_TRY(activate(ctx));
    const int64_t n = s->n;
    // step buffers: xp, vp, acc_new, jerk_new (3n each) + active (n int32)
    const size_t vec = (size_t)3 * n * sizeof(double);
    NB_TRY(ensure(ctx, &ctx->bs, &ctx->bs_bytes, 4 * vec + (size_t)n * sizeof(int32_t)));
    NB_TRY(ensure(ctx, &ctx->jrec, &ctx->jrec_bytes, (size_t)n * sizeof(JRec)));
    double *xp = (double *)ctx->bs;
    double *vp = (double *)((char *)ctx->bs + vec);
    double *an = (double *)((char *)ctx->bs + 2 * vec);
    double *kn = (double *)((char *)ctx->bs + 3 * vec);
    int32_t *act = (int32_t *)((char *)ctx->bs + 4 * vec);
    JRec *jr = (JRec *)ctx->jrec;

    set_info_kernel<<<1, 64, 0, ctx->stream>>>(ctx->info, t_end, 1);
    NB_TRY(hip_check(ctx, hipGetLastError(), "set_info"));

    ForceCall c;
    c.mode = acc_mode(s->flags);
    c.shape = shape_for(dynamic_shape(ctx, n), c.mode);
    c.jl_shape = shape_for(dynamic_small_shape(ctx, n, &c.jl_max), c.mode);
    if (c.shape.rep != REP_F64) c.jl_max = 0;  // the j-lane kernel reads float64 records
    c.jrec = jr;
    c.n_j = n;
    c.pos = xp;
    c.vel = vp;
    c.active = act;
    c.n_i_dev = &ctx->info->n_i;
    c.n_i_cap = n;
    c.eps2 = s->eps2;
    c.acc = an;
    c.jerk = kn;
    c.pot = nullptr;
    c.out_stride = n;

    // Systems of up to kSmallStep particles schedule and predict in one
    // workgroup per step.  Larger ones take three launches besides the pair
    // sums (step_scan_kernel, step_compact_kernel, the corrector with its
    // per-block minima); the first t_next of the call comes from
    // sched_min_kernel, the later ones are folded by step_scan_kernel.
    const bool small = n <= kSmallStep;
    const unsigned gp = grid_for(n, 256, 16 * ctx->cus);
    const unsigned gs = grid_for(n, 256, 1024);  // step_scan / step_compact chunks
    const unsigned gc = grid_for(n, 256, 1024);  // corrector blocks (driver)
    double *rmin = nullptr, *cmin = nullptr;
    int64_t *counts = nullptr;
    if (!small) {
        NB_TRY(ensure(ctx, &ctx->work, &ctx->work_bytes, 4096 * sizeof(double)));
        double *partial = (double *)ctx->work;
        counts = (int64_t *)ctx->work + 1024;
        rmin = (double *)ctx->work + 2048;
        cmin = (double *)ctx->work + 3072;
        unsigned g1, g2;
        sched_grids(n, &g1, &g2);
        sched_min_kernel<<<g1, 256, 0, ctx->stream>>>(n, s->t, s->dt, partial, ctx->info);
        NB_TRY(hip_check(ctx, hipGetLastError(), "sched_min_kernel"));
    }
    int fold = 0;
    int64_t enq = 0, chunk = 4;
    while (enq < max_steps) {
        int64_t todo = max_steps - enq < chunk ? max_steps - enq : chunk;
        for (int64_t q = 0; q < todo; ++q) {
            if (small) {
                small_step_kernel<<<1, kSmallThreads, 0, ctx->stream>>>(
                    n, ctx->info, s->t, s->dt, s->x, s->v, s->a, s->k, xp, vp, s->m, jr,
                    c.shape.rep, act, 1);
                NB_TRY(hip_check(ctx, hipGetLastError(), "small_step_kernel"));
            } else {
                step_scan_kernel<<<gs, 256, 0, ctx->stream>>>(
                    n, ctx->info, fold, cmin, (int)gc, s->t, s->dt, s->x, s->v, s->a, s->k, xp,
                    vp, s->m, jr, c.shape.rep, counts, rmin);
                NB_TRY(hip_check(ctx, hipGetLastError(), "step_scan_kernel"));
                fold = 1;
                step_compact_kernel<<<gs, 256, 0, ctx->stream>>>(n, ctx->info, s->t, s->dt,
                                                                 counts, rmin, act);
                NB_TRY(hip_check(ctx, hipGetLastError(), "step_compact_kernel"));
            }
            NB_TRY(launch_force(ctx, c));
            correct_kernel<<<small ? gp : gc, 256, 0, ctx->stream>>>(
                n, 0, nullptr, ctx->info, ctx->info, act, xp, vp, an, kn, n, s->eta, s->dt_max, s->dt_min,
                (s->flags & NBODY_FIXED_DT) ? 1 : 0, s->t, s->dt, s->x, s->v, s->a, s->k,
                small ? nullptr : cmin);
            NB_TRY(hip_check(ctx, hipGetLastError(), "correct_kernel"));
        }
        enq += todo;
        NB_TRY(hip_check(ctx, hipMemcpyAsync(ctx->info_host, ctx->info, sizeof(StepInfo),
                                             hipMemcpyDeviceToHost, ctx->stream),
                         "info read"));
        NB_TRY(hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"));
        if (ctx->prof.on) prof_resolve(ctx);
        if (ctx->info_host->done || ctx->info_host->status) break;
        if (chunk < 64) chunk *= 2;
    }
    if (steps_done) *steps_done = ctx->info_host->steps;
    if (interactions) *interactions = ctx->info_host->interactions;
    if (ctx->info_host->status) return nbody_sync_status(ctx);
    return NBODY_OK;
}

}  // extern "C"
