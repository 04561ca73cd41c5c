// Batched ensemble: many independent clusters integrated with Hermite block
// steps (Section 2) in one persistent, cooperative launch.
//
// Every workgroup of the grid is co-resident (cooperative launch).  The
// groups are partitioned into teams; a team owns a list of clusters and
// integrates them one after the other, each from initialisation (pair sums
// of every particle, initial steps) to t_end.  Within a team, each phase of
// a block step -- minimum of t + dt, compaction of the active block,
// prediction, pair sums, split reduction, correction -- is spread over the
// team's groups and closed by a team barrier (an arrival counter and a
// generation word in global memory, with agent-scope release/acquire).
// Barrier waits are bounded by a wall-clock limit: if one expires the launch
// raises an abort flag that every group checks, so the grid always drains.
//
// The host plans the teams from a time model.  A cluster of N particles
// takes about S = c N^p t_end block steps with blocks of 0.20 N^0.81
// particles (the paper fits c = 247, p = 0.35 for the steps per time unit,
// and that block size; c and p are recalibrated from measured runs), so on a
// team of g groups it takes
//     T(N, g) = S (step + [g > 1] (b0 + b1 g) + 0.20 N^1.81 / (g rate))
// where step is the fixed latency of one block step on one group, b0 + b1 g
// the extra cost of a step of a team of g groups and rate the pair
// interactions per second of one group (all calibrated by the autotuner).  With at
// least as many groups as clusters every cluster gets its own team and the
// spare groups go, one at a time, to the team with the largest T (while
// that lowers it); otherwise clusters are packed onto single-group teams,
// longest first onto the least-loaded team.
//
// The j particles of a pair-sum pass are staged through LDS in tiles (the
// predicted state is written during this launch, so it cannot be read
// through the scalar cache as in the standalone kernel); the four waves of a
// group share one tile, each taking a quarter of it for the group's 64
// i-particles, and their sums are combined in float64 in wave order.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <queue>
#include <vector>

#include "common.hpp"
#include "integ.hpp"

namespace nb {

constexpr int EW = 4;            // waves per group
constexpr int ETH = 64 * EW;     // threads per group
constexpr int ETILE = 256;       // j records per LDS tile
constexpr int EMAXSPLIT = 64;    // largest j split of a team's pair pass

struct EnsCluster {
    int64_t off;
    int32_t n;
    float eps2;
};

struct EnsTeam {
    int32_t size, cl_begin, cl_end, n_max;
    int32_t s_max, pad;
    int64_t scratch_off;  // in doubles
};

struct EnsArgs {
    int64_t nt;  // particles in the ensemble (component stride)
    double *t, *dt, *x, *v, *a, *k;
    const double *m;
    double *xp, *vp;
    double eta, eta_s, dt_max, dt_min, t_end;
    const EnsCluster *cl;
    const int32_t *cl_order;
    const EnsTeam *teams;
    const int32_t *wg_team, *wg_rank;
    double *scratch;
    uint32_t *bars;  // 64 arrival words per team (one per group rank)
    int64_t *steps, *inter;
    uint64_t *clock;  // per cluster: wall clock at its start and end
    int32_t *status, *abort;
    int64_t spin_limit;  // wall-clock ticks
};

struct TileRec {
    double x, y, z, u, v, w;
    float m, pad;
    double pad2;
};

__device__ __forceinline__ bool aborted(const int32_t *abort) {
    return __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Team barrier; returns false if the launch is being aborted.
// Each group of a team owns one arrival word (64 words per team, one per
// possible rank).  Arriving, thread 0 releases the group's writes at agent
// scope (the groups of a team sit on different XCDs, whose L2 caches are
// made coherent only by release/acquire) and stores the group's new epoch in
// its word; wave 0 then polls all g words of the team with one coalesced
// relaxed load per poll until every word has reached the epoch, and issues
// one agent-scope acquire.  No read-modify-write is contended, and no
// acquire is issued while polling (each would invalidate the L2 under the
// groups still computing on that XCD).  Polls are bounded by a wall-clock
// limit that raises the launch-wide abort flag.
__device__ bool team_barrier(uint32_t *flags, int g, int rank, uint32_t &epoch, int32_t *abort,
                             int64_t limit) {
    __shared__ int ok;
    __syncthreads();
    epoch += 1;
    if (g > 1) {
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(&flags[rank], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            const uint64_t t0 = wall_clock64();
            int good = 1;
            for (;;) {
                const uint32_t v = lane < g ? __hip_atomic_load(&flags[lane], __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT)
                                            : epoch;
                if (__ballot((int32_t)(v - epoch) < 0) == 0ull) break;
                if (aborted(abort)) {
                    good = 0;
                    break;
                }
                if ((int64_t)(wall_clock64() - t0) > limit) {
                    if (lane == 0)
                        __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    good = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (lane == 0) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                ok = good && !aborted(abort);
            }
        }
    } else if (threadIdx.x == 0) {
        ok = !aborted(abort);
    }
    __syncthreads();
    return ok != 0;
}

__device__ __forceinline__ void ds_fold(float &hi, float &lo, float x, bool ds) {
    if (ds) {
        const float s = hi + x;
        const float bp = s - hi;
        lo += (hi - (s - bp)) + (x - bp);
        hi = s;
    } else {
        hi += x;
    }
}

// Pair sums of one work item (64 * EIT i-slots x a j range) of a cluster.
// src_x/src_v: state to read (component stride nt); i-slot s is particle
// act[s] (or s when act is null); lane l holds slots ib*64*EIT + t*64 + l.
// Result: 7 float64 per slot and t in wave 0.
constexpr int EIT = 2;

template <bool DS>
__device__ void ens_pair_item(const EnsArgs &A, const double *src_x, const double *src_v,
                              int64_t base, int n, float eps2, const int32_t *act, int n_i,
                              int64_t ib, int j0, int j1, TileRec *tile,
                              double (*red)[7 * EIT][64], double tot[EIT][7]) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t nt = A.nt;
    double xi[EIT], yi[EIT], zi[EIT], ui[EIT], vi[EIT], wi[EIT];
    int ip[EIT];
    int lo = 0x7fffffff, hi = -1;
#pragma unroll
    for (int t = 0; t < EIT; ++t) {
        const int slot = (int)(ib * 64 * EIT + t * 64 + lane);
        const int sl = slot < n_i ? slot : n_i - 1;
        ip[t] = act ? act[sl] : sl;  // cluster-local index
        const int64_t q = base + ip[t];
        xi[t] = src_x[q];
        yi[t] = src_x[nt + q];
        zi[t] = src_x[2 * nt + q];
        ui[t] = src_v[q];
        vi[t] = src_v[nt + q];
        wi[t] = src_v[2 * nt + q];
        lo = min(lo, ip[t]);
        hi = max(hi, ip[t]);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o, 64));
        hi = max(hi, __shfl_xor(hi, o, 64));
    }
    float sh[EIT][7], sl7[EIT][7];
#pragma unroll
    for (int t = 0; t < EIT; ++t)
#pragma unroll
        for (int c = 0; c < 7; ++c) sh[t][c] = sl7[t][c] = 0.0f;
    for (int jt = j0; jt < j1; jt += ETILE) {
        const int cnt = min(ETILE, j1 - jt);
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const int64_t q = base + jt + threadIdx.x;
            TileRec r;
            r.x = src_x[q];
            r.y = src_x[nt + q];
            r.z = src_x[2 * nt + q];
            r.u = src_v[q];
            r.v = src_v[nt + q];
            r.w = src_v[2 * nt + q];
            r.m = (float)A.m[q];
            tile[threadIdx.x] = r;
        }
        __syncthreads();
        const int r0 = wave * 64, r1 = min(cnt, r0 + 64);
        float in[EIT][7];
#pragma unroll
        for (int t = 0; t < EIT; ++t)
#pragma unroll
            for (int c = 0; c < 7; ++c) in[t][c] = 0.0f;
        auto body = [&](const TileRec &R, const int j, const bool mask)
            __attribute__((always_inline)) {
#pragma unroll
            for (int t = 0; t < EIT; ++t) {
                const float dx = (float)(R.x - xi[t]), dy = (float)(R.y - yi[t]);
                const float dz = (float)(R.z - zi[t]);
                const float du = (float)(R.u - ui[t]), dv = (float)(R.v - vi[t]);
                const float dw = (float)(R.w - wi[t]);
                float s2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
                float mj = R.m;
                if (mask) {
                    const bool self = (j == ip[t]);
                    s2 = self ? 1.0f : s2;
                    mj = self ? 0.0f : mj;
                }
                const float rv = fmaf(dz, dw, fmaf(dy, dv, dx * du));
                const float rinv = __builtin_amdgcn_rsqf(s2);
                const float rinv2 = rinv * rinv;
                const float mr1 = mj * rinv;
                const float mr3 = mr1 * rinv2;
                const float w3 = (rv * rinv2) * -3.0f;
                in[t][0] = fmaf(mr3, dx, in[t][0]);
                in[t][1] = fmaf(mr3, dy, in[t][1]);
                in[t][2] = fmaf(mr3, dz, in[t][2]);
                in[t][3] = fmaf(mr3, fmaf(w3, dx, du), in[t][3]);
                in[t][4] = fmaf(mr3, fmaf(w3, dy, dv), in[t][4]);
                in[t][5] = fmaf(mr3, fmaf(w3, dz, dw), in[t][5]);
                in[t][6] = fmaf(mj, rinv, in[t][6]);
            }
        };
        if ((jt + r0 <= hi) && (jt + r1 > lo)) {
            for (int r = r0; r < r1; ++r) body(tile[r], jt + r, true);
        } else {
#pragma unroll 4
            for (int r = r0; r < r1; ++r) body(tile[r], jt + r, false);
        }
#pragma unroll
        for (int t = 0; t < EIT; ++t)
#pragma unroll
            for (int c = 0; c < 7; ++c) ds_fold(sh[t][c], sl7[t][c], in[t][c], DS);
    }
#pragma unroll
    for (int t = 0; t < EIT; ++t) {
#pragma unroll
        for (int c = 0; c < 7; ++c) tot[t][c] = (double)sh[t][c] + (double)sl7[t][c];
        tot[t][6] = -tot[t][6];
    }
    __syncthreads();
    if (wave > 0)
#pragma unroll
        for (int t = 0; t < EIT; ++t)
#pragma unroll
            for (int c = 0; c < 7; ++c) red[wave - 1][t * 7 + c][lane] = tot[t][c];
    __syncthreads();
    if (wave == 0)
        for (int w = 1; w < EW; ++w)
#pragma unroll
            for (int t = 0; t < EIT; ++t)
#pragma unroll
                for (int c = 0; c < 7; ++c) tot[t][c] += red[w - 1][t * 7 + c][lane];
}

// Pair sums of a whole active block of a cluster, spread over the team:
// results in anew/knew (component stride n_max); returns false on abort.
template <bool DS>
__device__ bool ens_pairs(const EnsArgs &A, const double *src_x, const double *src_v,
                          int64_t base, int n, float eps2, const int32_t *act, int n_i, int g,
                          int rank, int s_max, int n_max, double *anew, double *knew,
                          double *part, uint32_t *bar, uint32_t &epoch, TileRec *tile,
                          double (*red)[7 * EIT][64]) {
    const int64_t nb = (n_i + 64 * EIT - 1) / (64 * EIT);
    int64_t S = (g + nb - 1) / nb;  // about one item per group
    int64_t smax = max(1, n / ETILE);
    if (smax > s_max) smax = s_max;
    if (S > smax) S = smax;
    if (S < 1) S = 1;
    const int64_t items = nb * S;
    const int jchunk = (int)((n + S - 1) / S);
    const int lane = threadIdx.x & 63;
    for (int64_t it = rank; it < items; it += g) {
        const int64_t ib = it % nb, sp = it / nb;
        const int j0 = (int)(sp * jchunk), j1 = min(n, j0 + jchunk);
        double tot[EIT][7];
        ens_pair_item<DS>(A, src_x, src_v, base, n, eps2, act, n_i, ib, j0, j1, tile, red, tot);
        if ((threadIdx.x >> 6) == 0) {
#pragma unroll
            for (int t = 0; t < EIT; ++t) {
                const int slot = (int)(ib * 64 * EIT + t * 64 + lane);
                if (slot >= n_i) continue;
                if (S == 1) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        anew[c * n_max + slot] = tot[t][c];
                        knew[c * n_max + slot] = tot[t][3 + c];
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 6; ++c) part[(sp * 6 + c) * n_max + slot] = tot[t][c];
                }
            }
        }
    }
    if (S > 1) {
        if (!team_barrier(bar, g, rank, epoch, A.abort, A.spin_limit)) return false;
        const int64_t total = 6 * (int64_t)n_i;
        for (int64_t e = (int64_t)rank * ETH + threadIdx.x; e < total; e += (int64_t)g * ETH) {
            const int c = (int)(e / n_i), s = (int)(e - (int64_t)c * n_i);
            double acc = 0.0;
            for (int64_t p = 0; p < S; ++p) acc += part[(p * 6 + c) * n_max + s];
            if (c < 3)
                anew[c * n_max + s] = acc;
            else
                knew[(c - 3) * n_max + s] = acc;
        }
    }
    return team_barrier(bar, g, rank, epoch, A.abort, A.spin_limit);
}

template <bool DS>
__global__ __launch_bounds__(ETH) void ensemble_kernel(const EnsArgs A) {
    __shared__ TileRec tile[ETILE];
    __shared__ double red[EW - 1][7 * EIT][64];
    __shared__ double smin[ETH];
    __shared__ int scount[ETH];
    const int team = A.wg_team[blockIdx.x];
    const int rank = A.wg_rank[blockIdx.x];
    const EnsTeam T = A.teams[team];
    const int g = T.size;
    uint32_t *bar = A.bars + 64 * (int64_t)team;  // arrival words of the team
    uint32_t epoch = 0;
    double *scr = A.scratch + T.scratch_off;
    const int n_max = T.n_max;
    // scratch layout (doubles): pmin[g] | pcnt[g] | active[n_max] (int32) |
    // anew[3 n_max] | knew[3 n_max] | part[s_max * 6 * n_max]
    double *pmin = scr;
    int64_t *pcnt = (int64_t *)(scr + g);
    int32_t *act = (int32_t *)(scr + 2 * g);
    double *anew = scr + 2 * g + (n_max + 1) / 2;
    double *knew = anew + 3 * (int64_t)n_max;
    double *part = knew + 3 * (int64_t)n_max;
    const int64_t nt = A.nt;
    const int tid = threadIdx.x;

    for (int ci = T.cl_begin; ci < T.cl_end; ++ci) {
        const int c = A.cl_order[ci];
        const EnsCluster C = A.cl[c];
        const int64_t base = C.off;
        const int n = C.n;
        const float eps2 = C.eps2;
        const int per = (n + g - 1) / g;
        const int p0 = min(n, rank * per), p1 = min(n, p0 + per);
        if (rank == 0 && tid == 0) A.clock[2 * c] = wall_clock64();

        // ---- initialisation: pair sums of every particle, initial steps
        if (!ens_pairs<DS>(A, A.x, A.v, base, n, eps2, nullptr, n, g, rank, T.s_max, n_max, anew,
                           knew, part, bar, epoch, tile, red))
            return;
        for (int i = p0 + tid; i < p1; i += ETH) {
            const int64_t q = base + i;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                A.a[cc * nt + q] = anew[cc * n_max + i];
                A.k[cc * nt + q] = knew[cc * n_max + i];
            }
            int32_t st = 0;
            A.t[q] = 0.0;
            A.dt[q] = initial_dt_one(q, nt, 0.0, A.a, A.k, A.eta_s, A.dt_max, A.dt_min, &st);
            if (st) atomicOr(A.status, st);
        }
        if (!team_barrier(bar, g, rank, epoch, A.abort, A.spin_limit)) return;

        int64_t my_steps = 0, my_inter = 0;
        for (;;) {
            // ---- t_next = min(t + dt) over the cluster
            double mn = INFINITY;
            for (int i = p0 + tid; i < p1; i += ETH) mn = fmin(mn, A.t[base + i] + A.dt[base + i]);
            smin[tid] = mn;
            __syncthreads();
            for (int o = ETH / 2; o > 0; o >>= 1) {
                if (tid < o) smin[tid] = fmin(smin[tid], smin[tid + o]);
                __syncthreads();
            }
            if (tid == 0) pmin[rank] = smin[0];
            if (!team_barrier(bar, g, rank, epoch, A.abort, A.spin_limit)) return;
            double tn = INFINITY;
            for (int r = 0; r < g; ++r)
                tn = fmin(tn, __hip_atomic_load(&pmin[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (!(tn <= A.t_end)) break;

            // ---- active block, ascending: count per group, then place
            int cnt = 0;
            for (int i = p0 + tid; i < p1; i += ETH) cnt += (A.t[base + i] + A.dt[base + i] == tn);
            scount[tid] = cnt;
            __syncthreads();
            for (int o = ETH / 2; o > 0; o >>= 1) {
                if (tid < o) scount[tid] += scount[tid + o];
                __syncthreads();
            }
            if (tid == 0) pcnt[rank] = scount[0];
            if (!team_barrier(bar, g, rank, epoch, A.abort, A.spin_limit)) return;
            int64_t before = 0, n_i = 0;
            for (int r = 0; r < g; ++r) {
                const int64_t cr = __hip_atomic_load(&pcnt[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (r < rank) before += cr;
                n_i += cr;
            }
            {
                // place the active indices (ascending) and predict every
                // particle of the slice to tn in the same pass
                const int lane = tid & 63, wave = tid >> 6;
                int64_t off = before;
                for (int pbase = p0; pbase < p1; pbase += ETH) {
                    const int i = pbase + tid;
                    bool f = false;
                    if (i < p1) {
                        const int64_t q = base + i;
                        const double tq = A.t[q];
                        f = (tq + A.dt[q] == tn);
                        double px[3], pv[3];
                        predict_one(tn - tq, A.x, A.v, A.a, A.k, q, nt, px, pv);
#pragma unroll
                        for (int cc = 0; cc < 3; ++cc) {
                            A.xp[cc * nt + q] = px[cc];
                            A.vp[cc * nt + q] = pv[cc];
                        }
                    }
                    const unsigned long long bal = __ballot(f);
                    const int bef = __popcll(bal & ((1ull << lane) - 1ull));
                    __syncthreads();
                    if (lane == 0) scount[wave] = __popcll(bal);
                    __syncthreads();
                    int woff = 0, tot = 0;
                    for (int w = 0; w < EW; ++w) {
                        if (w < wave) woff += scount[w];
                        tot += scount[w];
                    }
                    if (f) act[off + woff + bef] = i;
                    off += tot;
                }
            }
            if (!team_barrier(bar, g, rank, epoch, A.abort, A.spin_limit)) return;

            // ---- pair sums of the block at the predicted state
            if (!ens_pairs<DS>(A, A.xp, A.vp, base, n, eps2, act, (int)n_i, g, rank, T.s_max, n_max,
                               anew, knew, part, bar, epoch, tile, red))
                return;

            // ---- correct the block
            const int per_i = (int)((n_i + g - 1) / g);
            const int s0 = min((int)n_i, rank * per_i), s1 = min((int)n_i, s0 + per_i);
            for (int s = s0 + tid; s < s1; s += ETH) {
                const int64_t q = base + act[s];
                double a1v[3], k1v[3];
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    a1v[cc] = anew[cc * n_max + s];
                    k1v[cc] = knew[cc * n_max + s];
                }
                const int32_t st = correct_one(q, nt, A.xp, A.vp, a1v, k1v, A.eta, A.dt_max,
                                               A.dt_min, 0, A.t, A.dt, A.x, A.v, A.a, A.k);
                if (st) atomicOr(A.status, st);
            }
            my_steps += 1;
            my_inter += n_i * n;
            if (!team_barrier(bar, g, rank, epoch, A.abort, A.spin_limit)) return;
        }
        if (rank == 0 && tid == 0) {
            A.steps[c] = my_steps;
            A.inter[c] = my_inter;
            A.clock[2 * c + 1] = wall_clock64();
        }
        // the next cluster's initialisation writes anew/knew and act: make
        // sure every group of the team is past this cluster
        if (!team_barrier(bar, g, rank, epoch, A.abort, A.spin_limit)) return;
    }
}

__global__ void ens_clear_kernel(uint32_t *bars, int64_t nbars, int64_t *steps, int64_t *inter,
                                 uint64_t *clock, int64_t nc, int32_t *flags) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < nbars) bars[i] = 0;
    if (i < nc) {
        steps[i] = 0;
        inter[i] = 0;
        clock[2 * i] = clock[2 * i + 1] = 0;
    }
    if (i < 2) flags[i] = 0;
}

// ---- host-side team planning ----------------------------------------------
struct Plan {
    std::vector<EnsTeam> teams;
    std::vector<int32_t> order, wg_team, wg_rank;
    int64_t scratch = 0;  // doubles
};

struct TimeModel {
    double step_s, barrier_s, barrier_g_s, rate, t_end, coef, expo;
    double steps(double n) const { return std::max(1.0, coef * std::pow(n, expo) * t_end); }
    double time(double n, int g) const {
        const double per_step = step_s + (g > 1 ? barrier_s + barrier_g_s * g : 0.0) +
                                0.20 * std::pow(n, 1.81) / ((double)g * rate);
        return steps(n) * per_step;
    }
};

static Plan plan_teams(const std::vector<int64_t> &sizes, int G, int max_team,
                       const TimeModel &M) {
    const int nc = (int)sizes.size();
    std::vector<std::vector<int>> tcl;
    std::vector<int> tsize;
    if (G >= nc) {
        // one team per cluster, then spare groups to the slowest team
        std::vector<int> gsz(nc, 1);
        typedef std::pair<double, int> TT;
        std::priority_queue<TT> heap;
        for (int c = 0; c < nc; ++c) heap.push(TT(M.time((double)sizes[c], 1), c));
        int spare = G - nc;
        while (spare > 0 && !heap.empty()) {
            TT top = heap.top();
            heap.pop();
            const int c = top.second;
            if (gsz[c] >= max_team) continue;
            const double t1 = M.time((double)sizes[c], gsz[c] + 1);
            if (!(t1 < top.first)) continue;  // more groups no longer help
            gsz[c] += 1;
            --spare;
            heap.push(TT(t1, c));
        }
        std::vector<int> idx(nc);
        std::iota(idx.begin(), idx.end(), 0);
        std::sort(idx.begin(), idx.end(), [&](int p, int q) {
            const double a = M.time((double)sizes[p], gsz[p]), b = M.time((double)sizes[q], gsz[q]);
            return a > b || (a == b && p < q);
        });
        for (int c : idx) {
            tcl.push_back({c});
            tsize.push_back(gsz[c]);
        }
    } else {
        // more clusters than groups: longest first onto the least-loaded group
        std::vector<int> idx(nc);
        std::iota(idx.begin(), idx.end(), 0);
        std::sort(idx.begin(), idx.end(), [&](int p, int q) {
            return sizes[p] > sizes[q] || (sizes[p] == sizes[q] && p < q);
        });
        tcl.assign(G, {});
        tsize.assign(G, 1);
        typedef std::pair<double, int> LT;
        std::priority_queue<LT, std::vector<LT>, std::greater<LT>> heap;
        for (int t = 0; t < G; ++t) heap.push(LT(0.0, t));
        for (int c : idx) {
            LT top = heap.top();
            heap.pop();
            tcl[top.second].push_back(c);
            heap.push(LT(top.first + M.time((double)sizes[c], 1), top.second));
        }
    }
    Plan P;
    for (int t = 0; t < (int)tcl.size(); ++t) {
        if (tcl[t].empty()) continue;
        EnsTeam T = {};
        T.size = tsize[t];
        T.cl_begin = (int32_t)P.order.size();
        int nmax = 1;
        for (int c : tcl[t]) {
            P.order.push_back(c);
            nmax = std::max<int>(nmax, (int)sizes[c]);
        }
        T.cl_end = (int32_t)P.order.size();
        T.n_max = nmax;
        T.s_max = std::min(EMAXSPLIT, std::max(1, T.size));
        T.scratch_off = P.scratch;
        P.scratch += 2 * T.size + (nmax + 1) / 2 + 6 * (int64_t)nmax +
                     (int64_t)T.s_max * 6 * nmax + 8;
        const int team_id = (int)P.teams.size();
        P.teams.push_back(T);
        for (int r = 0; r < T.size; ++r) {
            P.wg_team.push_back(team_id);
            P.wg_rank.push_back(r);
        }
    }
    return P;
}

}  // namespace nb

using namespace nb;

extern "C" int nbody_ensemble_run(nbody_ctx *ctx, const nbody_ensemble *e, double t_end,
                                  int64_t *steps, int64_t *interactions) {
    if (!ctx) return NBODY_E_INVAL;
    if (!e || e->n_clusters < 1 || !e->offsets || !e->eps2)
        return fail(ctx, NBODY_E_INVAL, "nbody_ensemble_run: bad description");
    const int nc = e->n_clusters;
    std::vector<int64_t> sizes(nc);
    if (e->offsets[0] != 0) return fail(ctx, NBODY_E_INVAL, "ensemble: offsets[0] must be 0");
    for (int c = 0; c < nc; ++c) {
        sizes[c] = e->offsets[c + 1] - e->offsets[c];
        if (sizes[c] < 1) return fail(ctx, NBODY_E_INVAL, "ensemble: empty cluster %d", c);
        if (!(e->eps2[c] >= 0) || std::isinf(e->eps2[c]))
            return fail(ctx, NBODY_E_INVAL, "ensemble: bad eps2 of cluster %d", c);
    }
    const int64_t nt = e->offsets[nc];
    if (nt > 0x7fffffffLL) return fail(ctx, NBODY_E_INVAL, "ensemble: too many particles");
    if (!e->t || !e->dt || !e->x || !e->v || !e->a || !e->k || !e->m)
        return fail(ctx, NBODY_E_INVAL, "ensemble: null array");
    int ex;
    if (!(e->dt_max > 0) || std::frexp(e->dt_max, &ex) != 0.5 || !(e->dt_min > 0) ||
        !(e->dt_max >= e->dt_min) || !(e->eta > 0) || !(e->eta_s > 0) || std::isnan(t_end))
        return fail(ctx, NBODY_E_INVAL, "ensemble: bad parameters");
    if (e->flags & ~NBODY_ACC_DS) return fail(ctx, NBODY_E_INVAL, "ensemble: unknown flags");
    NB_TRY(activate(ctx));

    const bool ds = (e->flags & NBODY_ACC_DS) != 0;
    const void *kfn = ds ? (const void *)ensemble_kernel<true> : (const void *)ensemble_kernel<false>;
    int occ = 0;
    NB_TRY(hip_check(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kfn, ETH, 0),
                     "occupancy"));
    int per_cu = std::min(occ, ctx->ens_cfg.groups_per_cu);
    if (per_cu < 1) return fail(ctx, NBODY_E_DEVICE, "ensemble kernel does not fit a CU");
    const int G = per_cu * ctx->cus;
    const nbody_ensemble_config &cf = ctx->ens_cfg;
    TimeModel M{cf.step_us * 1e-6,   cf.barrier_us * 1e-6, cf.barrier_group_us * 1e-6,
                cf.group_rate,       t_end > 0 ? t_end : 0.0, cf.steps_coef, cf.steps_exp};
    Plan P = plan_teams(sizes, G, std::min(cf.max_team, 64), M);
    const int grid = (int)P.wg_team.size();
    const int nteams = (int)P.teams.size();

    std::vector<EnsCluster> hc(nc);
    for (int c = 0; c < nc; ++c) hc[c] = EnsCluster{e->offsets[c], (int32_t)sizes[c], (float)e->eps2[c]};

    // one device block: tables, counters, scratch, predicted state
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t b_cl = al(sizeof(EnsCluster) * nc), b_ord = al(4 * P.order.size()),
                 b_tm = al(sizeof(EnsTeam) * nteams), b_wg = al(4 * (size_t)grid),
                 b_bar = al(4 * 64 * (size_t)nteams), b_cnt = al(8 * (size_t)nc),
                 b_clk = al(16 * (size_t)nc),
                 b_fl = al(8), b_scr = al(8 * (size_t)P.scratch), b_st = al(8 * 3 * (size_t)nt);
    const size_t total =
        b_cl + b_ord + b_tm + 2 * b_wg + b_bar + 2 * b_cnt + b_clk + b_fl + b_scr + 2 * b_st;
    NB_TRY(ensure(ctx, &ctx->ens, &ctx->ens_bytes, total));
    char *p = (char *)ctx->ens;
    EnsCluster *d_cl = (EnsCluster *)p; p += b_cl;
    int32_t *d_ord = (int32_t *)p; p += b_ord;
    EnsTeam *d_tm = (EnsTeam *)p; p += b_tm;
    int32_t *d_wgt = (int32_t *)p; p += b_wg;
    int32_t *d_wgr = (int32_t *)p; p += b_wg;
    uint32_t *d_bar = (uint32_t *)p; p += b_bar;
    int64_t *d_steps = (int64_t *)p; p += b_cnt;
    int64_t *d_inter = (int64_t *)p; p += b_cnt;
    uint64_t *d_clock = (uint64_t *)p; p += b_clk;
    int32_t *d_flags = (int32_t *)p; p += b_fl;
    double *d_scr = (double *)p; p += b_scr;
    double *d_xp = (double *)p; p += b_st;
    double *d_vp = (double *)p;

    NB_TRY(hip_check(ctx, hipMemcpyAsync(d_cl, hc.data(), sizeof(EnsCluster) * nc, hipMemcpyHostToDevice, ctx->stream), "copy"));
    NB_TRY(hip_check(ctx, hipMemcpyAsync(d_ord, P.order.data(), 4 * P.order.size(), hipMemcpyHostToDevice, ctx->stream), "copy"));
    NB_TRY(hip_check(ctx, hipMemcpyAsync(d_tm, P.teams.data(), sizeof(EnsTeam) * nteams, hipMemcpyHostToDevice, ctx->stream), "copy"));
    NB_TRY(hip_check(ctx, hipMemcpyAsync(d_wgt, P.wg_team.data(), 4 * (size_t)grid, hipMemcpyHostToDevice, ctx->stream), "copy"));
    NB_TRY(hip_check(ctx, hipMemcpyAsync(d_wgr, P.wg_rank.data(), 4 * (size_t)grid, hipMemcpyHostToDevice, ctx->stream), "copy"));
    const int64_t nclr = std::max<int64_t>(64 * (int64_t)nteams, nc) + 2;
    ens_clear_kernel<<<(unsigned)((nclr + 255) / 256), 256, 0, ctx->stream>>>(
        d_bar, 64 * (int64_t)nteams, d_steps, d_inter, d_clock, nc, d_flags);
    NB_TRY(hip_check(ctx, hipGetLastError(), "ens_clear_kernel"));

    int wclk_khz = 0;
    if (hipDeviceGetAttribute(&wclk_khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess ||
        wclk_khz <= 0) {
        (void)hipGetLastError();
        wclk_khz = 100000;
    }
    EnsArgs A;
    A.nt = nt;
    A.t = e->t; A.dt = e->dt; A.x = e->x; A.v = e->v; A.a = e->a; A.k = e->k; A.m = e->m;
    A.xp = d_xp; A.vp = d_vp;
    A.eta = e->eta; A.eta_s = e->eta_s; A.dt_max = e->dt_max; A.dt_min = e->dt_min;
    A.t_end = t_end;
    A.cl = d_cl; A.cl_order = d_ord; A.teams = d_tm; A.wg_team = d_wgt; A.wg_rank = d_wgr;
    A.scratch = d_scr; A.bars = d_bar; A.steps = d_steps; A.inter = d_inter; A.clock = d_clock;
    A.status = d_flags; A.abort = d_flags + 1;
    A.spin_limit = (int64_t)wclk_khz * 1000 * 20;  // 20 s of wall clock per barrier wait
    void *args[] = {&A};
    NB_TRY(hip_check(ctx, hipLaunchCooperativeKernel(kfn, dim3(grid), dim3(ETH), args, 0, ctx->stream),
                     "ensemble_kernel (cooperative launch)"));
    int32_t hflags[2] = {0, 0};
    std::vector<int64_t> hs(nc), hi(nc);
    std::vector<uint64_t> hclk(2 * (size_t)nc);
    NB_TRY(hip_check(ctx, hipMemcpyAsync(hflags, d_flags, 8, hipMemcpyDeviceToHost, ctx->stream), "copy"));
    NB_TRY(hip_check(ctx, hipMemcpyAsync(hs.data(), d_steps, 8 * (size_t)nc, hipMemcpyDeviceToHost, ctx->stream), "copy"));
    NB_TRY(hip_check(ctx, hipMemcpyAsync(hi.data(), d_inter, 8 * (size_t)nc, hipMemcpyDeviceToHost, ctx->stream), "copy"));
    NB_TRY(hip_check(ctx, hipMemcpyAsync(hclk.data(), d_clock, 16 * (size_t)nc, hipMemcpyDeviceToHost, ctx->stream), "copy"));
    NB_TRY(hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"));
    if (steps)
        for (int c = 0; c < nc; ++c) steps[c] = hs[c];
    if (interactions)
        for (int c = 0; c < nc; ++c) interactions[c] = hi[c];
    ctx->ens_last_grid = grid;
    ctx->ens_last_teams = nteams;
    ctx->ens_last_seconds.assign(nc, 0.0);
    ctx->ens_last_groups.assign(nc, 0);
    for (int c = 0; c < nc; ++c)
        ctx->ens_last_seconds[c] = (double)(hclk[2 * c + 1] - hclk[2 * c]) / ((double)wclk_khz * 1e3);
    for (const EnsTeam &T : P.teams)
        for (int q = T.cl_begin; q < T.cl_end; ++q) ctx->ens_last_groups[P.order[q]] = T.size;
    if (hflags[1]) return fail(ctx, NBODY_E_DEVICE, "ensemble: a team barrier timed out");
    if (hflags[0] & ST_NONFINITE) return fail(ctx, NBODY_E_NONFINITE, "ensemble: non-finite value");
    if (hflags[0] & ST_RANGE) return fail(ctx, NBODY_E_RANGE, "ensemble: time step below dt_min");
    return NBODY_OK;
}
