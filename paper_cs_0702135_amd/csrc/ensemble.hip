// Batched ensemble: many independent clusters integrated with Hermite block
// steps (Section 2) in one persistent, cooperative launch.
//
// Every workgroup of the grid is co-resident (cooperative launch).  The
// groups are partitioned into teams; a team owns a list of clusters and
// integrates them one after the other, each from initialisation (pair sums
// of every particle, initial steps) to t_end.  Within a team, the two phases
// of a block step (block selection and pair sums; split reduction and
// correction) are spread over the team's groups and each is closed by a team
// barrier (one arrival word per group in global memory, agent-scope
// release/acquire).  Barrier waits are bounded by a wall-clock limit: if one
// expires the launch raises an abort flag that every group checks, so the
// grid always drains.
//
// The host plans the teams from a time model.  A cluster of N particles
// takes about S = c N^p t_end block steps with blocks of B = b N^q particles
// (the paper's Section 5 fits, c = 247, p = 0.35, b = 0.20, q = 0.81, are the
// defaults; the autotuner can refit them), so on a team of g groups it takes
//     T(N, g) = P(N) + S (step + [g > 1] (b0 + b1 g) + P(B))
// where P(n_i) is the busiest group's share of a pair pass over n_i
// particles (its j tiles times a tile latency plus n_i N / (g rate)), step
// the fixed latency of one block step on one group and b0 + b1 g the extra
// cost of a step of a team of g groups.  The plan minimises the modelled
// makespan: clusters that one group finishes in time share single-group
// teams, the others get the fewest groups that finish them in time, and
// spare groups go to the slowest teams.
//
// The j particles of a pair-sum pass are staged through LDS in tiles (the
// state is rewritten during this launch, so it cannot be read through the
// scalar cache as in the standalone kernel); the W waves of a group share
// one tile, each taking a W-th of it for the group's 64 * IT block slots,
// and their sums are combined in float64 in wave order.  W, the tile and IT
// are compile-time shapes (ESh) among which the autotuner chooses.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <queue>
#include <vector>

#include "common.hpp"
#include "integ.hpp"

namespace nb {

// Launch shape of the ensemble kernel.
template <int W_, int TILE_, int IT_>
struct ESh {
    static constexpr int W = W_;        // waves per group (2, 4 or 8)
    static constexpr int TH = 64 * W_;  // threads per group
    static constexpr int TILE = TILE_;  // j records per LDS tile (a multiple of 64 W)
    static constexpr int IT = IT_;      // most i-slots per lane (1 or 2)
    static_assert(W_ >= 2 && TILE_ % (64 * W_) == 0 && (IT_ == 1 || IT_ == 2), "shape");
};
constexpr int EMAXSPLIT = 64;    // largest j split of a team's pair pass

struct EnsCluster {
    int64_t off;
    int32_t n;
    float eps2;    // softening^2 for the float32 pair terms
    double eps2d;  // and for the float64 pair terms of the compensated mode
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
    double md;  // the mass in float64 (compensated mode)
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

// Members of an active block, ascending: every group of a team compacts
// the whole cluster into its own copy act[0..n_i) (block slot s is particle
// act[s]).  A null act stands for the whole cluster in index order.
struct Block {
    const int32_t *act;
};

__device__ __forceinline__ int block_member(const Block &B, int s) {
    return B.act ? B.act[s] : s;
}

// State of one particle as loaded, before prediction.
struct Raw {
    double t, x[3], v[3], a[3], k[3];
    double m;
};

template <bool PRED>
__device__ __forceinline__ void load_raw(const EnsArgs &A, int64_t q, Raw &r) {
    const int64_t nt = A.nt;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        r.x[c] = A.x[c * nt + q];
        r.v[c] = A.v[c * nt + q];
        if (PRED) {
            r.a[c] = A.a[c * nt + q];
            r.k[c] = A.k[c * nt + q];
        }
    }
    if (PRED) r.t = A.t[q];
    r.m = A.m[q];
}

// Position and velocity predicted to tn (PRED) or as stored.
template <bool PRED>
__device__ __forceinline__ void raw_state(const Raw &r, double tn, double px[3], double pv[3]) {
    if (PRED) {
        predict_vals(tn - r.t, r.x, r.v, r.a, r.k, px, pv);
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            px[c] = r.x[c];
            pv[c] = r.v[c];
        }
    }
}

// Minimum over the group (every thread gets it).
template <class Sh>
__device__ __forceinline__ double group_min(double v, double *smin) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) smin[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = smin[0];
#pragma unroll
    for (int w = 1; w < Sh::W; ++w) r = fmin(r, smin[w]);
    return r;
}

// Pair sums of one work item of a cluster: block slots
// [slot0, slot0 + NI * 64 / L) against the j range [j0, j1).  Lane l holds
// slots slot0 + t * (64 / L) + l / L (t < NI) and takes every L-th j of its
// wave's share of each tile, starting at l % L; the L partial sums of a
// slot are added in float64 (butterfly, fixed order), then the waves' sums
// in wave order.  With PRED every particle, i and j, is predicted to tn as
// it is loaded; otherwise the stored state is used.  Only acceleration and
// jerk are summed: the ensemble never reports the potential.  The self pair
// adds exactly zero when eps2 is not tiny (r = w = 0 and m s^-3/2 finite), so
// it is masked by index only for eps2 < 1e-12.  (Holding the next j tile
// in registers while the current one is summed would cost the third group
// per CU its registers; the co-resident groups hide the tile loads.)
// Float32 mode (DS false): float32 pair terms of float64-formed relative
// coordinates, summed in float32 per tile and over the item's tiles.
// Compensated mode (DS true): float64 pair terms (s^-1/2 from the float32
// estimate and one float64 Newton step) summed in float64.
constexpr float EMASK = 1e-12f;  // below this eps2 the self pair is masked

template <class Sh, bool DS, bool PRED, int NI, int L>
__device__ void ens_pair_item(const EnsArgs &A, int64_t base, float eps2, double eps2d,
                              double tn, const Block &B, int n_i, int slot0, int j0, int j1,
                              TileRec *tile, double (*red)[6 * Sh::IT][64],
                              double (&tot)[Sh::IT][6]) {
    constexpr int SPL = 64 / L;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int ph = lane % L;
    double xi[NI], yi[NI], zi[NI], ui[NI], vi[NI], wi[NI];
    int ip[NI];
    int lo = 0x7fffffff, hi = -1;
#pragma unroll
    for (int t = 0; t < NI; ++t) {
        const int slot = slot0 + t * SPL + lane / L;
        ip[t] = block_member(B, slot < n_i ? slot : n_i - 1);  // cluster-local index
        Raw r;
        load_raw<PRED>(A, base + ip[t], r);
        double px[3], pv[3];
        raw_state<PRED>(r, tn, px, pv);
        xi[t] = px[0];
        yi[t] = px[1];
        zi[t] = px[2];
        ui[t] = pv[0];
        vi[t] = pv[1];
        wi[t] = pv[2];
        lo = min(lo, ip[t]);
        hi = max(hi, ip[t]);
    }
    const bool maskable = !(eps2 >= EMASK);
    if (maskable) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            lo = min(lo, __shfl_xor(lo, o, 64));
            hi = max(hi, __shfl_xor(hi, o, 64));
        }
    }
    float sh[NI][6];   // float32 mode: running sums over the item's tiles
    double sd[NI][6];  // compensated mode: float64 sums
#pragma unroll
    for (int t = 0; t < NI; ++t)
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            sh[t][c] = 0.0f;
            sd[t][c] = 0.0;
        }
    constexpr int PER = Sh::TILE / Sh::W;  // tile records per wave
    for (int jt = j0; jt < j1; jt += Sh::TILE) {
        const int cnt = min(Sh::TILE, j1 - jt);
        __syncthreads();
        for (int q = tid; q < cnt; q += Sh::TH) {
            Raw nxt;
            load_raw<PRED>(A, base + jt + q, nxt);
            double px[3], pv[3];
            raw_state<PRED>(nxt, tn, px, pv);
            TileRec R;
            R.x = px[0];
            R.y = px[1];
            R.z = px[2];
            R.u = pv[0];
            R.v = pv[1];
            R.w = pv[2];
            R.m = (float)nxt.m;
            R.md = nxt.m;
            tile[q] = R;
        }
        __syncthreads();
        const int r0 = wave * PER, r1 = min(cnt, r0 + PER);
        float in[NI][6];
#pragma unroll
        for (int t = 0; t < NI; ++t)
#pragma unroll
            for (int c = 0; c < 6; ++c) in[t][c] = 0.0f;
        auto body64 = [&](const TileRec &R, const int j, const bool mask)
            __attribute__((always_inline)) {
#pragma unroll
            for (int t = 0; t < NI; ++t) {
                const double dx = R.x - xi[t], dy = R.y - yi[t], dz = R.z - zi[t];
                const double du = R.u - ui[t], dv = R.v - vi[t], dw = R.w - wi[t];
                double s2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2d)));
                double mj = R.md;
                if (mask) {
                    const bool self = (j == ip[t]);
                    s2 = self ? 1.0 : s2;
                    mj = self ? 0.0 : mj;
                }
                const double rv = fma(dz, dw, fma(dy, dv, dx * du));
                const double y0 = (double)__builtin_amdgcn_rsqf((float)s2);
                const double e = fma(-(s2 * y0), y0, 1.0);
                const double y = fma(0.5 * y0, e, y0);
                const double y2 = y * y;
                const double mr3 = (mj * y) * y2;
                const double w3 = (rv * y2) * -3.0;
                sd[t][0] = fma(mr3, dx, sd[t][0]);
                sd[t][1] = fma(mr3, dy, sd[t][1]);
                sd[t][2] = fma(mr3, dz, sd[t][2]);
                sd[t][3] = fma(mr3, fma(w3, dx, du), sd[t][3]);
                sd[t][4] = fma(mr3, fma(w3, dy, dv), sd[t][4]);
                sd[t][5] = fma(mr3, fma(w3, dz, dw), sd[t][5]);
            }
        };
        auto body = [&](const TileRec &R, const int j, const bool mask)
            __attribute__((always_inline)) {
#pragma unroll
            for (int t = 0; t < NI; ++t) {
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
                const float mr3 = (mj * rinv) * rinv2;
                const float w3 = (rv * rinv2) * -3.0f;
                in[t][0] = fmaf(mr3, dx, in[t][0]);
                in[t][1] = fmaf(mr3, dy, in[t][1]);
                in[t][2] = fmaf(mr3, dz, in[t][2]);
                in[t][3] = fmaf(mr3, fmaf(w3, dx, du), in[t][3]);
                in[t][4] = fmaf(mr3, fmaf(w3, dy, dv), in[t][4]);
                in[t][5] = fmaf(mr3, fmaf(w3, dz, dw), in[t][5]);
            }
        };
        if constexpr (DS) {
            if (maskable && (jt + r0 <= hi) && (jt + r1 > lo)) {
                for (int r = r0 + ph; r < r1; r += L) body64(tile[r], jt + r, true);
            } else {
#pragma unroll 2
                for (int r = r0 + ph; r < r1; r += L) body64(tile[r], jt + r, false);
            }
        } else {
            if (maskable && (jt + r0 <= hi) && (jt + r1 > lo)) {
                for (int r = r0 + ph; r < r1; r += L) body(tile[r], jt + r, true);
            } else {
#pragma unroll 4
                for (int r = r0 + ph; r < r1; r += L) body(tile[r], jt + r, false);
            }
#pragma unroll
            for (int t = 0; t < NI; ++t)
#pragma unroll
                for (int c = 0; c < 6; ++c) sh[t][c] += in[t][c];
        }
    }
#pragma unroll
    for (int t = 0; t < NI; ++t)
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            double s = DS ? sd[t][c] : (double)sh[t][c];
#pragma unroll
            for (int o = 1; o < L; o <<= 1) s += __shfl_xor(s, o, 64);
            tot[t][c] = s;
        }
    __syncthreads();
    if (wave > 0)
#pragma unroll
        for (int t = 0; t < NI; ++t)
#pragma unroll
            for (int c = 0; c < 6; ++c) red[wave - 1][t * 6 + c][lane] = tot[t][c];
    __syncthreads();
    if (wave == 0)
        for (int w = 1; w < Sh::W; ++w)
#pragma unroll
            for (int t = 0; t < NI; ++t)
#pragma unroll
                for (int c = 0; c < 6; ++c) tot[t][c] += red[w - 1][t * 6 + c][lane];
}

// Width of the item of a block that starts at slot0: 128 slots (two per
// lane, with IT = 2) while more than 64 remain, else the narrowest of 64,
// 32, 16, 8 that holds the rest (the last three split j over 2, 4, 8 lanes).
template <int IT>
__device__ __forceinline__ int item_width(int rem, bool narrow) {
    const int w = (IT == 2 && rem > 64) ? 128
                  : rem > 32             ? 64
                  : rem > 16             ? 32
                  : rem > 8              ? 16
                                         : 8;
    return narrow ? w : max(w, 64);
}

// The j split of a block of n_i slots on a team of g groups.  The block is
// cut into nb i-items of 64 IT slots and each into S j ranges; the S that
// minimises the items of the busiest group per split, ceil(nb S / g) / S
// (the busiest group's share of the work), is taken, the smallest on ties,
// with at most s_max splits and no split below one tile.
template <class Sh>
__device__ __forceinline__ int ens_splits(int n_i, int n, int g, int s_max) {
    const int nb = (n_i + 64 * Sh::IT - 1) / (64 * Sh::IT);
    const int smax = max(1, min(s_max, n / Sh::TILE));
    int best = 1, bq = (nb + g - 1) / g;  // cost ceil(nb S / g) / S as bq / best
    for (int S = 2; S <= smax; ++S) {
        const int q = (nb * S + g - 1) / g;
        if ((int64_t)q * best < (int64_t)bq * S) {
            best = S;
            bq = q;
        }
    }
    return best;
}

// Pair sums of a whole block (n_i slots) of a cluster of n particles,
// spread over the team as items (128 slots by one of S j ranges).  With
// S = 1 an item writes the slot's sums to anew/knew (component stride
// n_max), otherwise its split's partial sums to part; share_sums adds the S
// partials of a slot in split order once the team has passed a barrier.
template <class Sh, bool DS, bool PRED>
__device__ void ens_pairs(const EnsArgs &A, int64_t base, int n, float eps2, double eps2d,
                          double tn,
                          const Block &B, int n_i, int g, int rank, int S, int n_max,
                          double *anew, double *knew, double *part, TileRec *tile,
                          double (*red)[6 * Sh::IT][64]) {
    if (n_i < 1) return;
    const int64_t nb = (n_i + 64 * Sh::IT - 1) / (64 * Sh::IT);
    const int64_t items = nb * S;
    const int jchunk = (int)((n + S - 1) / S);
    const int lane = threadIdx.x & 63;
    for (int64_t it = rank; it < items; it += g) {
        const int64_t ib = it % nb, sp = it / nb;
        const int j0 = (int)(sp * jchunk), j1 = min(n, j0 + jchunk);
        const int slot0 = (int)(ib * 64 * Sh::IT);
        const int w = item_width<Sh::IT>(n_i - slot0, PRED);
        double tot[Sh::IT][6];
        int ni = 1, L = 1;
        if (Sh::IT == 2 && w == 128) {
            ens_pair_item<Sh, DS, PRED, Sh::IT, 1>(A, base, eps2, eps2d, tn, B, n_i, slot0, j0, j1,
                                                   tile, red, tot);
            ni = 2;
        } else if (w == 64) {
            ens_pair_item<Sh, DS, PRED, 1, 1>(A, base, eps2, eps2d, tn, B, n_i, slot0, j0, j1, tile, red,
                                              tot);
        } else if (PRED && w == 32) {
            ens_pair_item<Sh, DS, PRED, 1, 2>(A, base, eps2, eps2d, tn, B, n_i, slot0, j0, j1, tile, red,
                                              tot);
            L = 2;
        } else if (PRED && w == 16) {
            ens_pair_item<Sh, DS, PRED, 1, 4>(A, base, eps2, eps2d, tn, B, n_i, slot0, j0, j1, tile, red,
                                              tot);
            L = 4;
        } else if (PRED) {
            ens_pair_item<Sh, DS, PRED, 1, 8>(A, base, eps2, eps2d, tn, B, n_i, slot0, j0, j1, tile, red,
                                              tot);
            L = 8;
        }
        if ((threadIdx.x >> 6) == 0 && lane % L == 0) {
#pragma unroll
            for (int t = 0; t < Sh::IT; ++t) {
                const int slot = slot0 + t * (64 / L) + lane / L;
                if (t >= ni || slot >= n_i) continue;
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
}

// Acceleration and jerk of block slots [b0, b0 + cnt), cnt <= TH: with
// S = 1 the item sums, otherwise the S partial sums of each slot added in
// float64 in split order, one (slot, component) per thread with the partial
// loads batched; the six components of slot b0 + l land in buf[c * TH + l].
template <class Sh>
__device__ __forceinline__ void share_sums(int b0, int cnt, int S, int n_max, const double *anew,
                                           const double *knew, const double *part, double *buf) {
    for (int e = threadIdx.x; e < 6 * cnt; e += Sh::TH) {
        const int c = e / cnt, l = e - c * cnt, s = b0 + l;
        double acc;
        if (S == 1) {
            acc = c < 3 ? anew[c * n_max + s] : knew[(c - 3) * n_max + s];
        } else {
            const double *pp = part + (int64_t)c * n_max + s;
            const int64_t stride = 6 * (int64_t)n_max;
            acc = 0.0;
            int p = 0;
            for (; p + 4 <= S; p += 4) {
                const double v0 = pp[p * stride], v1 = pp[(p + 1) * stride];
                const double v2 = pp[(p + 2) * stride], v3 = pp[(p + 3) * stride];
                acc += v0;
                acc += v1;
                acc += v2;
                acc += v3;
            }
            for (; p < S; ++p) acc += pp[p * stride];
        }
        buf[c * Sh::TH + l] = acc;
    }
    __syncthreads();
}

// One block step of a cluster is two team phases, each closed by a team
// barrier:
//   B  every group finds the block on its own: t_next is the smaller of the
//      least t + dt among the particles the last step did not move (known
//      from the last scan) and the least new t + dt that the groups
//      published in the last correction; one pass over the cluster's t + dt
//      then compacts the members (t + dt == t_next), ascending, into the
//      group's own member list and takes the least t + dt of the others;
//      then the pair sums of the block, every particle predicted to t_next
//      as it is loaded (no predicted copy of the state is stored);
//   C  every group takes a contiguous share of the block's slots, adds their
//      split partial sums, corrects them (predicting them again, bitwise the
//      same) and publishes the least new t + dt of its share.
// t + dt changes in phase C alone, and every group reaches phase C of a step
// only after every group has finished that step's scan, so the groups always
// see the same block.
template <class Sh, bool DS>
__global__ __launch_bounds__(Sh::TH, 3) void ensemble_kernel(const EnsArgs A) {
    constexpr int ETH = Sh::TH;
    constexpr int EW = Sh::W;
    constexpr int SCAN = 8;  // particles per thread and pass of the block scan
    __shared__ TileRec tile[Sh::TILE];
    __shared__ double red[EW - 1][6 * Sh::IT][64];
    __shared__ double smin[EW];
    __shared__ int scount[SCAN * EW];
    // the slot sums of phase C reuse the tile (6 TH doubles <= 8 TILE)
    static_assert(6 * Sh::TH <= 8 * Sh::TILE, "slot sums fit the tile");
    double *sbuf = reinterpret_cast<double *>(tile);
    const int team = A.wg_team[blockIdx.x];
    const int rank = A.wg_rank[blockIdx.x];
    const EnsTeam T = A.teams[team];
    const int g = T.size;
    uint32_t *bar = A.bars + 64 * (int64_t)team;  // arrival words of the team
    uint32_t epoch = 0;
    double *scr = A.scratch + T.scratch_off;
    const int n_max = T.n_max;
    // scratch layout (doubles): pmin[64] | tnext[n_max] | anew[3 n_max] |
    // knew[3 n_max] | part[s_max * 6 * n_max] | act[g][n_max] (int32, one
    // member list per group)
    double *pmin = scr;
    double *tnext = scr + 64;
    double *anew = tnext + n_max;
    double *knew = anew + 3 * (int64_t)n_max;
    double *part = knew + 3 * (int64_t)n_max;
    int32_t *act = (int32_t *)(part + (int64_t)T.s_max * 6 * n_max) + (int64_t)rank * n_max;
    const int64_t nt = A.nt;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;

    for (int ci = T.cl_begin; ci < T.cl_end; ++ci) {
        const int c = A.cl_order[ci];
        const EnsCluster C = A.cl[c];
        const int64_t base = C.off;
        const int n = C.n;
        const float eps2 = C.eps2;
        const double eps2d = C.eps2d;
        if (rank == 0 && tid == 0) A.clock[2 * c] = wall_clock64();

        // ---- initialisation: pair sums of every particle, initial steps
        {
            const int S = ens_splits<Sh>(n, n, g, T.s_max);
            ens_pairs<Sh, DS, false>(A, base, n, eps2, eps2d, 0.0, Block{nullptr}, n, g, rank, S,
                                     n_max, anew, knew, part, tile, red);
            if (!team_barrier(bar, g, rank, epoch, A.abort, A.spin_limit)) return;
            const int per = (n + g - 1) / g;
            const int s0 = min(n, rank * per), s1 = min(n, s0 + per);
            double mn = INFINITY;
            for (int b0 = s0; b0 < s1; b0 += ETH) {
                const int cnt = min(ETH, s1 - b0);
                share_sums<Sh>(b0, cnt, S, n_max, anew, knew, part, sbuf);
                if (tid < cnt) {
                    const int i = b0 + tid;
                    const int64_t q = base + i;
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) {
                        A.a[cc * nt + q] = sbuf[cc * ETH + tid];
                        A.k[cc * nt + q] = sbuf[(3 + cc) * ETH + tid];
                    }
                    int32_t st = 0;
                    A.t[q] = 0.0;
                    const double d =
                        initial_dt_one(q, nt, 0.0, A.a, A.k, A.eta_s, A.dt_max, A.dt_min, &st);
                    A.dt[q] = d;
                    tnext[i] = 0.0 + d;
                    mn = fmin(mn, 0.0 + d);
                    if (st) atomicOr(A.status, st);
                }
                __syncthreads();
            }
            mn = group_min<Sh>(mn, smin);
            if (tid == 0) pmin[rank] = mn;
            if (!team_barrier(bar, g, rank, epoch, A.abort, A.spin_limit)) return;
        }

        int64_t my_steps = 0, my_inter = 0;
        double rest = INFINITY;  // least t + dt of the particles the last step left alone
        for (;;) {
            // ---- B: the block time, the block's members, their pair sums
            double tn = rest;
            if (tid < 64) {
                double v = tid < g ? pmin[tid] : INFINITY;
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
                if (tid == 0) smin[0] = v;
            }
            __syncthreads();
            tn = fmin(tn, smin[0]);
            if (!(tn <= A.t_end)) break;
            int n_i = 0;
            double rmin = INFINITY;
            const unsigned long long below = (1ull << lane) - 1ull;
            for (int pb = 0; pb < n; pb += SCAN * ETH) {
                double s[SCAN];
#pragma unroll
                for (int u = 0; u < SCAN; ++u) {
                    const int i = pb + u * ETH + tid;
                    s[u] = i < n ? tnext[i] : INFINITY;
                }
                bool f[SCAN];
                unsigned long long bal[SCAN];
#pragma unroll
                for (int u = 0; u < SCAN; ++u) {
                    f[u] = (s[u] == tn);
                    if (!f[u]) rmin = fmin(rmin, s[u]);
                    bal[u] = __ballot(f[u]);
                    if (lane == 0) scount[u * EW + wave] = __popcll(bal[u]);
                }
                __syncthreads();
#pragma unroll
                for (int u = 0; u < SCAN; ++u) {
                    int woff = 0, tot = 0;
#pragma unroll
                    for (int w = 0; w < EW; ++w) {
                        const int cw = scount[u * EW + w];
                        woff += (w < wave) ? cw : 0;
                        tot += cw;
                    }
                    if (f[u]) act[n_i + woff + __popcll(bal[u] & below)] = pb + u * ETH + tid;
                    n_i += tot;
                }
                __syncthreads();
            }
            rest = group_min<Sh>(rmin, smin);
            const int S = ens_splits<Sh>(n_i, n, g, T.s_max);
            ens_pairs<Sh, DS, true>(A, base, n, eps2, eps2d, tn, Block{act}, n_i, g, rank, S,
                                    n_max,
                                    anew, knew, part, tile, red);
            if (!team_barrier(bar, g, rank, epoch, A.abort, A.spin_limit)) return;

            // ---- C: correct this group's share of the block's slots
            const int per = (n_i + g - 1) / g;
            const int s0 = min(n_i, rank * per), s1 = min(n_i, s0 + per);
            double nmin = INFINITY;
            for (int b0 = s0; b0 < s1; b0 += ETH) {
                const int cnt = min(ETH, s1 - b0);
                share_sums<Sh>(b0, cnt, S, n_max, anew, knew, part, sbuf);
                if (tid < cnt) {
                    const int i = act[b0 + tid];
                    const int64_t q = base + i;
                    Raw r;
                    load_raw<true>(A, q, r);
                    double px[3], pv[3];
                    raw_state<true>(r, tn, px, pv);
                    double a1v[3], k1v[3];
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) {
                        a1v[cc] = sbuf[cc * ETH + tid];
                        k1v[cc] = sbuf[(3 + cc) * ETH + tid];
                    }
                    double tq;
                    const int32_t st =
                        correct_vals(q, nt, px, pv, a1v, k1v, A.eta, A.dt_max, A.dt_min, 0, A.t,
                                     A.dt, A.x, A.v, A.a, A.k, &tq);
                    if (st) atomicOr(A.status, st);
                    tnext[i] = tq;
                    nmin = fmin(nmin, tq);
                }
                __syncthreads();
            }
            nmin = group_min<Sh>(nmin, smin);
            if (tid == 0) pmin[rank] = nmin;
            my_steps += 1;
            my_inter += (int64_t)n_i * n;
            if (!team_barrier(bar, g, rank, epoch, A.abort, A.spin_limit)) return;
        }
        if (rank == 0 && tid == 0) {
            A.steps[c] = my_steps;
            A.inter[c] = my_inter;
            A.clock[2 * c + 1] = wall_clock64();
        }
        // the next cluster's initialisation rewrites the scratch: make sure
        // every group of the team is past this cluster
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

// ---- compiled launch shapes ------------------------------------------------
struct EnsVariant {
    int w, tile, it, th;
    const void *fn[2];  // float32 sums, compensated sums
};

template <int W, int TILE, int IT>
static EnsVariant ens_variant() {
    typedef ESh<W, TILE, IT> S;
    return EnsVariant{W, TILE, IT, S::TH,
                      {(const void *)ensemble_kernel<S, false>,
                       (const void *)ensemble_kernel<S, true>}};
}

const EnsVariant *find_variant(int w, int tile, int it) {
    static const EnsVariant v[] = {
        ens_variant<4, 256, 2>(), ens_variant<4, 256, 1>(), ens_variant<2, 128, 2>(),
        ens_variant<2, 256, 2>(), ens_variant<4, 512, 2>(), ens_variant<8, 512, 2>(),
    };
    for (const EnsVariant &x : v)
        if (x.w == w && x.tile == tile && x.it == it) return &x;
    return nullptr;
}

// ---- host-side team planning ----------------------------------------------
struct Plan {
    std::vector<EnsTeam> teams;
    std::vector<int32_t> order, wg_team, wg_rank;
    int64_t scratch = 0;  // doubles
};

struct TimeModel {
    double step_s, barrier_s, barrier_g_s, rate, t_end, coef, expo, tile_s, bcoef, bexpo;
    int slots, tile;  // block slots per item (64 i_per_lane), j records per tile
    double steps(double n) const { return std::max(1.0, coef * std::pow(n, expo) * t_end); }
    double block(double n) const { return std::min(n, std::max(1.0, bcoef * std::pow(n, bexpo))); }
    // j tiles of the busiest group in a pair pass of n_i slots (the kernel's
    // split rule, ens_splits)
    double tiles(int64_t n_i, int64_t n, int g) const {
        const int64_t nb = (n_i + slots - 1) / slots;
        const int64_t smax = std::max<int64_t>(1, std::min<int64_t>(std::min(EMAXSPLIT, g), n / tile));
        int64_t best = 1, bq = (nb + g - 1) / g;
        for (int64_t S = 2; S <= smax; ++S) {
            const int64_t q = (nb * S + g - 1) / g;
            if (q * best < bq * S) {
                best = S;
                bq = q;
            }
        }
        const int64_t jchunk = (n + best - 1) / best;
        return (double)(bq * ((jchunk + tile - 1) / tile));
    }
    double pass(double n_i, double n, int g) const {
        return tiles((int64_t)std::ceil(n_i), (int64_t)n, g) * tile_s + n_i * n / ((double)g * rate);
    }
    // time of a cluster of n particles with `st` steps of blocks of `blk`
    double time_sb(double n, double st, double blk, int g) const {
        return pass(n, n, g) + st * (step_s + (g > 1 ? barrier_s + barrier_g_s * g : 0.0) +
                                     pass(blk, n, g));
    }
    double time(double n, int g) const { return time_sb(n, steps(n), block(n), g); }
    static TimeModel of(const nbody_ensemble_config &c, double t_end) {
        return TimeModel{c.step_us * 1e-6,  c.barrier_us * 1e-6, c.barrier_group_us * 1e-6,
                         c.group_rate,      t_end,              c.steps_coef,
                         c.steps_exp,       c.tile_us * 1e-6,   c.block_coef,
                         c.block_exp,       64 * c.i_per_lane,  c.j_tile};
    }
};

// Team plan of least modelled makespan.  For a target time T every cluster
// needs the fewest groups g(T) whose modelled time is within T; the clusters
// that one group finishes within T are packed onto shared single-group teams
// (longest first onto the least-loaded one: a team runs its clusters one
// after the other),
// the others get teams of g(T) groups.  T is bisected down to the least
// value whose plan fits the grid; the groups left over then go, one at a
// time, to the team with the longest modelled time while that shortens it.
static Plan plan_teams(const std::vector<int64_t> &sizes, int G, int max_team,
                       const TimeModel &M) {
    const int nc = (int)sizes.size();
    // modelled time of cluster c on g groups (its step count and block size
    // computed once)
    std::vector<double> st(nc), blk(nc);
    for (int c = 0; c < nc; ++c) {
        st[c] = M.steps((double)sizes[c]);
        blk[c] = M.block((double)sizes[c]);
    }
    auto tm = [&](int c, int g) { return M.time_sb((double)sizes[c], st[c], blk[c], g); };
    std::vector<double> t1(nc);
    double lo = 0.0, hi = 0.0;
    for (int c = 0; c < nc; ++c) {
        t1[c] = tm(c, 1);
        double best = t1[c];
        for (int g = 2; g <= max_team; ++g) best = std::min(best, tm(c, g));
        lo = std::max(lo, best);
        hi += t1[c];
    }
    std::vector<int> by_t1(nc);
    std::iota(by_t1.begin(), by_t1.end(), 0);
    std::sort(by_t1.begin(), by_t1.end(), [&](int p, int q) {
        return t1[p] > t1[q] || (t1[p] == t1[q] && p < q);
    });
    std::vector<int> gsz(nc);
    std::vector<std::vector<int>> bins;
    std::vector<double> bin_load;
    // groups that the plan for target T needs (gsz, bins filled), or -1
    auto build = [&](double T) -> int64_t {
        int64_t used = 0;
        bins.clear();
        bin_load.clear();
        for (int c = 0; c < nc; ++c) {
            gsz[c] = 0;
            if (t1[c] <= T) continue;  // packed below
            int g = 2;
            while (g <= max_team && tm(c, g) > T) ++g;
            if (g > max_team) return -1;
            gsz[c] = g;
            used += g;
        }
        // longest first onto the least-loaded shared team, a new one when
        // even that would pass T (O(log teams) per cluster)
        typedef std::pair<double, int> LB;
        std::priority_queue<LB, std::vector<LB>, std::greater<LB>> least;
        for (int c : by_t1) {
            if (gsz[c] != 0) continue;
            gsz[c] = 1;
            int b;
            if (!least.empty() && least.top().first + t1[c] <= T) {
                b = least.top().second;
                least.pop();
            } else {
                b = (int)bins.size();
                bins.push_back({});
                bin_load.push_back(0.0);
            }
            bins[b].push_back(c);
            bin_load[b] += t1[c];
            least.push(LB(bin_load[b], b));
        }
        return used + (int64_t)bins.size();
    };
    for (int it = 0; it < 60 && hi - lo > 1e-7 * hi; ++it) {
        const double mid = 0.5 * (lo + hi);
        const int64_t u = build(mid);
        if (u >= 0 && u <= G)
            hi = mid;
        else
            lo = mid;
    }
    build(hi);

    std::vector<std::vector<int>> tcl;
    std::vector<int> tsize;
    for (int c = 0; c < nc; ++c)
        if (gsz[c] > 1) {
            tcl.push_back({c});
            tsize.push_back(gsz[c]);
        }
    for (const std::vector<int> &b : bins) {
        tcl.push_back(b);
        tsize.push_back(1);
    }
    const int nteam = (int)tcl.size();
    auto team_time = [&](int t, int g) {
        double s = 0.0;
        for (int c : tcl[t]) s += tm(c, g);
        return s;
    };
    int spare = G - std::accumulate(tsize.begin(), tsize.end(), 0);
    typedef std::pair<double, int> TT;
    std::priority_queue<TT> heap;
    for (int t = 0; t < nteam; ++t) heap.push(TT(team_time(t, tsize[t]), t));
    while (spare > 0 && !heap.empty()) {
        const TT top = heap.top();
        heap.pop();
        const int t = top.second;
        if (tsize[t] >= max_team) continue;
        const double t_next = team_time(t, tsize[t] + 1);
        if (!(t_next < top.first)) continue;  // more groups no longer help
        tsize[t] += 1;
        --spare;
        heap.push(TT(t_next, t));
    }
    // longest teams first in the grid
    std::vector<int> torder(nteam);
    std::iota(torder.begin(), torder.end(), 0);
    std::vector<double> tt(nteam);
    for (int t = 0; t < nteam; ++t) tt[t] = team_time(t, tsize[t]);
    std::sort(torder.begin(), torder.end(),
              [&](int p, int q) { return tt[p] > tt[q] || (tt[p] == tt[q] && p < q); });

    Plan P;
    for (int t : torder) {
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
        P.scratch += 64 + 7 * (int64_t)nmax + (int64_t)T.s_max * 6 * nmax +
                     ((int64_t)T.size * nmax + 1) / 2 + 8;
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

extern "C" int nbody_ensemble_plan(const int64_t *sizes, int32_t n_clusters, int32_t groups,
                                   const nbody_ensemble_config *cfg, double t_end,
                                   int32_t *team_of, int32_t *team_size, double *model_seconds,
                                   int32_t *n_teams) {
    if (!sizes || !cfg || !team_of || !team_size || !n_teams || n_clusters < 1 || groups < 1 ||
        !(t_end >= 0.0) || !(cfg->group_rate > 0.0) || !(cfg->steps_coef > 0.0) ||
        !(cfg->block_coef > 0.0) || !(cfg->tile_us >= 0.0) ||
        !find_variant(cfg->waves, cfg->j_tile, cfg->i_per_lane) ||
        cfg->max_team < 1)
        return NBODY_E_INVAL;
    std::vector<int64_t> sz(sizes, sizes + n_clusters);
    for (int64_t v : sz)
        if (v < 1) return NBODY_E_INVAL;
    const TimeModel M = TimeModel::of(*cfg, t_end);
    Plan P = plan_teams(sz, groups, std::min(cfg->max_team, 64), M);
    for (int q = 0; q < (int)P.teams.size(); ++q) {
        const EnsTeam &T = P.teams[q];
        team_size[q] = T.size;
        for (int r = T.cl_begin; r < T.cl_end; ++r) {
            const int c = P.order[r];
            team_of[c] = q;
            if (model_seconds) model_seconds[c] = M.time((double)sz[c], T.size);
        }
    }
    *n_teams = (int32_t)P.teams.size();
    return NBODY_OK;
}

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
    const EnsVariant *var = find_variant(ctx->ens_cfg.waves, ctx->ens_cfg.j_tile,
                                         ctx->ens_cfg.i_per_lane);
    if (!var) return fail(ctx, NBODY_E_INVAL, "ensemble: shape not compiled");
    const void *kfn = var->fn[ds ? 1 : 0];
    const int ETH = var->th;
    int occ = 0;
    NB_TRY(hip_check(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kfn, ETH, 0),
                     "occupancy"));
    int per_cu = std::min(occ, ctx->ens_cfg.groups_per_cu);
    if (per_cu < 1) return fail(ctx, NBODY_E_DEVICE, "ensemble kernel does not fit a CU");
    const int G = per_cu * ctx->cus;
    const nbody_ensemble_config &cf = ctx->ens_cfg;
    const TimeModel M = TimeModel::of(cf, t_end > 0 ? t_end : 0.0);
    Plan P = plan_teams(sizes, G, std::min(cf.max_team, 64), M);
    const int grid = (int)P.wg_team.size();
    const int nteams = (int)P.teams.size();

    std::vector<EnsCluster> hc(nc);
    for (int c = 0; c < nc; ++c)
        hc[c] = EnsCluster{e->offsets[c], (int32_t)sizes[c], (float)e->eps2[c], e->eps2[c]};

    // one device block: tables, counters, team scratch
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t b_cl = al(sizeof(EnsCluster) * nc), b_ord = al(4 * P.order.size()),
                 b_tm = al(sizeof(EnsTeam) * nteams), b_wg = al(4 * (size_t)grid),
                 b_bar = al(4 * 64 * (size_t)nteams), b_cnt = al(8 * (size_t)nc),
                 b_clk = al(16 * (size_t)nc),
                 b_fl = al(8), b_scr = al(8 * (size_t)P.scratch);
    const size_t total = b_cl + b_ord + b_tm + 2 * b_wg + b_bar + 2 * b_cnt + b_clk + b_fl + b_scr;
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
    double *d_scr = (double *)p;

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
