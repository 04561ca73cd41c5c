// Pair sums of acceleration, jerk and potential (Section 2, Eq. (1), in the
// softened form of the Appendix A listing) on gfx950.
//
// Mapping (one lane per i-particle, j streamed through the scalar path):
//   * the j side is a packed 64-byte record per particle; the j loop index
//     is wave-uniform, so each record is fetched with scalar loads into SGPRs
//     and every lane reads it as an instruction operand: no LDS traffic and
//     no VGPRs for j data in the inner loop;
//   * each lane keeps IT i-particles;
//   * r = x_j - x_i and w = v_j - v_i are formed to float64 accuracy (see the
//     record forms in records.hpp);
//   * float32 mode: the pair arithmetic is float32 with the VALU reciprocal
//     square root; a wave sums `tile` consecutive j in float32, adds the
//     tile sums of up to kFoldTiles tiles in float32 and that sum to a
//     per-lane float64 total in LDS;
//   * compensated mode: the pair arithmetic is float64 (it issues at about
//     half the float32 rate, but needs no float64-to-float32 conversions),
//     s^(-1/2) from the float32 estimate refined by one float64 Newton step,
//     float64 sums;
//   * the W waves of a workgroup share the same i-particles and split their
//     j range; their sums are combined in float64 through LDS in wave order;
//   * the j range is also split across S workgroups when the active block
//     is too small to fill the GPU, and into chunks of a few MB at any size
//     so that the groups resident on an XCD share them in its L2; the
//     partial sums (float32 in the float32 mode, float64 otherwise) are
//     added in split order, in float64, by a second kernel;
//   * workgroups take their items XCD by XCD (xcd_item in pairs.hpp).
// The self pair is skipped by index: tiles whose j range can contain one of
// the wave's own indices take a masked path.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "pairs.hpp"

namespace nb {

template <int REP>
__global__ void pack_kernel(int64_t n, const double *__restrict__ pos,
                            const double *__restrict__ vel, const double *__restrict__ mass,
                            JRec *__restrict__ out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    store_rec(REP, out + i, pos[i], pos[n + i], pos[2 * n + i], vel[i], vel[n + i],
              vel[2 * n + i], mass[i]);
}

int launch_pack(nbody_ctx *ctx, int rep, int64_t n, const double *pos, const double *vel,
                const double *mass, JRec *out) {
    if (n <= 0) return NBODY_OK;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    if (rep == REP_FF)
        pack_kernel<REP_FF><<<g, b, 0, ctx->stream>>>(n, pos, vel, mass, out);
    else if (rep == REP_F64V)
        pack_kernel<REP_F64V><<<g, b, 0, ctx->stream>>>(n, pos, vel, mass, out);
    else
        pack_kernel<REP_F64><<<g, b, 0, ctx->stream>>>(n, pos, vel, mass, out);
    return hip_check(ctx, hipGetLastError(), "pack_kernel");
}

// ---- record forms: scalar-path loads and relative coordinates -------------
template <int REP>
struct Form;

template <>
struct Form<REP_F64> {
    typedef RecF64 Rec;
    struct I {
        double x, y, z, u, v, w;
    };
    static __device__ __forceinline__ Rec load(CONSTP(JRec) base, int j) {
        CONSTP(Rec) R = (CONSTP(Rec))base;
        Rec r;
        r.x = R[j].x; r.y = R[j].y; r.z = R[j].z; r.m = R[j].m;
        r.u = R[j].u; r.v = R[j].v; r.w = R[j].w;
        return r;
    }
    static __device__ __forceinline__ I own(double x, double y, double z, double u, double v,
                                            double w) {
        return I{x, y, z, u, v, w};
    }
    static __device__ __forceinline__ void rel(const Rec &r, const I &s, float &dx, float &dy,
                                               float &dz, float &du, float &dv, float &dw) {
        dx = (float)(r.x - s.x);
        dy = (float)(r.y - s.y);
        dz = (float)(r.z - s.z);
        du = (float)(r.u - s.u);
        dv = (float)(r.v - s.v);
        dw = (float)(r.w - s.w);
    }
};

template <>
struct Form<REP_FF> {
    typedef RecFF Rec;
    struct I {
        float xh, yh, zh, uh, vh, wh, xl, yl, zl, ul, vl, wl;
    };
    static __device__ __forceinline__ Rec load(CONSTP(JRec) base, int j) {
        CONSTP(Rec) R = (CONSTP(Rec))base;
        Rec r;
        r.xh = R[j].xh; r.yh = R[j].yh; r.zh = R[j].zh; r.m = R[j].m;
        r.uh = R[j].uh; r.vh = R[j].vh; r.wh = R[j].wh;
        r.xl = R[j].xl; r.yl = R[j].yl; r.zl = R[j].zl;
        r.ul = R[j].ul; r.vl = R[j].vl; r.wl = R[j].wl;
        return r;
    }
    static __device__ __forceinline__ I own(double x, double y, double z, double u, double v,
                                            double w) {
        I s;
        split_ff(x, s.xh, s.xl);
        split_ff(y, s.yh, s.yl);
        split_ff(z, s.zh, s.zl);
        split_ff(u, s.uh, s.ul);
        split_ff(v, s.vh, s.vl);
        split_ff(w, s.wh, s.wl);
        return s;
    }
    static __device__ __forceinline__ void rel(const Rec &r, const I &s, float &dx, float &dy,
                                               float &dz, float &du, float &dv, float &dw) {
        dx = (r.xh - s.xh) + (r.xl - s.xl);
        dy = (r.yh - s.yh) + (r.yl - s.yl);
        dz = (r.zh - s.zh) + (r.zl - s.zl);
        du = (r.uh - s.uh) + (r.ul - s.ul);
        dv = (r.vh - s.vh) + (r.vl - s.vl);
        dw = (r.wh - s.wh) + (r.wl - s.wl);
    }
};

template <>
struct Form<REP_F64V> {
    typedef RecF64V Rec;
    struct I {
        double x, y, z;
        float u, v, w;
    };
    static __device__ __forceinline__ Rec load(CONSTP(JRec) base, int j) {
        CONSTP(Rec) R = (CONSTP(Rec))base;
        Rec r;
        r.x = R[j].x; r.y = R[j].y; r.z = R[j].z; r.m = R[j].m;
        r.u = R[j].u; r.v = R[j].v; r.w = R[j].w;
        return r;
    }
    static __device__ __forceinline__ I own(double x, double y, double z, double u, double v,
                                            double w) {
        return I{x, y, z, (float)u, (float)v, (float)w};
    }
    static __device__ __forceinline__ void rel(const Rec &r, const I &s, float &dx, float &dy,
                                               float &dz, float &du, float &dv, float &dw) {
        dx = (float)(r.x - s.x);
        dy = (float)(r.y - s.y);
        dz = (float)(r.z - s.z);
        du = r.u - s.u;
        dv = r.v - s.v;
        dw = r.w - s.w;
    }
};

// Float32 tile sums added in float32 before each float64 fold (so no
// float32 sum spans more than kFoldTiles * tile j, whatever the launch shape).
constexpr int kFoldTiles = 8;

template <int REP, int IT, int W, int ACC>
__global__ __launch_bounds__(64 * W) void force_kernel(const KArgs a) {
    typedef Form<REP> F;
    typedef typename F::Rec Rec;
    static_assert(ACC != ACC_F64 || REP == REP_F64, "float64 pair terms need float64 records");
    const int64_t n_i = block_size(a);
    if (n_i <= 0 || n_i <= a.jl_max) return;  // (j-lane kernel's blocks)
    const int n_j = a.n_j;
    const int64_t ostride = a.out_stride > 0 ? a.out_stride : n_i;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nb = (n_i + 64 * IT - 1) / (64 * IT);
    const int64_t S = choose_splits(n_i, n_j, IT, W, a.min_j_wave, a.target_groups, a.max_splits);
    const int64_t items = nb * S;
    const int64_t jchunk = (n_j + S - 1) / S;
    const float eps2 = a.eps2;
    const double eps2d = a.eps2d;
    const int tile = a.tile;
    // Constant address space: the records are read-only during the kernel
    // and their addresses are wave-uniform, so every field is fetched with a
    // scalar load into SGPRs.
    const CONSTP(JRec) J = (CONSTP(JRec))a.jrec;

    // Per-wave float64 totals of each lane's sums: the running totals of
    // the float32 tile sums (ACC_F32), and the slices the waves of the
    // group combine in wave order at the end of an item.
    __shared__ double red[W][7 * IT][64];

    for (int64_t q = blockIdx.x; q < items; q += gridDim.x) {
        const int64_t item = xcd_item(q, items);
        const int64_t ib = item % nb;
        const int64_t sp = item / nb;
        const int j0 = (int)(sp * jchunk);
        const int j1 = (int)min((int64_t)n_j, (int64_t)j0 + jchunk);
        const int jw = (j1 - j0 + W - 1) / W;
        const int jb = __builtin_amdgcn_readfirstlane(min(j1, j0 + wave * jw));
        const int je = __builtin_amdgcn_readfirstlane(min(j1, jb + jw));

        typename F::I own[IT];
        int idx[IT];
        int64_t slot[IT];
        int lo_idx = 0x7fffffff, hi_idx = -1;
#pragma unroll
        for (int t = 0; t < IT; ++t) {
            slot[t] = ib * (64 * IT) + t * 64 + lane;
            const int64_t sl = slot[t] < n_i ? slot[t] : n_i - 1;
            idx[t] = a.active ? a.active[sl] : (int)sl;
            if ((unsigned)idx[t] >= (unsigned)n_j) {
                atomicOr(a.status, (int32_t)ST_INDEX);
                idx[t] = 0;
            }
            const int64_t q = idx[t];
            own[t] = F::own(a.pos[q], a.pos[n_j + q], a.pos[2 * (int64_t)n_j + q], a.vel[q],
                            a.vel[n_j + q], a.vel[2 * (int64_t)n_j + q]);
            lo_idx = min(lo_idx, idx[t]);
            hi_idx = max(hi_idx, idx[t]);
        }
        lo_idx = __builtin_amdgcn_readfirstlane(wave_min(lo_idx));
        hi_idx = __builtin_amdgcn_readfirstlane(wave_max(hi_idx));

        // Running sums: ACC_F32 adds the float32 tile sums of up to
        // kFoldTiles tiles in float32, then that sum to a float64 total kept
        // in LDS (folding every tile measured 1.3 % slower: each LDS wait also
        // drains the scalar j loads in flight); ACC_F64 keeps float64 sums in
        // registers.  The potential is accumulated as +sum m/r and negated
        // when stored.
        double sd[IT][7];
        float sr[IT][7];
        int nfold = 0;
#pragma unroll
        for (int t = 0; t < IT; ++t)
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                sd[t][k] = 0.0;
                sr[t][k] = 0.0f;
                if (ACC == ACC_F32) red[wave][t * 7 + k][lane] = 0.0;
            }

        for (int jt = jb; jt < je; jt += tile) {
            const int jend = min(je, jt + tile);
            const bool masked = jt <= hi_idx && jend > lo_idx;
            if constexpr (ACC == ACC_F64) {
                // float64 relative coordinates and pair terms; s^(-1/2)
                // from the float32 hardware estimate, refined by one
                // Newton step in float64 (relative error ~1e-14)
                auto body64 = [&](const RecF64 &r, const int j, const bool mask)
                    __attribute__((always_inline)) {
#pragma unroll
                    for (int t = 0; t < IT; ++t) {
                        const double dx = r.x - own[t].x, dy = r.y - own[t].y,
                                     dz = r.z - own[t].z;
                        const double du = r.u - own[t].u, dv = r.v - own[t].v,
                                     dw = r.w - own[t].w;
                        double s2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2d)));
                        double mj = r.md;
                        if (mask) {
                            const bool self = (j == idx[t]);
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
                        sd[t][6] = fma(mj, y, sd[t][6]);
                    }
                };
                CONSTP(RecF64) R = (CONSTP(RecF64))J;
                auto load64 = [&](int j) __attribute__((always_inline)) {
                    RecF64 r;
                    r.x = R[j].x; r.y = R[j].y; r.z = R[j].z; r.md = R[j].md;
                    r.u = R[j].u; r.v = R[j].v; r.w = R[j].w;
                    return r;
                };
                if (masked) {
                    for (int j = jt; j < jend; ++j) body64(load64(j), j, true);
                } else {
                    RecF64 cur = load64(jt);
#pragma unroll 2
                    for (int j = jt; j < jend; ++j) {
                        const RecF64 nxt = load64(min(j + 1, jend - 1));
                        body64(cur, j, false);
                        cur = nxt;
                    }
                }
            } else {
                float ts[IT][7];
#pragma unroll
                for (int t = 0; t < IT; ++t)
#pragma unroll
                    for (int k = 0; k < 7; ++k) ts[t][k] = 0.0f;

                auto body = [&](const Rec &r, const int j, const bool mask)
                    __attribute__((always_inline)) {
#pragma unroll
                    for (int t = 0; t < IT; ++t) {
                        float dx, dy, dz, du, dv, dw;
                        F::rel(r, own[t], dx, dy, dz, du, dv, dw);
                        float s2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
                        float mj = r.m;
                        if (mask) {
                            const bool self = (j == idx[t]);
                            s2 = self ? 1.0f : s2;
                            mj = self ? 0.0f : mj;
                        }
                        const float rv = fmaf(dz, dw, fmaf(dy, dv, dx * du));
                        const float rinv = __builtin_amdgcn_rsqf(s2);
                        const float rinv2 = rinv * rinv;
                        const float mr1 = mj * rinv;
                        const float mr3 = mr1 * rinv2;
                        const float w3 = (rv * rinv2) * -3.0f;
                        ts[t][0] = fmaf(mr3, dx, ts[t][0]);
                        ts[t][1] = fmaf(mr3, dy, ts[t][1]);
                        ts[t][2] = fmaf(mr3, dz, ts[t][2]);
                        ts[t][3] = fmaf(mr3, fmaf(w3, dx, du), ts[t][3]);
                        ts[t][4] = fmaf(mr3, fmaf(w3, dy, dv), ts[t][4]);
                        ts[t][5] = fmaf(mr3, fmaf(w3, dz, dw), ts[t][5]);
                        ts[t][6] = fmaf(mj, rinv, ts[t][6]);
                    }
                };

                if (masked) {
                    for (int j = jt; j < jend; ++j) {
                        const Rec r = F::load(J, j);
                        body(r, j, true);
                    }
                } else {
                    // software pipelined: the next record's scalar loads are
                    // in flight while the current one is used
                    Rec cur = F::load(J, jt);
#pragma unroll 4
                    for (int j = jt; j < jend; ++j) {
                        const Rec nxt = F::load(J, min(j + 1, jend - 1));
                        body(cur, j, false);
                        cur = nxt;
                    }
                }

#pragma unroll
                for (int t = 0; t < IT; ++t)
#pragma unroll
                    for (int k = 0; k < 7; ++k) sr[t][k] += ts[t][k];
                if (++nfold == kFoldTiles || jt + tile >= je) {
                    nfold = 0;
                    // (the barrier keeps the LDS totals from being loaded
                    // before the j loop, which would hold them in registers)
                    __asm__ volatile("" ::: "memory");
#pragma unroll
                    for (int t = 0; t < IT; ++t)
#pragma unroll
                        for (int k = 0; k < 7; ++k) {
                            red[wave][t * 7 + k][lane] += (double)sr[t][k];
                            sr[t][k] = 0.0f;
                        }
                }
            }
        }

        // per-wave totals in float64
        double tot[IT][7];
#pragma unroll
        for (int t = 0; t < IT; ++t)
#pragma unroll
            for (int k = 0; k < 7; ++k)
                tot[t][k] = ACC == ACC_F32 ? red[wave][t * 7 + k][lane] : sd[t][k];
        if (W > 1) {
            if (ACC != ACC_F32 && wave > 0) {
#pragma unroll
                for (int t = 0; t < IT; ++t)
#pragma unroll
                    for (int k = 0; k < 7; ++k) red[wave][t * 7 + k][lane] = tot[t][k];
            }
            __syncthreads();
            if (wave == 0) {
                for (int w = 1; w < W; ++w)
#pragma unroll
                    for (int t = 0; t < IT; ++t)
#pragma unroll
                        for (int k = 0; k < 7; ++k) tot[t][k] += red[w][t * 7 + k][lane];
            }
        }
        if (wave == 0) {
#pragma unroll
            for (int t = 0; t < IT; ++t) {
                tot[t][6] = -tot[t][6];
                if (slot[t] < n_i) {
                    const int64_t s = slot[t];
                    if (S == 1) {
                        a.acc[s] = tot[t][0];
                        a.acc[ostride + s] = tot[t][1];
                        a.acc[2 * ostride + s] = tot[t][2];
                        a.jerk[s] = tot[t][3];
                        a.jerk[ostride + s] = tot[t][4];
                        a.jerk[2 * ostride + s] = tot[t][5];
                        if (a.pot) a.pot[s] = tot[t][6];
                    } else if (!a.part_f32) {
                        double *p = a.part + (sp * 7) * n_i + s;
#pragma unroll
                        for (int k = 0; k < 7; ++k) p[k * n_i] = tot[t][k];
                    } else {
                        // float32 sums: the partial is kept to float32
                        // precision (half the traffic of the split partials)
                        float *p = (float *)a.part + (sp * 7) * n_i + s;
#pragma unroll
                        for (int k = 0; k < 7; ++k) p[k * n_i] = (float)tot[t][k];
                    }
                }
            }
        }
        if (W > 1) __syncthreads();
    }
}

// j-lane layout for small active blocks.  With few i-particles the i-lane
// kernel leaves most lanes idle and each wave walks its j range as a chain of
// dependent scalar loads; here the C i-particles of a workgroup are
// wave-uniform (scalar registers) and every lane takes its own j, fetched
// with coalesced vector loads (64 consecutive records per wave and step).
// A lane sums its j terms in float32 (at most `tile` of them, see
// choose_splits_jl) or float64; the lane sums are added in float64 by a
// fixed-order butterfly over the wave, the waves' totals in wave order
// through LDS, and the splits by reduce_parts_kernel.  Lanes past the end of
// the range and the self pair are masked (only in the 64-j steps that can
// contain them).
template <int C, int W, int ACC>
__global__ __launch_bounds__(64 * W) void force_jl_kernel(const KArgs a) {
    const int64_t n_i = block_size(a);
    if (n_i <= 0 || n_i > a.jl_max) return;  // (i-lane kernel's blocks)
    const int n_j = a.n_j;
    const int64_t ostride = a.out_stride > 0 ? a.out_stride : n_i;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nb = (n_i + C - 1) / C;
    const int64_t S = choose_splits_jl(n_i, n_j, C, W, a.jl_tile, a.jl_min_j_wave,
                                       a.jl_target_groups, a.max_splits);
    const int64_t items = nb * S;
    const int64_t jchunk = (n_j + S - 1) / S;
    const float eps2 = a.eps2;
    const double eps2d = a.eps2d;
    const RecF64 *__restrict__ R = (const RecF64 *)a.jrec;

    __shared__ double red[W > 1 ? W - 1 : 1][7 * C];

    for (int64_t q = blockIdx.x; q < items; q += gridDim.x) {
        const int64_t item = xcd_item(q, items);
        const int64_t ib = item % nb;
        const int64_t sp = item / nb;
        const int j0 = (int)(sp * jchunk);
        const int j1 = (int)min((int64_t)n_j, (int64_t)j0 + jchunk);
        // wave ranges in whole steps of 64 j
        const int jw = (((j1 - j0 + W - 1) / W) + 63) & ~63;
        const int jb = __builtin_amdgcn_readfirstlane(min(j1, j0 + wave * jw));
        const int je = __builtin_amdgcn_readfirstlane(min(j1, jb + jw));

        // the workgroup's i-particles, wave-uniform: read through the
        // constant address space, so with scalar loads into SGPRs
        int idx[C];
        double xi[C], yi[C], zi[C], ui[C], vi[C], wi[C];
        const CONSTP(int32_t) Act = (CONSTP(int32_t))a.active;
        const CONSTP(double) Pos = (CONSTP(double))a.pos;
        const CONSTP(double) Vel = (CONSTP(double))a.vel;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int64_t slot = ib * C + c;
            const int64_t sl = slot < n_i ? slot : n_i - 1;
            const int raw = Act ? Act[sl] : (int)sl;
            const bool bad = (unsigned)raw >= (unsigned)n_j;
            if (bad && lane == 0) atomicOr(a.status, (int32_t)ST_INDEX);
            const int id = __builtin_amdgcn_readfirstlane(bad ? 0 : raw);
            idx[c] = id;
            xi[c] = Pos[id];
            yi[c] = Pos[n_j + (int64_t)id];
            zi[c] = Pos[2 * (int64_t)n_j + id];
            ui[c] = Vel[id];
            vi[c] = Vel[n_j + (int64_t)id];
            wi[c] = Vel[2 * (int64_t)n_j + id];
        }

        // per-lane sums; the potential as +sum m/r (negated when stored)
        float s32[C][7];
        double s64[C][7];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                s32[c][k] = 0.0f;
                s64[c][k] = 0.0;
            }

        auto body = [&](const RecF64 &r, const int j, const bool mask)
            __attribute__((always_inline)) {
            const bool dead_j = j >= je;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if constexpr (ACC == ACC_F64) {
                    const double dx = r.x - xi[c], dy = r.y - yi[c], dz = r.z - zi[c];
                    const double du = r.u - ui[c], dv = r.v - vi[c], dw = r.w - wi[c];
                    double s2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2d)));
                    double mj = r.md;
                    if (mask) {
                        const bool dead = dead_j || j == idx[c];
                        s2 = dead ? 1.0 : s2;
                        mj = dead ? 0.0 : mj;
                    }
                    const double rv = fma(dz, dw, fma(dy, dv, dx * du));
                    const double y0 = (double)__builtin_amdgcn_rsqf((float)s2);
                    const double e = fma(-(s2 * y0), y0, 1.0);
                    const double y = fma(0.5 * y0, e, y0);
                    const double y2 = y * y;
                    const double mr3 = (mj * y) * y2;
                    const double w3 = (rv * y2) * -3.0;
                    s64[c][0] = fma(mr3, dx, s64[c][0]);
                    s64[c][1] = fma(mr3, dy, s64[c][1]);
                    s64[c][2] = fma(mr3, dz, s64[c][2]);
                    s64[c][3] = fma(mr3, fma(w3, dx, du), s64[c][3]);
                    s64[c][4] = fma(mr3, fma(w3, dy, dv), s64[c][4]);
                    s64[c][5] = fma(mr3, fma(w3, dz, dw), s64[c][5]);
                    s64[c][6] = fma(mj, y, s64[c][6]);
                } else {
                    const float dx = (float)(r.x - xi[c]), dy = (float)(r.y - yi[c]);
                    const float dz = (float)(r.z - zi[c]);
                    const float du = (float)(r.u - ui[c]), dv = (float)(r.v - vi[c]);
                    const float dw = (float)(r.w - wi[c]);
                    float s2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
                    float mj = r.m;
                    if (mask) {
                        const bool dead = dead_j || j == idx[c];
                        s2 = dead ? 1.0f : s2;
                        mj = dead ? 0.0f : mj;
                    }
                    const float rv = fmaf(dz, dw, fmaf(dy, dv, dx * du));
                    const float rinv = __builtin_amdgcn_rsqf(s2);
                    const float rinv2 = rinv * rinv;
                    const float mr3 = (mj * rinv) * rinv2;
                    const float w3 = (rv * rinv2) * -3.0f;
                    s32[c][0] = fmaf(mr3, dx, s32[c][0]);
                    s32[c][1] = fmaf(mr3, dy, s32[c][1]);
                    s32[c][2] = fmaf(mr3, dz, s32[c][2]);
                    s32[c][3] = fmaf(mr3, fmaf(w3, dx, du), s32[c][3]);
                    s32[c][4] = fmaf(mr3, fmaf(w3, dy, dv), s32[c][4]);
                    s32[c][5] = fmaf(mr3, fmaf(w3, dz, dw), s32[c][5]);
                    s32[c][6] = fmaf(mj, rinv, s32[c][6]);
                }
            }
        };
        auto load = [&](int j) __attribute__((always_inline)) {
            RecF64 r;
            r.x = R[j].x; r.y = R[j].y; r.z = R[j].z;
            r.u = R[j].u; r.v = R[j].v; r.w = R[j].w;
            if constexpr (ACC == ACC_F64) r.md = R[j].md; else r.m = R[j].m;
            return r;
        };

        if (jb < je) {
            // the next step's records are in flight while this one is used
            RecF64 cur = load(min(jb + lane, je - 1));
            for (int jt = jb; jt < je; jt += 64) {
                const RecF64 nxt = load(min(jt + 64 + lane, je - 1));
                bool edge = jt + 64 > je;
#pragma unroll
                for (int c = 0; c < C; ++c) edge |= (unsigned)(idx[c] - jt) < 64u;
                if (edge)
                    body(cur, jt + lane, true);
                else
                    body(cur, jt + lane, false);
                cur = nxt;
            }
        }

        // lane sums -> wave totals (float64 butterfly, fixed order)
        double tot[C][7];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                double v = ACC == ACC_F64 ? s64[c][k] : (double)s32[c][k];
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
                tot[c][k] = v;
            }
        if (W > 1) {
            if (wave > 0 && lane == 0) {
#pragma unroll
                for (int c = 0; c < C; ++c)
#pragma unroll
                    for (int k = 0; k < 7; ++k) red[wave - 1][c * 7 + k] = tot[c][k];
            }
            __syncthreads();
            if (wave == 0) {
                for (int w = 1; w < W; ++w)
#pragma unroll
                    for (int c = 0; c < C; ++c)
#pragma unroll
                        for (int k = 0; k < 7; ++k) tot[c][k] += red[w - 1][c * 7 + k];
            }
        }
        if (wave == 0) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int64_t slot = ib * C + c;
                if (lane == c && slot < n_i) {
                    tot[c][6] = -tot[c][6];
                    if (S == 1) {
                        a.acc[slot] = tot[c][0];
                        a.acc[ostride + slot] = tot[c][1];
                        a.acc[2 * ostride + slot] = tot[c][2];
                        a.jerk[slot] = tot[c][3];
                        a.jerk[ostride + slot] = tot[c][4];
                        a.jerk[2 * ostride + slot] = tot[c][5];
                        if (a.pot) a.pot[slot] = tot[c][6];
                    } else if (!a.part_f32) {
                        double *p = a.part + (sp * 7) * n_i + slot;
#pragma unroll
                        for (int k = 0; k < 7; ++k) p[k * n_i] = tot[c][k];
                    } else {
                        float *p = (float *)a.part + (sp * 7) * n_i + slot;
#pragma unroll
                        for (int k = 0; k < 7; ++k) p[k * n_i] = (float)tot[c][k];
                    }
                }
            }
        }
        if (W > 1) __syncthreads();
    }
}

// Adds the S float64 partial sums of every output in a fixed order: the 64
// lanes of a wave take 64 consecutive outputs, the RW waves of a workgroup
// take contiguous eighths of the splits, and the wave sums are combined in
// wave order through LDS.  A lane issues its loads eight at a time and adds
// them in split order, so a small block (few outputs, many splits) waits for
// one memory latency per eight splits rather than per split.  At most four
// workgroups per CU loop over the outputs: when the block size is counted on
// the device the launch is sized for the largest block, and a grid that large
// spends several microseconds dispatching groups that find nothing to do.
__global__ __launch_bounds__(64 * RW) void reduce_parts_kernel(const KArgs a, int it, int waves) {
    __shared__ double red[RW][64];
    const int64_t n_i = block_size(a);
    if (n_i <= 0) return;
    const int64_t S = n_i <= a.jl_max
                          ? choose_splits_jl(n_i, a.n_j, a.jl_c, a.jl_waves, a.jl_tile,
                                             a.jl_min_j_wave, a.jl_target_groups, a.max_splits)
                          : choose_splits(n_i, a.n_j, it, waves, a.min_j_wave, a.target_groups,
                                          a.max_splits);
    if (S == 1) return;
    const int64_t ostride = a.out_stride > 0 ? a.out_stride : n_i;
    const int64_t total = 7 * n_i;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t per = (S + RW - 1) / RW;
    const int64_t p0 = wave * per, p1 = min(S, p0 + per);
    for (int64_t base = blockIdx.x * (int64_t)64; base < total; base += (int64_t)gridDim.x * 64) {
        const int64_t e = base + lane;
        double acc = 0.0;
        if (e < total) {
            const int64_t q = e / n_i, s = e - q * n_i;
            if (a.part_f32) {
                const float *src = (const float *)a.part + q * n_i + s;
                int64_t p = p0;
                for (; p + 8 <= p1; p += 8) {
                    float v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v[u] = src[(p + u) * 7 * n_i];
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc += (double)v[u];
                }
                for (; p < p1; ++p) acc += (double)src[p * 7 * n_i];
            } else {
                const double *src = a.part + q * n_i + s;
                int64_t p = p0;
                for (; p + 8 <= p1; p += 8) {
                    double v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v[u] = src[(p + u) * 7 * n_i];
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc += v[u];
                }
                for (; p < p1; ++p) acc += src[p * 7 * n_i];
            }
        }
        red[wave][lane] = acc;
        __syncthreads();
        if (wave == 0 && e < total) {
            double t = red[0][lane];
            for (int w = 1; w < RW; ++w) t += red[w][lane];
            const int64_t q = e / n_i, s = e - q * n_i;
            double *dst = q < 3 ? &a.acc[q * ostride + s]
                                : (q < 6 ? &a.jerk[(q - 3) * ostride + s] : a.pot ? &a.pot[s] : nullptr);
            if (dst) *dst = a.accumulate ? *dst + t : t;
        }
        __syncthreads();
    }
}

int launch_reduce_parts(nbody_ctx *ctx, const KArgs &a, int it, int waves, int64_t n_i_max) {
    int64_t blocks = (7 * n_i_max + 63) / 64;
    if (blocks > 4 * (int64_t)ctx->cus) blocks = 4 * (int64_t)ctx->cus;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)blocks), dim3(64 * RW), 0, ctx->stream,
                       a, it, waves);
    return hip_check(ctx, hipGetLastError(), "reduce_parts_kernel");
}

typedef void (*force_fn)(const KArgs);

template <int REP, int IT, int ACC>
static force_fn pick_w(int w) {
    switch (w) {
        case 1: return force_kernel<REP, IT, 1, ACC>;
        case 2: return force_kernel<REP, IT, 2, ACC>;
        case 4: return force_kernel<REP, IT, 4, ACC>;
        case 8: return force_kernel<REP, IT, 8, ACC>;
        default: return nullptr;
    }
}

template <int REP, int ACC>
static force_fn pick_w4(int w) {
    switch (w) {
        case 1: return force_kernel<REP, 4, 1, ACC>;
        case 2: return force_kernel<REP, 4, 2, ACC>;
        case 4: return force_kernel<REP, 4, 4, ACC>;
        default: return nullptr;
    }
}

template <int REP, int ACC>
static force_fn pick_it(int it, int w) {
    if (it == 1) return pick_w<REP, 1, ACC>(w);
    if (it == 2) return pick_w<REP, 2, ACC>(w);
    if (it == 4) return pick_w4<REP, ACC>(w);
    return nullptr;
}

static force_fn pick_kernel(const ForceShape &s, int acc) {
    if (acc == ACC_F64) {
        if (s.rep != REP_F64) return nullptr;
        if (s.it == 1) return pick_w<REP_F64, 1, ACC_F64>(s.waves);
        if (s.it == 2) return pick_w<REP_F64, 2, ACC_F64>(s.waves);
        return nullptr;
    }
    switch (s.rep) {
        case REP_F64: return pick_it<REP_F64, ACC_F32>(s.it, s.waves);
        case REP_FF: return pick_it<REP_FF, ACC_F32>(s.it, s.waves);
        case REP_F64V: return pick_it<REP_F64V, ACC_F32>(s.it, s.waves);
        default: return nullptr;
    }
}

template <int C, int ACC>
static force_fn pick_jl_w(int w) {
    switch (w) {
        case 1: return force_jl_kernel<C, 1, ACC>;
        case 2: return force_jl_kernel<C, 2, ACC>;
        case 4: return force_jl_kernel<C, 4, ACC>;
        default: return nullptr;
    }
}

static force_fn pick_jl_kernel(const ForceShape &s, int acc) {
    if (s.rep != REP_F64) return nullptr;
    if (acc == ACC_F64) {
        switch (s.it) {
            case 1: return pick_jl_w<1, ACC_F64>(s.waves);
            case 2: return pick_jl_w<2, ACC_F64>(s.waves);
            case 4: return pick_jl_w<4, ACC_F64>(s.waves);
            default: return nullptr;
        }
    }
    switch (s.it) {
        case 1: return pick_jl_w<1, ACC_F32>(s.waves);
        case 2: return pick_jl_w<2, ACC_F32>(s.waves);
        case 4: return pick_jl_w<4, ACC_F32>(s.waves);
        case 8: return pick_jl_w<8, ACC_F32>(s.waves);
        default: return nullptr;
    }
}

int acc_mode(uint32_t flags) { return (flags & NBODY_ACC_DS) ? ACC_F64 : ACC_F32; }

ForceShape shape_for(ForceShape s, int acc) {
    if (s.layout == 1) s.rep = REP_F64;  // the j-lane kernel reads float64 records
    if (acc == ACC_F64) {
        s.rep = REP_F64;
        if (s.it > (s.layout == 1 ? 4 : 2)) s.it = s.layout == 1 ? 4 : 2;
    }
    return s;
}

// Largest active block the built-in shapes give to the j-lane kernel.
constexpr int64_t kJlDefaultMax = 128;

// Built-in shape for an active block of about n_i particles against n_j,
// following what the autotuner and the block-step runs find on the MI355X:
// blocks below 256 keep one i per lane and four waves splitting j; larger
// blocks take two i per lane (two independent chains per lane hide the rsq
// and FMA latencies) and two waves.  The target of 128 groups per CU (32768
// in all) makes the j splits small enough for the groups resident on an
// XCD to share their j chunk in L2.  Up to n_j = 8192 a wave may take as
// few as n_j / 256 j (2 ... 16): a lone wave walking a long chain of scalar
// j loads is latency-bound, so small systems split j over more workgroups
// (13-28 % faster block steps at N = 256 ... 8192 with 16 j, another 6-19 %
// at N = 256 ... 2048 with 2-8 j); beyond, finer splits cost more in
// partial sums than they hide (64 j per wave).
static ForceShape default_shape(const nbody_ctx *ctx, int64_t n_i, int64_t n_j) {
    ForceShape s;
    if (n_i <= kJlDefaultMax && n_j > 8192) {
        // small blocks of large systems: one j per lane (2.5x faster than
        // one i per lane at n_i = 1 ... 64, N = 2^20; 2x at N = 65536)
        s.layout = 1;
        s.it = n_i <= 4 ? 1 : (n_i <= 16 ? 2 : 4);
        s.waves = 4;
        s.tile = 128;
        s.min_j_wave = 64;
        s.target_groups = 512;
        return s;
    }
    s.rep = REP_F64;
    s.it = n_i >= 256 ? 2 : 1;
    s.waves = n_i >= 1024 ? 2 : 4;
    s.tile = 128;
    s.min_j_wave = n_j <= 8192 ? (int)std::min<int64_t>(16, std::max<int64_t>(2, n_j / 256)) : 64;
    s.target_groups = 128 * ctx->cus;
    return s;
}

ForceShape pick_shape(const nbody_ctx *ctx, int64_t n_i, int64_t n_j) {
    for (const TuneEntry &e : ctx->tune)
        if (e.n_i_lo >= 0 && n_i >= e.n_i_lo && n_i < e.n_i_hi) return e.shape;
    return default_shape(ctx, n_i, n_j);
}

// Shape of the block-step launches, whose n_i is only known on the device:
// the tuned entry for them, else the built-in shape for a typical block of
// a system of n particles (about 0.1 n^0.9 at eta = 0.02).  For 8192 < n
// <= 131072 the block sizes of one run spread over orders of magnitude, and
// one i per lane and four waves while the typical block is below 2048
// (resp. 4096), with 64 groups per CU, measured 6-8 % faster steps at
// N = 16384 ... 65536 than the static rule (the same at 131072; slower at
// 8192 and below, which keep it, as do larger systems, not measured).
ForceShape dynamic_small_shape(const nbody_ctx *ctx, int64_t n, int64_t *jl_max) {
    (void)n;
    for (const TuneEntry &e : ctx->tune)
        if (e.n_i_lo == -2) {
            *jl_max = e.n_i_hi;
            return e.shape;
        }
    // systems above 8192 particles: blocks of up to kJlDefaultMax take the
    // j-lane kernel (below, a step is bound by launch latencies and the extra
    // launch would not pay)
    *jl_max = n > 8192 ? kJlDefaultMax : 0;
    ForceShape s;
    s.layout = 1;
    s.it = 2;
    s.waves = 4;
    s.tile = 128;
    s.min_j_wave = 64;
    s.target_groups = 512;
    return s;
}

ForceShape dynamic_shape(const nbody_ctx *ctx, int64_t n) {
    for (const TuneEntry &e : ctx->tune)
        if (e.n_i_lo == -1) return e.shape;
    const int64_t typ = (int64_t)(0.1 * std::pow((double)n, 0.9));
    ForceShape s = default_shape(ctx, typ, n);
    if (n > 8192 && n <= 131072) {
        s.it = typ >= 2048 ? 2 : 1;
        s.waves = typ < 4096 ? 4 : 2;
        s.target_groups = 64 * ctx->cus;
    }
    return s;
}

// Upper bound of (i-blocks x splits) of the i-lane kernel over every block
// size up to n_i_max, so that each item gets its own workgroup (dispatch
// order = item order, which keeps the concurrently running groups on one or
// two j chunks).
static int64_t il_items_bound(const ForceShape &sh, int64_t n_i_max, int64_t n_j,
                              int max_splits) {
    const int64_t bi = 64 * sh.it;
    const int64_t nb_max = (n_i_max + bi - 1) / bi;
    int64_t smax = n_j / ((int64_t)sh.waves * sh.min_j_wave);
    if (smax > max_splits) smax = max_splits;
    if (smax < 1) smax = 1;
    const int64_t tg = sh.target_groups;
    int64_t a1 = (tg + smax - 1) / smax;  // below this nb, S = smax
    if (a1 > nb_max) a1 = nb_max;
    int64_t items = a1 * smax;
    int64_t b2 = tg + nb_max;  // nb * ceil(tg / nb) < tg + nb
    if (b2 > nb_max * smax) b2 = nb_max * smax;
    if (b2 > items) items = b2;
    if (nb_max > items) items = nb_max;
    return items;
}

// The same for the j-lane kernel: nb * S <= tg + nb * s_lo and <= nb * smax.
static int64_t jl_items_bound(const ForceShape &sh, int64_t n_i_max, int64_t n_j,
                              int max_splits) {
    const int64_t nb_max = (n_i_max + sh.it - 1) / sh.it;
    const int64_t per_split = (int64_t)sh.waves * 64 * sh.tile;
    const int64_t s_lo = (n_j + per_split - 1) / per_split;
    int64_t smax = n_j / ((int64_t)sh.waves * sh.min_j_wave);
    if (smax > max_splits) smax = max_splits;
    if (smax < 1) smax = 1;
    int64_t items = (int64_t)sh.target_groups + nb_max * s_lo;
    if (items > nb_max * smax) items = nb_max * smax;
    if (items < nb_max) items = nb_max;
    return items;
}

int launch_force(nbody_ctx *ctx, const ForceCall &c) {
    const bool dev_count = c.n_i_dev != nullptr;
    const int64_t n_i_max = dev_count ? c.n_i_cap : c.n_i;
    if (n_i_max <= 0) return NBODY_OK;
    // Kernels: the shape's layout; a device-counted launch with jl_max > 0
    // runs the j-lane kernel on blocks of up to jl_max particles and the
    // i-lane kernel on larger ones (each returns early on the other's).
    ForceShape il = c.shape, jl = c.shape;
    bool use_il = true, use_jl = false;
    int64_t jl_max = 0;
    if (c.shape.layout == 1) {
        use_il = false;
        use_jl = true;
        jl_max = INT64_MAX;
    } else if (dev_count && c.jl_max > 0) {
        use_jl = true;
        jl = c.jl_shape;
        jl_max = std::min(c.jl_max, n_i_max);
    }
    force_fn fil = use_il ? pick_kernel(il, c.mode) : nullptr;
    force_fn fjl = use_jl ? pick_jl_kernel(jl, c.mode) : nullptr;
    if ((use_il && !fil) || (use_jl && !fjl))
        return fail(ctx, NBODY_E_INVAL, "no pair kernel for layout=%d rep=%d it=%d waves=%d acc=%d",
                    use_jl && !fjl ? jl.layout : il.layout, use_jl && !fjl ? jl.rep : il.rep,
                    use_jl && !fjl ? jl.it : il.it, use_jl && !fjl ? jl.waves : il.waves, c.mode);

    KArgs a;
    a.jrec = c.jrec;
    a.pos = c.pos;
    a.vel = c.vel;
    a.active = c.active;
    a.n_i_dev = c.n_i_dev;
    a.acc = c.acc;
    a.jerk = c.jerk;
    a.pot = c.pot;
    a.part = nullptr;
    a.status = &ctx->info->status;
    a.n_i = dev_count ? n_i_max : c.n_i;  // (the capacity when counted on the device)
    a.out_stride = c.out_stride;
    a.n_j = (int32_t)c.n_j;
    a.eps2 = (float)c.eps2;
    a.eps2d = c.eps2;
    a.tile = il.tile;
    a.min_j_wave = il.min_j_wave;
    a.target_groups = il.target_groups;
    a.max_splits = c.max_splits > 0 && c.max_splits < kMaxSplits ? c.max_splits : kMaxSplits;
    a.accumulate = 0;
    a.part_f32 = c.mode == ACC_F32 ? 1 : 0;
    a.jl_max = jl_max;
    a.jl_c = jl.it;
    a.jl_waves = jl.waves;
    a.jl_tile = jl.tile;
    a.jl_min_j_wave = jl.min_j_wave;
    a.jl_target_groups = jl.target_groups;
    const int64_t part_elem = a.part_f32 ? (int64_t)sizeof(float) : (int64_t)sizeof(double);

    // Grids and partial-sum scratch (S * 7 * n_i values: float32 in the
    // float32 mode, float64 otherwise).
    int64_t items_il = 0, items_jl = 0, need_part = 0;
    if (use_il) {
        const int64_t bi = 64 * il.it;
        if (dev_count) {
            items_il = il_items_bound(il, n_i_max, c.n_j, a.max_splits);
            // S * n_i <= S * nb * bi <= items * bi, and <= 2 * target_groups *
            // bi (S > 1 only while nb < target_groups)
            const int64_t rows = std::min<int64_t>(2 * (int64_t)il.target_groups, items_il) * bi;
            need_part = std::max(need_part, rows * 7 * part_elem);
        } else {
            const int64_t S = choose_splits(c.n_i, c.n_j, il.it, il.waves, il.min_j_wave,
                                            il.target_groups, a.max_splits);
            items_il = ((c.n_i + bi - 1) / bi) * S;
            if (S > 1) need_part = std::max(need_part, S * 7 * c.n_i * part_elem);
        }
    }
    if (use_jl) {
        if (dev_count) {
            const int64_t cap = std::min<int64_t>(jl_max, n_i_max);
            items_jl = jl_items_bound(jl, cap, c.n_j, a.max_splits);
            // S * n_i <= S * nb * C = items * C
            need_part = std::max(need_part, items_jl * jl.it * 7 * part_elem);
        } else {
            const int64_t S = choose_splits_jl(c.n_i, c.n_j, jl.it, jl.waves, jl.tile,
                                               jl.min_j_wave, jl.target_groups, a.max_splits);
            items_jl = ((c.n_i + jl.it - 1) / jl.it) * S;
            if (S > 1) need_part = std::max(need_part, S * 7 * c.n_i * part_elem);
        }
    }
    items_il = std::min<int64_t>(items_il, 1 << 24);
    items_jl = std::min<int64_t>(items_jl, 1 << 24);
    const bool prof = ctx->prof.on && !c.part_buf;
    if (need_part > 0) {
        if (c.part_buf) {
            if ((size_t)need_part > c.part_cap)
                return fail(ctx, NBODY_E_INVAL, "partial sums need %lld bytes, %zu available",
                            (long long)need_part, c.part_cap);
            a.part = (double *)c.part_buf;
        } else {
            NB_TRY(ensure(ctx, &ctx->part, &ctx->part_bytes, (size_t)need_part));
            a.part = (double *)ctx->part;
        }
    }
    hipEvent_t e0 = prof ? prof_mark(ctx) : nullptr;
    if (use_jl) {
        hipLaunchKernelGGL(fjl, dim3((unsigned)items_jl), dim3(64 * jl.waves), 0, ctx->stream, a);
        NB_TRY(hip_check(ctx, hipGetLastError(), "force_jl_kernel"));
    }
    if (use_il) {
        hipLaunchKernelGGL(fil, dim3((unsigned)items_il), dim3(64 * il.waves), 0, ctx->stream, a);
        NB_TRY(hip_check(ctx, hipGetLastError(), "force_kernel"));
    }
    if (prof) prof_push(ctx, e0, prof_mark(ctx), 0);
    if (need_part > 0) {
        hipEvent_t r0 = prof ? prof_mark(ctx) : nullptr;
        NB_TRY(launch_reduce_parts(ctx, a, il.it, il.waves, n_i_max));
        if (prof) prof_push(ctx, r0, prof_mark(ctx), 1);
    }
    return NBODY_OK;
}

}  // namespace nb

using namespace nb;

extern "C" int nbody_force(nbody_ctx *ctx, const int32_t *active_idx, int64_t n_i,
                           const double *pos, const double *vel, const double *mass,
                           int64_t n_j, double eps2, double *acc, double *jerk, double *pot,
                           uint32_t flags) {
    if (!ctx) return NBODY_E_INVAL;
    if (n_i < 0 || n_j < 1 || n_i > 0x7fffffffLL || n_j > 0x7fffffffLL)
        return fail(ctx, NBODY_E_INVAL, "nbody_force: bad sizes n_i=%lld n_j=%lld",
                    (long long)n_i, (long long)n_j);
    if (!(eps2 >= 0.0) || std::isinf(eps2))
        return fail(ctx, NBODY_E_INVAL, "nbody_force: eps2 must be finite and >= 0");
    if (flags & ~NBODY_ACC_DS) return fail(ctx, NBODY_E_INVAL, "nbody_force: unknown flags");
    if (!pos || !vel || !mass || (n_i > 0 && (!acc || !jerk)))
        return fail(ctx, NBODY_E_INVAL, "nbody_force: null array");
    if (n_i == 0) return NBODY_OK;
    NB_TRY(activate(ctx));
    ForceCall c;
    c.mode = acc_mode(flags);
    c.shape = shape_for(pick_shape(ctx, n_i, n_j), c.mode);
    NB_TRY(ensure(ctx, &ctx->jrec, &ctx->jrec_bytes, (size_t)n_j * sizeof(JRec)));
    NB_TRY(launch_pack(ctx, c.shape.rep, n_j, pos, vel, mass, (JRec *)ctx->jrec));
    c.jrec = (const JRec *)ctx->jrec;
    c.n_j = n_j;
    c.pos = pos;
    c.vel = vel;
    c.active = active_idx;
    c.n_i = n_i;
    c.eps2 = eps2;
    c.acc = acc;
    c.jerk = jerk;
    c.pot = pot;
    c.out_stride = n_i;
    return launch_force(ctx, c);
}

extern "C" int nbody_force_dev(nbody_ctx *ctx, const int32_t *active_idx, const int64_t *n_i_dev,
                               int64_t n_i_cap, const double *pos, const double *vel,
                               const double *mass, int64_t n_j, double eps2, double *acc,
                               double *jerk, double *pot, uint32_t flags) {
    if (!ctx) return NBODY_E_INVAL;
    if (n_i_cap < 0 || n_j < 1 || n_i_cap > 0x7fffffffLL || n_j > 0x7fffffffLL ||
        (!active_idx && n_i_cap > n_j))
        return fail(ctx, NBODY_E_INVAL, "nbody_force_dev: bad sizes n_i_cap=%lld n_j=%lld",
                    (long long)n_i_cap, (long long)n_j);
    if (!(eps2 >= 0.0) || std::isinf(eps2))
        return fail(ctx, NBODY_E_INVAL, "nbody_force_dev: eps2 must be finite and >= 0");
    if (flags & ~NBODY_ACC_DS) return fail(ctx, NBODY_E_INVAL, "nbody_force_dev: unknown flags");
    if (!n_i_dev || !pos || !vel || !mass || (n_i_cap > 0 && (!acc || !jerk)))
        return fail(ctx, NBODY_E_INVAL, "nbody_force_dev: null array");
    if (n_i_cap == 0) return NBODY_OK;
    NB_TRY(activate(ctx));
    // the block-step driver's launch: shapes for a block size known only on
    // the device
    ForceCall c;
    c.mode = acc_mode(flags);
    c.shape = shape_for(dynamic_shape(ctx, n_j), c.mode);
    c.jl_shape = shape_for(dynamic_small_shape(ctx, n_j, &c.jl_max), c.mode);
    if (c.shape.rep != REP_F64) c.jl_max = 0;
    NB_TRY(ensure(ctx, &ctx->jrec, &ctx->jrec_bytes, (size_t)n_j * sizeof(JRec)));
    NB_TRY(launch_pack(ctx, c.shape.rep, n_j, pos, vel, mass, (JRec *)ctx->jrec));
    c.jrec = (const JRec *)ctx->jrec;
    c.n_j = n_j;
    c.pos = pos;
    c.vel = vel;
    c.active = active_idx;
    c.n_i_dev = n_i_dev;
    c.n_i_cap = n_i_cap;
    c.eps2 = eps2;
    c.acc = acc;
    c.jerk = jerk;
    c.pot = pot;
    c.out_stride = n_i_cap;
    return launch_force(ctx, c);
}
