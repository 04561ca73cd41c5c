// Adjoint of the pair sums and of the shared-step Hermite chain.
//
// The paper has no adjoint; this is the transpose of the force law of the
// Appendix A listing (Section 2, Eq. (1), softened).  For cotangents
// (abar_i, kbar_i, pbar_i) of (a_i, k_i, phi_i) and a pair (i, j) with
// r = x_j - x_i, w = v_j - v_i, s = r.r + eps^2, q = r.w, al = s^(-3/2),
// be = s^(-5/2), ga = s^(-7/2):
//   g_r(i,j) = m_j [al abar_i - 3 q be kbar_i - 3 be (kbar_i.r) w
//                   + (pbar_i al - 3 be (abar_i.r + kbar_i.w) + 15 q ga (kbar_i.r)) r]
//   g_v(i,j) = m_j [al kbar_i - 3 be (kbar_i.r) r]
//   g_m(i,j) = al (abar_i.r + kbar_i.w) - 3 q be (kbar_i.r) - pbar_i s^(-1/2)
// and xbar_j += g_r, xbar_i -= g_r, vbar_j += g_v, vbar_i -= g_v,
// mbar_j += g_m.  A lane owns particle p and sums, over every other q, both
// its role as the receiver i (-g(p,q)) and as the source j (+g(q,p)); the
// two share the pair geometry, so one pass over q gives xbar_p, vbar_p and
// mbar_p with no atomics.  The pair arithmetic is float32 on float64-formed
// relative coordinates; sums are two-level float32 or compensated, and the
// work decomposition (waves and workgroups splitting q, float64 partials
// reduced in a fixed order) is the one of the forward pair kernel.
#include <cmath>

#include "common.hpp"
#include "pairs.hpp"

namespace nb {

// Source record of the adjoint pass (128 bytes, two scalar cache lines).
struct __attribute__((aligned(128))) AdjRec {
    double x, y, z, u, v, w;
    float m, ax, ay, az, kx, ky, kz, ph;
    float pad[12];
};
static_assert(sizeof(AdjRec) == 128, "AdjRec is two 64-byte lines");

__global__ void adj_pack_kernel(int64_t n, const double *__restrict__ pos,
                                const double *__restrict__ vel, const double *__restrict__ mass,
                                const double *__restrict__ ab, const double *__restrict__ kb,
                                const double *__restrict__ pb, AdjRec *__restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    AdjRec r;
    r.x = pos[i];
    r.y = pos[n + i];
    r.z = pos[2 * n + i];
    r.u = vel[i];
    r.v = vel[n + i];
    r.w = vel[2 * n + i];
    r.m = (float)mass[i];
    r.ax = (float)ab[i];
    r.ay = (float)ab[n + i];
    r.az = (float)ab[2 * n + i];
    r.kx = (float)kb[i];
    r.ky = (float)kb[n + i];
    r.kz = (float)kb[2 * n + i];
    r.ph = pb ? (float)pb[i] : 0.0f;
    for (int q = 0; q < 12; ++q) r.pad[q] = 0.0f;
    out[i] = r;
}

struct AdjCot {
    float m, ax, ay, az, kx, ky, kz, ph;
};

template <int W, bool DS>
__global__ __launch_bounds__(64 * W) void force_adjoint_kernel(const KArgs a,
                                                               const AdjRec *__restrict__ rec) {
    const int64_t n = a.n_i;
    const int n_j = a.n_j;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nb = (n + 63) / 64;
    const int64_t S = choose_splits(n, n_j, 1, W, a.min_j_wave, a.target_groups, a.max_splits);
    const int64_t items = nb * S;
    const int64_t jchunk = (n_j + S - 1) / S;
    const float eps2 = a.eps2;
    const int tile = a.tile;
    const CONSTP(AdjRec) R = (CONSTP(AdjRec))rec;

    __shared__ double red[W > 1 ? W - 1 : 1][7][64];

    for (int64_t q = blockIdx.x; q < items; q += gridDim.x) {
        const int64_t item = xcd_item(q, items);
        const int64_t ib = item % nb;
        const int64_t sp = item / nb;
        const int j0 = (int)(sp * jchunk);
        const int j1 = (int)min((int64_t)n_j, (int64_t)j0 + jchunk);
        const int jw = (j1 - j0 + W - 1) / W;
        const int jb = __builtin_amdgcn_readfirstlane(min(j1, j0 + wave * jw));
        const int je = __builtin_amdgcn_readfirstlane(min(j1, jb + jw));

        const int64_t slot = ib * 64 + lane;
        const int p = (int)(slot < n ? slot : n - 1);
        const double px = rec[p].x, py = rec[p].y, pz = rec[p].z;
        const double pu = rec[p].u, pv = rec[p].v, pw = rec[p].w;
        const AdjCot own{rec[p].m, rec[p].ax, rec[p].ay, rec[p].az,
                         rec[p].kx, rec[p].ky, rec[p].kz, rec[p].ph};
        const int lo_idx = __builtin_amdgcn_readfirstlane(wave_min(p));
        const int hi_idx = __builtin_amdgcn_readfirstlane(wave_max(p));

        float s_hi[7], s_lo[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) s_hi[c] = s_lo[c] = 0.0f;

        for (int jt = jb; jt < je; jt += tile) {
            const int jend = min(je, jt + tile);
            float in[7];
#pragma unroll
            for (int c = 0; c < 7; ++c) in[c] = 0.0f;
            for (int q = jt; q < jend; ++q) {
                const float rx = (float)(R[q].x - px);
                const float ry = (float)(R[q].y - py);
                const float rz = (float)(R[q].z - pz);
                const float wx = (float)(R[q].u - pu);
                const float wy = (float)(R[q].v - pv);
                const float wz = (float)(R[q].w - pw);
                const AdjCot o{R[q].m, R[q].ax, R[q].ay, R[q].az,
                               R[q].kx, R[q].ky, R[q].kz, R[q].ph};
                float s2 = fmaf(rz, rz, fmaf(ry, ry, fmaf(rx, rx, eps2)));
                float live = 1.0f;
                if (q >= lo_idx && q <= hi_idx && q == p) {
                    s2 = 1.0f;
                    live = 0.0f;
                }
                const float rinv = __builtin_amdgcn_rsqf(s2);
                const float rinv2 = rinv * rinv;
                const float al = rinv * rinv2 * live;
                const float be = al * rinv2;
                const float ga = be * rinv2;
                const float qv = rx * wx + ry * wy + rz * wz;
                // own (receiver) and other (source) projections
                const float ar_p = own.ax * rx + own.ay * ry + own.az * rz;
                const float kr_p = own.kx * rx + own.ky * ry + own.kz * rz;
                const float kw_p = own.kx * wx + own.ky * wy + own.kz * wz;
                const float ar_q = o.ax * rx + o.ay * ry + o.az * rz;
                const float kr_q = o.kx * rx + o.ky * ry + o.kz * rz;
                const float kw_q = o.kx * wx + o.ky * wy + o.kz * wz;
                // -g(p,q) with factor m_q, and +g(q,p) with factor m_p: the
                // source's geometry is (-r, -w), same s and q
                const float cp = own.ph * al - 3.0f * be * (ar_p + kw_p) + 15.0f * qv * ga * kr_p;
                const float cq = o.ph * al + 3.0f * be * (ar_q + kw_q) - 15.0f * qv * ga * kr_q;
                const float mp = own.m, mq = o.m;
                const float t_a_x = mp * o.ax - mq * own.ax;
                const float t_a_y = mp * o.ay - mq * own.ay;
                const float t_a_z = mp * o.az - mq * own.az;
                const float t_k_x = mp * o.kx - mq * own.kx;
                const float t_k_y = mp * o.ky - mq * own.ky;
                const float t_k_z = mp * o.kz - mq * own.kz;
                const float t_kr = mp * kr_q - mq * kr_p;
                const float t_c = mp * cq + mq * cp;
                const float b3q = 3.0f * qv * be;
                const float b3 = 3.0f * be;
                in[0] += al * t_a_x - b3q * t_k_x - b3 * t_kr * wx - t_c * rx;
                in[1] += al * t_a_y - b3q * t_k_y - b3 * t_kr * wy - t_c * ry;
                in[2] += al * t_a_z - b3q * t_k_z - b3 * t_kr * wz - t_c * rz;
                in[3] += al * t_k_x - b3 * t_kr * rx;
                in[4] += al * t_k_y - b3 * t_kr * ry;
                in[5] += al * t_k_z - b3 * t_kr * rz;
                in[6] += -al * (ar_q + kw_q) + b3q * kr_q - o.ph * rinv * live;
            }
#pragma unroll
            for (int c = 0; c < 7; ++c) {
                if (DS)
                    two_sum_acc(s_hi[c], s_lo[c], in[c]);
                else
                    s_hi[c] += in[c];
            }
        }

        double tot[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) tot[c] = (double)s_hi[c] + (double)s_lo[c];
        if (W > 1) {
            if (wave > 0) {
#pragma unroll
                for (int c = 0; c < 7; ++c) red[wave - 1][c][lane] = tot[c];
            }
            __syncthreads();
            if (wave == 0)
                for (int w = 1; w < W; ++w)
#pragma unroll
                    for (int c = 0; c < 7; ++c) tot[c] += red[w - 1][c][lane];
        }
        if (wave == 0 && slot < n) {
            if (S == 1) {
                double *dst[7] = {&a.acc[slot],  &a.acc[n + slot],  &a.acc[2 * n + slot],
                                  &a.jerk[slot], &a.jerk[n + slot], &a.jerk[2 * n + slot],
                                  &a.pot[slot]};
#pragma unroll
                for (int c = 0; c < 7; ++c) *dst[c] = a.accumulate ? *dst[c] + tot[c] : tot[c];
            } else {
                double *dst = a.part + (sp * 7) * n + slot;
#pragma unroll
                for (int c = 0; c < 7; ++c) dst[c * n] = tot[c];
            }
        }
        if (W > 1) __syncthreads();
    }
}

// Predictor transpose (shared step h), accumulating:
//   xbar += xpbar,  vbar += h xpbar + vpbar,
//   abar += (h^2/2) xpbar + h vpbar,  kbar += (h^3/6) xpbar + (h^2/2) vpbar.
__global__ void predict_adjoint_kernel(int64_t m3, double h, const double *__restrict__ xpb,
                                       const double *__restrict__ vpb, double *__restrict__ xb,
                                       double *__restrict__ vb, double *__restrict__ ab,
                                       double *__restrict__ kb) {
    const double h2 = h * h / 2.0, h3 = h * h * h / 6.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m3;
         e += (int64_t)gridDim.x * blockDim.x) {
        const double x = xpb[e], v = vpb[e];
        xb[e] += x;
        vb[e] += h * x + v;
        ab[e] += h2 * x + h * v;
        kb[e] += h3 * x + h2 * v;
    }
}

// Corrector transpose (shared step h).  Expanding the corrector's a2, a3
// makes it linear:
//   x1 = xp - (3/20) h^2 (a0 - a1) - h^3 (7 k0/60 + k1/30)
//   v1 = vp - (h/2) (a0 - a1)       - h^2 (5 k0/12 + k1/12)
// so, accumulating: xpbar += x1bar, vpbar += v1bar,
//   a0bar += -(3/20) h^2 x1bar - (h/2) v1bar,  a1bar += -(that),
//   k0bar += -(7/60) h^3 x1bar - (5/12) h^2 v1bar,
//   k1bar += -(1/30) h^3 x1bar - (1/12) h^2 v1bar.
__global__ void correct_adjoint_kernel(int64_t m3, double h, const double *__restrict__ x1b,
                                       const double *__restrict__ v1b, double *__restrict__ xpb,
                                       double *__restrict__ vpb, double *__restrict__ a0b,
                                       double *__restrict__ k0b, double *__restrict__ a1b,
                                       double *__restrict__ k1b) {
    const double ca = 0.15 * h * h, cv = 0.5 * h;
    const double k0x = 7.0 / 60.0 * h * h * h, k0v = 5.0 / 12.0 * h * h;
    const double k1x = 1.0 / 30.0 * h * h * h, k1v = 1.0 / 12.0 * h * h;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m3;
         e += (int64_t)gridDim.x * blockDim.x) {
        const double x = x1b[e], v = v1b[e];
        const double ga = ca * x + cv * v;
        xpb[e] += x;
        vpb[e] += v;
        a0b[e] -= ga;
        a1b[e] += ga;
        k0b[e] -= k0x * x + k0v * v;
        k1b[e] -= k1x * x + k1v * v;
    }
}

}  // namespace nb

using namespace nb;

extern "C" {

int nbody_force_adjoint(nbody_ctx *ctx, int64_t n, const double *pos, const double *vel,
                        const double *mass, double eps2, const double *acc_bar,
                        const double *jerk_bar, const double *pot_bar, double *pos_bar,
                        double *vel_bar, double *mass_bar, uint32_t flags) {
    if (!ctx) return NBODY_E_INVAL;
    if (n < 1 || n > 0x7fffffffLL || !(eps2 >= 0.0) || std::isinf(eps2))
        return fail(ctx, NBODY_E_INVAL, "nbody_force_adjoint: bad arguments");
    if (flags & ~(NBODY_ACC_DS | NBODY_ADJ_ACCUMULATE))
        return fail(ctx, NBODY_E_INVAL, "nbody_force_adjoint: unknown flags");
    if (!pos || !vel || !mass || !acc_bar || !jerk_bar || !pos_bar || !vel_bar || !mass_bar)
        return fail(ctx, NBODY_E_INVAL, "nbody_force_adjoint: null array");
    NB_TRY(activate(ctx));
    NB_TRY(ensure(ctx, &ctx->adj, &ctx->adj_bytes, (size_t)n * sizeof(AdjRec)));
    AdjRec *rec = (AdjRec *)ctx->adj;
    adj_pack_kernel<<<(unsigned)((n + 255) / 256), 256, 0, ctx->stream>>>(
        n, pos, vel, mass, acc_bar, jerk_bar, pot_bar, rec);
    NB_TRY(hip_check(ctx, hipGetLastError(), "adj_pack_kernel"));

    const int W = 4;
    KArgs a = {};
    a.acc = pos_bar;
    a.jerk = vel_bar;
    a.pot = mass_bar;
    a.status = &ctx->info->status;
    a.n_i = n;
    a.out_stride = n;
    a.n_j = (int32_t)n;
    a.eps2 = (float)eps2;
    a.tile = 128;
    a.min_j_wave = 64;
    a.target_groups = 8 * ctx->cus;
    a.max_splits = kMaxSplits;
    a.accumulate = (flags & NBODY_ADJ_ACCUMULATE) ? 1 : 0;
    const int64_t S = choose_splits(n, n, 1, W, a.min_j_wave, a.target_groups, a.max_splits);
    const int64_t nb = (n + 63) / 64;
    if (S > 1) {
        NB_TRY(ensure(ctx, &ctx->part, &ctx->part_bytes, (size_t)S * 7 * n * sizeof(double)));
        a.part = (double *)ctx->part;
    }
    const bool ds = (flags & NBODY_ACC_DS) != 0;
    if (ds)
        force_adjoint_kernel<W, true><<<(unsigned)(nb * S), 64 * W, 0, ctx->stream>>>(a, rec);
    else
        force_adjoint_kernel<W, false><<<(unsigned)(nb * S), 64 * W, 0, ctx->stream>>>(a, rec);
    NB_TRY(hip_check(ctx, hipGetLastError(), "force_adjoint_kernel"));
    if (S > 1) NB_TRY(launch_reduce_parts(ctx, a, 1, W, n));
    return NBODY_OK;
}

int nbody_predict_adjoint(nbody_ctx *ctx, int64_t n, double h, const double *xp_bar,
                          const double *vp_bar, double *x_bar, double *v_bar, double *a_bar,
                          double *k_bar) {
    if (!ctx) return NBODY_E_INVAL;
    if (n < 0 || !std::isfinite(h)) return fail(ctx, NBODY_E_INVAL, "nbody_predict_adjoint: bad args");
    if (n == 0) return NBODY_OK;
    if (!xp_bar || !vp_bar || !x_bar || !v_bar || !a_bar || !k_bar)
        return fail(ctx, NBODY_E_INVAL, "nbody_predict_adjoint: null array");
    NB_TRY(activate(ctx));
    const int64_t m3 = 3 * n;
    int64_t g = (m3 + 255) / 256;
    if (g > 16 * (int64_t)ctx->cus) g = 16 * (int64_t)ctx->cus;
    predict_adjoint_kernel<<<(unsigned)g, 256, 0, ctx->stream>>>(m3, h, xp_bar, vp_bar, x_bar,
                                                                 v_bar, a_bar, k_bar);
    return hip_check(ctx, hipGetLastError(), "predict_adjoint_kernel");
}

int nbody_correct_adjoint(nbody_ctx *ctx, int64_t n, double h, const double *x1_bar,
                          const double *v1_bar, double *xp_bar, double *vp_bar, double *a0_bar,
                          double *k0_bar, double *a1_bar, double *k1_bar) {
    if (!ctx) return NBODY_E_INVAL;
    if (n < 0 || !std::isfinite(h)) return fail(ctx, NBODY_E_INVAL, "nbody_correct_adjoint: bad args");
    if (n == 0) return NBODY_OK;
    if (!x1_bar || !v1_bar || !xp_bar || !vp_bar || !a0_bar || !k0_bar || !a1_bar || !k1_bar)
        return fail(ctx, NBODY_E_INVAL, "nbody_correct_adjoint: null array");
    NB_TRY(activate(ctx));
    const int64_t m3 = 3 * n;
    int64_t g = (m3 + 255) / 256;
    if (g > 16 * (int64_t)ctx->cus) g = 16 * (int64_t)ctx->cus;
    correct_adjoint_kernel<<<(unsigned)g, 256, 0, ctx->stream>>>(m3, h, x1_bar, v1_bar, xp_bar,
                                                                 vp_bar, a0_bar, k0_bar, a1_bar,
                                                                 k1_bar);
    return hip_check(ctx, hipGetLastError(), "correct_adjoint_kernel");
}

}  // extern "C"
