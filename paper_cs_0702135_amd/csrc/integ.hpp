// Per-particle float64 Hermite arithmetic shared by the standalone kernels
// and the ensemble kernel (Section 2).  Compiled without contraction so the
// results follow the printed formulas operation by operation.
#pragma once

#include "common.hpp"

namespace nb {

// Predictor from values: h = t_target - t_i.
__device__ __forceinline__ void predict_vals(double h, const double x[3], const double v[3],
                                             const double a[3], const double k[3], double px[3],
                                             double pv[3]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        px[c] = x[c] + (v[c] + (h / 2.0) * (a[c] + (h / 3.0) * k[c])) * h;
        pv[c] = v[c] + (a[c] + (h / 2.0) * k[c]) * h;
    }
}

// Predictor: h = t_target - t_i; q points at component 0, stride cs.
__device__ __forceinline__ void predict_one(double h, const double *x, const double *v,
                                            const double *a, const double *k, int64_t q,
                                            int64_t cs, double px[3], double pv[3]) {
    double xs[3], vs[3], as[3], ks[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t e = q + c * cs;
        xs[c] = x[e];
        vs[c] = v[e];
        as[c] = a[e];
        ks[c] = k[e];
    }
    predict_vals(h, xs, vs, as, ks, px, pv);
}

// Corrector and new step of one particle.  xp, vp: its predicted position
// and velocity; a1, k1: the new force and jerk.  State arrays at element q
// (component stride cs); returns status bits.  If t_next is given it
// receives the particle's new t + dt.
__device__ __forceinline__ int32_t correct_vals(int64_t q, int64_t cs, const double xp[3],
                                                const double vp[3], const double a1v[3],
                                                const double k1v[3], double eta, double dt_max,
                                                double dt_min, int fixed_dt, double *t,
                                                double *dtv, double *x, double *v, double *a,
                                                double *k, double *t_next = nullptr) {
#pragma clang fp contract(off)
    int32_t st = 0;
    const double h = dtv[q];
    const double t_new = t[q] + h;
    double a2v[3], a3v[3];
    bool bad = false;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t e = q + c * cs;
        const double a0 = a[e], k0 = k[e];
        const double a1 = a1v[c], k1 = k1v[c];
        const double A3 = 2.0 * (a0 - a1) + (k0 + k1) * h;
        const double A2 = -3.0 * (a0 - a1) - (2.0 * k0 + k1) * h;
        const double xn = xp[c] + (A2 / 12.0 + A3 / 20.0) * h * h;
        const double vn = vp[c] + (A2 / 3.0 + A3 / 4.0) * h;
        x[e] = xn;
        v[e] = vn;
        a[e] = a1;
        k[e] = k1;
        a2v[c] = (2.0 * A2 + 6.0 * A3) / (h * h);
        a3v[c] = 6.0 * A3 / (h * h * h);
        bad = bad || !isfinite(xn) || !isfinite(vn) || !isfinite(a1) || !isfinite(k1);
    }
    t[q] = t_new;
    // a non-finite corrected state is reported and keeps its step
    if (bad) st |= ST_NONFINITE;
    if (!fixed_dt) {
        const double an = sqrt(a1v[0] * a1v[0] + a1v[1] * a1v[1] + a1v[2] * a1v[2]);
        const double kn = sqrt(k1v[0] * k1v[0] + k1v[1] * k1v[1] + k1v[2] * k1v[2]);
        const double a2n = sqrt(a2v[0] * a2v[0] + a2v[1] * a2v[1] + a2v[2] * a2v[2]);
        const double a3n = sqrt(a3v[0] * a3v[0] + a3v[1] * a3v[1] + a3v[2] * a3v[2]);
        const double num = eta * (an * a2n + kn * kn);
        const double den = kn * a3n + a2n * a2n;
        double crit = den > 0.0 ? sqrt(num / den) : INFINITY;
        double d = h;
        if (bad || !(crit == crit)) {
            st |= ST_NONFINITE;
            crit = d;
        }
        if (d > crit) {
            while (d > crit) d = d / 2.0;
        } else if (2.0 * d <= crit && fmod(t_new, 2.0 * d) == 0.0 && 2.0 * d <= dt_max) {
            d = 2.0 * d;
        }
        if (d < dt_min) {
            st |= ST_RANGE;
            d = dt_min;
        }
        dtv[q] = d;
        if (t_next) *t_next = t_new + d;
    } else if (t_next) {
        *t_next = t_new + h;
    }
    return st;
}

// Corrector reading the predicted state from arrays (element q, stride cs).
__device__ __forceinline__ int32_t correct_one(int64_t q, int64_t cs, const double *xp,
                                               const double *vp, const double a1v[3],
                                               const double k1v[3], double eta, double dt_max,
                                               double dt_min, int fixed_dt, double *t,
                                               double *dtv, double *x, double *v, double *a,
                                               double *k) {
    double px[3], pv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        px[c] = xp[q + c * cs];
        pv[c] = vp[q + c * cs];
    }
    return correct_vals(q, cs, px, pv, a1v, k1v, eta, dt_max, dt_min, fixed_dt, t, dtv, x, v, a,
                        k);
}

// Initial step of one particle (a, k at element q, stride cs).
__device__ __forceinline__ double initial_dt_one(int64_t q, int64_t cs, double t0,
                                                 const double *a, const double *k, double eta_s,
                                                 double dt_max, double dt_min, int32_t *st) {
#pragma clang fp contract(off)
    const double ax = a[q], ay = a[q + cs], az = a[q + 2 * cs];
    const double kx = k[q], ky = k[q + cs], kz = k[q + 2 * cs];
    const double an = sqrt(ax * ax + ay * ay + az * az);
    const double kn = sqrt(kx * kx + ky * ky + kz * kz);
    double want = kn > 0.0 ? eta_s * an / kn : dt_max;
    // a non-finite norm carries no step information
    if (!(want == want) || !isfinite(an) || !isfinite(kn)) {
        *st |= ST_NONFINITE;
        want = dt_min;
    }
    double d = dt_max;
    while (d > want && d >= 2.0 * dt_min) d = d / 2.0;
    while (fmod(t0, d) != 0.0 && d >= 2.0 * dt_min) d = d / 2.0;
    if (d > want || fmod(t0, d) != 0.0) *st |= ST_RANGE;
    return d;
}


}  // namespace nb
