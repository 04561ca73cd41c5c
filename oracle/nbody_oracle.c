/*
 * FP64 CPU oracle for the direct-summation Hermite hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never calls it and shares no code, header or constant with it.
 *
 * Everything is IEEE double precision, compiled without floating-point
 * contraction, and every sum runs over j in ascending index order.  OpenMP
 * parallelises only over independent outputs (one i per thread), so the
 * result does not depend on the thread count.
 *
 * Layout: structure-of-arrays, component-major.  A vector field q of n
 * particles is q[0..n) = x components, q[n..2n) = y, q[2n..3n) = z.
 *
 * Paper: Portegies Zwart, Belleman & Geldof, "High Performance Direct
 * Gravitational N-body Simulations on Graphics Processing Units".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_INVAL (-1)
#define ORC_E_RANGE (-3)
#define ORC_E_NONFINITE (-4)

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------
 * Pair sums: acceleration, jerk and potential.
 *
 * Section 2, Eq. (1) gives the acceleration as a sum over all j != i of
 * G m_j times the separation over its cube; the Appendix A listing gives the
 * softened form the code evaluates: with r = x_j - x_i and v = v_j - v_i,
 * s = r.r + eps^2,
 *     a_i   +=  m_j r / s^(3/2)
 *     k_i   +=  m_j ( v / s^(3/2) - 3 (r.v) r / s^(5/2) )
 *     phi_i -=  m_j / s^(1/2)
 * with G = 1 (N-body units, Section 4).  Eq. (1) writes the separation as
 * r_i - r_j, which would make gravity repulsive; the listing subtracts the
 * own position from the other one, which is the attractive sign used here.
 * The potential is per unit mass of i.  j == i is excluded by index, as in
 * Eq. (1), so eps^2 = 0 is allowed for distinct positions.
 *
 * active == NULL means i = s for s in [0, n_i).  Outputs are indexed by the
 * slot s: acc[c * n_i + s].
 * ---------------------------------------------------------------------- */
void oracle_force(int64_t n_i, const int32_t *active, int64_t n_j,
                  const double *pos, const double *vel, const double *mass,
                  double eps2, double *acc, double *jerk, double *pot)
{
    int64_t s;
#pragma omp parallel for schedule(dynamic, 16)
    for (s = 0; s < n_i; ++s) {
        const int64_t i = active ? (int64_t)active[s] : s;
        const double xi = pos[i], yi = pos[n_j + i], zi = pos[2 * n_j + i];
        const double ui = vel[i], vi = vel[n_j + i], wi = vel[2 * n_j + i];
        double ax = 0.0, ay = 0.0, az = 0.0;
        double jx = 0.0, jy = 0.0, jz = 0.0;
        double ph = 0.0;
        int64_t j;
        for (j = 0; j < n_j; ++j) {
            double rx, ry, rz, vx, vy, vz, s2, rv, rinv, r3inv, r5inv, mj;
            if (j == i) continue;
            rx = pos[j] - xi;
            ry = pos[n_j + j] - yi;
            rz = pos[2 * n_j + j] - zi;
            vx = vel[j] - ui;
            vy = vel[n_j + j] - vi;
            vz = vel[2 * n_j + j] - wi;
            s2 = rx * rx + ry * ry + rz * rz + eps2;
            rv = rx * vx + ry * vy + rz * vz;
            rinv = 1.0 / sqrt(s2);            /* s^(-1/2) */
            r3inv = rinv * rinv * rinv;       /* s^(-3/2) */
            r5inv = r3inv * rinv * rinv;      /* s^(-5/2) */
            mj = mass[j];
            ax += mj * rx * r3inv;
            ay += mj * ry * r3inv;
            az += mj * rz * r3inv;
            jx += mj * (vx * r3inv - 3.0 * rv * rx * r5inv);
            jy += mj * (vy * r3inv - 3.0 * rv * ry * r5inv);
            jz += mj * (vz * r3inv - 3.0 * rv * rz * r5inv);
            ph -= mj * rinv;
        }
        acc[s] = ax; acc[n_i + s] = ay; acc[2 * n_i + s] = az;
        jerk[s] = jx; jerk[n_i + s] = jy; jerk[2 * n_i + s] = jz;
        pot[s] = ph;
    }
}

/* ------------------------------------------------------------------------
 * Pair sums accumulated in float32, in index order or smallest force first.
 *
 * Section 6 notes that the accuracy of single-precision sums could be
 * improved by sorting the forces by size and adding the smallest first.
 * This is that arithmetic, written out: for each i every pair term of the
 * sums above is evaluated in float64 and rounded once to float32; the terms
 * are then added in float32, one after the other, either in ascending j
 * (order 0) or in ascending size of the pair force m_j |r| / s^(3/2)
 * (order 1; ties by j), the same order for all seven sums.  Outputs are the
 * float32 sums widened to float64, indexed by slot as in oracle_force.
 * ---------------------------------------------------------------------- */
typedef struct {
    double key;
    int64_t j;
} SizeKey;

static int cmp_size(const void *pa, const void *pb)
{
    const SizeKey *a = (const SizeKey *)pa, *b = (const SizeKey *)pb;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->j > b->j) - (a->j < b->j);
}

int oracle_force_sum32(int64_t n_i, const int32_t *active, int64_t n_j,
                       const double *pos, const double *vel, const double *mass,
                       double eps2, int order, double *acc, double *jerk,
                       double *pot)
{
    int fail = 0;
#pragma omp parallel
    {
        float *term = (float *)malloc(sizeof(float) * 7 * (size_t)(n_j > 0 ? n_j : 1));
        SizeKey *keys = (SizeKey *)malloc(sizeof(SizeKey) * (size_t)(n_j > 0 ? n_j : 1));
        int64_t s;
        if (!term || !keys) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (s = 0; s < n_i; ++s) {
            const int64_t i = active ? (int64_t)active[s] : s;
            const double xi = pos[i], yi = pos[n_j + i], zi = pos[2 * n_j + i];
            const double ui = vel[i], vi = vel[n_j + i], wi = vel[2 * n_j + i];
            float sum[7] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            int64_t j, m = 0, q;
            int c;
            if (!term || !keys) continue;
            for (j = 0; j < n_j; ++j) {
                double rx, ry, rz, vx, vy, vz, s2, rv, rinv, r3inv, r5inv, mj;
                if (j == i) continue;
                rx = pos[j] - xi;
                ry = pos[n_j + j] - yi;
                rz = pos[2 * n_j + j] - zi;
                vx = vel[j] - ui;
                vy = vel[n_j + j] - vi;
                vz = vel[2 * n_j + j] - wi;
                s2 = rx * rx + ry * ry + rz * rz + eps2;
                rv = rx * vx + ry * vy + rz * vz;
                rinv = 1.0 / sqrt(s2);
                r3inv = rinv * rinv * rinv;
                r5inv = r3inv * rinv * rinv;
                mj = mass[j];
                term[7 * m + 0] = (float)(mj * rx * r3inv);
                term[7 * m + 1] = (float)(mj * ry * r3inv);
                term[7 * m + 2] = (float)(mj * rz * r3inv);
                term[7 * m + 3] = (float)(mj * (vx * r3inv - 3.0 * rv * rx * r5inv));
                term[7 * m + 4] = (float)(mj * (vy * r3inv - 3.0 * rv * ry * r5inv));
                term[7 * m + 5] = (float)(mj * (vz * r3inv - 3.0 * rv * rz * r5inv));
                term[7 * m + 6] = (float)(-mj * rinv);
                keys[m].key = fabs(mj) * sqrt(rx * rx + ry * ry + rz * rz) * r3inv;
                keys[m].j = m;
                ++m;
            }
            if (order == 1) qsort(keys, (size_t)m, sizeof(SizeKey), cmp_size);
            for (q = 0; q < m; ++q) {
                const int64_t t = (order == 1) ? keys[q].j : q;
                for (c = 0; c < 7; ++c) sum[c] = sum[c] + term[7 * t + c];
            }
            acc[s] = sum[0]; acc[n_i + s] = sum[1]; acc[2 * n_i + s] = sum[2];
            jerk[s] = sum[3]; jerk[n_i + s] = sum[4]; jerk[2 * n_i + s] = sum[5];
            pot[s] = sum[6];
        }
        free(term);
        free(keys);
    }
    return fail ? ORC_E_INVAL : ORC_OK;
}

/* ------------------------------------------------------------------------
 * Predictor (Section 2): with dt = t_target - t_i,
 *     x_p = x + (v + (dt/2) (a + (dt/3) k)) dt
 *     v_p = v + (a + (dt/2) k) dt
 * evaluated in exactly this nesting, for all n particles.
 * ---------------------------------------------------------------------- */
void oracle_predict(int64_t n, double t_target, const double *t,
                    const double *x, const double *v, const double *a,
                    const double *k, double *xp, double *vp)
{
    int64_t i;
    int c;
    for (i = 0; i < n; ++i) {
        const double dt = t_target - t[i];
        for (c = 0; c < 3; ++c) {
            const int64_t q = c * n + i;
            xp[q] = x[q] + (v[q] + (dt / 2.0) * (a[q] + (dt / 3.0) * k[q])) * dt;
            vp[q] = v[q] + (a[q] + (dt / 2.0) * k[q]) * dt;
        }
    }
}

/* ------------------------------------------------------------------------
 * Block scheduler (Section 2, first item of the integration step): the
 * particles to advance are those with the smallest t_i + dt_i.  Returns the
 * count; writes t_next and the ascending list of indices.
 * ---------------------------------------------------------------------- */
int64_t oracle_schedule(int64_t n, const double *t, const double *dt,
                        double *t_next, int32_t *active)
{
    int64_t i, m = 0;
    double tn = INFINITY;
    for (i = 0; i < n; ++i)
        if (t[i] + dt[i] < tn) tn = t[i] + dt[i];
    for (i = 0; i < n; ++i)
        if (t[i] + dt[i] == tn) active[m++] = (int32_t)i;
    *t_next = tn;
    return m;
}

/* ------------------------------------------------------------------------
 * Time steps.  The paper does not state its criterion (it says the codes use
 * the same one).  Reading: the Aarseth (1985) criterion with eta, the usual
 * companion of the Makino & Aarseth (1992) Hermite scheme the paper follows,
 * quantised to powers of two as Section 2 requires for block steps.
 * ---------------------------------------------------------------------- */
static double norm3(const double *q, int64_t n, int64_t i)
{
    const double x = q[i], y = q[n + i], z = q[2 * n + i];
    return sqrt(x * x + y * y + z * z);
}

/* Initial step: eta_s |a| / |k|, floored to a power of two not above dt_max,
 * halved until t0 is a multiple of it.  A non-finite |a| or |k| carries no
 * step information: the particle gets dt_min and the call reports it. */
int oracle_initial_dt(int64_t n, double t0, const double *a, const double *k,
                      double eta_s, double dt_max, double dt_min, double *dt)
{
    int64_t i;
    int rc = ORC_OK;
    for (i = 0; i < n; ++i) {
        const double an = norm3(a, n, i), kn = norm3(k, n, i);
        double want, d;
        if (kn > 0.0) want = eta_s * an / kn;
        else want = dt_max;
        if (!(want == want) || !isfinite(an) || !isfinite(kn)) {
            rc = ORC_E_NONFINITE;
            want = dt_min;
        }
        d = dt_max;
        while (d > want && d >= 2.0 * dt_min) d = d / 2.0;
        while (fmod(t0, d) != 0.0 && d >= 2.0 * dt_min) d = d / 2.0;
        if (d > want || fmod(t0, d) != 0.0) rc = ORC_E_RANGE;
        dt[i] = d;
    }
    return rc;
}

/* ------------------------------------------------------------------------
 * Corrector (Section 2) for the active particles, then the new time step.
 *     a3 = 2 (a - a_p) + (k + k_p) dt
 *     a2 = -3 (a - a_p) - (2 k + k_p) dt
 *     x  = x_p + (a2/12 + a3/20) dt^2
 *     v  = v_p + (a2/3 + a3/4) dt
 * where a, k are the old values at t_i and a_p, k_p the new force evaluated
 * at the predicted state.  Afterwards a <- a_p, k <- k_p, t_i <- t_i + dt.
 *
 * New step (reading): with a2 = (d^2a/dt^2) dt^2/2 and a3 = (d^3a/dt^3)
 * dt^3/6 as the paper defines them, the second derivative at the end of the
 * step is (2 a2 + 6 a3) / dt^2 and the third 6 a3 / dt^3; then
 *     dt_crit = sqrt( eta (|a||a''| + |k|^2) / (|k||a'''| + |a''|^2) ).
 * The step is halved while above dt_crit; otherwise it is doubled once if
 * 2 dt <= dt_crit, t_new is a multiple of 2 dt, and 2 dt <= dt_max.  If the
 * denominator is zero the criterion places no limit.  A step that would fall
 * below dt_min is an error.  fixed_dt != 0 keeps every step as it is.
 *
 * acc_new/jerk_new are indexed by slot with stride n_i (as oracle_force
 * writes them); x, v, a, k, t, dt by particle with stride n.
 * ---------------------------------------------------------------------- */
int oracle_correct(int64_t n, int64_t n_i, const int32_t *active,
                   const double *xp, const double *vp,
                   const double *acc_new, const double *jerk_new,
                   double eta, double dt_max, double dt_min, int fixed_dt,
                   double *t, double *dt, double *x, double *v,
                   double *a, double *k)
{
    int64_t s;
    int rc = ORC_OK;
    for (s = 0; s < n_i; ++s) {
        const int64_t i = active ? (int64_t)active[s] : s;
        const double h = dt[i];
        const double t_new = t[i] + h;
        double a2v[3], a3v[3], a1v[3], k1v[3];
        int c, bad = 0;
        for (c = 0; c < 3; ++c) {
            const int64_t q = c * n + i;
            const double a0 = a[q], k0 = k[q];
            const double a1 = acc_new[c * n_i + s], k1 = jerk_new[c * n_i + s];
            const double A3 = 2.0 * (a0 - a1) + (k0 + k1) * h;
            const double A2 = -3.0 * (a0 - a1) - (2.0 * k0 + k1) * h;
            x[q] = xp[q] + (A2 / 12.0 + A3 / 20.0) * h * h;
            v[q] = vp[q] + (A2 / 3.0 + A3 / 4.0) * h;
            a[q] = a1;
            k[q] = k1;
            a1v[c] = a1;
            k1v[c] = k1;
            a2v[c] = (2.0 * A2 + 6.0 * A3) / (h * h);
            a3v[c] = 6.0 * A3 / (h * h * h);
            if (!isfinite(x[q]) || !isfinite(v[q]) || !isfinite(a1) || !isfinite(k1)) bad = 1;
        }
        t[i] = t_new;
        /* a non-finite corrected state is reported and keeps its step */
        if (bad) rc = ORC_E_NONFINITE;
        if (!fixed_dt) {
            const double an = sqrt(a1v[0] * a1v[0] + a1v[1] * a1v[1] + a1v[2] * a1v[2]);
            const double kn = sqrt(k1v[0] * k1v[0] + k1v[1] * k1v[1] + k1v[2] * k1v[2]);
            const double a2n = sqrt(a2v[0] * a2v[0] + a2v[1] * a2v[1] + a2v[2] * a2v[2]);
            const double a3n = sqrt(a3v[0] * a3v[0] + a3v[1] * a3v[1] + a3v[2] * a3v[2]);
            const double num = eta * (an * a2n + kn * kn);
            const double den = kn * a3n + a2n * a2n;
            double crit, d = h;
            if (den > 0.0) crit = sqrt(num / den);
            else crit = INFINITY;
            if (bad || !(crit == crit)) { rc = ORC_E_NONFINITE; crit = d; }
            if (d > crit) {
                while (d > crit) d = d / 2.0;
            } else if (2.0 * d <= crit && fmod(t_new, 2.0 * d) == 0.0 &&
                       2.0 * d <= dt_max) {
                d = 2.0 * d;
            }
            if (d < dt_min) { rc = ORC_E_RANGE; d = dt_min; }
            dt[i] = d;
        }
    }
    return rc;
}

/* ------------------------------------------------------------------------
 * Energy diagnostic (Section 6 quotes energy errors; reading: the total
 * energy E = K + W with K = sum 1/2 m |v|^2 and W = 1/2 sum_i m_i phi_i for
 * the softened potential of the force law above).  out[0] = K, out[1] = W.
 * ---------------------------------------------------------------------- */
void oracle_energy(int64_t n, const double *pos, const double *vel,
                   const double *mass, double eps2, double *out)
{
    double kin = 0.0, wsum = 0.0;
    double *phi = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < n; ++i) {
        double ph = 0.0;
        int64_t j;
        for (j = 0; j < n; ++j) {
            double rx, ry, rz;
            if (j == i) continue;
            rx = pos[j] - pos[i];
            ry = pos[n + j] - pos[n + i];
            rz = pos[2 * n + j] - pos[2 * n + i];
            ph -= mass[j] / sqrt(rx * rx + ry * ry + rz * rz + eps2);
        }
        phi[i] = ph;
    }
    for (i = 0; i < n; ++i) {
        const double u = vel[i], w = vel[n + i], z = vel[2 * n + i];
        kin += 0.5 * mass[i] * (u * u + w * w + z * z);
        wsum += mass[i] * phi[i];
    }
    free(phi);
    out[0] = kin;
    out[1] = 0.5 * wsum;
}

/* ------------------------------------------------------------------------
 * Initialisation: force on all particles at t0, then the initial steps.
 * ---------------------------------------------------------------------- */
int oracle_init(int64_t n, double t0, const double *m, double eps2,
                double eta_s, double dt_max, double dt_min,
                double *t, double *dt, const double *x, const double *v,
                double *a, double *k)
{
    double *pot = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t i;
    int rc;
    oracle_force(n, NULL, n, x, v, m, eps2, a, k, pot);
    free(pot);
    for (i = 0; i < n; ++i) t[i] = t0;
    rc = oracle_initial_dt(n, t0, a, k, eta_s, dt_max, dt_min, dt);
    return rc;
}

/* ------------------------------------------------------------------------
 * One block step (Section 2, the four items of the integration step):
 * select the block, predict all particles to the new time, recompute the
 * force on the block, correct it.  Returns n_i (0 if t_next > t_end, in
 * which case nothing changes), or a negative error code.
 * ---------------------------------------------------------------------- */
int64_t oracle_blockstep(int64_t n, const double *m, double eps2, double eta,
                         double dt_max, double dt_min, double t_end,
                         double *t, double *dt, double *x, double *v,
                         double *a, double *k, double *t_next_out,
                         int32_t *active_out)
{
    double t_next;
    int32_t *act = active_out ? active_out
                              : (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *xp = (double *)malloc(sizeof(double) * (size_t)(3 * n));
    double *vp = (double *)malloc(sizeof(double) * (size_t)(3 * n));
    int64_t n_i = oracle_schedule(n, t, dt, &t_next, act);
    int64_t ret = n_i;
    if (t_next_out) *t_next_out = t_next;
    if (!(t_next <= t_end)) {
        ret = 0;
    } else {
        double *an = (double *)malloc(sizeof(double) * (size_t)(3 * n_i));
        double *kn = (double *)malloc(sizeof(double) * (size_t)(3 * n_i));
        double *pn = (double *)malloc(sizeof(double) * (size_t)n_i);
        int rc;
        oracle_predict(n, t_next, t, x, v, a, k, xp, vp);
        oracle_force(n_i, act, n, xp, vp, m, eps2, an, kn, pn);
        rc = oracle_correct(n, n_i, act, xp, vp, an, kn, eta, dt_max, dt_min,
                            0, t, dt, x, v, a, k);
        if (rc != ORC_OK) ret = rc;
        free(an); free(kn); free(pn);
    }
    free(xp); free(vp);
    if (!active_out) free(act);
    return ret;
}

/* Repeated block steps until the next block would pass t_end or max_steps
 * is reached.  stats[0] += steps taken, stats[1] += sum of block sizes. */
int oracle_integrate(int64_t n, const double *m, double eps2, double eta,
                     double dt_max, double dt_min, double t_end,
                     int64_t max_steps, double *t, double *dt, double *x,
                     double *v, double *a, double *k, int64_t *stats)
{
    int64_t step;
    for (step = 0; step < max_steps; ++step) {
        int64_t r = oracle_blockstep(n, m, eps2, eta, dt_max, dt_min, t_end,
                                     t, dt, x, v, a, k, NULL, NULL);
        if (r < 0) return (int)r;
        if (r == 0) break;
        stats[0] += 1;
        stats[1] += r;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Shared-step Hermite run (every particle, one common dt): the initial a, k
 * come from the force at t = 0, then n_steps of predict / force / correct.
 * x, v are advanced in place; a, k hold the last force.
 * ---------------------------------------------------------------------- */
void oracle_shared_run(int64_t n, int64_t n_steps, double h, const double *m,
                       double eps2, double *x, double *v, double *a, double *k)
{
    double *t = (double *)calloc((size_t)n, sizeof(double));
    double *dt = (double *)malloc(sizeof(double) * (size_t)n);
    double *xp = (double *)malloc(sizeof(double) * (size_t)(3 * n));
    double *vp = (double *)malloc(sizeof(double) * (size_t)(3 * n));
    double *an = (double *)malloc(sizeof(double) * (size_t)(3 * n));
    double *kn = (double *)malloc(sizeof(double) * (size_t)(3 * n));
    double *pn = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t i, st;
    for (i = 0; i < n; ++i) dt[i] = h;
    oracle_force(n, NULL, n, x, v, m, eps2, a, k, pn);
    for (st = 0; st < n_steps; ++st) {
        oracle_predict(n, t[0] + h, t, x, v, a, k, xp, vp);
        oracle_force(n, NULL, n, xp, vp, m, eps2, an, kn, pn);
        oracle_correct(n, n, NULL, xp, vp, an, kn, 0.0, h, h, 1,
                       t, dt, x, v, a, k);
    }
    free(t); free(dt); free(xp); free(vp); free(an); free(kn); free(pn);
}

/* ------------------------------------------------------------------------
 * Adjoint of the pair sums (not in the paper; derived from the force law of
 * the Appendix A listing).  Given cotangents abar, kbar, pbar of the outputs
 * a, k, phi of every particle (full set, n_i = n_j = n), returns
 *     xbar = dL/dx, vbar = dL/dv, mbar = dL/dm  for L = sum_i abar_i.a_i +
 *     kbar_i.k_i + pbar_i phi_i.
 * Per pair (i, j), with r = x_j - x_i, v = v_j - v_i, s = r.r + eps^2,
 * q = r.v, al = s^(-3/2), be = s^(-5/2), ga = s^(-7/2):
 *   g_r = m_j [ al abar - 3 q be kbar - 3 be (kbar.r) v
 *             + (pbar al - 3 be (abar.r + kbar.v) + 15 q ga (kbar.r)) r ]
 *   g_v = m_j [ al kbar - 3 be (kbar.r) r ]
 *   g_m = al (abar.r + kbar.v) - 3 q be (kbar.r) - pbar s^(-1/2)
 * and xbar_j += g_r, xbar_i -= g_r, vbar_j += g_v, vbar_i -= g_v,
 * mbar_j += g_m.  Two plain loops: the i-side sums over j, the j-side over i.
 * ---------------------------------------------------------------------- */
static void pair_adjoint(int64_t n, const double *pos, const double *vel,
                         const double *mass, double eps2,
                         const double *abar, const double *kbar,
                         const double *pbar, int64_t i, int64_t j,
                         double gr[3], double gv[3], double *gm)
{
    const double r[3] = {pos[j] - pos[i], pos[n + j] - pos[n + i],
                         pos[2 * n + j] - pos[2 * n + i]};
    const double w[3] = {vel[j] - vel[i], vel[n + j] - vel[n + i],
                         vel[2 * n + j] - vel[2 * n + i]};
    const double A[3] = {abar[i], abar[n + i], abar[2 * n + i]};
    const double K[3] = {kbar[i], kbar[n + i], kbar[2 * n + i]};
    const double P = pbar[i];
    const double s = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
    const double q = r[0] * w[0] + r[1] * w[1] + r[2] * w[2];
    const double rinv = 1.0 / sqrt(s);
    const double al = rinv * rinv * rinv;
    const double be = al * rinv * rinv;
    const double ga = be * rinv * rinv;
    const double ar = A[0] * r[0] + A[1] * r[1] + A[2] * r[2];
    const double kr = K[0] * r[0] + K[1] * r[1] + K[2] * r[2];
    const double kv = K[0] * w[0] + K[1] * w[1] + K[2] * w[2];
    const double mj = mass[j];
    const double coef = P * al - 3.0 * be * (ar + kv) + 15.0 * q * ga * kr;
    int c;
    for (c = 0; c < 3; ++c) {
        gr[c] = mj * (al * A[c] - 3.0 * q * be * K[c] - 3.0 * be * kr * w[c] +
                      coef * r[c]);
        gv[c] = mj * (al * K[c] - 3.0 * be * kr * r[c]);
    }
    *gm = al * (ar + kv) - 3.0 * q * be * kr - P * rinv;
}

void oracle_force_adjoint(int64_t n, const double *pos, const double *vel,
                          const double *mass, double eps2, const double *abar,
                          const double *kbar, const double *pbar, double *xbar,
                          double *vbar, double *mbar)
{
    int64_t i, j;
    /* i-side: particle i as the receiver of the force */
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < n; ++i) {
        double sx[3] = {0, 0, 0}, sv[3] = {0, 0, 0};
        int64_t jj;
        int c;
        for (jj = 0; jj < n; ++jj) {
            double gr[3], gv[3], gm;
            if (jj == i) continue;
            pair_adjoint(n, pos, vel, mass, eps2, abar, kbar, pbar, i, jj, gr,
                         gv, &gm);
            for (c = 0; c < 3; ++c) { sx[c] -= gr[c]; sv[c] -= gv[c]; }
        }
        for (c = 0; c < 3; ++c) { xbar[c * n + i] = sx[c]; vbar[c * n + i] = sv[c]; }
        mbar[i] = 0.0;
    }
    /* j-side: particle j as the source of the force on every other i */
#pragma omp parallel for schedule(dynamic, 16)
    for (j = 0; j < n; ++j) {
        double sx[3] = {0, 0, 0}, sv[3] = {0, 0, 0}, sm = 0.0;
        int64_t ii;
        int c;
        for (ii = 0; ii < n; ++ii) {
            double gr[3], gv[3], gm;
            if (ii == j) continue;
            pair_adjoint(n, pos, vel, mass, eps2, abar, kbar, pbar, ii, j, gr,
                         gv, &gm);
            for (c = 0; c < 3; ++c) { sx[c] += gr[c]; sv[c] += gv[c]; }
            sm += gm;
        }
        for (c = 0; c < 3; ++c) { xbar[c * n + j] += sx[c]; vbar[c * n + j] += sv[c]; }
        mbar[j] += sm;
    }
}
