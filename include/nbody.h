/*
 * nbody.h -- C ABI of libnbody.so, the MI355X (gfx950) direct-summation
 * Hermite library.
 *
 * What it computes (Portegies Zwart, Belleman & Geldof, "High Performance
 * Direct Gravitational N-body Simulations on Graphics Processing Units"):
 *   - the softened pair sums of acceleration, jerk and potential of
 *     Section 2, Eq. (1), in the softened form of the Appendix A listing;
 *   - the fourth-order Hermite predictor and corrector of Section 2;
 *   - the power-of-two block time steps of Section 2 (selection of the
 *     particles with the smallest t_i + dt_i);
 *   - the energy diagnostic behind the energy errors of Section 6;
 *   - an adjoint of the pair sums and of the shared-step Hermite chain, and
 *     a batched ensemble driver (extensions of the method; see each entry).
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers owned by the caller; the library
 *     never frees them.  Scalars are host values.  A few outputs are
 *     explicitly host pointers; they say so.
 *   - Vectors are structure-of-arrays, component-major float64: for n
 *     particles q[0..n) holds x, q[n..2n) y, q[2n..3n) z.  Scalars per
 *     particle are float64 arrays of length n.  Index lists are int32.
 *   - Work is enqueued on the context's HIP stream and is asynchronous
 *     unless an entry says it synchronises.
 *   - Every entry returns NBODY_OK (0) or a negative status; no C++
 *     exception crosses the ABI.  nbody_last_error() gives the text of the
 *     last failure on that context.  Errors found by kernels (a time step
 *     below dt_min, a non-finite value, an active index out of range) are
 *     latched in a device status word
 *     and reported by the next synchronising call (nbody_sync_status,
 *     nbody_blockstep, nbody_ensemble_run).
 *   - Results are deterministic for a fixed device and configuration: no
 *     floating-point atomics; every reduction has a fixed order.
 *   - Calls on one context must not overlap from several host threads.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define NBODY_OK 0
#define NBODY_E_INVAL (-1)     /* bad argument, detected on the host       */
#define NBODY_E_DEVICE (-2)    /* HIP runtime error                         */
#define NBODY_E_RANGE (-3)     /* a time step fell below dt_min             */
#define NBODY_E_NONFINITE (-4) /* a non-finite state, force or step norm    */
#define NBODY_E_NOMEM (-5)     /* device allocation failed                  */

/* ---- flags for the force and adjoint entries ------------------------- */
/* Relative positions and velocities are always formed in float64.  The flag
 * selects the pair arithmetic and its accumulation:
 *   NBODY_ACC_FP32  relative coordinates rounded to float32, float32 pair
 *                   terms (rsqrt on the VALU) summed in float32 over at most
 *                   8 tiles of consecutive j, those sums added in float64;
 *   NBODY_ACC_DS    the compensated (accurate) mode.  nbody_force,
 *                   nbody_init / nbody_blockstep, nbody_shared_run and
 *                   nbody_ensemble_run evaluate the pair terms in float64
 *                   (s^(-1/2) from the float32 estimate refined by a float64
 *                   Newton step) with float64 sums; the adjoint keeps float32
 *                   pair terms and folds its tile sums by TwoSum into
 *                   float-float sums. */
#define NBODY_ACC_FP32 0u
#define NBODY_ACC_DS 1u
/* nbody_system.flags only: every particle keeps the step it has (dt_max after
 * nbody_init), i.e. shared steps in which every block step advances all
 * particles; the step criterion is not evaluated. */
#define NBODY_FIXED_DT 2u
/* nbody_force_adjoint only: add into pos_bar, vel_bar, mass_bar instead of
 * overwriting them. */
#define NBODY_ADJ_ACCUMULATE 4u

typedef struct nbody_ctx nbody_ctx;

/* Library version, major*10000 + minor*100 + patch. */
int nbody_version(void);

/* Create a context bound to HIP device `device` and stream `stream`
 * (a hipStream_t, or NULL for the null stream).  The context owns its
 * scratch buffers and tuning table.  Allocates device memory lazily. */
int nbody_create(nbody_ctx **out, int device, void *stream);
int nbody_destroy(nbody_ctx *ctx);
/* Re-bind the stream (e.g. torch.cuda.current_stream().cuda_stream). */
int nbody_set_stream(nbody_ctx *ctx, void *stream);
/* Text of the last error on ctx (never NULL; "" if none). */
const char *nbody_last_error(const nbody_ctx *ctx);
/* Synchronise the stream, return and clear the device status word:
 * NBODY_OK, NBODY_E_RANGE or NBODY_E_NONFINITE. */
int nbody_sync_status(nbody_ctx *ctx);

/* ---- pair sums ---------------------------------------------------------
 * Section 2, Eq. (1) with the softening, jerk and potential of the
 * Appendix A listing, G = 1: for each active slot s with particle
 * i = active_idx[s] (or i = s when active_idx is NULL), over all j != i:
 *   r = x_j - x_i,  w = v_j - v_i,  S = r.r + eps2,
 *   acc[s]  = sum m_j r S^(-3/2)
 *   jerk[s] = sum m_j ( w S^(-3/2) - 3 (r.w) r S^(-5/2) )
 *   pot[s]  = -sum m_j S^(-1/2)            (per unit mass of i)
 * The self pair is excluded by index, so eps2 = 0 is valid for distinct
 * positions; coincident distinct particles with eps2 = 0 give non-finite
 * values (not trapped).
 *   active_idx : int32[n_i] indices in [0, n_j), or NULL.  Any order,
 *                duplicates allowed.
 *   pos, vel   : float64[3*n_j];  mass : float64[n_j]
 *   acc, jerk  : float64[3*n_i] (component stride n_i);  pot : float64[n_i]
 *                (pot may be NULL).
 *   flags      : NBODY_ACC_FP32 or NBODY_ACC_DS.
 * Errors: NBODY_E_INVAL for NULL arrays, n_i < 0, n_j < 1, n_i > 2^31-1,
 * eps2 < 0 or NaN, unknown flags. */
int nbody_force(nbody_ctx *ctx, const int32_t *active_idx, int64_t n_i,
                const double *pos, const double *vel, const double *mass,
                int64_t n_j, double eps2, double *acc, double *jerk,
                double *pot, uint32_t flags);

/* ---- smallest-first float32 pair sums (Section 6) -----------------------
 * The accuracy improvement Section 6 proposes for float32 sums: the same
 * acceleration, jerk and potential as nbody_force, with every pair term
 * evaluated in float64 and rounded once to float32, and each particle's
 * terms added in float32 in ascending order of the pair-acceleration
 * magnitude m_j |x_j - x_i| S^(-3/2) (ties by j), all seven sums in that
 * order.  An accuracy mode, not a fast path: one workgroup per particle sorts
 * its n_j - 1 keys in LDS.
 *   n_j : 1 <= n_j <= 8192, else NBODY_E_INVAL.  Other arguments, layouts
 *   and errors as nbody_force (no flags).  eps2 = 0 with coincident
 *   particles gives non-finite keys and an unspecified order. */
int nbody_force_sorted(nbody_ctx *ctx, const int32_t *active_idx, int64_t n_i,
                       const double *pos, const double *vel, const double *mass,
                       int64_t n_j, double eps2, double *acc, double *jerk,
                       double *pot);

/* ---- pair sums without allocation ----------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, arithmetic and errors as nbody_force, but the j records and the
 * split partial sums live in a static array of NBODY_NOALLOC_SCRATCH_MB MiB
 * that every device the library runs on holds until the process ends; the
 * call makes no hipMalloc / hipFree and records no timing events (the
 * context itself, including its status word, is allocated by nbody_create).
 * The j split is capped so that the partial sums fit next to the records,
 * so the launch shape (and the last bits of the float32 sums) can differ
 * from nbody_force's for large n_i.
 *   n_j : 1 <= n_j <= NBODY_NOALLOC_MAX_NJ, else NBODY_E_INVAL (host check).
 * Every call on a device shares that device's array: calls that overlap on
 * one device (other streams, other threads, other contexts) race. */
#define NBODY_NOALLOC_SCRATCH_MB 96
#define NBODY_NOALLOC_MAX_NJ 1048576
int nbody_force_noalloc(nbody_ctx *ctx, const int32_t *active_idx, int64_t n_i,
                        const double *pos, const double *vel, const double *mass,
                        int64_t n_j, double eps2, double *acc, double *jerk,
                        double *pot, uint32_t flags);

/* ---- predictor ---------------------------------------------------------
 * Section 2: for every particle, with h = t_target - t[i],
 *   xp = x + (v + (h/2)(a + (h/3) k)) h,    vp = v + (a + (h/2) k) h
 * evaluated in float64 in this nesting (no contraction).
 *   t : float64[n];  x, v, a, k, xp, vp : float64[3n]. */
int nbody_predict(nbody_ctx *ctx, int64_t n, double t_target, const double *t,
                  const double *x, const double *v, const double *a,
                  const double *k, double *xp, double *vp);

/* ---- block scheduler ---------------------------------------------------
 * Section 2, first item of a step: t_next = min_i (t[i] + dt[i]); the
 * active block is every i with t[i] + dt[i] == t_next (exact float64
 * comparison), written in ascending index order.
 *   active_idx : int32[n] output (first n_i entries valid)
 *   n_i_out    : int64[1] device output;  t_next_out : float64[1] device. */
int nbody_schedule(nbody_ctx *ctx, int64_t n, const double *t,
                   const double *dt, int32_t *active_idx, int64_t *n_i_out,
                   double *t_next_out);

/* ---- corrector and new time step ---------------------------------------
 * Section 2, for each active slot s, particle i = active_idx[s] (or s), with
 * h = dt[i], a, k the old values and a_p = acc_new[s], k_p = jerk_new[s]:
 *   a3 = 2(a - a_p) + (k + k_p) h,   a2 = -3(a - a_p) - (2k + k_p) h,
 *   x = xp + (a2/12 + a3/20) h^2,    v = vp + (a2/3 + a3/4) h,
 *   a <- a_p, k <- k_p, t <- t + h.
 * New step (the paper does not state its criterion; this library uses
 * Aarseth's, with the end-of-step derivatives (2 a2 + 6 a3)/h^2 and
 * 6 a3/h^3):
 *   dt_crit = sqrt(eta (|a||a''| + |k|^2) / (|k||a'''| + |a''|^2)),
 * halved while dt > dt_crit, else doubled once if 2dt <= dt_crit, t is a
 * multiple of 2dt and 2dt <= dt_max.  A zero denominator sets no limit.  A
 * step below dt_min latches NBODY_E_RANGE; a NaN criterion latches
 * NBODY_E_NONFINITE.  fixed_dt != 0 leaves dt unchanged (shared steps).
 *   acc_new, jerk_new : float64[3*n_i], component stride n_i.
 *   xp, vp, x, v, a, k : float64[3n];  t, dt : float64[n]. */
int nbody_correct(nbody_ctx *ctx, int64_t n, int64_t n_i,
                  const int32_t *active_idx, const double *xp,
                  const double *vp, const double *acc_new,
                  const double *jerk_new, double eta, double dt_max,
                  double dt_min, int fixed_dt, double *t, double *dt,
                  double *x, double *v, double *a, double *k);

/* ---- device-counted variants ---------------------------------------------
 * nbody_predict, nbody_force and nbody_correct with the block time and the
 * block size read from device memory (nbody_schedule's t_next_out and
 * n_i_out), so that schedule -> predict -> force -> correct is enqueued with
 * no host synchronisation in between.  Same arithmetic as the host-counted
 * entries; nbody_force_dev uses the launch shapes of the block-step driver.
 *   t_target_dev : float64[1] device;  n_i_dev : int64[1] device.
 *   n_i_cap      : capacity of the outputs and largest accepted block; a
 *                  device block size above it is clamped to it and latches
 *                  the index error (NBODY_E_INVAL at the next sync).
 *   acc, jerk / acc_new, jerk_new : float64[3 n_i_cap], component stride
 *                  n_i_cap;  pot : float64[n_i_cap] or NULL. */
int nbody_predict_dev(nbody_ctx *ctx, int64_t n, const double *t_target_dev,
                      const double *t, const double *x, const double *v,
                      const double *a, const double *k, double *xp, double *vp);
int nbody_force_dev(nbody_ctx *ctx, const int32_t *active_idx, const int64_t *n_i_dev,
                    int64_t n_i_cap, const double *pos, const double *vel,
                    const double *mass, int64_t n_j, double eps2, double *acc,
                    double *jerk, double *pot, uint32_t flags);
int nbody_correct_dev(nbody_ctx *ctx, int64_t n, const int64_t *n_i_dev, int64_t n_i_cap,
                      const int32_t *active_idx, const double *xp, const double *vp,
                      const double *acc_new, const double *jerk_new, double eta,
                      double dt_max, double dt_min, int fixed_dt, double *t, double *dt,
                      double *x, double *v, double *a, double *k);

/* ---- initial time steps ------------------------------------------------
 * dt[i] = largest power of two <= min(eta_s |a_i|/|k_i|, dt_max) of which
 * t0 is a multiple (|k_i| = 0 gives dt_max).  A value below dt_min latches
 * NBODY_E_RANGE.  dt_max must be a power of two. */
int nbody_initial_dt(nbody_ctx *ctx, int64_t n, double t0, const double *a,
                     const double *k, double eta_s, double dt_max,
                     double dt_min, double *dt);

/* ---- energy diagnostic -------------------------------------------------
 * Section 6 quotes energy errors; the energy is E = K + W with
 * K = sum 1/2 m |v|^2 and W = 1/2 sum_i m_i phi_i for the softened
 * potential of the force law above, all in float64 (float64 pair
 * arithmetic).  out : float64[2] device output {K, W}. */
int nbody_energy(nbody_ctx *ctx, int64_t n, const double *pos,
                 const double *vel, const double *mass, double eps2,
                 double *out);

/* ---- device-resident block-step integrator -------------------------------
 * A system of n particles whose state lives in caller-owned device arrays.
 * eta: step criterion accuracy; eta_s: initial-step factor; dt_max (a power
 * of two) and dt_min bound the steps; flags as for nbody_force. */
typedef struct nbody_system {
    int64_t n;
    double *t, *dt;       /* float64[n]                      */
    double *x, *v;        /* float64[3n]                     */
    double *a, *k;        /* float64[3n] last force and jerk */
    const double *m;      /* float64[n]                      */
    double eps2, eta, eta_s, dt_max, dt_min;
    uint32_t flags;
} nbody_system;

/* Set t = t0 for all particles, evaluate a and k on all of them, and set
 * the initial steps (as nbody_initial_dt; dt_max for every particle with
 * NBODY_FIXED_DT). */
int nbody_init(nbody_ctx *ctx, const nbody_system *sys, double t0);

/* Run block steps (schedule -> predict all -> force on the block ->
 * correct the block, Section 2) without any per-step host traffic, until
 * max_steps steps are done or the next block would pass t_end.
 * Synchronises.  steps_done and interactions (sum over steps of n_i * n)
 * are HOST outputs (either may be NULL).  Returns the latched device
 * status (NBODY_E_RANGE / NBODY_E_NONFINITE) if any. */
int nbody_blockstep(nbody_ctx *ctx, const nbody_system *sys,
                    int64_t max_steps, double t_end, int64_t *steps_done,
                    int64_t *interactions);

/* ---- batched ensemble ----------------------------------------------------
 * Many independent clusters, each integrated with the block steps of
 * nbody_blockstep (same predictor, pair sums, corrector and step rules),
 * all in ONE persistent cooperative launch.  Cluster c is particles
 * [offsets[c], offsets[c+1]) of the concatenated arrays, with its own eps2;
 * clusters do not interact.  Every cluster is initialised at t = 0 (pair
 * sums of all its particles, initial steps as nbody_initial_dt) and
 * advanced until its next block would pass t_end (so all its particles end
 * at t_end when t_end is a multiple of dt_max).  Synchronises.
 *   offsets, eps2 : HOST arrays int64[n_clusters + 1] (offsets[0] = 0,
 *                   strictly increasing) and float64[n_clusters].
 *   t, dt, m      : device float64[n_total];  x, v, a, k : device
 *                   float64[3 n_total] with component stride n_total
 *                   (t, dt, a, k are outputs; x, v are advanced in place).
 *   steps, interactions : HOST int64[n_clusters] outputs (may be NULL):
 *                   block steps and sum of n_i * N per cluster.
 * Returns NBODY_E_DEVICE if the launch could not be made co-resident or a
 * team barrier timed out, else the latched step / non-finite status. */
typedef struct nbody_ensemble {
    int32_t n_clusters;
    const int64_t *offsets;
    const double *eps2;
    double *t, *dt;
    double *x, *v, *a, *k;
    const double *m;
    double eta, eta_s, dt_max, dt_min;
    uint32_t flags; /* NBODY_ACC_FP32 or NBODY_ACC_DS */
} nbody_ensemble;

int nbody_ensemble_run(nbody_ctx *ctx, const nbody_ensemble *e, double t_end,
                       int64_t *steps, int64_t *interactions);

/* Launch shape and team-planning model of the ensemble.  The persistent grid
 * has groups_per_cu workgroups per CU (capped by occupancy).  A cluster of N
 * particles is modelled to take S = steps_coef N^steps_exp t_end block steps
 * with blocks of B = block_coef N^block_exp particles (the paper's fits,
 * 247 N^0.35 steps per time unit and 0.20 N^0.81, are the defaults).  A pair
 * pass over n_i particles costs the busiest group of a team of g groups
 *   P(n_i) = tiles(n_i, g) tile_us 1e-6 + n_i N / (g group_rate),
 * where tiles(n_i, g) counts the j tiles of its items under the kernel's
 * split rule (items of 64 i_per_lane slots by S j ranges), and the cluster
 *   T = P(N) + S (1e-6 (step_us + [g > 1] (barrier_us + barrier_group_us g))
 *                + P(B)).
 * The plan minimises the largest modelled team time: clusters that one group
 * finishes in time share single-group teams (run one after the other), the
 * others get teams of the fewest groups (at most min(max_team, 64)) that
 * finish them in time, and spare groups go to the slowest teams.
 * The workgroup shape (waves, j_tile, i_per_lane) must be one of the
 * compiled ones: (4, 256, 2), (4, 256, 1), (2, 128, 2), (2, 256, 2),
 * (4, 512, 2), (8, 512, 2). */
typedef struct nbody_ensemble_config {
    int32_t groups_per_cu; /* 1..8 */
    int32_t max_team;      /* 1..4096 */
    double step_us;        /* fixed latency of one block step on one group */
    double barrier_us;     /* extra per-step cost of a multi-group team ... */
    double barrier_group_us; /* ... plus this much per group of the team */
    double group_rate;     /* pair interactions per second of one group */
    double steps_coef;     /* block steps per time unit = steps_coef N^steps_exp */
    double steps_exp;
    int32_t waves;         /* waves per workgroup, sharing each j tile */
    int32_t j_tile;        /* j particles staged in LDS per tile */
    int32_t i_per_lane;    /* block slots per lane (1 or 2) */
    double tile_us;        /* latency of one j tile of a pair item (load, predict, LDS) */
    double block_coef;     /* mean block size = block_coef N^block_exp */
    double block_exp;
} nbody_ensemble_config;

int nbody_ensemble_set(nbody_ctx *ctx, const nbody_ensemble_config *cfg);
/* Current configuration (HOST output). */
int nbody_ensemble_get(nbody_ctx *ctx, nbody_ensemble_config *cfg);

/* Per cluster of the last ensemble launch (HOST outputs, n_clusters entries,
 * either may be NULL): wall-clock seconds from the start of its
 * initialisation to its last step, and the number of groups of its team. */
int nbody_ensemble_timing(nbody_ctx *ctx, int32_t n_clusters, double *seconds,
                          int32_t *groups);
/* Grid size and number of teams of the last ensemble launch (HOST outputs). */
int nbody_ensemble_info(nbody_ctx *ctx, int32_t *grid, int32_t *teams);

/* The team plan nbody_ensemble_run would use, computed on the host only (no
 * context, no device): the same planner, for a grid of `groups` workgroups.
 *   sizes         : HOST int64[n_clusters], particles per cluster (>= 1).
 *   cfg           : the planning model, as nbody_ensemble_set takes it.
 *   t_end         : end time the model's step count scales with (>= 0).
 *   team_of       : HOST int32[n_clusters] output, team of each cluster.
 *   team_size     : HOST int32[n_clusters] output, groups of team q for
 *                   q < *n_teams (there are never more teams than clusters).
 *   model_seconds : HOST float64[n_clusters] output (may be NULL), modelled
 *                   time of each cluster on its team.
 *   n_teams       : HOST output.
 * Clusters that share a team (several clusters on one single-group team)
 * run one after the other; the team's time is the sum of theirs.
 * Returns NBODY_E_INVAL on null pointers, n_clusters < 1, groups < 1, a
 * cluster size < 1, a model with non-positive rates or a workgroup shape
 * that is not compiled. */
int nbody_ensemble_plan(const int64_t *sizes, int32_t n_clusters, int32_t groups,
                        const nbody_ensemble_config *cfg, double t_end, int32_t *team_of,
                        int32_t *team_size, double *model_seconds, int32_t *n_teams);

/* ---- adjoint (not in the paper: the transpose of the pair sums above) ----
 * For the full set (every particle is both i and j, n_i = n_j = n) and
 * cotangents abar, kbar, pbar of acc, jerk, pot, writes
 *   pos_bar = dL/dx,  vel_bar = dL/dv,  mass_bar = dL/dm
 * of L = sum_i abar_i.acc_i + kbar_i.jerk_i + pbar_i pot_i.  Per pair (i, j),
 * with r, w, S as for nbody_force, q = r.w, al = S^(-3/2), be = S^(-5/2),
 * ga = S^(-7/2):
 *   g_r = m_j [al abar_i - 3 q be kbar_i - 3 be (kbar_i.r) w
 *              + (pbar_i al - 3 be (abar_i.r + kbar_i.w) + 15 q ga (kbar_i.r)) r]
 *   g_v = m_j [al kbar_i - 3 be (kbar_i.r) r]
 *   g_m = al (abar_i.r + kbar_i.w) - 3 q be (kbar_i.r) - pbar_i S^(-1/2)
 * contribute pos_bar_j += g_r, pos_bar_i -= g_r, vel_bar_j += g_v,
 * vel_bar_i -= g_v, mass_bar_j += g_m.  float32 pair arithmetic on float64
 * relative coordinates, accumulation as selected by flags (NBODY_ACC_*, and
 * NBODY_ADJ_ACCUMULATE to add into the outputs).
 *   pos, vel, acc_bar, jerk_bar, pos_bar, vel_bar : float64[3n]
 *   mass, pot_bar (may be NULL = zero), mass_bar  : float64[n]
 * Outputs are overwritten unless NBODY_ADJ_ACCUMULATE is set. */
int nbody_force_adjoint(nbody_ctx *ctx, int64_t n, const double *pos,
                        const double *vel, const double *mass, double eps2,
                        const double *acc_bar, const double *jerk_bar,
                        const double *pot_bar, double *pos_bar, double *vel_bar,
                        double *mass_bar, uint32_t flags);

/* Transpose of the predictor for one shared step h (Section 2 predictor is
 * linear in x, v, a, k), ACCUMULATED into the outputs:
 *   x_bar += xp_bar;  v_bar += h xp_bar + vp_bar;
 *   a_bar += (h^2/2) xp_bar + h vp_bar;  k_bar += (h^3/6) xp_bar + (h^2/2) vp_bar.
 * All arrays float64[3n]. */
int nbody_predict_adjoint(nbody_ctx *ctx, int64_t n, double h, const double *xp_bar,
                          const double *vp_bar, double *x_bar, double *v_bar,
                          double *a_bar, double *k_bar);

/* Transpose of the corrector for one shared step h (Section 2 corrector,
 * linear in xp, vp, a0, k0, a1, k1 once a2, a3 are expanded:
 *   x1 = xp - (3/20) h^2 (a0 - a1) - h^3 (7 k0/60 + k1/30),
 *   v1 = vp - (h/2) (a0 - a1) - h^2 (5 k0/12 + k1/12)),
 * ACCUMULATED into xp_bar, vp_bar, a0_bar, k0_bar, a1_bar, k1_bar.  The
 * step's outputs a <- a1, k <- k1 pass their cotangents through unchanged
 * (the caller adds them to a1_bar, k1_bar).  All arrays float64[3n]. */
int nbody_correct_adjoint(nbody_ctx *ctx, int64_t n, double h, const double *x1_bar,
                          const double *v1_bar, double *xp_bar, double *vp_bar,
                          double *a0_bar, double *k0_bar, double *a1_bar,
                          double *k1_bar);

/* ---- differentiable shared-step run (an extension: the chain of the
 * entry points above, orchestrated natively) ------------------------------
 * nbody_shared_run: a, k = pair sums at (x0, v0) (nbody_force, all n
 * particles); then n_steps shared steps of h, each nbody_predict to h,
 * nbody_force at the predicted state, nbody_correct with the step held fixed
 * (Section 2).  Outputs the final x, v, a, k (device float64[3n], distinct
 * from x0, v0).  If ckpt is not NULL (device float64[ceil(n_steps /
 * ckpt_every) * 12n]), the state (x, v, a, k, each 3n, in that order)
 * before steps 0, ckpt_every, 2 ckpt_every, ... is stored there.
 *   m: device float64[n]; flags: NBODY_ACC_FP32 or NBODY_ACC_DS.
 * nbody_shared_run_adjoint: the gradient of a loss of the final (x, v, a, k)
 * with respect to x0, v0 and m, from its cotangents x_bar, v_bar, a_bar,
 * k_bar (device float64[3n]) and the checkpoints of nbody_shared_run with
 * the same arguments: each segment is recomputed from its checkpoint, then
 * nbody_correct_adjoint, nbody_force_adjoint (at the predicted state) and
 * nbody_predict_adjoint run back through its steps; last, the transpose of
 * the initial pair sums.  Outputs x0_bar, v0_bar (float64[3n]) and m_bar
 * (float64[n]), overwritten.  Workspace (about (16 + 2 ckpt_every) * 3n
 * doubles) is owned by the context.  Both return NBODY_E_INVAL for n < 1,
 * h <= 0, n_steps < 0, ckpt_every < 1, eps2 < 0 or null arrays. */
int nbody_shared_run(nbody_ctx *ctx, int64_t n, const double *m, double eps2, double h,
                     int64_t n_steps, int64_t ckpt_every, const double *x0,
                     const double *v0, double *x, double *v, double *a, double *k,
                     double *ckpt, uint32_t flags);
int nbody_shared_run_adjoint(nbody_ctx *ctx, int64_t n, const double *m, double eps2,
                             double h, int64_t n_steps, int64_t ckpt_every,
                             const double *x0, const double *v0, const double *ckpt,
                             const double *x_bar, const double *v_bar,
                             const double *a_bar, const double *k_bar, double *x0_bar,
                             double *v0_bar, double *m_bar, uint32_t flags);

/* ---- launch shape of the pair kernels (autotuning) ----------------------
 * The pair kernels are compiled in several shapes; a context keeps a table
 * of which shape to use for which active-block size.  Without entries a
 * built-in default is used.
 *   rep           form of the relative coordinates: 0 = float64 differences
 *                 rounded to float32; 1 = float-float (hi/lo float32 pairs)
 *                 differences, float32 instructions only; 2 = float64
 *                 position differences, float32 velocity differences (the
 *                 jerk then carries float32 rounding of the velocities).
 *   i_per_lane    i-particles per lane: 1, 2 or 4.
 *   waves         waves per workgroup splitting the j range: 1, 2, 4 or 8
 *                 (at most 4 with 4 i-particles per lane).
 *   tile          j-particles summed in float32 before each fold (>= 1).
 *   min_j_wave    smallest j range per wave when the j range is split (>= 1).
 *   target_groups workgroups to aim for before splitting j (>= 1).
 *   layout        0: one i-particle per lane, every j broadcast to the wave;
 *                 1: one j-particle per lane (vector loads), the workgroup's
 *                 i_per_lane (1, 2, 4 or 8; at most 4 with NBODY_ACC_DS)
 *                 i-particles shared by all lanes, lane sums added by a
 *                 fixed-order butterfly -- for small active blocks.  Layout 1
 *                 takes rep 0 and 1, 2 or 4 waves; `tile` bounds the terms of
 *                 a lane's float32 sum. */
typedef struct nbody_force_config {
    int32_t rep;
    int32_t i_per_lane;
    int32_t waves;
    int32_t tile;
    int32_t min_j_wave;
    int32_t target_groups;
    int32_t layout;
} nbody_force_config;

/* Use `cfg` for active-block sizes n_i in [n_i_lo, n_i_hi).  n_i_lo = -1
 * sets the shape of the block-step driver's pair launches (block size known
 * only on the device); n_i_lo = -2 sets the driver's small-block shape (a
 * layout-1 shape) and n_i_hi its largest block, i.e. blocks of up to n_i_hi
 * particles take that shape (n_i_hi = 0: no small-block shape).  Later entries do not override earlier ones
 * that cover the same n_i.  NBODY_E_INVAL for an unsupported shape. */
int nbody_tune_set(nbody_ctx *ctx, int64_t n_i_lo, int64_t n_i_hi,
                   const nbody_force_config *cfg);
/* Timing of the pair kernels with HIP events recorded on the context's
 * stream around each launch made by nbody_force and nbody_blockstep.
 * enable = 1 clears the totals and starts timing, 0 stops it, -1 leaves it
 * as it is.  Synchronises, then writes the totals so far to the HOST
 * pointers (each may be NULL): milliseconds in the pair kernel, in the
 * split-reduction kernel, and the number of pair-kernel launches. */
int nbody_profile(nbody_ctx *ctx, int enable, double *force_ms, double *reduce_ms,
                  int64_t *launches);

/* ---- VALU issue rates (diagnostic, not an operation of the paper) --------
 * For callers that state how close the float32-mode pair kernel (Eq. (1))
 * runs to the hardware: its inner loop is made of five vector instruction
 * kinds that do not issue at one rate.  For each kind a grid of
 * waves_per_simd waves per SIMD on the context's device issues only that
 * instruction (eight independent chains per lane, long unrolled runs), and
 * rates[k] (HOST pointer, NBODY_VALU_KINDS doubles) receives the
 * wave-instructions per second of the whole device (event-timed over three
 * launches, at whatever clock the card holds under that load).  Kinds, in
 * order: v_fmac_f32, v_mul_f32, v_add_f64, v_cvt_f32_f64, v_rsq_f32.  A
 * loop's issue-bound time is the sum over kinds of its wave-instructions of
 * that kind divided by the rate.  Uses the context's partial-sum buffer
 * (grown if needed) and synchronises; about 50 ms.
 *   waves_per_simd : 1..8, else NBODY_E_INVAL. */
#define NBODY_VALU_KINDS 5
int nbody_valu_rates(nbody_ctx *ctx, int waves_per_simd, double *rates);

/* Remove every entry (back to the built-in default). */
int nbody_tune_clear(nbody_ctx *ctx);
/* The shape used for n_i (n_i < 0: the block-step shape); `out` is a HOST
 * pointer. */
int nbody_tune_get(nbody_ctx *ctx, int64_t n_i, nbody_force_config *out);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */
