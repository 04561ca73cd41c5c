// Differentiable shared-step Hermite run, forward and adjoint, orchestrated
// natively: the chain that the per-step entry points compose (Section 2
// predictor, pair sums at the predicted state, corrector with the step held
// fixed), with its state checkpointed every few steps so that the adjoint
// pass recomputes one segment at a time.
//
// Forward: a, k = pair sums at (x0, v0); then for each step: x_p, v_p =
// predict(x, v, a, k; h); a_1, k_1 = pair sums at (x_p, v_p); x, v =
// correct(...); a, k = a_1, k_1.  The state (x, v, a, k) before every
// segment of ckpt_every steps is copied to the checkpoint buffer.
//
// Adjoint: from the cotangents of the final (x, v, a, k), for each segment
// from the last: restore its checkpoint, recompute its steps keeping every
// predicted state, then for each step in reverse apply the transposes of
// the corrector, of the pair sums at the predicted state and of the
// predictor (the cotangents of a, k after a step pass to the new force, and
// those of the predicted state return to the step's input); finally the
// transpose of the initial pair sums.  Each call is the library's own entry
// point, so the result equals that of chaining those entry points by hand.
#include <cstring>
#include <utility>

#include "common.hpp"

namespace nb {

__global__ void chain_fill_kernel(double *p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static int chain_fill(nbody_ctx *ctx, double *p, int64_t n, double v) {
    if (n <= 0) return NBODY_OK;
    int64_t g = (n + 255) / 256;
    if (g > 16 * (int64_t)ctx->cus) g = 16 * (int64_t)ctx->cus;
    chain_fill_kernel<<<(unsigned)g, 256, 0, ctx->stream>>>(p, n, v);
    return hip_check(ctx, hipGetLastError(), "chain_fill_kernel");
}

static int chain_copy(nbody_ctx *ctx, double *dst, const double *src, int64_t n) {
    return hip_check(ctx, hipMemcpyAsync(dst, src, (size_t)n * sizeof(double),
                                         hipMemcpyDeviceToDevice, ctx->stream),
                     "copy");
}

static int chain_args(nbody_ctx *ctx, int64_t n, const double *m, double eps2, double h,
                      int64_t n_steps, int64_t ckpt_every, uint32_t flags) {
    if (n < 1 || n > 0x7fffffffLL || !m || !(eps2 >= 0.0) || std::isinf(eps2) ||
        !(h > 0.0) || std::isinf(h) || n_steps < 0 || ckpt_every < 1)
        return fail(ctx, NBODY_E_INVAL, "shared run: bad arguments");
    if (flags & ~NBODY_ACC_DS) return fail(ctx, NBODY_E_INVAL, "shared run: unknown flags");
    return NBODY_OK;
}

// One step of the forward chain on state (x, v, a, k) in place; the
// predicted state goes to (xp, vp), the new pair sums through (a1, k1).
static int chain_step(nbody_ctx *ctx, int64_t n, const double *m, double eps2, double h,
                      uint32_t flags, const double *t0, double *tw, double *dtv, double *x,
                      double *v, double *a, double *k, double *xp, double *vp, double *a1,
                      double *k1) {
    NB_TRY(nbody_predict(ctx, n, h, t0, x, v, a, k, xp, vp));
    NB_TRY(nbody_force(ctx, nullptr, n, xp, vp, m, n, eps2, a1, k1, nullptr, flags));
    return nbody_correct(ctx, n, n, nullptr, xp, vp, a1, k1, 1.0, h, h, 1, tw, dtv, x, v, a, k);
}

}  // namespace nb

using namespace nb;

extern "C" {

int nbody_shared_run(nbody_ctx *ctx, int64_t n, const double *m, double eps2, double h,
                     int64_t n_steps, int64_t ckpt_every, const double *x0, const double *v0,
                     double *x, double *v, double *a, double *k, double *ckpt, uint32_t flags) {
    if (!ctx) return NBODY_E_INVAL;
    NB_TRY(chain_args(ctx, n, m, eps2, h, n_steps, ckpt_every, flags));
    if (!x0 || !v0 || !x || !v || !a || !k) return fail(ctx, NBODY_E_INVAL, "shared run: null array");
    NB_TRY(activate(ctx));
    const int64_t n3 = 3 * n;
    // workspace: t0 (zeros), t (corrector's clock), dt (h), xp, vp, a1, k1
    NB_TRY(ensure(ctx, &ctx->chain, &ctx->chain_bytes, (size_t)(3 * n + 4 * n3) * sizeof(double)));
    double *t0 = (double *)ctx->chain, *tw = t0 + n, *dtv = tw + n;
    double *xp = dtv + n, *vp = xp + n3, *a1 = vp + n3, *k1 = a1 + n3;
    NB_TRY(chain_fill(ctx, t0, 2 * n, 0.0));
    NB_TRY(chain_fill(ctx, dtv, n, h));
    NB_TRY(chain_copy(ctx, x, x0, n3));
    NB_TRY(chain_copy(ctx, v, v0, n3));
    NB_TRY(nbody_force(ctx, nullptr, n, x0, v0, m, n, eps2, a, k, nullptr, flags));
    for (int64_t s = 0; s < n_steps; ++s) {
        if (ckpt && s % ckpt_every == 0) {
            double *c = ckpt + (s / ckpt_every) * 4 * n3;
            NB_TRY(chain_copy(ctx, c, x, n3));
            NB_TRY(chain_copy(ctx, c + n3, v, n3));
            NB_TRY(chain_copy(ctx, c + 2 * n3, a, n3));
            NB_TRY(chain_copy(ctx, c + 3 * n3, k, n3));
        }
        NB_TRY(chain_step(ctx, n, m, eps2, h, flags, t0, tw, dtv, x, v, a, k, xp, vp, a1, k1));
    }
    return NBODY_OK;
}

int nbody_shared_run_adjoint(nbody_ctx *ctx, int64_t n, const double *m, double eps2, double h,
                             int64_t n_steps, int64_t ckpt_every, const double *x0,
                             const double *v0, const double *ckpt, const double *x_bar,
                             const double *v_bar, const double *a_bar, const double *k_bar,
                             double *x0_bar, double *v0_bar, double *m_bar, uint32_t flags) {
    if (!ctx) return NBODY_E_INVAL;
    NB_TRY(chain_args(ctx, n, m, eps2, h, n_steps, ckpt_every, flags));
    if (!x0 || !v0 || (n_steps > 0 && !ckpt) || !x_bar || !v_bar || !a_bar || !k_bar ||
        !x0_bar || !v0_bar || !m_bar)
        return fail(ctx, NBODY_E_INVAL, "shared run adjoint: null array");
    NB_TRY(activate(ctx));
    const int64_t n3 = 3 * n;
    const int64_t seg = ckpt_every < n_steps ? ckpt_every : (n_steps > 0 ? n_steps : 1);
    // workspace: t0, t, dt | state x v a k | a1 k1 | xp vp per step of a
    // segment | two sets of cotangents (x, v, a, k), each contiguous | the
    // predicted state's cotangents xpb, vpb
    const size_t doubles = (size_t)(3 * n + 4 * n3 + 2 * n3 + 2 * n3 * seg + 10 * n3);
    NB_TRY(ensure(ctx, &ctx->chain, &ctx->chain_bytes, doubles * sizeof(double)));
    double *t0 = (double *)ctx->chain, *tw = t0 + n, *dtv = tw + n;
    double *xs = dtv + n, *vs = xs + n3, *as = vs + n3, *ks = as + n3;
    double *a1 = ks + n3, *k1 = a1 + n3;
    double *xps = k1 + n3, *vps = xps + n3 * seg;
    double *cur = vps + n3 * seg, *nxt = cur + 4 * n3;  // x v a k cotangents
    double *xpb = nxt + 4 * n3, *vpb = xpb + n3;
    NB_TRY(chain_fill(ctx, t0, 2 * n, 0.0));
    NB_TRY(chain_fill(ctx, dtv, n, h));
    NB_TRY(chain_copy(ctx, cur, x_bar, n3));
    NB_TRY(chain_copy(ctx, cur + n3, v_bar, n3));
    NB_TRY(chain_copy(ctx, cur + 2 * n3, a_bar, n3));
    NB_TRY(chain_copy(ctx, cur + 3 * n3, k_bar, n3));
    NB_TRY(chain_fill(ctx, m_bar, n, 0.0));
    const int64_t n_seg = (n_steps + ckpt_every - 1) / ckpt_every;
    for (int64_t sg = n_seg - 1; sg >= 0; --sg) {
        const int64_t s0 = sg * ckpt_every;
        const int64_t len = (s0 + ckpt_every < n_steps ? s0 + ckpt_every : n_steps) - s0;
        const double *c = ckpt + sg * 4 * n3;
        NB_TRY(chain_copy(ctx, xs, c, 4 * n3));  // x v a k are contiguous in a checkpoint
        for (int64_t j = 0; j < len; ++j)
            NB_TRY(chain_step(ctx, n, m, eps2, h, flags, t0, tw, dtv, xs, vs, as, ks,
                              xps + j * n3, vps + j * n3, a1, k1));
        for (int64_t j = len - 1; j >= 0; --j) {
            // cur: cotangents of the step's outputs (x1, v1, a1, k1); the
            // corrector's transpose adds into cur's a, k, which then are
            // those of the step's new pair sums; nxt collects the cotangents
            // of the step's input state
            NB_TRY(chain_fill(ctx, nxt, 4 * n3, 0.0));
            NB_TRY(chain_fill(ctx, xpb, 2 * n3, 0.0));  // xpb, vpb
            NB_TRY(nbody_correct_adjoint(ctx, n, h, cur, cur + n3, xpb, vpb, nxt + 2 * n3,
                                         nxt + 3 * n3, cur + 2 * n3, cur + 3 * n3));
            NB_TRY(nbody_force_adjoint(ctx, n, xps + j * n3, vps + j * n3, m, eps2, cur + 2 * n3,
                                       cur + 3 * n3, nullptr, xpb, vpb, m_bar,
                                       flags | NBODY_ADJ_ACCUMULATE));
            NB_TRY(nbody_predict_adjoint(ctx, n, h, xpb, vpb, nxt, nxt + n3, nxt + 2 * n3,
                                         nxt + 3 * n3));
            std::swap(cur, nxt);
        }
    }
    // the initial pair sums at (x0, v0)
    NB_TRY(nbody_force_adjoint(ctx, n, x0, v0, m, eps2, cur + 2 * n3, cur + 3 * n3, nullptr, cur,
                               cur + n3, m_bar, flags | NBODY_ADJ_ACCUMULATE));
    NB_TRY(chain_copy(ctx, x0_bar, cur, n3));
    return chain_copy(ctx, v0_bar, cur + n3, n3);
}

}  // extern "C"
