// Context management, errors and scratch buffers of libnbody.so.
#include <cmath>
#include <cstdarg>
#include <new>

#include "common.hpp"

namespace nb {

int fail(nbody_ctx *ctx, int code, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

int hip_check(nbody_ctx *ctx, hipError_t e, const char *what) {
    if (e == hipSuccess) return NBODY_OK;
    (void)hipGetLastError();  // clear the sticky non-fatal error
    return fail(ctx, e == hipErrorOutOfMemory ? NBODY_E_NOMEM : NBODY_E_DEVICE,
                "%s: %s", what, hipGetErrorString(e));
}

int activate(nbody_ctx *ctx) {
    return hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice");
}

// Grow a device buffer to at least `need` bytes (contents not preserved).
int ensure(nbody_ctx *ctx, void **buf, size_t *have, size_t need) {
    if (need <= *have && *buf) return NBODY_OK;
    if (*buf) {
        // the stream may still use the old buffer
        NB_TRY(hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"));
        NB_TRY(hip_check(ctx, hipFree(*buf), "hipFree"));
        *buf = nullptr;
        *have = 0;
    }
    size_t sz = need < 256 ? 256 : need;
    sz = (sz + 4095) & ~size_t(4095);
    NB_TRY(hip_check(ctx, hipMalloc(buf, sz), "hipMalloc"));
    *have = sz;
    return NBODY_OK;
}

__global__ void clear_info_kernel(StepInfo *info) {
    if (threadIdx.x == 0) {
        StepInfo z = {};
        *info = z;
    }
}

int ensure_info(nbody_ctx *ctx) {
    if (ctx->info) return NBODY_OK;
    NB_TRY(hip_check(ctx, hipMalloc(&ctx->info, sizeof(StepInfo)), "hipMalloc"));
    NB_TRY(hip_check(ctx, hipHostMalloc(&ctx->info_host, sizeof(StepInfo), hipHostMallocDefault),
                     "hipHostMalloc"));
    clear_info_kernel<<<1, 64, 0, ctx->stream>>>(ctx->info);
    return hip_check(ctx, hipGetLastError(), "clear_info");
}

hipEvent_t prof_mark(nbody_ctx *ctx) {
    hipEvent_t e = nullptr;
    if (!ctx->prof.pool.empty()) {
        e = ctx->prof.pool.back();
        ctx->prof.pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (hipEventRecord(e, ctx->stream) != hipSuccess) {
        (void)hipGetLastError();
        ctx->prof.pool.push_back(e);
        return nullptr;
    }
    return e;
}

void prof_push(nbody_ctx *ctx, hipEvent_t a, hipEvent_t b, int kind) {
    if (a && b) {
        ctx->prof.pending.push_back({a, b, kind});
    } else {
        if (a) ctx->prof.pool.push_back(a);
        if (b) ctx->prof.pool.push_back(b);
    }
}

void prof_resolve(nbody_ctx *ctx) {
    for (const NbProf::Rec &r : ctx->prof.pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            if (r.kind == 0) {
                ctx->prof.force_ms += ms;
                ctx->prof.launches += 1;
            } else {
                ctx->prof.reduce_ms += ms;
            }
        } else {
            (void)hipGetLastError();
        }
        ctx->prof.pool.push_back(r.a);
        ctx->prof.pool.push_back(r.b);
    }
    ctx->prof.pending.clear();
}

}  // namespace nb

using namespace nb;

extern "C" {

int nbody_version(void) { return 10000; }

int nbody_create(nbody_ctx **out, int device, void *stream) {
    if (!out) return NBODY_E_INVAL;
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return NBODY_E_DEVICE;
    }
    if (device < 0 || device >= count) return NBODY_E_INVAL;
    nbody_ctx *ctx = new (std::nothrow) nbody_ctx();
    if (!ctx) return NBODY_E_NOMEM;
    ctx->device = device;
    ctx->stream = reinterpret_cast<hipStream_t>(stream);
    int rc = activate(ctx);
    if (rc == NBODY_OK) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) ==
                hipSuccess && cus > 0)
            ctx->cus = cus;
        rc = ensure_info(ctx);
        if (rc == NBODY_OK) static_scratch_setup(ctx);
    }
    if (rc != NBODY_OK) {
        nbody_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return NBODY_OK;
}

int nbody_destroy(nbody_ctx *ctx) {
    if (!ctx) return NBODY_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    void *bufs[] = {ctx->jrec, ctx->part, ctx->work, ctx->bs, ctx->adj, ctx->chain, ctx->ens,
                    ctx->info};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (ctx->info_host) (void)hipHostFree(ctx->info_host);
    for (const NbProf::Rec &r : ctx->prof.pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : ctx->prof.pool) (void)hipEventDestroy(e);
    delete ctx;
    return NBODY_OK;
}

int nbody_set_stream(nbody_ctx *ctx, void *stream) {
    if (!ctx) return NBODY_E_INVAL;
    ctx->stream = reinterpret_cast<hipStream_t>(stream);
    return NBODY_OK;
}

const char *nbody_last_error(const nbody_ctx *ctx) {
    return ctx ? ctx->err.c_str() : "null context";
}

int nbody_sync_status(nbody_ctx *ctx) {
    if (!ctx) return NBODY_E_INVAL;
    NB_TRY(activate(ctx));
    NB_TRY(hip_check(ctx, hipMemcpyAsync(ctx->info_host, ctx->info, sizeof(StepInfo),
                                         hipMemcpyDeviceToHost, ctx->stream),
                     "status read"));
    NB_TRY(hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"));
    int32_t st = ctx->info_host->status;
    if (st) {
        // clear the latched bits with a tiny kernel (no memset node)
        clear_info_kernel<<<1, 64, 0, ctx->stream>>>(ctx->info);
        NB_TRY(hip_check(ctx, hipGetLastError(), "clear_info"));
        NB_TRY(hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"));
    }
    if (st & ST_INDEX) return fail(ctx, NBODY_E_INVAL, "active index out of range");
    if (st & ST_NONFINITE) return fail(ctx, NBODY_E_NONFINITE, "non-finite value in a kernel");
    if (st & ST_RANGE) return fail(ctx, NBODY_E_RANGE, "time step below dt_min");
    return NBODY_OK;
}

static int shape_ok(const nbody_force_config *c) {
    if (!c) return 0;
    if (c->tile < 1 || c->min_j_wave < 1 || c->target_groups < 1) return 0;
    if (c->target_groups > (1 << 20)) return 0;
    if (c->layout == 1) {
        // j-lane kernel: float64 records, 1/2/4/8 i-particles, 1/2/4 waves
        if (c->rep != REP_F64) return 0;
        if (c->i_per_lane != 1 && c->i_per_lane != 2 && c->i_per_lane != 4 && c->i_per_lane != 8)
            return 0;
        return c->waves == 1 || c->waves == 2 || c->waves == 4;
    }
    if (c->layout != 0) return 0;
    if (c->rep < REP_F64 || c->rep > REP_F64V) return 0;
    if (c->i_per_lane != 1 && c->i_per_lane != 2 && c->i_per_lane != 4) return 0;
    if (c->waves != 1 && c->waves != 2 && c->waves != 4 && c->waves != 8) return 0;
    if (c->i_per_lane == 4 && c->waves == 8) return 0;
    return 1;
}

int nbody_tune_set(nbody_ctx *ctx, int64_t n_i_lo, int64_t n_i_hi,
                   const nbody_force_config *cfg) {
    if (!ctx) return NBODY_E_INVAL;
    if (!shape_ok(cfg)) return fail(ctx, NBODY_E_INVAL, "nbody_tune_set: unsupported shape");
    if (n_i_lo >= 0 && n_i_hi <= n_i_lo)
        return fail(ctx, NBODY_E_INVAL, "nbody_tune_set: empty range");
    if (n_i_lo == -2 && (cfg->layout != 1 || n_i_hi < 0))
        return fail(ctx, NBODY_E_INVAL,
                    "nbody_tune_set: the small-block entry needs layout 1 and n_i_hi >= 0");
    TuneEntry e;
    e.n_i_lo = n_i_lo == -2 ? -2 : (n_i_lo < 0 ? -1 : n_i_lo);
    e.n_i_hi = n_i_hi;
    e.shape.rep = cfg->rep;
    e.shape.it = cfg->i_per_lane;
    e.shape.waves = cfg->waves;
    e.shape.tile = cfg->tile;
    e.shape.min_j_wave = cfg->min_j_wave;
    e.shape.target_groups = cfg->target_groups;
    e.shape.layout = cfg->layout;
    ctx->tune.push_back(e);
    return NBODY_OK;
}

int nbody_profile(nbody_ctx *ctx, int enable, double *force_ms, double *reduce_ms,
                  int64_t *launches) {
    if (!ctx) return NBODY_E_INVAL;
    NB_TRY(activate(ctx));
    NB_TRY(hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"));
    prof_resolve(ctx);
    if (enable == 1) {
        ctx->prof.on = true;
        ctx->prof.force_ms = ctx->prof.reduce_ms = 0;
        ctx->prof.launches = 0;
    } else if (enable == 0) {
        ctx->prof.on = false;
    }
    if (force_ms) *force_ms = ctx->prof.force_ms;
    if (reduce_ms) *reduce_ms = ctx->prof.reduce_ms;
    if (launches) *launches = ctx->prof.launches;
    return NBODY_OK;
}

int nbody_ensemble_set(nbody_ctx *ctx, const nbody_ensemble_config *cfg) {
    if (!ctx || !cfg) return NBODY_E_INVAL;
    if (cfg->groups_per_cu < 1 || cfg->groups_per_cu > 8 || cfg->max_team < 1 ||
        cfg->max_team > 4096 || !(cfg->step_us >= 0) || !(cfg->barrier_us >= 0) ||
        !(cfg->barrier_group_us >= 0) || std::isinf(cfg->barrier_group_us) ||
        !(cfg->group_rate > 0) || std::isinf(cfg->step_us) || std::isinf(cfg->barrier_us) ||
        std::isinf(cfg->group_rate) || !(cfg->steps_coef > 0) || !(cfg->steps_exp >= 0) ||
        !(cfg->steps_exp < 3) || std::isinf(cfg->steps_coef) || !(cfg->tile_us >= 0) ||
        std::isinf(cfg->tile_us) || !(cfg->block_coef > 0) || std::isinf(cfg->block_coef) ||
        !(cfg->block_exp >= 0) || !(cfg->block_exp <= 1))
        return fail(ctx, NBODY_E_INVAL, "nbody_ensemble_set: bad values");
    if (!find_variant(cfg->waves, cfg->j_tile, cfg->i_per_lane))
        return fail(ctx, NBODY_E_INVAL,
                    "nbody_ensemble_set: no compiled shape with %d waves, tile %d, %d per lane",
                    cfg->waves, cfg->j_tile, cfg->i_per_lane);
    ctx->ens_cfg = *cfg;
    return NBODY_OK;
}

int nbody_ensemble_get(nbody_ctx *ctx, nbody_ensemble_config *cfg) {
    if (!ctx || !cfg) return NBODY_E_INVAL;
    *cfg = ctx->ens_cfg;
    return NBODY_OK;
}

int nbody_ensemble_info(nbody_ctx *ctx, int32_t *grid, int32_t *teams) {
    if (!ctx) return NBODY_E_INVAL;
    if (grid) *grid = ctx->ens_last_grid;
    if (teams) *teams = ctx->ens_last_teams;
    return NBODY_OK;
}

int nbody_ensemble_timing(nbody_ctx *ctx, int32_t n_clusters, double *seconds,
                          int32_t *groups) {
    if (!ctx) return NBODY_E_INVAL;
    if (n_clusters != (int32_t)ctx->ens_last_seconds.size())
        return fail(ctx, NBODY_E_INVAL, "nbody_ensemble_timing: %d clusters in the last run",
                    (int)ctx->ens_last_seconds.size());
    for (int c = 0; c < n_clusters; ++c) {
        if (seconds) seconds[c] = ctx->ens_last_seconds[c];
        if (groups) groups[c] = ctx->ens_last_groups[c];
    }
    return NBODY_OK;
}

int nbody_tune_clear(nbody_ctx *ctx) {
    if (!ctx) return NBODY_E_INVAL;
    ctx->tune.clear();
    return NBODY_OK;
}

int nbody_tune_get(nbody_ctx *ctx, int64_t n_i, nbody_force_config *out) {
    if (!ctx || !out) return NBODY_E_INVAL;
    ForceShape s;
    if (n_i == -2) {
        int64_t jl_max = 0;
        s = dynamic_small_shape(ctx, 0, &jl_max);
    } else {
        s = n_i < 0 ? dynamic_shape(ctx, 0) : pick_shape(ctx, n_i, 0);
    }
    out->rep = s.rep;
    out->i_per_lane = s.it;
    out->waves = s.waves;
    out->tile = s.tile;
    out->min_j_wave = s.min_j_wave;
    out->target_groups = s.target_groups;
    out->layout = s.layout;
    return NBODY_OK;
}

}  // extern "C"
