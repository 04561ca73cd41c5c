// Internal declarations shared by the HIP sources of libnbody.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/nbody.h"
#include "records.hpp"

namespace nb {

// Step bookkeeping kept in device memory so that a block step needs no
// host round trip (the scheduler writes it, the other kernels read it).
struct StepInfo {
    double t_next;        // time of the current block
    double t_end;         // no block beyond this time is executed
    int64_t n_i;          // size of the current block (0 once done)
    int64_t done;         // 1 once the next block would pass t_end
    int64_t steps;        // block steps executed since the last reset
    int64_t interactions; // sum of n_i * n over those steps
    double rest_min;      // min of t + dt outside the current block (driver)
    int32_t status;       // latched NBODY_E_* bits (see status_bits)
    uint32_t ticket0;     // arrival counters of the last-block reductions
    uint32_t ticket1;
    uint32_t ticket2;
    int32_t pad;
};

enum : int32_t { ST_RANGE = 1, ST_NONFINITE = 2, ST_INDEX = 4 };

// Tunable launch shape of the pair kernels.
struct ForceShape {
    int rep = REP_F64;     // form of the relative coordinates (REP_*)
    int it = 1;            // i-particles per lane (i-lanes: 1, 2, 4; j-lanes: 1, 2, 4, 8)
    int waves = 4;         // waves per workgroup (split j inside the group)
    int tile = 128;        // j per float32 inner sum before folding
    int min_j_wave = 64;   // smallest j range per wave when splitting j
    int target_groups = 4096;  // workgroups to aim for before splitting j
    int layout = 0;        // 0: one i per lane (force_kernel); 1: one j per lane
                           // (force_jl_kernel), the `it` i-particles wave-uniform
};

struct TuneEntry {
    int64_t n_i_lo, n_i_hi;  // applies to n_i in [lo, hi)
    ForceShape shape;
};

}  // namespace nb

struct NbProf {
    bool on = false;
    std::vector<hipEvent_t> pool;
    // pending (start, stop, kind) triples: kind 0 = pair kernel, 1 = reduction
    struct Rec {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<Rec> pending;
    double force_ms = 0, reduce_ms = 0;
    int64_t launches = 0;
};

struct nbody_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int cus = 256;
    // scratch (grown on demand, owned by the context)
    void *jrec = nullptr;
    size_t jrec_bytes = 0;
    void *part = nullptr;
    size_t part_bytes = 0;
    void *work = nullptr;  // scheduler / reduction scratch
    size_t work_bytes = 0;
    void *adj = nullptr;  // adjoint source records
    size_t adj_bytes = 0;
    void *chain = nullptr;  // differentiable shared-step run workspace
    size_t chain_bytes = 0;
    void *ens = nullptr;  // ensemble tables and team scratch
    size_t ens_bytes = 0;
    void *static_scratch = nullptr;  // this device's copy of the static scratch
    int static_scratch_rc = 0;       // hipGetSymbolAddress status (hipError_t)
    nbody_ensemble_config ens_cfg = {2, 64, 30.0, 15.0, 0.5, 2.0e9, 247.0, 0.35, 4, 256, 2,
                                      0.0, 0.20, 0.81};
    int ens_last_grid = 0;
    int ens_last_teams = 0;
    std::vector<double> ens_last_seconds;  // per cluster, last ensemble launch
    std::vector<int> ens_last_groups;
    nb::StepInfo *info = nullptr;  // device
    nb::StepInfo *info_host = nullptr;  // pinned host mirror
    // block-step buffers
    void *bs = nullptr;
    size_t bs_bytes = 0;
    std::vector<nb::TuneEntry> tune;
    NbProf prof;
};

namespace nb {

int fail(nbody_ctx *ctx, int code, const char *fmt, ...);
int hip_check(nbody_ctx *ctx, hipError_t e, const char *what);
int ensure(nbody_ctx *ctx, void **buf, size_t *have, size_t need);
int ensure_info(nbody_ctx *ctx);
int activate(nbody_ctx *ctx);
// Event timing (active when ctx->prof.on): mark() records an event on the
// stream; resolve() (stream already synchronised) accumulates the pairs.
hipEvent_t prof_mark(nbody_ctx *ctx);
void prof_push(nbody_ctx *ctx, hipEvent_t a, hipEvent_t b, int kind);
void prof_resolve(nbody_ctx *ctx);

ForceShape pick_shape(const nbody_ctx *ctx, int64_t n_i, int64_t n_j);
// Compiled launch shapes of the ensemble kernel (ensemble.hip): the one with
// w waves per group, j tiles of `tile` records and `it` slots per lane, or
// null.
struct EnsVariant;
const EnsVariant *find_variant(int w, int tile, int it);

// Pair-arithmetic mode (ACC_* in pairs.hpp) of the NBODY_ACC_* flags, and
// the shape a mode runs in: float64 pair terms need float64 records and take
// at most two i-particles per lane.
int acc_mode(uint32_t flags);
ForceShape shape_for(ForceShape s, int acc);

// Pair-sum launch used by nbody_force and the block-step driver.
//   n_i_dev != nullptr: the block size is read on the device (at most
//   n_i_cap); otherwise n_i is used.  Outputs have component stride
//   out_stride (n_i_cap in the device-count case).
struct ForceCall {
    ForceShape shape;
    const JRec *jrec = nullptr;
    int64_t n_j = 0;
    const double *pos = nullptr, *vel = nullptr;  // i side (stride n_j)
    const int32_t *active = nullptr;
    int64_t n_i = 0;
    const int64_t *n_i_dev = nullptr;
    int64_t n_i_cap = 0;
    double eps2 = 0;
    double *acc = nullptr, *jerk = nullptr, *pot = nullptr;
    int64_t out_stride = 0;
    int mode = 0;  // accumulation, ACC_* (pairs.hpp)
    // Device-counted launches only: blocks of at most jl_max particles take
    // the j-lane kernel in shape jl_shape (0: none).
    ForceShape jl_shape;
    int64_t jl_max = 0;
    // Caller-provided partial-sum buffer (static scratch): when set, the j
    // split is capped at max_splits so that the partials fit in part_cap
    // bytes, nothing is allocated and no timing events are recorded.
    void *part_buf = nullptr;
    size_t part_cap = 0;
    int max_splits = 0;  // 0: the library's limit
};
int launch_force(nbody_ctx *ctx, const ForceCall &c);
int launch_pack(nbody_ctx *ctx, int rep, int64_t n, const double *pos,
                const double *vel, const double *mass, JRec *out);
// Shape used by the block-step driver (block size known only on the device).
ForceShape dynamic_shape(const nbody_ctx *ctx, int64_t n);
// The driver's small-block shape (j-lane layout) and the largest block it
// takes (*jl_max = 0: none) for a system of n particles.
ForceShape dynamic_small_shape(const nbody_ctx *ctx, int64_t n, int64_t *jl_max);
// Address of the static scratch array on the context's device (called by
// nbody_create with that device current; sets static_scratch(_rc)).
void static_scratch_setup(nbody_ctx *ctx);

}  // namespace nb

#define NB_TRY(expr)                 \
    do {                             \
        int _rc = (expr);            \
        if (_rc != NBODY_OK) return _rc; \
    } while (0)
