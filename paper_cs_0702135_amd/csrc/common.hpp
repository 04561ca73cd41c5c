// Internal declarations shared by the HIP sources of libnbody.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/nbody.h"

namespace nb {

// Packed j-particle records read by the pair kernels through the scalar
// data path: one 64-byte record per particle (whole-record scalar loads), so
// the record lands in SGPRs that every lane of a wave reads as operands.
// The mass is float32 in every form (it only enters float32 products).  The
// form of the relative coordinates r = x_j - x_i, w = v_j - v_i is a launch
// choice (ForceShape::rep):
//   REP_F64  positions and velocities in float64; r and w are float64
//            differences rounded once to float32 (v_add_f64 + v_cvt_f32_f64);
//   REP_FF   float-float pairs (hi = float32 rounding, lo = float32 rounding
//            of the remainder, ~48 bits); r = (hi_j - hi_i) + (lo_j - lo_i),
//            float32 instructions only, same accuracy as REP_F64 to within
//            one float32 rounding;
//   REP_F64V float64 positions as REP_F64, float32 velocities (w is a plain
//            float32 difference: jerk loses ~u |v| / |w| relative accuracy).
enum { REP_F64 = 0, REP_FF = 1, REP_F64V = 2 };

struct __attribute__((aligned(64))) RecF64 {
    double x, y, z;
    float m, pad0;
    double u, v, w;
    double pad1;
};
struct __attribute__((aligned(64))) RecFF {
    float xh, yh, zh, m;
    float uh, vh, wh, pad0;
    float xl, yl, zl, pad1;
    float ul, vl, wl, pad2;
};
struct __attribute__((aligned(64))) RecF64V {
    double x, y, z;
    float m, u, v, w;
    float pad[6];
};
static_assert(sizeof(RecF64) == 64 && sizeof(RecFF) == 64 && sizeof(RecF64V) == 64,
              "records are one 64-byte line");
typedef RecF64 JRec;  // storage unit of the record buffers (64 bytes)

__host__ __device__ inline void split_ff(double x, float &hi, float &lo) {
    hi = (float)x;
    lo = (float)(x - (double)hi);
}

// Write particle data as a record of form `rep` (64 bytes at `out`).
__device__ inline void store_rec(int rep, JRec *out, double x, double y, double z, double u,
                                 double v, double w, double m) {
    if (rep == REP_FF) {
        RecFF r;
        split_ff(x, r.xh, r.xl);
        split_ff(y, r.yh, r.yl);
        split_ff(z, r.zh, r.zl);
        split_ff(u, r.uh, r.ul);
        split_ff(v, r.vh, r.vl);
        split_ff(w, r.wh, r.wl);
        r.m = (float)m;
        r.pad0 = r.pad1 = r.pad2 = 0.0f;
        *reinterpret_cast<RecFF *>(out) = r;
    } else if (rep == REP_F64V) {
        RecF64V r;
        r.x = x;
        r.y = y;
        r.z = z;
        r.m = (float)m;
        r.u = (float)u;
        r.v = (float)v;
        r.w = (float)w;
        for (int q = 0; q < 6; ++q) r.pad[q] = 0.0f;
        *reinterpret_cast<RecF64V *>(out) = r;
    } else {
        RecF64 r;
        r.x = x;
        r.y = y;
        r.z = z;
        r.m = (float)m;
        r.pad0 = 0.0f;
        r.u = u;
        r.v = v;
        r.w = w;
        r.pad1 = 0.0;
        *out = r;
    }
}

// Step bookkeeping kept in device memory so that a block step needs no
// host round trip (the scheduler writes it, the other kernels read it).
struct StepInfo {
    double t_next;        // time of the current block
    double t_end;         // no block beyond this time is executed
    int64_t n_i;          // size of the current block (0 once done)
    int64_t done;         // 1 once the next block would pass t_end
    int64_t steps;        // block steps executed since the last reset
    int64_t interactions; // sum of n_i * n over those steps
    int32_t status;       // latched NBODY_E_* bits (see status_bits)
    uint32_t ticket0;     // arrival counters of the last-block reductions
    uint32_t ticket1;
    uint32_t ticket2;
    int32_t pad;
};

enum : int32_t { ST_RANGE = 1, ST_NONFINITE = 2, ST_INDEX = 4 };

// Tunable launch shape of the pair kernel.
struct ForceShape {
    int rep = REP_F64;     // form of the relative coordinates (REP_*)
    int it = 1;            // i-particles per lane (1 or 2)
    int waves = 4;         // waves per workgroup (split j inside the group)
    int tile = 128;        // j per float32 inner sum before folding
    int min_j_wave = 64;   // smallest j range per wave when splitting j
    int target_groups = 4096;  // workgroups to aim for before splitting j
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
    bool ds = false;
};
int launch_force(nbody_ctx *ctx, const ForceCall &c);
int launch_pack(nbody_ctx *ctx, int rep, int64_t n, const double *pos,
                const double *vel, const double *mass, JRec *out);
// Shape used by the block-step driver (block size known only on the device).
ForceShape dynamic_shape(const nbody_ctx *ctx, int64_t n);

}  // namespace nb

#define NB_TRY(expr)                 \
    do {                             \
        int _rc = (expr);            \
        if (_rc != NBODY_OK) return _rc; \
    } while (0)
