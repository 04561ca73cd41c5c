// j-particle record forms of the pair kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nb {

// Packed j-particle records read by the pair kernels through the scalar
// data path: one 64-byte record per particle (whole-record scalar loads), so
// the record lands in SGPRs that every lane of a wave reads as operands.
// The mass is float32 in every form (it enters the float32 products); the
// float64 form also carries it in float64 for float64 pair terms.  The
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
    double md;  // the mass in float64
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
        r.md = m;
        *out = r;
    }
}

}  // namespace nb
