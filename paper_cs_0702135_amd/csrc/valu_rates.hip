// Issue rates of the VALU instruction kinds that make up the pair kernel's
// inner loop (a diagnostic, not an operation of the paper).
//
// The float32-mode pair kernel executes, per interaction, 15 v_fmac_f32,
// 6 v_mul_f32 and one v_rsq_f32 for the pair arithmetic and 6 v_add_f64 plus
// 6 v_cvt_f32_f64 that form the relative coordinates in float64; nothing else
// in its loop is a vector instruction.  Those kinds do not all issue at one
// rate (the float64 adds and the conversions take more cycles per wave than
// float32 arithmetic, the reciprocal square root more still), so a float32
// FLOP/s peak alone does not say how close the loop runs to the hardware.
// This measures each kind on the device it runs on: every lane keeps eight
// independent chains, and a grid of W waves per SIMD issues nothing but that
// kind in long unrolled runs (written as inline assembly so that exactly that
// instruction is issued), timed with events over three launches.  The
// loop's issue bound is then the sum over kinds of its wave-instructions of
// that kind divided by the kind's rate.
#include "common.hpp"

namespace nb {

constexpr int kRateChains = 8;
constexpr int kRateUnroll = 16;
constexpr int kRateIters = 2000;

template <int KIND>
__global__ __launch_bounds__(256) void valu_rate_kernel(float *__restrict__ outf,
                                                        double *__restrict__ outd, float a,
                                                        float b, double e) {
    float f[kRateChains];
    double d[kRateChains];
#pragma unroll
    for (int c = 0; c < kRateChains; ++c) {
        f[c] = 1.0f + 1.0e-3f * (float)(threadIdx.x + c);
        d[c] = 1.0 + 1.0e-3 * (double)(threadIdx.x + c);
    }
    for (int it = 0; it < kRateIters; ++it) {
#pragma unroll
        for (int u = 0; u < kRateUnroll; ++u) {
#pragma unroll
            for (int c = 0; c < kRateChains; ++c) {
                if (KIND == 0) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(f[c]) : "v"(a), "v"(b));
                if (KIND == 1) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(f[c]) : "v"(a));
                if (KIND == 2) asm volatile("v_add_f64 %0, %0, %1" : "+v"(d[c]) : "v"(e));
                if (KIND == 3) asm volatile("v_cvt_f32_f64 %0, %1" : "+v"(f[c]) : "v"(d[c]));
                if (KIND == 4)
                    asm volatile("v_rsq_f32 %0, %1"
                                 : "+v"(f[c])
                                 : "v"(f[(c + 1) % kRateChains]));
            }
        }
    }
    float sf = 0.0f;
    double sd = 0.0;
#pragma unroll
    for (int c = 0; c < kRateChains; ++c) {
        sf += f[c];
        sd += d[c];
    }
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    outf[g] = sf;
    outd[g] = sd;
}

}  // namespace nb

using namespace nb;

extern "C" int nbody_valu_rates(nbody_ctx *ctx, int waves_per_simd, double *rates) {
    if (!ctx) return NBODY_E_INVAL;
    if (!rates || waves_per_simd < 1 || waves_per_simd > 8)
        return fail(ctx, NBODY_E_INVAL, "nbody_valu_rates: waves_per_simd must be 1..8");
    NB_TRY(activate(ctx));
    // 256-thread groups of four waves: waves_per_simd groups per CU
    const int64_t blocks = (int64_t)ctx->cus * waves_per_simd;
    const int64_t lanes = blocks * 256;
    NB_TRY(ensure(ctx, &ctx->part, &ctx->part_bytes,
                  (size_t)lanes * (sizeof(float) + sizeof(double))));
    double *outd = (double *)ctx->part;
    float *outf = (float *)(outd + lanes);
    typedef void (*rate_fn)(float *, double *, float, float, double);
    const rate_fn fns[NBODY_VALU_KINDS] = {valu_rate_kernel<0>, valu_rate_kernel<1>,
                                           valu_rate_kernel<2>, valu_rate_kernel<3>,
                                           valu_rate_kernel<4>};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    NB_TRY(hip_check(ctx, hipEventCreate(&e0), "event"));
    int rc = hip_check(ctx, hipEventCreate(&e1), "event");
    const int reps = 3;
    const double instr = (double)blocks * 4.0 * kRateIters * kRateUnroll * kRateChains * reps;
    for (int k = 0; k < NBODY_VALU_KINDS && rc == NBODY_OK; ++k) {
        // one untimed launch, then `reps` timed back to back
        for (int r = 0; r <= reps && rc == NBODY_OK; ++r) {
            if (r == 1) rc = hip_check(ctx, hipEventRecord(e0, ctx->stream), "event");
            hipLaunchKernelGGL(fns[k], dim3((unsigned)blocks), dim3(256), 0, ctx->stream, outf,
                               outd, 1.0f, 0.0f, 0.0);
            if (rc == NBODY_OK) rc = hip_check(ctx, hipGetLastError(), "valu_rate_kernel");
        }
        if (rc == NBODY_OK) rc = hip_check(ctx, hipEventRecord(e1, ctx->stream), "event");
        if (rc == NBODY_OK) rc = hip_check(ctx, hipEventSynchronize(e1), "sync");
        float ms = 0.0f;
        if (rc == NBODY_OK) rc = hip_check(ctx, hipEventElapsedTime(&ms, e0, e1), "event time");
        if (rc == NBODY_OK) rates[k] = ms > 0.0f ? instr / (ms * 1e-3) : 0.0;
    }
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}
