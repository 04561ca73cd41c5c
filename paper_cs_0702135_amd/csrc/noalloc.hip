// Pair sums that allocate nothing: nbody_force_noalloc.
//
// The same pair kernels as nbody_force (force.hip), with the j records and
// the split partial sums placed in a file-scope static device array instead
// of context-owned buffers grown with hipMalloc.  Each device holds its own
// copy of the array; its address is taken once per device with
// hipGetSymbolAddress when a context is created on it (the array's name is
// only a host-side stand-in, never a device address).  Every call on a
// device shares that device's array, so calls that overlap on one device
// (on different streams or from different threads) race.  Nothing in the
// array needs clearing between calls: the records are rewritten by each
// call and every partial sum a call reads is written by the same call.
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "pairs.hpp"

namespace nb {

constexpr size_t kStaticBytes = (size_t)NBODY_NOALLOC_SCRATCH_MB << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];
static int g_scratch_rc[kMaxDevices];
static bool g_scratch_done[kMaxDevices];

void static_scratch_setup(nbody_ctx *ctx) {
    ctx->static_scratch = nullptr;
    const int dev = ctx->device;
    if (dev < 0 || dev >= kMaxDevices) {
        ctx->static_scratch_rc = (int)hipErrorInvalidDevice;
        return;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
        g_scratch_ptr[dev] = p;
        g_scratch_rc[dev] = (int)e;
        g_scratch_done[dev] = true;
    }
    ctx->static_scratch = g_scratch_ptr[dev];
    ctx->static_scratch_rc = g_scratch_rc[dev];
}

}  // namespace nb

using namespace nb;

extern "C" int nbody_force_noalloc(nbody_ctx *ctx, const int32_t *active_idx, int64_t n_i,
                                   const double *pos, const double *vel, const double *mass,
                                   int64_t n_j, double eps2, double *acc, double *jerk,
                                   double *pot, uint32_t flags) {
    if (!ctx) return NBODY_E_INVAL;
    if (n_i < 0 || n_j < 1 || n_i > 0x7fffffffLL || n_j > 0x7fffffffLL)
        return fail(ctx, NBODY_E_INVAL, "nbody_force_noalloc: bad sizes n_i=%lld n_j=%lld",
                    (long long)n_i, (long long)n_j);
    if (!(eps2 >= 0.0) || std::isinf(eps2))
        return fail(ctx, NBODY_E_INVAL, "nbody_force_noalloc: eps2 must be finite and >= 0");
    if (flags & ~NBODY_ACC_DS)
        return fail(ctx, NBODY_E_INVAL, "nbody_force_noalloc: unknown flags");
    if (!pos || !vel || !mass || (n_i > 0 && (!acc || !jerk)))
        return fail(ctx, NBODY_E_INVAL, "nbody_force_noalloc: null array");
    // j records fill the front of the array; at least 1/4 of it is left for
    // the partial sums
    const size_t rec_bytes = (((size_t)n_j * sizeof(JRec)) + 255) & ~(size_t)255;
    if (n_j > NBODY_NOALLOC_MAX_NJ || rec_bytes > kStaticBytes - kStaticBytes / 4)
        return fail(ctx, NBODY_E_INVAL,
                    "nbody_force_noalloc: n_j = %lld exceeds the static scratch limit "
                    "(n_j <= %d, %d MiB per device)",
                    (long long)n_j, NBODY_NOALLOC_MAX_NJ, NBODY_NOALLOC_SCRATCH_MB);
    if (n_i == 0) return NBODY_OK;
    if (!ctx->static_scratch)
        return fail(ctx, NBODY_E_DEVICE,
                    "nbody_force_noalloc: static scratch unavailable on device %d (%s)",
                    ctx->device, hipGetErrorString((hipError_t)ctx->static_scratch_rc));
    NB_TRY(activate(ctx));
    unsigned char *base = (unsigned char *)ctx->static_scratch;
    ForceCall c;
    c.mode = acc_mode(flags);
    c.shape = shape_for(pick_shape(ctx, n_i, n_j), c.mode);
    JRec *rec = (JRec *)base;
    NB_TRY(launch_pack(ctx, c.shape.rep, n_j, pos, vel, mass, rec));
    c.jrec = rec;
    c.n_j = n_j;
    c.pos = pos;
    c.vel = vel;
    c.active = active_idx;
    c.n_i = n_i;
    c.eps2 = eps2;
    c.acc = acc;
    c.jerk = jerk;
    c.pot = pot;
    c.out_stride = n_i;
    // cap the j split so that S * 7 * n_i partial sums fit behind the records
    c.part_buf = base + rec_bytes;
    c.part_cap = kStaticBytes - rec_bytes;
    const size_t elem = c.mode == ACC_F32 ? sizeof(float) : sizeof(double);
    const size_t per_split = (size_t)7 * (size_t)n_i * elem;
    const size_t fit = c.part_cap / per_split;
    c.max_splits = fit < 1 ? 1 : (fit > (size_t)kMaxSplits ? kMaxSplits : (int)fit);
    return launch_force(ctx, c);
}
