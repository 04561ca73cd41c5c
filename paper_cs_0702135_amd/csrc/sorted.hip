// Smallest-first float32 pair sums (Section 6): the paper proposes adding
// the pair forces in order of increasing size to improve its float32 sums.
// Here every pair term of Eq. (1) (softened as in the Appendix A listing)
// is evaluated in float64 and rounded once to float32; the terms of each
// particle are added in float32 in ascending order of the pair-acceleration
// magnitude m_j |r| s^(-3/2) (ties by j), all seven sums in that one order.
//
// One 1024-thread workgroup per active particle (16 waves, so that the LDS
// latency of the sort is hidden): its n_j - 1 keys (float64) and j indices
// are sorted in LDS by a bitonic network, then the sorted terms are
// evaluated 1024 at a time into LDS and seven lanes add one component each
// in sorted order.  The float64 expressions are evaluated without
// contraction, in the order they are written, so that the rounding of each
// term and key is the plain IEEE rounding of that expression.
#include <cmath>

#include "common.hpp"
#include "pairs.hpp"

namespace nb {

constexpr int kSortMax = 8192;     // largest n_j (LDS: 8 + 2 bytes per j)
constexpr int kSortThreads = 1024;
constexpr uint16_t kInvalid = 0xFFFF;  // the self pair and the padding

struct PairTerms {
    double rx, ry, rz, vx, vy, vz, mj;
};

__device__ __forceinline__ PairTerms pair_of(const double *pos, const double *vel,
                                             const double *mass, int n_j, int j, double xi,
                                             double yi, double zi, double ui, double vi,
                                             double wi) {
#pragma clang fp contract(off)
    PairTerms p;
    p.rx = pos[j] - xi;
    p.ry = pos[n_j + j] - yi;
    p.rz = pos[2 * n_j + j] - zi;
    p.vx = vel[j] - ui;
    p.vy = vel[n_j + j] - vi;
    p.vz = vel[2 * n_j + j] - wi;
    p.mj = mass[j];
    return p;
}

__global__ __launch_bounds__(kSortThreads) void force_sorted_kernel(
    int64_t n_i, const int32_t *__restrict__ active, int n_j, const double *__restrict__ pos,
    const double *__restrict__ vel, const double *__restrict__ mass, double eps2,
    double *__restrict__ acc, double *__restrict__ jerk, double *__restrict__ pot,
    int32_t *status) {
#pragma clang fp contract(off)
    __shared__ double key[kSortMax];
    __shared__ uint16_t idx[kSortMax];
    // rows padded by four floats: rows stay 16-byte aligned for the summing
    // lanes' 4-float reads, and the seven lanes' reads of one column fall in
    // different banks
    constexpr int kRow = kSortThreads + 4;
    __shared__ __attribute__((aligned(16))) float term[7][kRow];
    const int tid = threadIdx.x;
    int n_pad = 1;
    while (n_pad < n_j) n_pad <<= 1;
    for (int64_t s = blockIdx.x; s < n_i; s += gridDim.x) {
        int i = active ? active[s] : (int)s;
        if ((unsigned)i >= (unsigned)n_j) {
            if (tid == 0) atomicOr(status, (int32_t)ST_INDEX);
            i = 0;
        }
        const double xi = pos[i], yi = pos[n_j + i], zi = pos[2 * n_j + i];
        const double ui = vel[i], vi = vel[n_j + i], wi = vel[2 * n_j + i];
        // keys: |pair acceleration| in float64
        for (int j = tid; j < n_pad; j += kSortThreads) {
            double kv = 0.0;
            uint16_t id = kInvalid;
            if (j < n_j && j != i) {
                const PairTerms p = pair_of(pos, vel, mass, n_j, j, xi, yi, zi, ui, vi, wi);
                const double r2 = p.rx * p.rx + p.ry * p.ry + p.rz * p.rz;
                const double s2 = r2 + eps2;
                const double rinv = 1.0 / sqrt(s2);
                const double r3inv = rinv * rinv * rinv;
                kv = fabs(p.mj) * sqrt(r2) * r3inv;
                id = (uint16_t)j;
            }
            key[j] = kv;
            idx[j] = id;
        }
        __syncthreads();
        // bitonic sort, ascending by (valid first, key, j); each thread takes
        // whole compare-exchange pairs (t, t + jj), t with a zero jj bit
        for (int kk = 2; kk <= n_pad; kk <<= 1) {
            for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                for (int c = tid; c < (n_pad >> 1); c += kSortThreads) {
                    const int t = ((c & ~(jj - 1)) << 1) | (c & (jj - 1));
                    const int p = t | jj;
                    const double kt = key[t], kp = key[p];
                    const uint16_t xt = idx[t], xp = idx[p];
                    const bool it = xt == kInvalid, ip = xp == kInvalid;
                    const bool gt = it != ip ? it : (kt > kp || (kt == kp && xt > xp));
                    if (gt == ((t & kk) == 0)) {
                        key[t] = kp;
                        key[p] = kt;
                        idx[t] = xp;
                        idx[p] = xt;
                    }
                }
                __syncthreads();
            }
        }
        // the n_j - 1 terms in sorted order, a workgroup's worth at a time;
        // lane c < 7 adds component c in float32
        const int m = n_j - 1;
        float sum = 0.0f;
        for (int base = 0; base < m; base += kSortThreads) {
            const int e = base + tid;
            if (e < m) {
                const int j = idx[e];
                const PairTerms p = pair_of(pos, vel, mass, n_j, j, xi, yi, zi, ui, vi, wi);
                const double s2 = p.rx * p.rx + p.ry * p.ry + p.rz * p.rz + eps2;
                const double rv = p.rx * p.vx + p.ry * p.vy + p.rz * p.vz;
                const double rinv = 1.0 / sqrt(s2);
                const double r3inv = rinv * rinv * rinv;
                const double r5inv = r3inv * rinv * rinv;
                term[0][tid] = (float)(p.mj * p.rx * r3inv);
                term[1][tid] = (float)(p.mj * p.ry * r3inv);
                term[2][tid] = (float)(p.mj * p.rz * r3inv);
                term[3][tid] = (float)(p.mj * (p.vx * r3inv - 3.0 * rv * p.rx * r5inv));
                term[4][tid] = (float)(p.mj * (p.vy * r3inv - 3.0 * rv * p.ry * r5inv));
                term[5][tid] = (float)(p.mj * (p.vz * r3inv - 3.0 * rv * p.rz * r5inv));
                term[6][tid] = (float)(-p.mj * rinv);
            }
            __syncthreads();
            if (tid < 7) {
                const int cnt = min(kSortThreads, m - base);
                const float4 *row = reinterpret_cast<const float4 *>(&term[tid][0]);
                int q = 0;
#pragma unroll 8
                for (; q + 4 <= cnt; q += 4) {
                    const float4 v = row[q >> 2];
                    sum = sum + v.x;
                    sum = sum + v.y;
                    sum = sum + v.z;
                    sum = sum + v.w;
                }
                for (; q < cnt; ++q) sum = sum + term[tid][q];
            }
            __syncthreads();
        }
        if (tid < 3)
            acc[tid * n_i + s] = sum;
        else if (tid < 6)
            jerk[(tid - 3) * n_i + s] = sum;
        else if (tid == 6 && pot)
            pot[s] = sum;
        __syncthreads();
    }
}

}  // namespace nb

using namespace nb;

extern "C" int nbody_force_sorted(nbody_ctx *ctx, const int32_t *active_idx, int64_t n_i,
                                  const double *pos, const double *vel, const double *mass,
                                  int64_t n_j, double eps2, double *acc, double *jerk,
                                  double *pot) {
    if (!ctx) return NBODY_E_INVAL;
    if (n_i < 0 || n_j < 1 || n_i > 0x7fffffffLL || n_j > kSortMax)
        return fail(ctx, NBODY_E_INVAL,
                    "nbody_force_sorted: bad sizes n_i=%lld n_j=%lld (n_j <= %d)",
                    (long long)n_i, (long long)n_j, kSortMax);
    if (!(eps2 >= 0.0) || std::isinf(eps2))
        return fail(ctx, NBODY_E_INVAL, "nbody_force_sorted: eps2 must be finite and >= 0");
    if (!pos || !vel || !mass || (n_i > 0 && (!acc || !jerk)))
        return fail(ctx, NBODY_E_INVAL, "nbody_force_sorted: null array");
    if (n_i == 0) return NBODY_OK;
    NB_TRY(activate(ctx));
    const int64_t grid = std::min<int64_t>(n_i, 8 * (int64_t)ctx->cus);
    force_sorted_kernel<<<(unsigned)grid, kSortThreads, 0, ctx->stream>>>(
        n_i, active_idx, (int)n_j, pos, vel, mass, eps2, acc, jerk, pot, &ctx->info->status);
    return hip_check(ctx, hipGetLastError(), "force_sorted_kernel");
}
