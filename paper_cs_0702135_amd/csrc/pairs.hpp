// Internal declarations shared by the pair kernels (sums and adjoint).
#pragma once

#include "common.hpp"

namespace nb {

// Pointer into the constant address space: wave-uniform loads through it
// become scalar loads (SGPR results).
#define CONSTP(T) const __attribute__((address_space(4))) T *

constexpr int kMaxSplits = 1024;  // largest j split across workgroups

// Arithmetic and accumulation of the pair terms:
//   ACC_F32  (NBODY_ACC_FP32) float32 pair terms summed in float32 over a
//            tile of consecutive j; the tile sums of a few tiles are added
//            in float32, then to a float64 total, so no float32 sum spans
//            more than a fixed number of j whatever the launch shape;
//   ACC_F64  (NBODY_ACC_DS) float64 pair terms and float64 sums (float64
//            records only).
enum { ACC_F32 = 0, ACC_F64 = 1 };
constexpr int RW = 8;             // waves per group of the split reduction

struct KArgs {
    const JRec *__restrict__ jrec;
    const double *__restrict__ pos;
    const double *__restrict__ vel;
    const int32_t *__restrict__ active;
    const int64_t *__restrict__ n_i_dev;
    double *__restrict__ acc;
    double *__restrict__ jerk;
    double *__restrict__ pot;
    double *__restrict__ part;
    int32_t *status;  // latched error bits (an active index out of range)
    int64_t n_i;
    int64_t out_stride;  // <= 0: use n_i
    int32_t n_j;
    float eps2;
    double eps2d;
    int32_t tile;
    int32_t min_j_wave;
    int32_t target_groups;
    int32_t max_splits;
    int32_t accumulate;  // 1: add into acc/jerk/pot instead of overwriting
    int32_t part_f32;    // 1: split partials stored as float32 (float32 sums)
    // j-lane layout (force_jl_kernel): its split rule, and the block sizes it
    // takes: n_i <= jl_max (the i-lane kernel takes n_i > jl_max).  Both
    // kernels and the split reduction read the block size on the device, so
    // the block-step driver launches both and each returns early on the
    // other's blocks.
    int64_t jl_max;
    int32_t jl_c, jl_waves, jl_tile, jl_min_j_wave, jl_target_groups;
};

// Active-block size of a launch: read on the device when n_i_dev is set
// (then a.n_i is the capacity of the outputs and larger values are clamped
// to it), else a.n_i.
__device__ __forceinline__ int64_t block_size(const KArgs &a) {
    if (!a.n_i_dev) return a.n_i;
    const int64_t v = *a.n_i_dev;
    return v < a.n_i ? v : a.n_i;
}

// Number of workgroups that share one i-block's j range.
__host__ __device__ inline int64_t choose_splits(int64_t n_i, int64_t n_j, int it, int waves,
                                                 int min_j_wave, int target_groups,
                                                 int max_splits) {
    int64_t nb = (n_i + 64 * it - 1) / (64 * it);
    if (nb < 1) nb = 1;
    int64_t s = (target_groups + nb - 1) / nb;
    int64_t smax = n_j / ((int64_t)waves * min_j_wave);
    if (smax > max_splits) smax = max_splits;
    if (s > smax) s = smax;
    if (s < 1) s = 1;
    return s;
}

// Splits of the j range in the j-lane layout: each workgroup takes C
// i-particles and its waves give each lane one j at a time, so a lane's
// float32 sum has (j range per wave) / 64 terms; the split keeps that at or
// below `tile` (as the i-lane kernel's tiles) while aiming at target_groups
// workgroups in all.
__host__ __device__ inline int64_t choose_splits_jl(int64_t n_i, int64_t n_j, int c, int waves,
                                                    int tile, int min_j_wave, int target_groups,
                                                    int max_splits) {
    int64_t nb = (n_i + c - 1) / c;
    if (nb < 1) nb = 1;
    int64_t s = (target_groups + nb - 1) / nb;
    const int64_t per_split = (int64_t)waves * 64 * tile;
    const int64_t s_lo = (n_j + per_split - 1) / per_split;
    if (s < s_lo) s = s_lo;
    int64_t smax = n_j / ((int64_t)waves * min_j_wave);
    if (smax > max_splits) smax = max_splits;
    if (s > smax) s = smax;
    if (s < 1) s = 1;
    return s;
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each
// with its own L2.  Items are numbered split-major (item = split * nb +
// i-block), so mapping workgroup q to item (q % 8) * (items / 8) + q / 8
// hands each XCD a contiguous run of items, i.e. one or two j chunks that
// its L2 serves to all of its groups, instead of every XCD streaming every
// chunk.  The map is a bijection on [0, items) (the remainder beyond a
// multiple of 8 maps to itself), so results never depend on the dispatch.
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_item(int64_t q, int64_t items) {
    const int64_t per = items / kXcds;
    return q < per * kXcds ? (q % kXcds) * per + q / kXcds : q;
}

__device__ __forceinline__ void two_sum_acc(float &hi, float &lo, float x) {
    const float s = hi + x;
    const float bp = s - hi;
    const float e = (hi - (s - bp)) + (x - bp);
    hi = s;
    lo += e;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Adds the S partial sums [S][7][n_i] of the 7 outputs (float64, or
// float32 with KArgs::part_f32) in split order, in float64, and writes acc
// (q < 3), jerk (q < 6) and pot (q = 6).
int launch_reduce_parts(nbody_ctx *ctx, const KArgs &a, int it, int waves, int64_t n_i_max);

}  // namespace nb
