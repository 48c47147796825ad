// Device helpers shared by the library's kernels (not public).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace flipmi {

constexpr int WAVE = 64;

__device__ inline int lane_id() { return threadIdx.x & (WAVE - 1); }

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8). Remap block b to a work index so that each XCD receives one
// contiguous range of the (spatially ordered) work list: neighbouring tiles
// then share that XCD's L2. Bijective for any block count.
__device__ inline int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, rem = nb & 7, x = b & 7, idx = b >> 3;
    return x * q + (x < rem ? x : rem) + idx;
}

// Floor of the exact real quotient x / dx, clamped to [0, n-1]. The first
// estimate comes from a rounded product; it is then corrected until
// q*dx <= x < (q+1)*dx, each test evaluated with one fused multiply-add whose
// rounding keeps the sign of the exact difference.
__device__ inline int exact_cell_floor(double x, double dx, double inv_dx, int n)
{
    double q = floor(x * inv_dx);
    q = fmin(fmax(q, -1.0), (double)n);  // also maps NaN to -1
    for (int it = 0; it < 3 && fma(q, dx, -x) > 0.0; ++it) q -= 1.0;
    for (int it = 0; it < 3 && fma(q + 1.0, dx, -x) <= 0.0; ++it) q += 1.0;
    q = fmin(fmax(q, 0.0), (double)(n - 1));
    return (int)q;
}

template <typename T>
__device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_down(v, o, WAVE);
    return v;
}

template <typename T>
__device__ inline T wave_max(T v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        T w = __shfl_down(v, o, WAVE);
        v = w > v ? w : v;
    }
    return v;
}

// Sum over the block in a fixed order (wave tree, then waves in index
// order); the result is valid in thread 0. `sh` holds >= NT/64 doubles.
template <int NT>
__device__ inline double block_sum(double v, double* sh)
{
    v = wave_sum(v);
    const int w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane_id() == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / WAVE; ++i) s += sh[i];
    return s;
}

template <int NT>
__device__ inline double block_max(double v, double* sh)
{
    v = wave_max(v);
    const int w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane_id() == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / WAVE; ++i) s = sh[i] > s ? sh[i] : s;
    return s;
}

// Publish this block's partial results and report whether it is the last
// block of the grid to do so. Called by every thread; the release fence
// makes the partials visible device-wide (across XCDs) before the counter
// increment, and the last block acquires before reading them.
__device__ inline bool last_block_arrives(unsigned* counter, bool* sh_flag)
{
    if (threadIdx.x == 0) {
        __threadfence();
        unsigned prev = atomicAdd(counter, 1u);
        *sh_flag = (prev == gridDim.x - 1);
    }
    __syncthreads();
    bool last = *sh_flag;
    if (last) __threadfence();
    return last;
}

// Fixed-order reduction of nb partials by one block (sum or max). Callers
// map non-finite magnitudes to +inf before a max so it cannot be lost.
template <int NT>
__device__ inline double reduce_partials_sum(const double* p, int nb, double* sh)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += NT) s += p[i];
    return block_sum<NT>(s, sh);
}

template <int NT>
__device__ inline double reduce_partials_max(const double* p, int nb, double* sh)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += NT) s = p[i] > s ? p[i] : s;
    return block_max<NT>(s, sh);
}

}  // namespace flipmi
