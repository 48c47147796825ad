// Device helpers shared by the library's kernels (not public).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cfloat>
#include <cmath>

#include "common.h"

namespace flipmi {

constexpr int WAVE = 64;

__device__ inline int lane_id() { return threadIdx.x & (WAVE - 1); }

// A workgroup's place in the grid of the scene it works on. A plain launch
// covers one scene: id = blockIdx.x, n = gridDim.x. A batched launch
// concatenates the grids of several scenes: scene s owns the workgroups
// [first[s], first[s + 1]) of the launch.
struct Blk {
    int id;
    int n;
};

__device__ inline Blk plain_blk() { return Blk{(int)blockIdx.x, (int)gridDim.x}; }

// Scene of virtual workgroup w in a batched launch of ns scenes (first[] is
// non-decreasing, first[0] = 0; scenes with no workgroups are skipped). Each
// wave counts, 64 entries at a time, the scenes that end at or before this
// workgroup. The result is uniform across the workgroup.
__device__ inline int batch_scene(const uint32_t* __restrict__ first, int ns, uint32_t w, Blk& b)
{
    int s = 0;
    for (int base = 1; base <= ns; base += WAVE) {
        const int i = base + lane_id();
        const bool ended = i <= ns && first[i] <= w;
        s += __popcll(__ballot(ended));
    }
    s = __builtin_amdgcn_readfirstlane(s);
    const uint32_t f0 = first[s], f1 = first[s + 1];
    b.id = (int)(w - f0);
    b.n = (int)(f1 - f0);
    return s;
}

// A pointer read from memory (not a kernel argument) is generic to the
// compiler, so its accesses become flat loads and stores, which count on the
// LDS counter too and make every wait a full one. The tables of batched
// launches hold global pointers only: passing one through an integer into
// the global address space restores global accesses.
template <typename T>
__device__ inline T* as_global(T* p)
{
    typedef __attribute__((address_space(1))) T GT;
    return (T*)(GT*)(uintptr_t)p;
}

// Runs body(b, args) for each workgroup of a batched launch's virtual grid
// (see batch.h): first[ns] workgroups in all, each with its scene's
// arguments and its place b in that scene's own grid. This workgroup takes
// virtual workgroups blockIdx.x, blockIdx.x + gridDim.x, ... (the physical
// grid is fixed when the batch is built, whatever its scenes are later), with
// a barrier between two of them, so each may use LDS from the start.
template <typename A, typename F>
__device__ __forceinline__ void batch_for_each(const A* __restrict__ tab, const uint32_t* __restrict__ first, int ns,
                                               F&& body)
{
    const uint32_t total = first[ns];
    for (uint32_t w = blockIdx.x; w < total; w += gridDim.x) {
        Blk b;
        const int s = batch_scene(first, ns, w, b);
        body(b, tab[s]);
        __syncthreads();
    }
}

// Workgroup barrier that orders LDS only. __syncthreads() fences every
// address space, which makes the compiler wait for all outstanding global
// loads (vmcnt(0)) before the barrier, including loads issued early for
// later use. Where waves exchange data through LDS alone, this barrier
// waits only for the wave's LDS operations, so prefetched global loads stay
// in flight across it.
// 1/d for a cell's neighbour count d in 0..6 (0 for 0) in the multigrid
// smoother. FP32 takes the hardware reciprocal (one instruction, within 1 ulp;
// exact for 1, 2 and 4) instead of the correctly rounded division sequence:
// the smoother only has to be the same linear operator every time it is
// applied, which it is. FP64 divides.
template <typename V>
__device__ inline V smoother_recip(int d)
{
    if constexpr (sizeof(V) == 4)
        return d ? __builtin_amdgcn_rcpf((float)d) : 0.0f;
    else
        return d ? V(1) / (V)d : V(0);
}

__device__ inline void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8). Remap block b to a work index so that each XCD receives one
// contiguous range of the (spatially ordered) work list: neighbouring tiles
// then share that XCD's L2. Bijective for any block count.
__device__ inline int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, rem = nb & 7, x = b & 7, idx = b >> 3;
    return x * q + (x < rem ? x : rem) + idx;
}

// contiguous range [t0, t1) of the n_tiles active tiles for this workgroup; the
// workgroups of one XCD get one contiguous chunk of the (spatially ordered) list
__device__ inline void tile_range(Blk blk, int n_tiles, int& t0, int& t1)
{
    const int L = xcd_remap(blk.id, blk.n);
    t0 = (int)((int64_t)n_tiles * L / blk.n);
    t1 = (int)((int64_t)n_tiles * (L + 1) / blk.n);
}

// a finite value, or +inf for inf and NaN (so a max over values flags both)
__device__ inline double finite_or_inf(double a) { return (a <= DBL_MAX) ? a : INFINITY; }

// The cell index of an FP32 coordinate when dx is a power of two: x / dx is
// then exact in FP32 and so is its floor, so this equals exact_cell_floor
// below (NaN maps to 0 there too).
__device__ inline int dyadic_cell_floor(float x, float inv_dx, int n)
{
    const float q = floorf(x * inv_dx);
    return (int)fminf(fmaxf(q, 0.0f), (float)(n - 1));
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

// The binning's cell of a position: the exact floor of x / dx per axis,
// clamped into the grid (FP32 positions on a power-of-two spacing take the
// FP32 floor, which is the same)
template <typename T>
__device__ inline void bin_cell(const Geo& g, T x, T y, T z, int& i, int& j, int& k)
{
    if (sizeof(T) == 4 && g.dyadic) {
        const float inv = (float)g.inv_dx;
        i = dyadic_cell_floor((float)x, inv, g.nx);
        j = dyadic_cell_floor((float)y, inv, g.ny);
        k = dyadic_cell_floor((float)z, inv, g.nz);
    } else {
        i = exact_cell_floor((double)x, g.dx, g.inv_dx, g.nx);
        j = exact_cell_floor((double)y, g.dx, g.inv_dx, g.ny);
        k = exact_cell_floor((double)z, g.dx, g.inv_dx, g.nz);
    }
}

// Provisional rank of a particle in cell c (i, j, k), for the wave's live
// lanes, which must be a prefix of the wave holding consecutive particles:
// the lanes of a run of equal cells (particles arrive mostly sorted, so a
// wave holds a few long runs) take theirs from one atomic on count[c] issued
// by the run's first lane; every run's atomic is issued by the same
// instruction, so a wave waits for one round trip, not one per run. A cell
// that appears in several runs gets several disjoint ranges; the gather makes
// the final ranks stable. tile_flag (optional): the run's first lane marks
// the cell's 8^3 tile.
__device__ inline uint32_t bin_rank(const Geo& g, uint32_t c, int i, int j, int k, uint32_t* __restrict__ count,
                                    uint32_t* __restrict__ tile_flag)
{
    const int lane = lane_id();
    const uint32_t prev = __shfl_up(c, 1, WAVE);
    const bool head = lane == 0 || prev != c;
    const uint64_t heads = __ballot(head);
    const uint64_t live = __ballot(true);
    // the run ends at the next head or at the wave's last live lane
    const uint64_t above = lane == WAVE - 1 ? 0ull : (~0ull << (lane + 1));
    const uint64_t after = heads & above & live;
    const int end = after ? __ffsll((unsigned long long)after) - 1 : 64 - __clzll((unsigned long long)live);
    uint32_t base = 0;
    if (head) {
        base = atomicAdd(&count[c], (uint32_t)(end - lane));
        // every writer stores the same value (flags cleared before the launch)
        if (tile_flag) tile_flag[(i >> 3) + (int64_t)g.tx * ((j >> 3) + (int64_t)g.ty * (k >> 3))] = 1u;
    }
    // this lane's run starts at the highest head at or below it
    const uint64_t upto = lane == WAVE - 1 ? ~0ull : (~0ull >> (WAVE - 1 - lane));
    const int first = 63 - __clzll((unsigned long long)(heads & upto));
    base = __shfl(base, first, WAVE);
    return base + (uint32_t)(lane - first);
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

// ---------------------------------------------------------------------------
// Completing a reduction in the next kernel. Each workgroup of a kernel
// stores its partial sums with plain stores; the kernel boundary makes them
// visible, and every workgroup of the next kernel combines all of them the
// same way (each thread strides over the slots in index order, then a fixed
// tree), so all workgroups hold the same value and no workgroup of the
// producing kernel has to wait for the others. The result is in every thread;
// `sh` holds 2 * NT / 64 doubles.
// ---------------------------------------------------------------------------

// Slots per thread loaded together (one round trip for up to 4 * NT slots).
constexpr int SLOT_UNROLL = 4;

template <int NT>
__device__ inline double reduce_slots_all(const double* __restrict__ slots, int nb, double* sh)
{
    double acc = 0.0;
    for (int base = threadIdx.x; base < nb; base += SLOT_UNROLL * NT) {
        double v[SLOT_UNROLL];
#pragma unroll
        for (int u = 0; u < SLOT_UNROLL; ++u) {
            const int i = base + u * NT;
            v[u] = i < nb ? slots[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < SLOT_UNROLL; ++u) acc += v[u];
    }
    acc = wave_sum(acc);
    __syncthreads();
    if (lane_id() == 0) sh[threadIdx.x / WAVE] = acc;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < NT / WAVE; ++i) s += sh[i];
    return s;
}

// sum of sum_slots[0..nb) and max of max_slots[0..nb), loaded together.
// Returned by value: a result written through a reference to a local that a
// caller then selects against a value from memory lets the compiler merge the
// two into one load through a selected pointer, which moves the local to
// scratch memory and makes that load a flat one.
struct SumMax {
    double sum, mx;
};

template <int NT>
__device__ inline SumMax reduce_slots_all(const double* __restrict__ sum_slots,
                                          const double* __restrict__ max_slots, int nb, double* sh)
{
    double a = 0.0, m = 0.0;
    for (int base = threadIdx.x; base < nb; base += SLOT_UNROLL * NT) {
        double v[SLOT_UNROLL], w[SLOT_UNROLL];
#pragma unroll
        for (int u = 0; u < SLOT_UNROLL; ++u) {
            const int i = base + u * NT;
            v[u] = i < nb ? sum_slots[i] : 0.0;
            w[u] = i < nb ? max_slots[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < SLOT_UNROLL; ++u) {
            a += v[u];
            m = w[u] > m ? w[u] : m;
        }
    }
    a = wave_sum(a);
    m = wave_max(m);
    __syncthreads();
    if (lane_id() == 0) {
        sh[threadIdx.x / WAVE] = a;
        sh[NT / WAVE + threadIdx.x / WAVE] = m;
    }
    __syncthreads();
    a = 0.0;
    m = 0.0;
    for (int i = 0; i < NT / WAVE; ++i) {
        a += sh[i];
        m = sh[NT / WAVE + i] > m ? sh[NT / WAVE + i] : m;
    }
    return SumMax{a, m};
}

// ---------------------------------------------------------------------------
// Grid-wide reduction without a device-scope fence.
//
// A release fence at device scope makes the issuing CU write back its XCD's
// whole L2, which costs far more than the kernel's own traffic when thousands
// of workgroups each issue one. Instead, each workgroup publishes its partial
// results into its own slots with relaxed device-scope atomic stores (coherent
// across XCDs, nothing else is flushed) and counts itself in with a relaxed
// atomic add. The workgroup that takes the count to the grid size reads every
// slot; a slot whose store is not visible yet still holds the EMPTY pattern and
// is re-read until it is (bounded; on exhaustion the error flag is set). Slots
// are summed in index order, so the result is the same on every run, and are
// reset to EMPTY for the next kernel.
// ---------------------------------------------------------------------------

// a signalling-NaN bit pattern: arithmetic never produces it
constexpr unsigned long long SLOT_EMPTY = SLOT_EMPTY_BITS;
constexpr int SLOT_MAX_POLLS = 1 << 20;

__device__ inline void slot_store(double* slot, double v)
{
    __hip_atomic_store((unsigned long long*)slot, (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline unsigned long long slot_load(const double* slot)
{
    return __hip_atomic_load((unsigned long long*)slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Arrival counters: ctr[0] counts arriving sets, ctr[SYNC_STRIDE * (1 + x)]
// counts the arriving workgroups of set x = (workgroup index) % 8. One counter per set
// (each on its own 128-byte line) keeps the relaxed atomic adds from queueing
// on a single address: a single counter cost microseconds per thousand
// workgroups.
constexpr int SYNC_SETS = 8;
constexpr int SYNC_STRIDE = 32;
static_assert(SYNC_STRIDE * (SYNC_SETS + 1) * 4 == SYNC_BYTES, "arrival counter layout");

// Thread 0 publishes vals[0..nq) into slots[q * stride + b.id]; returns (in
// every thread) whether this workgroup is the last of its scene's grid to arrive.
__device__ inline bool publish_partials(Blk b, double* slots, int64_t stride, const double* vals, int nq,
                                        unsigned* ctr, bool* sh_last)
{
    if (threadIdx.x == 0) {
        for (int q = 0; q < nq; ++q) slot_store(slots + q * stride + b.id, vals[q]);
        const unsigned nb = (unsigned)b.n;
        const unsigned set = (unsigned)b.id % SYNC_SETS;
        const unsigned in_set = nb / SYNC_SETS + (set < nb % SYNC_SETS ? 1u : 0u);
        const unsigned sets = nb < SYNC_SETS ? nb : SYNC_SETS;
        bool last = false;
        const unsigned prev = __hip_atomic_fetch_add(ctr + SYNC_STRIDE * (1 + set), 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        if (prev == in_set - 1) {
            const unsigned p2 = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last = (p2 == sets - 1);
        }
        *sh_last = last;
    }
    __syncthreads();
    return *sh_last;
}

// In the last workgroup, after the slots are collected: zero the counters.
__device__ inline void reset_arrivals(unsigned* ctr)
{
    if (threadIdx.x <= SYNC_SETS)
        __hip_atomic_store(ctr + SYNC_STRIDE * threadIdx.x, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// In the last workgroup: combine the slots of NQ quantities, quantity q in
// slots[q * stride + 0 .. nb), by sum, or by max where MAXMASK has bit q set,
// and reset them to EMPTY. Every quantity's loads are issued together, so
// the combine costs one round trip to memory whatever NQ is. *err is set
// when a slot stayed EMPTY for SLOT_MAX_POLLS re-reads; after that the
// thread stops waiting, so the block always finishes. Within a thread slots
// are taken in index order, then threads in a fixed tree: the result is the
// same on every run.
template <int NT, int NQ, unsigned MAXMASK>
__device__ inline void collect_slots(double* slots, int64_t stride, int nb, double* sh, int* err,
                                     double (&out)[NQ])
{
    constexpr int U = 8;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    for (int base = threadIdx.x; base < nb; base += U * NT) {
        unsigned long long v[NQ][U];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = base + u * NT;
                v[q][u] = i < nb ? slot_load(slots + q * stride + i) : 0ull;
            }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = base + u * NT;
                if (i >= nb) continue;
                double* slot = slots + q * stride + i;
                for (int polls = 0; v[q][u] == SLOT_EMPTY && polls < SLOT_MAX_POLLS && !*err; ++polls) {
                    __builtin_amdgcn_s_sleep(1);
                    v[q][u] = slot_load(slot);
                }
                if (v[q][u] == SLOT_EMPTY) {
                    *err = 1;
                    v[q][u] = 0ull;
                }
                const double x = __longlong_as_double((long long)v[q][u]);
                acc[q] = ((MAXMASK >> q) & 1u) ? (x > acc[q] ? x : acc[q]) : acc[q] + x;
                __hip_atomic_store((unsigned long long*)slot, SLOT_EMPTY, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        out[q] = ((MAXMASK >> q) & 1u) ? block_max<NT>(acc[q], sh) : block_sum<NT>(acc[q], sh);
}

}  // namespace flipmi
