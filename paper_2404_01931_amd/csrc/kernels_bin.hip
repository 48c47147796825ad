// Particle binning by cell (paper Sec. 3.1.5, Fig. 4; GPU variant Sec. 3.2.2):
// raw cell index per particle, per-cell counts, exclusive scan (the space
// hash's start offsets), a stable counting sort of the particles, and the
// list of active 8x8x8 tiles used by the pressure solve.
//
// Stability without a global order of atomics: each particle first takes a
// provisional slot inside its cell's segment (an atomic rank, order
// arbitrary), then its final slot is its rank by original index among the
// particles of the same cell. The result equals a stable sort by key and is
// the same on every run.
#include "batch.h"
#include "common.h"
#include "device_util.h"

namespace flipmi {

// ---------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------

__device__ __forceinline__ void fill_u32_body(Blk b, uint32_t* p, int64_t n, uint32_t v)
{
    int64_t i = (int64_t)b.id * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, int64_t n, uint32_t v)
{
    fill_u32_body(plain_blk(), p, n, v);
}

__global__ __launch_bounds__(256) void kb_fill_u32(const FillU32Args* __restrict__ tab,
                                                   const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const FillU32Args& a) {
        fill_u32_body(b, as_global(a.p), a.n, a.v);
    });
}

void launch_b_fill_u32(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_fill_u32, dim3(L.blocks), dim3(256), 0, st, (const FillU32Args*)L.args, L.first, L.ns);
}

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
}

__global__ __launch_bounds__(256) void k_fill_u64(uint64_t* p, int64_t n, uint64_t v)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

void launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
}

__global__ __launch_bounds__(256) void k_zero_bytes(uint8_t* p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

void launch_fill_bytes_zero(void* p, int64_t bytes, hipStream_t st)
{
    if (bytes <= 0) return;
    if ((bytes & 3) == 0 && ((uintptr_t)p & 3) == 0) {
        launch_fill_u32((uint32_t*)p, bytes / 4, 0u, st);
        return;
    }
    hipLaunchKernelGGL(k_zero_bytes, dim3((unsigned)((bytes + 255) / 256)), dim3(256), 0, st,
                       (uint8_t*)p, bytes);
}

// ---------------------------------------------------------------------------
// raw cell index and count (one thread per particle)
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void bin_keys_body(Blk b, Geo g, const T* __restrict__ px,
                                              const T* __restrict__ py, const T* __restrict__ pz,
                                              int64_t n, uint32_t* __restrict__ key,
                                              uint32_t* __restrict__ rank,
                                              uint32_t* __restrict__ count,
                                              uint32_t* __restrict__ tile_flag = nullptr)
{
    const int64_t p = (int64_t)b.id * 256 + threadIdx.x;
    if (p >= n) return;
    int i, j, k;
    bin_cell<T>(g, px[p], py[p], pz[p], i, j, k);
    const uint32_t c = (uint32_t)(i + (int64_t)g.nx * (j + (int64_t)g.ny * k));
    key[p] = c;
    rank[p] = bin_rank(g, c, i, j, k, count, tile_flag);
}

template <typename T>
__global__ __launch_bounds__(256) void k_bin_keys(Geo g, const T* __restrict__ px,
                                                  const T* __restrict__ py, const T* __restrict__ pz,
                                                  int64_t n, uint32_t* __restrict__ key,
                                                  uint32_t* __restrict__ rank,
                                                  uint32_t* __restrict__ count,
                                                  uint32_t* __restrict__ tile_flag)
{
    bin_keys_body<T>(plain_blk(), g, px, py, pz, n, key, rank, count, tile_flag);
}

template <typename T>
__global__ __launch_bounds__(256) void kb_bin_keys(const BinKeysArgs<T>* __restrict__ tab,
                                                   const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const BinKeysArgs<T>& a) {
        bin_keys_body<T>(b, a.g, as_global(a.px), as_global(a.py), as_global(a.pz), a.n, as_global(a.key), as_global(a.rank), as_global(a.count));
    });
}

template <typename T>
void launch_b_bin_keys(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_bin_keys<T>, dim3(L.blocks), dim3(256), 0, st, (const BinKeysArgs<T>*)L.args,
                       L.first, L.ns);
}
template void launch_b_bin_keys<float>(const BatchLaunch&, hipStream_t);
template void launch_b_bin_keys<double>(const BatchLaunch&, hipStream_t);

template <typename T>
void launch_bin_keys(const Geo& g, const T* pos, int64_t n, uint32_t* key, uint32_t* rank,
                     uint32_t* count, hipStream_t st, uint32_t* tile_flag)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bin_keys<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, pos,
                       pos + n, pos + 2 * n, n, key, rank, count, tile_flag);
}

template void launch_bin_keys<float>(const Geo&, const float*, int64_t, uint32_t*, uint32_t*,
                                     uint32_t*, hipStream_t, uint32_t*);
template void launch_bin_keys<double>(const Geo&, const double*, int64_t, uint32_t*, uint32_t*,
                                      uint32_t*, hipStream_t, uint32_t*);

// ---------------------------------------------------------------------------
// exclusive scan of u32 (all-prefix-sums with identity 0, Sec. 3.2.2)
// Three passes: per-block totals, a scan of the totals by one block, and a
// rescan of each block with its offset. 256 threads x 16 items per block.
// ---------------------------------------------------------------------------

__device__ inline uint32_t wave_incl_scan_u32(uint32_t v)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        uint32_t t = __shfl_up(v, o, WAVE);
        if (lane >= o) v += t;
    }
    return v;
}

// exclusive scan across the block of one value per thread; returns the
// thread's exclusive prefix and the block total in *total
template <int NT>
__device__ inline uint32_t block_excl_scan_u32(uint32_t v, uint32_t* sh, uint32_t* total)
{
    const int w = threadIdx.x / WAVE;
    uint32_t incl = wave_incl_scan_u32(v);
    __syncthreads();
    if (lane_id() == WAVE - 1) sh[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < NT / WAVE; ++i) {
            uint32_t t = sh[i];
            sh[i] = run;
            run += t;
        }
        sh[NT / WAVE] = run;
    }
    __syncthreads();
    *total = sh[NT / WAVE];
    return incl - v + sh[w];
}

__device__ __forceinline__ void scan_totals_body(Blk b, const uint32_t* __restrict__ in, int64_t n,
                                                 uint32_t* __restrict__ totals)
{
    __shared__ uint32_t sh[SCAN_NT / WAVE + 1];
    const int64_t base = (int64_t)b.id * SCAN_TILE;
    uint32_t s = 0;
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
        int64_t i = base + it * SCAN_NT + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t total;
    block_excl_scan_u32<SCAN_NT>(s, sh, &total);
    if (threadIdx.x == 0) totals[b.id] = total;
}

__global__ __launch_bounds__(SCAN_NT) void k_scan_totals(const uint32_t* __restrict__ in, int64_t n,
                                                         uint32_t* __restrict__ totals)
{
    scan_totals_body(plain_blk(), in, n, totals);
}

__global__ __launch_bounds__(SCAN_NT) void kb_scan_totals(const ScanTotalsArgs* __restrict__ tab,
                                                          const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const ScanTotalsArgs& a) {
        scan_totals_body(b, as_global(a.in), a.n, as_global(a.totals));
    });
}

void launch_b_scan_totals(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_scan_totals, dim3(L.blocks), dim3(SCAN_NT), 0, st, (const ScanTotalsArgs*)L.args,
                       L.first, L.ns);
}

// single block: exclusive scan of nb totals in place, chunk by chunk
__device__ __forceinline__ void scan_totals_scan_body(uint32_t* __restrict__ totals, int64_t nb)
{
    __shared__ uint32_t sh[1024 / WAVE + 1];
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
        int64_t i = c0 + threadIdx.x;
        uint32_t v = i < nb ? totals[i] : 0u;
        uint32_t total;
        uint32_t ex = block_excl_scan_u32<1024>(v, sh, &total);
        if (i < nb) totals[i] = ex + carry;
        carry += total;
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_scan_totals_scan(uint32_t* __restrict__ totals, int64_t nb)
{
    scan_totals_scan_body(totals, nb);
}

__global__ __launch_bounds__(1024) void kb_scan_totals_scan(const ScanTotalsScanArgs* __restrict__ tab,
                                                            const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const ScanTotalsScanArgs& a) {
        scan_totals_scan_body(as_global(a.totals), a.nb);
    });
}

void launch_b_scan_totals_scan(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_scan_totals_scan, dim3(L.blocks), dim3(1024), 0, st,
                       (const ScanTotalsScanArgs*)L.args, L.first, L.ns);
}

__device__ __forceinline__ void scan_apply_body(Blk b, const uint32_t* __restrict__ in,
                                                uint32_t* __restrict__ out, int64_t n,
                                                const uint32_t* __restrict__ offsets)
{
    // items of the tile staged in LDS; thread t owns items [16 t, 16 t + 16),
    // padded by one word per 32 to spread LDS banks
    __shared__ uint32_t tile[SCAN_TILE + SCAN_TILE / 32];
    __shared__ uint32_t sh[SCAN_NT / WAVE + 1];
    const int64_t base = (int64_t)b.id * SCAN_TILE;
#define PAD(i) ((i) + ((i) >> 5))
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
        int li = it * SCAN_NT + threadIdx.x;
        int64_t i = base + li;
        tile[PAD(li)] = i < n ? in[i] : 0u;
    }
    __syncthreads();
    uint32_t vals[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
        vals[it] = tile[PAD(threadIdx.x * SCAN_ITEMS + it)];
        s += vals[it];
    }
    uint32_t total;
    uint32_t run = block_excl_scan_u32<SCAN_NT>(s, sh, &total) + offsets[b.id];
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
        tile[PAD(threadIdx.x * SCAN_ITEMS + it)] = run;
        run += vals[it];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
        int li = it * SCAN_NT + threadIdx.x;
        int64_t i = base + li;
        if (i < n) out[i] = tile[PAD(li)];
    }
#undef PAD
}

__global__ __launch_bounds__(SCAN_NT) void k_scan_apply(const uint32_t* __restrict__ in,
                                                        uint32_t* __restrict__ out, int64_t n,
                                                        const uint32_t* __restrict__ offsets)
{
    scan_apply_body(plain_blk(), in, out, n, offsets);
}

__global__ __launch_bounds__(SCAN_NT) void kb_scan_apply(const ScanApplyArgs* __restrict__ tab,
                                                         const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const ScanApplyArgs& a) {
        scan_apply_body(b, as_global(a.in), as_global(a.out), a.n, as_global(a.offsets));
    });
}

void launch_b_scan_apply(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_scan_apply, dim3(L.blocks), dim3(SCAN_NT), 0, st, (const ScanApplyArgs*)L.args,
                       L.first, L.ns);
}

int64_t scan_tmp_words(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

void launch_exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp,
                               hipStream_t st)
{
    if (n <= 0) return;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)nb), dim3(SCAN_NT), 0, st, in, n, tmp);
    hipLaunchKernelGGL(k_scan_totals_scan, dim3(1), dim3(1024), 0, st, tmp, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_NT), 0, st, in, out, n, tmp);
}

// ---------------------------------------------------------------------------
// stable counting sort
// ---------------------------------------------------------------------------

__device__ __forceinline__ void bin_scatter_body(Blk b, const uint32_t* __restrict__ key,
                                                 const uint32_t* __restrict__ rank,
                                                 const uint32_t* __restrict__ start, int64_t n,
                                                 uint32_t* __restrict__ perm)
{
    const int64_t p = (int64_t)b.id * 256 + threadIdx.x;
    if (p >= n) return;
    perm[start[key[p]] + rank[p]] = (uint32_t)p;
}

__global__ __launch_bounds__(256) void k_bin_scatter(const uint32_t* __restrict__ key,
                                                     const uint32_t* __restrict__ rank,
                                                     const uint32_t* __restrict__ start, int64_t n,
                                                     uint32_t* __restrict__ perm)
{
    bin_scatter_body(plain_blk(), key, rank, start, n, perm);
}

__global__ __launch_bounds__(256) void kb_bin_scatter(const ScatterArgs* __restrict__ tab,
                                                      const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const ScatterArgs& a) {
        bin_scatter_body(b, as_global(a.key), as_global(a.rank), as_global(a.start), a.n, as_global(a.perm));
    });
}

void launch_b_bin_scatter(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_bin_scatter, dim3(L.blocks), dim3(256), 0, st, (const ScatterArgs*)L.args, L.first,
                       L.ns);
}

void launch_bin_scatter(const uint32_t* key, const uint32_t* rank, const uint32_t* start,
                        int64_t n, uint32_t* perm, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bin_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, key, rank,
                       start, n, perm);
}

// Slot s of the provisional order holds particle p; p's final slot is the
// start of its cell plus the number of particles of that cell with a smaller
// original index. The particle's state moves there (double buffer, Sec. 3.2.2).
// SPREAD (reseeding): the output has n_out >= n slots and cell c's particles
// move up by spread[c], the new particles of the cells before it.
template <typename T, bool SPREAD = false>
__device__ __forceinline__ void bin_gather_body(
    Blk b, const uint32_t* __restrict__ perm, const uint32_t* __restrict__ key,
    const uint32_t* __restrict__ start, const uint32_t* __restrict__ count, int64_t n,
    const T* __restrict__ pos_in, const T* __restrict__ vel_in, const uint32_t* __restrict__ id_in,
    T* __restrict__ pos_out, T* __restrict__ vel_out, uint32_t* __restrict__ id_out,
    const uint32_t* __restrict__ spread = nullptr, int64_t n_out = 0)
{
    // the workgroup's 256 slots of the provisional order, staged in LDS: a
    // cell's slots are mostly among them, and the rank below reads them from
    // there (the few outside the workgroup's range from memory)
    __shared__ uint32_t slots[256];
    const int64_t s0 = (int64_t)b.id * 256;
    const int64_t s = s0 + threadIdx.x;
    const bool live = s < n;
    const uint32_t p = live ? perm[s] : 0u;
    slots[threadIdx.x] = p;
    __syncthreads();
    if (!live) return;
    // the particle's state is read while its slot is worked out (those
    // loads do not depend on the rank)
    T pv[3], vv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        pv[a] = pos_in[a * n + p];
        vv[a] = vel_in[a * n + p];
    }
    const uint32_t idv = id_in[p];
    const uint32_t c = key[p];
    const uint32_t st = start[c];
    const uint32_t cnt = count[c];
    // the cell's slots four at a time (indices clamped into the cell)
    const uint32_t end = st + cnt;
    const uint32_t base = (uint32_t)s0;
    uint32_t r = 0;
    for (uint32_t q = st; q < end; q += 4) {
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t qq = min(q + k, end - 1);
            v[k] = qq - base < 256u ? slots[qq - base] : perm[qq];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) r += (q + k < end && v[k] < p) ? 1u : 0u;
    }
    const int64_t d = (int64_t)st + r + (SPREAD ? spread[c] : 0u);
    const int64_t m = SPREAD ? n_out : n;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        pos_out[a * m + d] = pv[a];
        vel_out[a * m + d] = vv[a];
    }
    id_out[d] = idv;
}

template <typename T>
__global__ __launch_bounds__(256) void k_bin_gather(
    const uint32_t* __restrict__ perm, const uint32_t* __restrict__ key,
    const uint32_t* __restrict__ start, const uint32_t* __restrict__ count, int64_t n,
    const T* __restrict__ pos_in, const T* __restrict__ vel_in, const uint32_t* __restrict__ id_in,
    T* __restrict__ pos_out, T* __restrict__ vel_out, uint32_t* __restrict__ id_out)
{
    bin_gather_body<T>(plain_blk(), perm, key, start, count, n, pos_in, vel_in, id_in, pos_out, vel_out,
                       id_out);
}

template <typename T>
__global__ __launch_bounds__(256) void kb_bin_gather(const GatherArgs<T>* __restrict__ tab,
                                                     const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const GatherArgs<T>& a) {
        bin_gather_body<T>(b, as_global(a.perm), as_global(a.key), as_global(a.start), as_global(a.count), a.n, as_global(a.pos_in), as_global(a.vel_in), as_global(a.id_in), as_global(a.pos_out),
                           as_global(a.vel_out), as_global(a.id_out));
    });
}

template <typename T>
void launch_b_bin_gather(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_bin_gather<T>, dim3(L.blocks), dim3(256), 0, st, (const GatherArgs<T>*)L.args,
                       L.first, L.ns);
}
template void launch_b_bin_gather<float>(const BatchLaunch&, hipStream_t);
template void launch_b_bin_gather<double>(const BatchLaunch&, hipStream_t);

template <typename T>
void launch_bin_gather(const uint32_t* perm, const uint32_t* key, const uint32_t* start,
                       const uint32_t* count, int64_t n, const T* pos_in, const T* vel_in,
                       const uint32_t* id_in, T* pos_out, T* vel_out, uint32_t* id_out,
                       hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bin_gather<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, perm,
                       key, start, count, n, pos_in, vel_in, id_in, pos_out, vel_out, id_out);
}

template void launch_bin_gather<float>(const uint32_t*, const uint32_t*, const uint32_t*,
                                       const uint32_t*, int64_t, const float*, const float*,
                                       const uint32_t*, float*, float*, uint32_t*, hipStream_t);
template void launch_bin_gather<double>(const uint32_t*, const uint32_t*, const uint32_t*,
                                        const uint32_t*, int64_t, const double*, const double*,
                                        const uint32_t*, double*, double*, uint32_t*, hipStream_t);

// ---------------------------------------------------------------------------
// reseeding (paper Sec. 3.1.2, closing paragraph): a fluid cell holding k
// particles, 0 < k < sub^3, is refilled to sub^3. Plan: the number of new
// particles per cell; its exclusive scan spreads the binned particles apart
// (the gather above) and numbers the new ones; fill: the new particles, in
// jitter subcells k .. sub^3 - 1, with the mean velocity of the cell's k.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_reseed_plan(const uint32_t* __restrict__ count, int64_t C,
                                                     uint32_t target, uint32_t* __restrict__ add)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= C) return;
    const uint32_t k = count[c];
    add[c] = (k > 0 && k < target) ? target - k : 0u;
}

void launch_reseed_plan(const uint32_t* count, int64_t C, uint32_t target, uint32_t* add, hipStream_t st)
{
    if (C <= 0) return;
    hipLaunchKernelGGL(k_reseed_plan, dim3((unsigned)((C + 255) / 256)), dim3(256), 0, st, count, C, target,
                       add);
}

// the last prefix plus the last count: the number of new particles
__global__ void k_reseed_total(const uint32_t* __restrict__ add, const uint32_t* __restrict__ off, int64_t C,
                               uint32_t* __restrict__ total)
{
    if (threadIdx.x == 0) total[0] = C > 0 ? off[C - 1] + add[C - 1] : 0u;
}

void launch_reseed_total(const uint32_t* add, const uint32_t* off, int64_t C, uint32_t* total, hipStream_t st)
{
    hipLaunchKernelGGL(k_reseed_total, dim3(1), dim3(64), 0, st, add, off, C, total);
}

// SplitMix64 (Steele, Lea & Flood 2014): element `index` of the sequence of
// `seed`, top 53 bits as a double in [0, 1)
__device__ inline double splitmix_unit(uint64_t seed, uint64_t index)
{
    uint64_t z = seed + (index + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * 0x1.0p-53;
}

// x rounded to T, then moved one representable value at a time until the
// binning's exact floor puts it in cell i (rounding can land it on a face)
template <typename T>
__device__ inline T into_cell(double x, int i, double dx, double inv_dx, int n)
{
    T v = (T)x;
    for (int it = 0; it < 8 && exact_cell_floor((double)v, dx, inv_dx, n) < i; ++it)
        v = nextafter(v, (T)INFINITY);
    for (int it = 0; it < 8 && exact_cell_floor((double)v, dx, inv_dx, n) > i; ++it)
        v = nextafter(v, (T)-INFINITY);
    return v;
}

// One thread per cell. count/start become those of the refilled cells; the
// cell's binned particles already sit at start + off (the spread gather).
template <typename T>
__global__ __launch_bounds__(256) void k_reseed_fill(Geo g, int sub, uint64_t seed, uint64_t step,
                                                     uint32_t* __restrict__ count, uint32_t* __restrict__ start,
                                                     const uint32_t* __restrict__ add,
                                                     const uint32_t* __restrict__ off, uint32_t n_old,
                                                     int64_t n, T* __restrict__ pos, T* __restrict__ vel,
                                                     uint32_t* __restrict__ id)
{
#pragma clang fp contract(off)
    const int64_t C = (int64_t)g.nx * g.ny * g.nz;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= C) return;
    const uint32_t k = count[c], a = add[c], o = off[c];
    const uint32_t s0 = start[c] + o;
    start[c] = s0;
    count[c] = k + a;
    if (a == 0) return;
    double mean[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        double sum = 0.0;
        for (uint32_t q = 0; q < k; ++q) sum += (double)vel[ax * n + s0 + q];
        mean[ax] = sum / (double)k;
    }
    const int i = (int)(c % g.nx), j = (int)((c / g.nx) % g.ny), kk = (int)(c / ((int64_t)g.nx * g.ny));
    const uint64_t per = (uint64_t)sub * sub * sub;
    for (uint32_t t = 0; t < a; ++t) {
        const uint32_t s = k + t;
        const int sx = (int)(s % sub), sy = (int)((s / sub) % sub), sz = (int)(s / (sub * sub));
        const uint64_t ctr = 3u * (per * ((uint64_t)C * (step + 1) + (uint64_t)c) + s);
        const double x = (((double)sx + splitmix_unit(seed, ctr + 0)) / sub + i) * g.dx;
        const double y = (((double)sy + splitmix_unit(seed, ctr + 1)) / sub + j) * g.dx;
        const double z = (((double)sz + splitmix_unit(seed, ctr + 2)) / sub + kk) * g.dx;
        const int64_t d = (int64_t)s0 + s;
        pos[d] = into_cell<T>(x, i, g.dx, g.inv_dx, g.nx);
        pos[n + d] = into_cell<T>(y, j, g.dx, g.inv_dx, g.ny);
        pos[2 * n + d] = into_cell<T>(z, kk, g.dx, g.inv_dx, g.nz);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) vel[ax * n + d] = (T)mean[ax];
        id[d] = n_old + o + t;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_bin_gather_spread(
    const uint32_t* __restrict__ perm, const uint32_t* __restrict__ key,
    const uint32_t* __restrict__ start, const uint32_t* __restrict__ count, int64_t n,
    const T* __restrict__ pos_in, const T* __restrict__ vel_in, const uint32_t* __restrict__ id_in,
    T* __restrict__ pos_out, T* __restrict__ vel_out, uint32_t* __restrict__ id_out,
    const uint32_t* __restrict__ spread, int64_t n_out)
{
    bin_gather_body<T, true>(plain_blk(), perm, key, start, count, n, pos_in, vel_in, id_in, pos_out, vel_out,
                             id_out, spread, n_out);
}

template <typename T>
void launch_reseed_move(const Geo& g, int sub, uint64_t seed, uint64_t step, const uint32_t* perm,
                        const uint32_t* key, uint32_t* start, uint32_t* count, const uint32_t* add,
                        const uint32_t* off, int64_t n, int64_t n_out, const T* pos_in, const T* vel_in,
                        const uint32_t* id_in, T* pos_out, T* vel_out, uint32_t* id_out, hipStream_t st)
{
    if (n > 0)
        hipLaunchKernelGGL(k_bin_gather_spread<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, perm,
                           key, start, count, n, pos_in, vel_in, id_in, pos_out, vel_out, id_out, off, n_out);
    const int64_t C = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_reseed_fill<T>, dim3((unsigned)((C + 255) / 256)), dim3(256), 0, st, g, sub, seed, step,
                       count, start, add, off, (uint32_t)n, n_out, pos_out, vel_out, id_out);
}

template void launch_reseed_move<float>(const Geo&, int, uint64_t, uint64_t, const uint32_t*, const uint32_t*,
                                        uint32_t*, uint32_t*, const uint32_t*, const uint32_t*, int64_t, int64_t,
                                        const float*, const float*, const uint32_t*, float*, float*, uint32_t*,
                                        hipStream_t);
template void launch_reseed_move<double>(const Geo&, int, uint64_t, uint64_t, const uint32_t*, const uint32_t*,
                                         uint32_t*, uint32_t*, const uint32_t*, const uint32_t*, int64_t,
                                         int64_t, const double*, const double*, const uint32_t*, double*,
                                         double*, uint32_t*, hipStream_t);

// ---------------------------------------------------------------------------
// active tiles (the fluid-cells vector of Sec. 3.1.5, at tile granularity)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void tile_flags_body(Blk b, Geo g, const uint32_t* __restrict__ count,
                                                uint32_t* __restrict__ tile_flag)
{
    const int t = b.id;
    const int ti = t % g.tx, tj = (t / g.tx) % g.ty, tk = t / (g.tx * g.ty);
    int any = 0;
    for (int l = threadIdx.x; l < TILE_CELLS; l += 256) {
        const int i = ti * TILE + (l & 7), j = tj * TILE + ((l >> 3) & 7), k = tk * TILE + (l >> 6);
        if (i < g.nx && j < g.ny && k < g.nz)
            any |= count[i + (int64_t)g.nx * (j + (int64_t)g.ny * k)] > 0;
    }
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) tile_flag[t] = any ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_tile_flags(Geo g, const uint32_t* __restrict__ count,
                                                    uint32_t* __restrict__ tile_flag)
{
    tile_flags_body(plain_blk(), g, count, tile_flag);
}

__global__ __launch_bounds__(256) void kb_tile_flags(const TileFlagsArgs* __restrict__ tab,
                                                     const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const TileFlagsArgs& a) {
        tile_flags_body(b, a.g, as_global(a.count), as_global(a.tile_flag));
    });
}

void launch_b_tile_flags(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_tile_flags, dim3(L.blocks), dim3(256), 0, st, (const TileFlagsArgs*)L.args, L.first,
                       L.ns);
}

// slot of each tile (-1 when inactive), the active list, and for every
// active tile the slots of its six face neighbours (-x,+x,-y,+y,-z,+z; -1 when
// outside the domain or inactive)
__device__ __forceinline__ void tile_compact_body(Blk b, Geo g, const uint32_t* __restrict__ flag,
                                                  const uint32_t* __restrict__ excl,
                                                  int32_t* __restrict__ tile_slot,
                                                  uint32_t* __restrict__ tile_list,
                                                  int32_t* __restrict__ tile_nbr,
                                                  uint32_t* __restrict__ d_nactive)
{
    const int64_t T = (int64_t)g.tx * g.ty * g.tz;
    const int64_t t = (int64_t)b.id * 256 + threadIdx.x;
    if (t >= T) return;
    if (t == T - 1) *d_nactive = excl[t] + flag[t];
    if (!flag[t]) {
        tile_slot[t] = -1;
        return;
    }
    const int32_t slot = (int32_t)excl[t];
    tile_slot[t] = slot;
    tile_list[slot] = (uint32_t)t;
    const int ti = (int)(t % g.tx), tj = (int)((t / g.tx) % g.ty), tk = (int)(t / ((int64_t)g.tx * g.ty));
    const int off[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const int a = ti + off[d][0], b = tj + off[d][1], c = tk + off[d][2];
        int32_t ns = -1;
        if (a >= 0 && a < g.tx && b >= 0 && b < g.ty && c >= 0 && c < g.tz) {
            const int64_t tn = a + (int64_t)g.tx * (b + (int64_t)g.ty * c);
            if (flag[tn]) ns = (int32_t)excl[tn];
        }
        tile_nbr[(int64_t)slot * 6 + d] = ns;
    }
}

__global__ __launch_bounds__(256) void k_tile_compact(Geo g, const uint32_t* __restrict__ flag,
                                                      const uint32_t* __restrict__ excl,
                                                      int32_t* __restrict__ tile_slot,
                                                      uint32_t* __restrict__ tile_list,
                                                      int32_t* __restrict__ tile_nbr,
                                                      uint32_t* __restrict__ d_nactive)
{
    tile_compact_body(plain_blk(), g, flag, excl, tile_slot, tile_list, tile_nbr, d_nactive);
}

__global__ __launch_bounds__(256) void kb_tile_compact(const TileCompactArgs* __restrict__ tab,
                                                       const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const TileCompactArgs& a) {
        tile_compact_body(b, a.g, as_global(a.flag), as_global(a.excl), as_global(a.tile_slot), as_global(a.tile_list), as_global(a.tile_nbr), as_global(a.d_nactive));
    });
}

void launch_b_tile_compact(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_tile_compact, dim3(L.blocks), dim3(256), 0, st, (const TileCompactArgs*)L.args,
                       L.first, L.ns);
}

void launch_tiles(const Geo& g, const uint32_t* count, uint32_t* tile_flag, uint32_t* tile_excl,
                  int32_t* tile_slot, uint32_t* tile_list, int32_t* tile_nbr, uint32_t* d_nactive,
                  uint32_t* scan_tmp, hipStream_t st, bool flags_set)
{
    const int64_t T = tiles_of(g);
    if (!flags_set) hipLaunchKernelGGL(k_tile_flags, dim3((unsigned)T), dim3(256), 0, st, g, count, tile_flag);
    launch_exclusive_scan_u32(tile_flag, tile_excl, T, scan_tmp, st);
    hipLaunchKernelGGL(k_tile_compact, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, st, g,
                       tile_flag, tile_excl, tile_slot, tile_list, tile_nbr, d_nactive);
}

__global__ __launch_bounds__(256) void k_flags_from_count(const uint32_t* __restrict__ count,
                                                          int64_t n, uint8_t* __restrict__ flags)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) flags[i] = count[i] > 0 ? 1 : 0;
}

void launch_flags_from_count(const uint32_t* count, int64_t ncells, uint8_t* flags,
                             hipStream_t st)
{
    if (ncells <= 0) return;
    hipLaunchKernelGGL(k_flags_from_count, dim3((unsigned)((ncells + 255) / 256)), dim3(256), 0,
                       st, count, ncells, flags);
}

}  // namespace flipmi
