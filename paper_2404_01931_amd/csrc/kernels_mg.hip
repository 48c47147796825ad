// Multigrid preconditioner for the pressure solve: one V-cycle z = M r per
// conjugate-gradient iteration (the preconditioned CG the paper solves the
// pressure Poisson equation with, Sec. 3.1.7; the paper leaves the
// preconditioner to its solver reference).
//
// Levels: level 0 is the fine grid in the solver's tile layout; each coarser
// level halves every axis (ceil) and is stored dense, i fastest, down to a
// grid of at most 8 cells per axis. A coarse cell is fluid when any of its
// (up to 8) children is; its n_c counts its neighbours inside the level's
// box, as on the fine grid, and air neighbours hold 0.
//
// One V-cycle, with damped Jacobi (w = 6/7) as the smoother:
//   down, level l:  x0 = w b / n;  t = b - A x0;  b_{l+1} = (R t) / 2
//   bottom:         x = 0, then 20 sweeps x += w (b - A x) / n
//   up, level l:    y = x0 + P x_{l+1};  x_l = y + w (b - A y) / n
// R sums the children of a coarse cell, P copies a coarse value to its fluid
// children (P = R^T), and the coarse equation is scaled by 1/2 (with these
// transfers the Galerkin product R A P is 4 times the coarse stencil, while
// a smooth error is corrected best with twice it). One pre- and one
// post-sweep with the same smoother, a fixed number of bottom sweeps and
// P = R^T make the cycle a fixed symmetric positive definite operator, as CG
// needs. Level 0 reads r and writes z; the fine up-kernel also forms the
// partial sums r . z and max |r| that the next direction kernel completes.
//
// Every kernel first reads the solver state and exits when the solve is over.
#include "batch.h"
#include "common.h"
#include "device_util.h"

namespace flipmi {

namespace {

template <typename V>
__device__ inline V mg_omega()
{
    return V(6) / V(7);
}

__device__ inline int level_count(const MgLevel& L) { return L.nx * L.ny * L.nz; }

__device__ inline int64_t level_index(const MgLevel& L, int i, int j, int k)
{
    return i + (int64_t)L.nx * (j + (int64_t)L.ny * k);
}

__device__ inline int level_nc(const MgLevel& L, int i, int j, int k)
{
    return (i > 0) + (i < L.nx - 1) + (j > 0) + (j < L.ny - 1) + (k > 0) + (k < L.nz - 1);
}

// a level whose pointers came from a batched launch's table, marked global
// (pointers loaded from memory are otherwise generic, and generic accesses
// make every wait a full one)
__device__ inline MgLevel glob(MgLevel L)
{
    L.b = as_global(L.b);
    L.x = as_global(L.x);
    L.d = as_global(L.d);
    return L;
}


}  // namespace

// ---- cell types of the coarse levels -----------------------------------------

__device__ __forceinline__ void mg_types_fine_body(Blk b, const Geo& g, const int32_t* __restrict__ tile_slot,
                                                   const uint8_t* __restrict__ diag, const MgLevel& c)
{
    const int64_t q = (int64_t)b.id * 256 + threadIdx.x;
    if (q >= level_count(c)) return;
    const int i = (int)(q % c.nx), j = (int)((q / c.nx) % c.ny), k = (int)(q / ((int64_t)c.nx * c.ny));
    bool fluid = false;
    for (int o = 0; o < 8; ++o) {
        const int gi = 2 * i + (o & 1), gj = 2 * j + ((o >> 1) & 1), gk = 2 * k + (o >> 2);
        if (gi >= g.nx || gj >= g.ny || gk >= g.nz) continue;
        const int32_t s = tile_slot[(gi >> 3) + (int64_t)g.tx * ((gj >> 3) + (int64_t)g.ty * (gk >> 3))];
        if (s >= 0 && diag[(int64_t)s * TILE_CELLS + (gi & 7) + 8 * (gj & 7) + 64 * (gk & 7)] > 0) fluid = true;
    }
    c.d[q] = fluid ? (uint8_t)level_nc(c, i, j, k) : (uint8_t)0;
}

__global__ __launch_bounds__(256) void k_mg_types_fine(Geo g, const int32_t* __restrict__ tile_slot,
                                                       const uint8_t* __restrict__ diag, MgLevel c)
{
    mg_types_fine_body(plain_blk(), g, tile_slot, diag, c);
}

__global__ __launch_bounds__(256) void kb_mg_types_fine(const MgTypesFineArgs* __restrict__ tab,
                                                        const uint32_t* __restrict__ first, int ns)
{
    Blk b;
    const MgTypesFineArgs& a = batch_args(tab, first, ns, b);
    mg_types_fine_body(b, a.g, as_global(a.tile_slot), as_global(a.diag), glob(a.c));
}

__device__ __forceinline__ void mg_types_body(Blk b, const MgLevel& f, const MgLevel& c)
{
    const int64_t q = (int64_t)b.id * 256 + threadIdx.x;
    if (q >= level_count(c)) return;
    const int i = (int)(q % c.nx), j = (int)((q / c.nx) % c.ny), k = (int)(q / ((int64_t)c.nx * c.ny));
    bool fluid = false;
    for (int o = 0; o < 8; ++o) {
        const int fi = 2 * i + (o & 1), fj = 2 * j + ((o >> 1) & 1), fk = 2 * k + (o >> 2);
        if (fi < f.nx && fj < f.ny && fk < f.nz && f.d[level_index(f, fi, fj, fk)] > 0) fluid = true;
    }
    c.d[q] = fluid ? (uint8_t)level_nc(c, i, j, k) : (uint8_t)0;
}

__global__ __launch_bounds__(256) void k_mg_types(MgLevel f, MgLevel c) { mg_types_body(plain_blk(), f, c); }

__global__ __launch_bounds__(256) void kb_mg_types(const MgPairArgs* __restrict__ tab,
                                                   const uint32_t* __restrict__ first, int ns)
{
    Blk b;
    const MgPairArgs& a = batch_args(tab, first, ns, b);
    mg_types_body(b, glob(a.f), glob(a.c));
}

// ---- down: dense level f to level c ---------------------------------------------

// One thread per level-f cell of a 16 x 4 x 4 block (x fastest, so a row is
// one 64-byte segment); t = (1 - w) b + w sum of b / n over the fluid
// neighbours goes to LDS, and 32 threads sum the 2x2x2 children of the
// block's 8 x 2 x 2 parents. Every load is issued unconditionally (clamped
// address, masked value), so a thread waits for memory once.
constexpr int MGD_X = 16, MGD_Y = 4, MGD_Z = 4;

template <typename V>
__device__ inline V recip_nc(int d)
{
    return d ? V(1) / (V)d : V(0);
}

// workgroups of a restriction from level f: one per 16 x 4 x 4 block, x fastest
__host__ __device__ inline int mg_down_blocks_x(const MgLevel& f) { return (f.nx + MGD_X - 1) / MGD_X; }
__host__ __device__ inline int mg_down_blocks_y(const MgLevel& f) { return (f.ny + MGD_Y - 1) / MGD_Y; }
__host__ __device__ inline int64_t mg_down_blocks(const MgLevel& f)
{
    return (int64_t)mg_down_blocks_x(f) * mg_down_blocks_y(f) * ((f.nz + MGD_Z - 1) / MGD_Z);
}

template <typename V>
__device__ __forceinline__ void mg_down_body(Blk blk, const MgLevel& f, const MgLevel& c,
                                             const PcgState* __restrict__ ps)
{
    __shared__ V tv[MGD_Z][MGD_Y][MGD_X];
    if (ps->done != PCG_RUNNING) return;
    const int gbx = mg_down_blocks_x(f), gby = mg_down_blocks_y(f);
    const int bx = blk.id % gbx, by = (blk.id / gbx) % gby, bz = blk.id / (gbx * gby);
    const int lx = threadIdx.x & 15, ly = (threadIdx.x >> 4) & 3, lz = threadIdx.x >> 6;
    const int i = bx * MGD_X + lx, j = by * MGD_Y + ly, k = bz * MGD_Z + lz;
    const bool in = i < f.nx && j < f.ny && k < f.nz;
    const int ic = min(i, f.nx - 1), jc = min(j, f.ny - 1), kc = min(k, f.nz - 1);
    const V* const fb = (const V*)f.b;
    const int64_t e = level_index(f, ic, jc, kc);
    const int sx = 1, sy = f.nx;
    const int64_t sz = (int64_t)f.nx * f.ny;
    // neighbours inside the level (a missing one reads the cell itself, masked)
    const bool hm[6] = {ic > 0, ic < f.nx - 1, jc > 0, jc < f.ny - 1, kc > 0, kc < f.nz - 1};
    const int64_t off[6] = {-sx, sx, -sy, sy, -sz, sz};
    int dn[6];
    V bn[6];
#pragma unroll
    for (int n = 0; n < 6; ++n) {
        const int64_t q = hm[n] ? e + off[n] : e;
        dn[n] = f.d[q];
        bn[n] = fb[q];
    }
    const int d = f.d[e];
    const V b = fb[e];
    const V w = mg_omega<V>();
    V nsum = V(0);
#pragma unroll
    for (int n = 0; n < 6; ++n) nsum += (hm[n] && dn[n]) ? bn[n] * recip_nc<V>(dn[n]) : V(0);
    tv[lz][ly][lx] = (in && d) ? (V(1) - w) * b + w * nsum : V(0);
    __syncthreads();
    if (threadIdx.x < 32) {
        const int px = threadIdx.x & 7, py = (threadIdx.x >> 3) & 1, pz = threadIdx.x >> 4;
        const int ci = bx * (MGD_X / 2) + px, cj = by * (MGD_Y / 2) + py, ck = bz * (MGD_Z / 2) + pz;
        if (ci < c.nx && cj < c.ny && ck < c.nz) {
            const V sum = ((tv[2 * pz][2 * py][2 * px] + tv[2 * pz][2 * py][2 * px + 1]) +
                           (tv[2 * pz][2 * py + 1][2 * px] + tv[2 * pz][2 * py + 1][2 * px + 1])) +
                          ((tv[2 * pz + 1][2 * py][2 * px] + tv[2 * pz + 1][2 * py][2 * px + 1]) +
                           (tv[2 * pz + 1][2 * py + 1][2 * px] + tv[2 * pz + 1][2 * py + 1][2 * px + 1]));
            ((V*)c.b)[level_index(c, ci, cj, ck)] = V(0.5) * sum;
        }
    }
}

template <typename V>
__global__ __launch_bounds__(256) void k_mg_down(MgLevel f, MgLevel c, const PcgState* __restrict__ ps)
{
    mg_down_body<V>(plain_blk(), f, c, ps);
}

template <typename V>
__global__ __launch_bounds__(256) void kb_mg_down(const MgPairArgs* __restrict__ tab,
                                                  const uint32_t* __restrict__ first, int ns)
{
    Blk b;
    const MgPairArgs& a = batch_args(tab, first, ns, b);
    mg_down_body<V>(b, glob(a.f), glob(a.c), as_global(a.ps));
}

// ---- bottom: the coarsest level (at most 8^3 cells), one workgroup -------------

template <typename V>
__device__ __forceinline__ void mg_bottom_body(const MgLevel& L, const PcgState* __restrict__ ps)
{
    __shared__ V xs[2][512];
    if (ps->done != PCG_RUNNING) return;
    const int q = threadIdx.x;
    const int n = level_count(L);
    const bool own = q < n;
    const int i = q % L.nx, j = (q / L.nx) % L.ny, k = q / (L.nx * L.ny);
    const int d = own ? L.d[q] : 0;
    const V b = own ? ((const V*)L.b)[q] : V(0);
    const V w = mg_omega<V>();
    xs[0][q] = V(0);
    for (int it = 0; it < MG_BOTTOM_SWEEPS; ++it) {
        __syncthreads();
        const V* x = xs[it & 1];
        V xn = V(0);
        if (own && d > 0) {
            V nsum = V(0);
            if (i > 0) nsum += x[q - 1];
            if (i < L.nx - 1) nsum += x[q + 1];
            if (j > 0) nsum += x[q - L.nx];
            if (j < L.ny - 1) nsum += x[q + L.nx];
            if (k > 0) nsum += x[q - L.nx * L.ny];
            if (k < L.nz - 1) nsum += x[q + L.nx * L.ny];
            xn = x[q] + w * (b - (V)d * x[q] + nsum) / (V)d;
        }
        xs[(it + 1) & 1][q] = xn;
    }
    __syncthreads();
    if (own) ((V*)L.x)[q] = xs[MG_BOTTOM_SWEEPS & 1][q];
}

template <typename V>
__global__ __launch_bounds__(512) void k_mg_bottom(MgLevel L, const PcgState* __restrict__ ps)
{
    mg_bottom_body<V>(L, ps);
}

template <typename V>
__global__ __launch_bounds__(512) void kb_mg_bottom(const MgPairArgs* __restrict__ tab,
                                                    const uint32_t* __restrict__ first, int ns)
{
    Blk b;
    const MgPairArgs& a = batch_args(tab, first, ns, b);  // the coarsest level is f
    mg_bottom_body<V>(glob(a.f), as_global(a.ps));
}

// ---- up: dense level f from level c --------------------------------------------

// One thread per level-f cell; loads issued unconditionally as in k_mg_down.
template <typename V>
__device__ __forceinline__ void mg_up_body(Blk blk, const MgLevel& f, const MgLevel& c,
                                           const PcgState* __restrict__ ps)
{
    if (ps->done != PCG_RUNNING) return;
    const int64_t q0 = (int64_t)blk.id * 256 + threadIdx.x;
    const int64_t ncell = level_count(f);
    const bool in = q0 < ncell;
    const int64_t e = in ? q0 : ncell - 1;
    const int i = (int)(e % f.nx), j = (int)((e / f.nx) % f.ny), k = (int)(e / ((int64_t)f.nx * f.ny));
    const V* const fb = (const V*)f.b;
    const V* const cx = (const V*)c.x;
    const int64_t sz = (int64_t)f.nx * f.ny;
    const bool hm[6] = {i > 0, i < f.nx - 1, j > 0, j < f.ny - 1, k > 0, k < f.nz - 1};
    const int64_t off[6] = {-1, 1, -f.nx, f.nx, -sz, sz};
    const int pi[6] = {i - 1, i + 1, i, i, i, i}, pj[6] = {j, j, j - 1, j + 1, j, j},
              pk[6] = {k, k, k, k, k - 1, k + 1};
    int dn[6];
    V bn[6], xn[6];
#pragma unroll
    for (int n = 0; n < 6; ++n) {
        const int64_t qn = hm[n] ? e + off[n] : e;
        dn[n] = f.d[qn];
        bn[n] = fb[qn];
        const int a = hm[n] ? pi[n] : i, b2 = hm[n] ? pj[n] : j, c2 = hm[n] ? pk[n] : k;
        xn[n] = cx[level_index(c, a >> 1, b2 >> 1, c2 >> 1)];
    }
    const int d = f.d[e];
    const V bc = fb[e], xc = cx[level_index(c, i >> 1, j >> 1, k >> 1)];
    const V w = mg_omega<V>();
    // y = w b / n + (P x_c) at this cell and its fluid neighbours
    const V rd = recip_nc<V>(d);
    const V yc = w * bc * rd + xc;
    V nsum = V(0);
#pragma unroll
    for (int n = 0; n < 6; ++n) nsum += (hm[n] && dn[n]) ? w * bn[n] * recip_nc<V>(dn[n]) + xn[n] : V(0);
    if (in) ((V*)f.x)[e] = d ? yc + w * ((bc - (V)d * yc) + nsum) * rd : V(0);
}

template <typename V>
__global__ __launch_bounds__(256) void k_mg_up(MgLevel f, MgLevel c, const PcgState* __restrict__ ps)
{
    mg_up_body<V>(plain_blk(), f, c, ps);
}

template <typename V>
__global__ __launch_bounds__(256) void kb_mg_up(const MgPairArgs* __restrict__ tab,
                                                const uint32_t* __restrict__ first, int ns)
{
    Blk b;
    const MgPairArgs& a = batch_args(tab, first, ns, b);
    mg_up_body<V>(b, glob(a.f), glob(a.c), as_global(a.ps));
}

// ---- launchers -----------------------------------------------------------------

namespace {
inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }
}  // namespace

void launch_mg_types_fine(const Geo& g, const int32_t* tile_slot, const uint8_t* diag, const MgLevel& c,
                          hipStream_t st)
{
    const int64_t n = (int64_t)c.nx * c.ny * c.nz;
    hipLaunchKernelGGL(k_mg_types_fine, dim3(blocks_for(n)), dim3(256), 0, st, g, tile_slot, diag, c);
}

void launch_mg_types(const MgLevel& f, const MgLevel& c, hipStream_t st)
{
    const int64_t n = (int64_t)c.nx * c.ny * c.nz;
    hipLaunchKernelGGL(k_mg_types, dim3(blocks_for(n)), dim3(256), 0, st, f, c);
}

template <typename V>
void launch_mg_coarse(const MgLevel* lv, int nlev, const PcgState* ps, hipStream_t st)
{
    for (int l = 0; l + 1 < nlev; ++l)
        hipLaunchKernelGGL(k_mg_down<V>, dim3((unsigned)mg_down_blocks(lv[l])), dim3(256), 0, st, lv[l], lv[l + 1],
                           ps);
    hipLaunchKernelGGL(k_mg_bottom<V>, dim3(1), dim3(512), 0, st, lv[nlev - 1], ps);
    for (int l = nlev - 2; l >= 0; --l) {
        const int64_t n = (int64_t)lv[l].nx * lv[l].ny * lv[l].nz;
        hipLaunchKernelGGL(k_mg_up<V>, dim3(blocks_for(n)), dim3(256), 0, st, lv[l], lv[l + 1], ps);
    }
}

template void launch_mg_coarse<float>(const MgLevel*, int, const PcgState*, hipStream_t);
template void launch_mg_coarse<double>(const MgLevel*, int, const PcgState*, hipStream_t);

// ---- batched launchers (grids: see mg_batch_blocks) ------------------------------

int64_t mg_blocks(int kind, const MgLevel& f, const MgLevel& c)
{
    switch (kind) {
    case MG_B_TYPES: return blocks_for((int64_t)c.nx * c.ny * c.nz);
    case MG_B_DOWN: return mg_down_blocks(f);
    case MG_B_BOTTOM: return 1;
    default: return blocks_for((int64_t)f.nx * f.ny * f.nz);  // MG_B_UP
    }
}

void launch_b_mg_types_fine(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_mg_types_fine, dim3(L.blocks), dim3(256), 0, st, (const MgTypesFineArgs*)L.args, L.first,
                       L.ns);
}

void launch_b_mg_types(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_mg_types, dim3(L.blocks), dim3(256), 0, st, (const MgPairArgs*)L.args, L.first, L.ns);
}

template <typename V>
void launch_b_mg_level(int kind, const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    const MgPairArgs* a = (const MgPairArgs*)L.args;
    if (kind == MG_B_DOWN)
        hipLaunchKernelGGL(kb_mg_down<V>, dim3(L.blocks), dim3(256), 0, st, a, L.first, L.ns);
    else if (kind == MG_B_BOTTOM)
        hipLaunchKernelGGL(kb_mg_bottom<V>, dim3(L.blocks), dim3(512), 0, st, a, L.first, L.ns);
    else
        hipLaunchKernelGGL(kb_mg_up<V>, dim3(L.blocks), dim3(256), 0, st, a, L.first, L.ns);
}
template void launch_b_mg_level<float>(int, const BatchLaunch&, hipStream_t);
template void launch_b_mg_level<double>(int, const BatchLaunch&, hipStream_t);

}  // namespace flipmi
