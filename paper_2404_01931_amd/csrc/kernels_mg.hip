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

// Index of the face neighbour f (-x,+x,-y,+y,-z,+z) of local cell (lx,ly,lz)
// of tile slot s, or -1 when that neighbour is in no active tile. nb[] holds
// the six neighbour-tile slots of s.
__device__ inline int64_t fine_neighbour(int s, int l, int lx, int ly, int lz, int f, const int32_t (&nb)[6])
{
    const int64_t base = (int64_t)s * TILE_CELLS;
    switch (f) {
    case 0: return lx > 0 ? base + l - 1 : (nb[0] >= 0 ? (int64_t)nb[0] * TILE_CELLS + l + 7 : -1);
    case 1: return lx < 7 ? base + l + 1 : (nb[1] >= 0 ? (int64_t)nb[1] * TILE_CELLS + l - 7 : -1);
    case 2: return ly > 0 ? base + l - 8 : (nb[2] >= 0 ? (int64_t)nb[2] * TILE_CELLS + l + 56 : -1);
    case 3: return ly < 7 ? base + l + 8 : (nb[3] >= 0 ? (int64_t)nb[3] * TILE_CELLS + l - 56 : -1);
    case 4: return lz > 0 ? base + l - 64 : (nb[4] >= 0 ? (int64_t)nb[4] * TILE_CELLS + l + 448 : -1);
    default: return lz < 7 ? base + l + 64 : (nb[5] >= 0 ? (int64_t)nb[5] * TILE_CELLS + l - 448 : -1);
    }
}

constexpr int MG_NT = 256;  // threads of the fine-level kernels (two cells each)

}  // namespace

// ---- cell types of the coarse levels -----------------------------------------

__global__ __launch_bounds__(256) void k_mg_types_fine(Geo g, const int32_t* __restrict__ tile_slot,
                                                       const uint8_t* __restrict__ diag, MgLevel c)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
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

__global__ __launch_bounds__(256) void k_mg_types(MgLevel f, MgLevel c)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= level_count(c)) return;
    const int i = (int)(q % c.nx), j = (int)((q / c.nx) % c.ny), k = (int)(q / ((int64_t)c.nx * c.ny));
    bool fluid = false;
    for (int o = 0; o < 8; ++o) {
        const int fi = 2 * i + (o & 1), fj = 2 * j + ((o >> 1) & 1), fk = 2 * k + (o >> 2);
        if (fi < f.nx && fj < f.ny && fk < f.nz && f.d[level_index(f, fi, fj, fk)] > 0) fluid = true;
    }
    c.d[q] = fluid ? (uint8_t)level_nc(c, i, j, k) : (uint8_t)0;
}

// ---- down: fine level (tile layout) to level 1 --------------------------------

// t = r - A (w r / n) on the fluid cells of each active tile, summed over the
// 2x2x2 children of every level-1 cell the tile covers (a tile of 8^3 cells
// covers a 4^3 block of level 1).
template <typename V>
__global__ __launch_bounds__(MG_NT) void k_mg_down_fine(int na_hint, Geo g, const uint32_t* __restrict__ tile_list,
                                                        const int32_t* __restrict__ nbr,
                                                        const uint8_t* __restrict__ diag,
                                                        const V* __restrict__ r, MgLevel c,
                                                        const PcgState* __restrict__ ps)
{
    __shared__ V tv[TILE_CELLS];
    if (ps->done != PCG_RUNNING) return;
    const Blk blk = plain_blk();
    const int na = na_hint >= 0 ? na_hint : ps->n_active;
    int t0, t1;
    tile_range(blk, na, t0, t1);
    const V w = mg_omega<V>();
    V* const cb = (V*)c.b;
    for (int s = t0; s < t1; ++s) {
        int32_t nb[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) nb[f] = nbr[(int64_t)s * 6 + f];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int l = threadIdx.x + h * MG_NT;
            const int lx = l & 7, ly = (l >> 3) & 7, lz = l >> 6;
            const int64_t e = (int64_t)s * TILE_CELLS + l;
            const int d = diag[e];
            V t = V(0);
            if (d > 0) {
                V nsum = V(0);
#pragma unroll
                for (int f = 0; f < 6; ++f) {
                    const int64_t q = fine_neighbour(s, l, lx, ly, lz, f, nb);
                    if (q >= 0) {
                        const int dn = diag[q];
                        if (dn > 0) nsum += r[q] / (V)dn;
                    }
                }
                t = (V(1) - w) * r[e] + w * nsum;
            }
            tv[l] = t;
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const int p = threadIdx.x, px = p & 3, py = (p >> 2) & 3, pz = p >> 4;
            const uint32_t tt = tile_list[s];
            const int ti = (int)(tt % g.tx), tj = (int)((tt / g.tx) % g.ty), tk = (int)(tt / ((uint32_t)g.tx * g.ty));
            const int ci = 4 * ti + px, cj = 4 * tj + py, ck = 4 * tk + pz;
            if (ci < c.nx && cj < c.ny && ck < c.nz) {
                V sum = V(0);
#pragma unroll
                for (int o = 0; o < 8; ++o)
                    sum += tv[(2 * px + (o & 1)) + 8 * (2 * py + ((o >> 1) & 1)) + 64 * (2 * pz + (o >> 2))];
                cb[level_index(c, ci, cj, ck)] = V(0.5) * sum;
            }
        }
        __syncthreads();
    }
}

// ---- down: dense level f to level c ---------------------------------------------

template <typename V>
__global__ __launch_bounds__(256) void k_mg_down(MgLevel f, MgLevel c, const PcgState* __restrict__ ps)
{
    if (ps->done != PCG_RUNNING) return;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= level_count(c)) return;
    const int i = (int)(q % c.nx), j = (int)((q / c.nx) % c.ny), k = (int)(q / ((int64_t)c.nx * c.ny));
    const V w = mg_omega<V>();
    const V* const fb = (const V*)f.b;
    V sum = V(0);
    for (int o = 0; o < 8; ++o) {
        const int fi = 2 * i + (o & 1), fj = 2 * j + ((o >> 1) & 1), fk = 2 * k + (o >> 2);
        if (fi >= f.nx || fj >= f.ny || fk >= f.nz) continue;
        const int64_t e = level_index(f, fi, fj, fk);
        if (f.d[e] == 0) continue;
        V nsum = V(0);
        const int ni[6] = {fi - 1, fi + 1, fi, fi, fi, fi};
        const int nj[6] = {fj, fj, fj - 1, fj + 1, fj, fj};
        const int nk[6] = {fk, fk, fk, fk, fk - 1, fk + 1};
        for (int n = 0; n < 6; ++n) {
            if (ni[n] < 0 || ni[n] >= f.nx || nj[n] < 0 || nj[n] >= f.ny || nk[n] < 0 || nk[n] >= f.nz) continue;
            const int64_t qn = level_index(f, ni[n], nj[n], nk[n]);
            const int dn = f.d[qn];
            if (dn > 0) nsum += fb[qn] / (V)dn;
        }
        sum += (V(1) - w) * fb[e] + w * nsum;
    }
    ((V*)c.b)[q] = V(0.5) * sum;
}

// ---- bottom: the coarsest level (at most 8^3 cells), one workgroup -------------

template <typename V>
__global__ __launch_bounds__(512) void k_mg_bottom(MgLevel L, const PcgState* __restrict__ ps)
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

// ---- up: dense level f from level c --------------------------------------------

template <typename V>
__global__ __launch_bounds__(256) void k_mg_up(MgLevel f, MgLevel c, const PcgState* __restrict__ ps)
{
    if (ps->done != PCG_RUNNING) return;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= level_count(f)) return;
    const int i = (int)(q % f.nx), j = (int)((q / f.nx) % f.ny), k = (int)(q / ((int64_t)f.nx * f.ny));
    const int d = f.d[q];
    V xo = V(0);
    if (d > 0) {
        const V w = mg_omega<V>();
        const V* const fb = (const V*)f.b;
        const V* const cx = (const V*)c.x;
        // y = w b / n + (P x_c) at this cell and its fluid neighbours
        auto y_at = [&](int a, int b2, int c2, int64_t e, int de) {
            return w * fb[e] / (V)de + cx[level_index(c, a >> 1, b2 >> 1, c2 >> 1)];
        };
        const V yc = y_at(i, j, k, q, d);
        V nsum = V(0);
        const int ni[6] = {i - 1, i + 1, i, i, i, i};
        const int nj[6] = {j, j, j - 1, j + 1, j, j};
        const int nk[6] = {k, k, k, k, k - 1, k + 1};
        for (int n = 0; n < 6; ++n) {
            if (ni[n] < 0 || ni[n] >= f.nx || nj[n] < 0 || nj[n] >= f.ny || nk[n] < 0 || nk[n] >= f.nz) continue;
            const int64_t qn = level_index(f, ni[n], nj[n], nk[n]);
            const int dn = f.d[qn];
            if (dn > 0) nsum += y_at(ni[n], nj[n], nk[n], qn, dn);
        }
        xo = yc + w * (fb[q] - (V)d * yc + nsum) / (V)d;
    }
    ((V*)f.x)[q] = xo;
}

// ---- up: fine level (tile layout) from level 1, with the CG partial sums -----

template <typename V>
__global__ __launch_bounds__(MG_NT) void k_mg_up_fine(int na_hint, Geo g, const uint32_t* __restrict__ tile_list,
                                                      const int32_t* __restrict__ nbr,
                                                      const uint8_t* __restrict__ diag,
                                                      const V* __restrict__ r, MgLevel c, V* __restrict__ z,
                                                      double* __restrict__ pslots, const PcgState* __restrict__ ps)
{
    __shared__ double red[2 * (MG_NT / WAVE)];
    if (ps->done != PCG_RUNNING) return;
    const Blk blk = plain_blk();
    const int na = na_hint >= 0 ? na_hint : ps->n_active;
    int t0, t1;
    tile_range(blk, na, t0, t1);
    const V w = mg_omega<V>();
    const V* const cx = (const V*)c.x;
    double rz = 0.0, rmax = 0.0;
    for (int s = t0; s < t1; ++s) {
        int32_t nb[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) nb[f] = nbr[(int64_t)s * 6 + f];
        const uint32_t tt = tile_list[s];
        const int ti = (int)(tt % g.tx), tj = (int)((tt / g.tx) % g.ty), tk = (int)(tt / ((uint32_t)g.tx * g.ty));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int l = threadIdx.x + h * MG_NT;
            const int lx = l & 7, ly = (l >> 3) & 7, lz = l >> 6;
            const int gi = 8 * ti + lx, gj = 8 * tj + ly, gk = 8 * tk + lz;
            const int64_t e = (int64_t)s * TILE_CELLS + l;
            const int d = diag[e];
            V zo = V(0);
            const V rc = r[e];
            if (d > 0) {
                const V yc = w * rc / (V)d + cx[level_index(c, gi >> 1, gj >> 1, gk >> 1)];
                const int oi[6] = {-1, 1, 0, 0, 0, 0}, oj[6] = {0, 0, -1, 1, 0, 0}, ok[6] = {0, 0, 0, 0, -1, 1};
                V nsum = V(0);
#pragma unroll
                for (int f = 0; f < 6; ++f) {
                    const int64_t q = fine_neighbour(s, l, lx, ly, lz, f, nb);
                    if (q >= 0) {
                        const int dn = diag[q];
                        if (dn > 0)
                            nsum += w * r[q] / (V)dn +
                                    cx[level_index(c, (gi + oi[f]) >> 1, (gj + oj[f]) >> 1, (gk + ok[f]) >> 1)];
                    }
                }
                zo = yc + w * (rc - (V)d * yc + nsum) / (V)d;
                rz += (double)rc * (double)zo;
                rmax = fmax(rmax, finite_or_inf(fabs((double)rc)));
            }
            z[e] = zo;
        }
    }
    const double prz = block_sum<MG_NT>(rz, red);
    const double pmx = block_max<MG_NT>(rmax, red);
    if (threadIdx.x == 0) {  // completed by the next direction kernel
        slot_rho(pslots, blk.n)[blk.id] = prz;
        slot_max(pslots, blk.n)[blk.id] = pmx;
    }
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
void launch_mg_vcycle(int groups, int na_hint, const Geo& g, const uint32_t* tile_list, const int32_t* tile_nbr,
                      const uint8_t* diag, const V* r, V* z, const MgLevel* lv, int nlev, double* pslots,
                      const PcgState* ps, hipStream_t st)
{
    hipLaunchKernelGGL(k_mg_down_fine<V>, dim3((unsigned)groups), dim3(MG_NT), 0, st, na_hint, g, tile_list, tile_nbr,
                       diag, r, lv[0], ps);
    for (int l = 0; l + 1 < nlev; ++l) {
        const int64_t n = (int64_t)lv[l + 1].nx * lv[l + 1].ny * lv[l + 1].nz;
        hipLaunchKernelGGL(k_mg_down<V>, dim3(blocks_for(n)), dim3(256), 0, st, lv[l], lv[l + 1], ps);
    }
    hipLaunchKernelGGL(k_mg_bottom<V>, dim3(1), dim3(512), 0, st, lv[nlev - 1], ps);
    for (int l = nlev - 2; l >= 0; --l) {
        const int64_t n = (int64_t)lv[l].nx * lv[l].ny * lv[l].nz;
        hipLaunchKernelGGL(k_mg_up<V>, dim3(blocks_for(n)), dim3(256), 0, st, lv[l], lv[l + 1], ps);
    }
    hipLaunchKernelGGL(k_mg_up_fine<V>, dim3((unsigned)groups), dim3(MG_NT), 0, st, na_hint, g, tile_list, tile_nbr,
                       diag, r, lv[0], z, pslots, ps);
}

template void launch_mg_vcycle<float>(int, int, const Geo&, const uint32_t*, const int32_t*, const uint8_t*,
                                      const float*, float*, const MgLevel*, int, double*, const PcgState*,
                                      hipStream_t);
template void launch_mg_vcycle<double>(int, int, const Geo&, const uint32_t*, const int32_t*, const uint8_t*,
                                       const double*, double*, const MgLevel*, int, double*, const PcgState*,
                                       hipStream_t);

}  // namespace flipmi
