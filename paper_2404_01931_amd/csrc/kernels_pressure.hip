// Pressure projection (paper Sec. 3.1.7): right-hand side from the discrete
// divergence (Eq. (6)), matrix-free seven-point operator, Jacobi-preconditioned
// conjugate gradient, and the pressure-gradient update of the faces (Eq. (5)).
//
// Layout: the solver's vectors are stored per active 8x8x8 tile (512 cells,
// x-fastest), so a workgroup of 512 threads owns one tile and reads it with
// fully coalesced accesses. The stencil reads of a tile are staged in LDS
// together with the six 8x8 face halos taken from the neighbouring tiles.
//
// System: multiplying the Poisson equation by rho dx^2 / dt gives integer
// coefficients, (A p)_c = n_c p_c - sum over fluid neighbours p_nb, with n_c
// the number of neighbours inside the domain (air neighbours carry p = 0, the
// free-surface condition; wall neighbours are left out), and
// b_c = -(rho dx / dt) * (sum of face differences of the cell).
//
// CG is written with the preconditioned residual z = r / n_c stored in place
// of r (r = n_c z is recovered on the fly), so the direction update
// s = z + beta s needs no division for the stencil's neighbours:
//   direction kernel: s = z + beta s_old; q = A s; sigma = s.q; alpha = rho/sigma
//   update kernel:    x += alpha s; r = n z - alpha A s; z = r / n;
//                     rho' = r.z; max|r|; beta = rho'/rho; convergence test
// Each kernel finishes with a fixed-order grid reduction by its last block, so
// results are identical from run to run.
#include <cfloat>

#include "common.h"
#include "device_util.h"

namespace flipmi {

constexpr int PNT = TILE_CELLS;          // threads per tile workgroup
constexpr int HALO = 6 * TILE * TILE;    // 384 face-halo cells
constexpr int STAGE = TILE_CELLS + HALO; // 896

__device__ inline double finite_or_inf(double a) { return (a <= DBL_MAX) ? a : INFINITY; }

// local index (in the neighbouring tile) of halo cell m of face f
__device__ inline int halo_source(int f, int m)
{
    const int a = m & 7, b = m >> 3;
    switch (f) {
        case 0: return 7 + 8 * a + 64 * b;   // -x face: (7, a, b)
        case 1: return 8 * a + 64 * b;       // +x face: (0, a, b)
        case 2: return a + 56 + 64 * b;      // -y face: (a, 7, b)
        case 3: return a + 64 * b;           // +y face: (a, 0, b)
        case 4: return a + 8 * b + 448;      // -z face: (a, b, 7)
        default: return a + 8 * b;           // +z face: (a, b, 0)
    }
}

// sum of the six neighbour values of local cell l from the staged tile
template <typename V>
__device__ inline V neighbour_sum(const V* st, int l)
{
    const int lx = l & 7, ly = (l >> 3) & 7, lz = l >> 6;
    const V xm = st[lx > 0 ? l - 1 : TILE_CELLS + 0 * 64 + ly + 8 * lz];
    const V xp = st[lx < 7 ? l + 1 : TILE_CELLS + 1 * 64 + ly + 8 * lz];
    const V ym = st[ly > 0 ? l - 8 : TILE_CELLS + 2 * 64 + lx + 8 * lz];
    const V yp = st[ly < 7 ? l + 8 : TILE_CELLS + 3 * 64 + lx + 8 * lz];
    const V zm = st[lz > 0 ? l - 64 : TILE_CELLS + 4 * 64 + lx + 8 * ly];
    const V zp = st[lz < 7 ? l + 64 : TILE_CELLS + 5 * 64 + lx + 8 * ly];
    return ((xm + xp) + (ym + yp)) + (zm + zp);
}

// ---------------------------------------------------------------------------
// right-hand side and solver start (x = 0, z = b / n, s = 0)
// ---------------------------------------------------------------------------

template <typename T, typename V>
__global__ __launch_bounds__(PNT) void k_rhs(Geo g, const uint32_t* __restrict__ tile_list,
                                             const uint32_t* __restrict__ count,
                                             const T* __restrict__ u, const T* __restrict__ v,
                                             const T* __restrict__ w, T scale,
                                             uint8_t* __restrict__ diag, V* __restrict__ b,
                                             V* __restrict__ z, V* __restrict__ x,
                                             V* __restrict__ s0, V* __restrict__ s1,
                                             double* __restrict__ partials, int64_t pstride,
                                             PcgState* __restrict__ ps, double tol, int max_iters)
{
    __shared__ double red[PNT / WAVE];
    __shared__ bool last;
    const int slot = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t t = tile_list[slot];
    const int ti = (int)(t % g.tx), tj = (int)((t / g.tx) % g.ty), tk = (int)(t / ((uint32_t)g.tx * g.ty));
    const int l = threadIdx.x;
    const int i = ti * TILE + (l & 7), j = tj * TILE + ((l >> 3) & 7), k = tk * TILE + (l >> 6);
    int d = 0;
    T bv = T(0);
    if (i < g.nx && j < g.ny && k < g.nz) {
        const int64_t c = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
        if (count[c] > 0) {
            d = (i > 0) + (i < g.nx - 1) + (j > 0) + (j < g.ny - 1) + (k > 0) + (k < g.nz - 1);
            const int64_t uX = g.nx + 1, vY = g.ny + 1;
            const int64_t fu = i + uX * (j + (int64_t)g.ny * k);
            const int64_t fv = i + (int64_t)g.nx * (j + vY * k);
            const int64_t fw = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
            const int64_t wZ = (int64_t)g.nx * g.ny;
            const T div = (u[fu + 1] - u[fu]) + (v[fv + g.nx] - v[fv]) + (w[fw + wZ] - w[fw]);
            bv = scale * div;
        }
    }
    const int64_t e = (int64_t)slot * TILE_CELLS + l;
    const V bq = (V)bv;
    const V zq = d ? bq / (V)d : V(0);
    diag[e] = (uint8_t)d;
    b[e] = bq;
    z[e] = zq;
    x[e] = V(0);
    s0[e] = V(0);
    s1[e] = V(0);
    const double rz = block_sum<PNT>((double)bq * (double)zq, red);
    const double mb = block_max<PNT>(finite_or_inf(fabs((double)bq)), red);
    const double nf = block_sum<PNT>(d ? 1.0 : 0.0, red);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = rz;
        partials[pstride + blockIdx.x] = mb;
        partials[2 * pstride + blockIdx.x] = nf;
    }
    if (!last_block_arrives(&ps->counter, &last)) return;
    const int nb = gridDim.x;
    const double rho = reduce_partials_sum<PNT>(partials, nb, red);
    const double max_b = reduce_partials_max<PNT>(partials + pstride, nb, red);
    const double nfl = reduce_partials_sum<PNT>(partials + 2 * pstride, nb, red);
    if (threadIdx.x == 0) {
        ps->rho = rho;
        ps->alpha = 0.0;
        ps->beta = 0.0;
        ps->max_b = max_b;
        ps->max_r = max_b;
        ps->tol = tol;
        ps->iter = 0;
        ps->max_iters = max_iters;
        ps->nfluid = (int)nfl;
        ps->n_active = nb;
        ps->done = !(max_b <= DBL_MAX) ? PCG_BREAKDOWN
                   : (max_b == 0.0)    ? PCG_CONVERGED
                   : (max_iters <= 0)  ? PCG_MAX_ITERS
                                       : PCG_RUNNING;
        ps->counter = 0u;
    }
}

template <typename T, typename V>
void launch_rhs(const Geo& g, int n_active, const uint32_t* tile_list, const uint32_t* count,
                const T* u, const T* v, const T* w, double scale, uint8_t* diag, V* b, V* z, V* x,
                V* s0, V* s1, double* partials, int64_t pstride, PcgState* st_dev, double tol,
                int max_iters, hipStream_t st)
{
    if (n_active <= 0) return;
    hipLaunchKernelGGL((k_rhs<T, V>), dim3((unsigned)n_active), dim3(PNT), 0, st, g, tile_list,
                       count, u, v, w, (T)scale, diag, b, z, x, s0, s1, partials, pstride, st_dev,
                       tol, max_iters);
}

template void launch_rhs<float, float>(const Geo&, int, const uint32_t*, const uint32_t*,
                                       const float*, const float*, const float*, double, uint8_t*,
                                       float*, float*, float*, float*, float*, double*, int64_t,
                                       PcgState*, double, int, hipStream_t);
template void launch_rhs<double, double>(const Geo&, int, const uint32_t*, const uint32_t*,
                                         const double*, const double*, const double*, double,
                                         uint8_t*, double*, double*, double*, double*, double*,
                                         double*, int64_t, PcgState*, double, int, hipStream_t);

// ---------------------------------------------------------------------------
// direction kernel: s = z + beta s_old, q = A s, sigma = s.q
// ---------------------------------------------------------------------------

template <typename V>
__global__ __launch_bounds__(PNT) void k_pcg_direction(const int32_t* __restrict__ nbr,
                                                       const uint8_t* __restrict__ diag,
                                                       const V* __restrict__ z,
                                                       const V* __restrict__ s_old,
                                                       V* __restrict__ s_new,
                                                       double* __restrict__ partials,
                                                       PcgState* __restrict__ ps)
{
    __shared__ V stg[STAGE];
    __shared__ double red[PNT / WAVE];
    __shared__ bool last;
    if (ps->done != PCG_RUNNING) return;
    const V beta = (V)ps->beta;
    const int slot = xcd_remap(blockIdx.x, gridDim.x);
    const int l = threadIdx.x;
    const int64_t e = (int64_t)slot * TILE_CELLS + l;
    const V sc = fma(beta, s_old[e], z[e]);
    const int d = diag[e];
    s_new[e] = sc;
    stg[l] = sc;
    if (l < HALO) {
        const int f = l >> 6;
        const int32_t ns = nbr[(int64_t)slot * 6 + f];
        V hv = V(0);
        if (ns >= 0) {
            const int64_t en = (int64_t)ns * TILE_CELLS + halo_source(f, l & 63);
            hv = fma(beta, s_old[en], z[en]);
        }
        stg[TILE_CELLS + l] = hv;
    }
    __syncthreads();
    const V q = d ? (V)d * sc - neighbour_sum(stg, l) : V(0);
    const double part = block_sum<PNT>((double)sc * (double)q, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = part;
    if (!last_block_arrives(&ps->counter, &last)) return;
    const double sigma = reduce_partials_sum<PNT>(partials, gridDim.x, red);
    if (threadIdx.x == 0) {
        if (!(sigma > 0.0) || !(sigma <= DBL_MAX))
            ps->done = PCG_BREAKDOWN;
        else
            ps->alpha = ps->rho / sigma;
        ps->counter = 0u;
    }
}

template <typename V>
void launch_pcg_direction(int n_active, const int32_t* tile_nbr, const uint8_t* diag, const V* z,
                          const V* s_old, V* s_new, double* partials, PcgState* st_dev,
                          hipStream_t st)
{
    if (n_active <= 0) return;
    hipLaunchKernelGGL(k_pcg_direction<V>, dim3((unsigned)n_active), dim3(PNT), 0, st, tile_nbr,
                       diag, z, s_old, s_new, partials, st_dev);
}

template void launch_pcg_direction<float>(int, const int32_t*, const uint8_t*, const float*,
                                          const float*, float*, double*, PcgState*, hipStream_t);
template void launch_pcg_direction<double>(int, const int32_t*, const uint8_t*, const double*,
                                           const double*, double*, double*, PcgState*,
                                           hipStream_t);

// ---------------------------------------------------------------------------
// update kernel: x += alpha s; r = n z - alpha A s; z = r / n; r.z; max|r|
// ---------------------------------------------------------------------------

template <typename V>
__global__ __launch_bounds__(PNT) void k_pcg_update(const int32_t* __restrict__ nbr,
                                                    const uint8_t* __restrict__ diag,
                                                    const V* __restrict__ s, V* __restrict__ x,
                                                    V* __restrict__ z, double* __restrict__ partials,
                                                    int64_t pstride, PcgState* __restrict__ ps)
{
    __shared__ V stg[STAGE];
    __shared__ double red[PNT / WAVE];
    __shared__ bool last;
    if (ps->done != PCG_RUNNING) return;
    const V alpha = (V)ps->alpha;
    const int slot = xcd_remap(blockIdx.x, gridDim.x);
    const int l = threadIdx.x;
    const int64_t e = (int64_t)slot * TILE_CELLS + l;
    const V sc = s[e];
    const int d = diag[e];
    stg[l] = sc;
    if (l < HALO) {
        const int f = l >> 6;
        const int32_t ns = nbr[(int64_t)slot * 6 + f];
        stg[TILE_CELLS + l] = ns >= 0 ? s[(int64_t)ns * TILE_CELLS + halo_source(f, l & 63)] : V(0);
    }
    __syncthreads();
    double rz = 0.0, rmax = 0.0;
    if (d) {
        const V q = (V)d * sc - neighbour_sum(stg, l);
        x[e] = fma(alpha, sc, x[e]);
        const V r = fma((V)d, z[e], -alpha * q);
        const V zn = r / (V)d;
        z[e] = zn;
        rz = (double)r * (double)zn;
        rmax = finite_or_inf(fabs((double)r));
    }
    const double prz = block_sum<PNT>(rz, red);
    const double pmx = block_max<PNT>(rmax, red);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = prz;
        partials[pstride + blockIdx.x] = pmx;
    }
    if (!last_block_arrives(&ps->counter, &last)) return;
    const double rho_new = reduce_partials_sum<PNT>(partials, gridDim.x, red);
    const double max_r = reduce_partials_max<PNT>(partials + pstride, gridDim.x, red);
    if (threadIdx.x == 0) {
        const int it = ps->iter + 1;
        ps->iter = it;
        ps->max_r = max_r;
        if (!(max_r <= DBL_MAX) || !(fabs(rho_new) <= DBL_MAX))
            ps->done = PCG_BREAKDOWN;
        else if (max_r <= ps->tol * ps->max_b)
            ps->done = PCG_CONVERGED;
        else if (it >= ps->max_iters)
            ps->done = PCG_MAX_ITERS;
        ps->beta = rho_new / ps->rho;
        ps->rho = rho_new;
        ps->counter = 0u;
    }
}

template <typename V>
void launch_pcg_update(int n_active, const int32_t* tile_nbr, const uint8_t* diag, const V* s, V* x,
                       V* z, double* partials, int64_t pstride, PcgState* st_dev, hipStream_t st)
{
    if (n_active <= 0) return;
    hipLaunchKernelGGL(k_pcg_update<V>, dim3((unsigned)n_active), dim3(PNT), 0, st, tile_nbr, diag,
                       s, x, z, partials, pstride, st_dev);
}

template void launch_pcg_update<float>(int, const int32_t*, const uint8_t*, const float*, float*,
                                       float*, double*, int64_t, PcgState*, hipStream_t);
template void launch_pcg_update<double>(int, const int32_t*, const uint8_t*, const double*, double*,
                                        double*, double*, int64_t, PcgState*, hipStream_t);

// ---------------------------------------------------------------------------
// projection, Eq. (5): u = u* - (dt / (rho dx)) (p+ - p-) on every non-wall
// face touching a fluid cell; p = 0 in air
// ---------------------------------------------------------------------------

template <typename V>
__device__ inline V tile_value(const Geo& g, const int32_t* __restrict__ tile_slot,
                               const V* __restrict__ p, int i, int j, int k)
{
    const int64_t t = (i >> 3) + (int64_t)g.tx * ((j >> 3) + (int64_t)g.ty * (k >> 3));
    const int32_t s = tile_slot[t];
    return s >= 0 ? p[(int64_t)s * TILE_CELLS + (i & 7) + 8 * (j & 7) + 64 * (k & 7)] : V(0);
}

template <typename T, typename V, int A>
__global__ __launch_bounds__(256) void k_project(Geo g, const uint32_t* __restrict__ count,
                                                 const int32_t* __restrict__ tile_slot,
                                                 const V* __restrict__ p, const T* __restrict__ star,
                                                 T* __restrict__ out, T scale)
{
    const int dX = g.nx + (A == 0), dY = g.ny + (A == 1), dZ = g.nz + (A == 2);
    const int64_t F = (int64_t)dX * dY * dZ;
    const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (f >= F) return;
    const int i = (int)(f % dX), j = (int)((f / dX) % dY), k = (int)(f / ((int64_t)dX * dY));
    const int idx = A == 0 ? i : (A == 1 ? j : k);
    const int lim = A == 0 ? g.nx : (A == 1 ? g.ny : g.nz);
    T o = star[f];
    if (idx > 0 && idx < lim) {
        const int im = i - (A == 0), jm = j - (A == 1), km = k - (A == 2);
        const bool fp = count[i + (int64_t)g.nx * (j + (int64_t)g.ny * k)] > 0;
        const bool fm = count[im + (int64_t)g.nx * (jm + (int64_t)g.ny * km)] > 0;
        if (fp || fm) {
            const T pp = fp ? (T)tile_value(g, tile_slot, p, i, j, k) : T(0);
            const T pm = fm ? (T)tile_value(g, tile_slot, p, im, jm, km) : T(0);
            o = o - scale * (pp - pm);
        }
    }
    out[f] = o;
}

template <typename T, typename V>
void launch_project(const Geo& g, int axis, const uint32_t* count, const int32_t* tile_slot,
                    const V* p, const T* star, T* out, T scale, hipStream_t st)
{
    const int64_t F = (int64_t)(g.nx + (axis == 0)) * (g.ny + (axis == 1)) * (g.nz + (axis == 2));
    const dim3 grid((unsigned)((F + 255) / 256)), block(256);
    if (axis == 0)
        hipLaunchKernelGGL((k_project<T, V, 0>), grid, block, 0, st, g, count, tile_slot, p, star, out, scale);
    else if (axis == 1)
        hipLaunchKernelGGL((k_project<T, V, 1>), grid, block, 0, st, g, count, tile_slot, p, star, out, scale);
    else
        hipLaunchKernelGGL((k_project<T, V, 2>), grid, block, 0, st, g, count, tile_slot, p, star, out, scale);
}

template void launch_project<float, float>(const Geo&, int, const uint32_t*, const int32_t*,
                                           const float*, const float*, float*, float, hipStream_t);
template void launch_project<double, double>(const Geo&, int, const uint32_t*, const int32_t*,
                                             const double*, const double*, double*, double,
                                             hipStream_t);

// ---------------------------------------------------------------------------
// compact tile storage -> dense cell array (readback of b and p)
// ---------------------------------------------------------------------------

template <typename V, typename O>
__global__ __launch_bounds__(256) void k_densify(Geo g, const int32_t* __restrict__ tile_slot,
                                                 const uint8_t* __restrict__ diag,
                                                 const V* __restrict__ src, O* __restrict__ dst)
{
    const int64_t C = (int64_t)g.nx * g.ny * g.nz;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= C) return;
    const int i = (int)(c % g.nx), j = (int)((c / g.nx) % g.ny), k = (int)(c / ((int64_t)g.nx * g.ny));
    const int64_t t = (i >> 3) + (int64_t)g.tx * ((j >> 3) + (int64_t)g.ty * (k >> 3));
    const int32_t s = tile_slot[t];
    O v = O(0);
    if (s >= 0) {
        const int64_t e = (int64_t)s * TILE_CELLS + (i & 7) + 8 * (j & 7) + 64 * (k & 7);
        if (diag[e]) v = (O)src[e];
    }
    dst[c] = v;
}

template <typename V, typename O>
void launch_densify(const Geo& g, const int32_t* tile_slot, const uint8_t* diag, const V* src,
                    O* dst, hipStream_t st)
{
    const int64_t C = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL((k_densify<V, O>), dim3((unsigned)((C + 255) / 256)), dim3(256), 0, st, g,
                       tile_slot, diag, src, dst);
}

template void launch_densify<float, float>(const Geo&, const int32_t*, const uint8_t*, const float*,
                                           float*, hipStream_t);
template void launch_densify<double, double>(const Geo&, const int32_t*, const uint8_t*,
                                             const double*, double*, hipStream_t);

}  // namespace flipmi
