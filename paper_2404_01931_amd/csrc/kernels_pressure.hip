// Pressure projection (paper Sec. 3.1.7): right-hand side from the discrete
// divergence (Eq. (6)), matrix-free seven-point operator, preconditioned
// conjugate gradient (Jacobi, or the multigrid V-cycle whose fine-level kernels
// live here and whose coarse levels are in kernels_mg.hip), the paper's
// red-black Gauss-Seidel solver as an alternative, the FP64 refinement of the
// mixed-precision solve, and the pressure-gradient update of the faces
// (Eq. (5)).
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
// The iteration kernels' grid reductions are completed by the kernel after
// them (every workgroup stores its partial sums; every workgroup of the next
// kernel sums all of them in workgroup order); the start kernels complete
// theirs in their last workgroup. Either way the order is fixed, so results
// are identical from run to run. With the multigrid preconditioner the update
// kernel keeps r instead of z = r / n_c and the V-cycle forms z = M r.
#include <cfloat>

#include <hip/hip_ext.h>

#include "batch.h"
#include "common.h"
#include "device_util.h"

namespace flipmi {

constexpr int PNT = TILE_CELLS;          // threads per tile workgroup
constexpr int HALO = 6 * TILE * TILE;    // 384 face-halo cells
constexpr int STAGE = TILE_CELLS + HALO; // 896


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
__device__ __forceinline__ void rhs_body(Blk blk, Geo g, const uint32_t* __restrict__ tile_list,
                                         const uint32_t* __restrict__ d_nactive,
                                         const uint32_t* __restrict__ count, const T* __restrict__ u,
                                         const T* __restrict__ v, const T* __restrict__ w, T scale,
                                         uint8_t* __restrict__ diag, V* __restrict__ b,
                                         V* __restrict__ z, V* __restrict__ x, V* __restrict__ s0,
                                         V* __restrict__ s1, double* __restrict__ partials,
                                         int64_t pstride, PcgState* __restrict__ ps, double tol,
                                         int max_iters, int r_form)
{
    __shared__ double red[PNT / WAVE];
    __shared__ bool last;
    unsigned* const sync = pcg_sync(ps);
    const int na = (int)*d_nactive;
    int t0, t1;
    tile_range(blk, na, t0, t1);
    const int l = threadIdx.x;
    double rz = 0.0, mb = 0.0, nf = 0.0;
    for (int slot = t0; slot < t1; ++slot) {
        const uint32_t t = tile_list[slot];
        const int ti = (int)(t % g.tx), tj = (int)((t / g.tx) % g.ty), tk = (int)(t / ((uint32_t)g.tx * g.ty));
        const int i = ti * TILE + (l & 7), j = tj * TILE + ((l >> 3) & 7), k = tk * TILE + (l >> 6);
        int d = 0;
        T bv = T(0);
        if (i < g.nx && j < g.ny && k < g.nz) {
            const int64_t c = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
            if (count[c] > 0) {
                d = (i > 0) + (i < g.nx - 1) + (j > 0) + (j < g.ny - 1) + (k > 0) + (k < g.nz - 1);
                const int64_t fu = i + (int64_t)(g.nx + 1) * (j + (int64_t)g.ny * k);
                const int64_t fv = i + (int64_t)g.nx * (j + (int64_t)(g.ny + 1) * k);
                const int64_t fw = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
                const int64_t wZ = (int64_t)g.nx * g.ny;
                const T div = (u[fu + 1] - u[fu]) + (v[fv + g.nx] - v[fv]) + (w[fw + wZ] - w[fw]);
                bv = scale * div;
            }
        }
        const int64_t e = (int64_t)slot * TILE_CELLS + l;
        const V bq = (V)bv;
        // z = b / n for the Jacobi-preconditioned form; r = b when a
        // preconditioner application follows (multigrid)
        const V zq = r_form ? bq : (d ? bq / (V)d : V(0));
        diag[e] = (uint8_t)d;
        b[e] = bq;
        z[e] = zq;
        x[e] = V(0);
        s0[e] = V(0);
        s1[e] = V(0);
        rz += (double)bq * (double)zq;
        mb = fmax(mb, finite_or_inf(fabs((double)bq)));
        nf += d ? 1.0 : 0.0;
    }
    const double vals[3] = {block_sum<PNT>(rz, red), block_max<PNT>(mb, red), block_sum<PNT>(nf, red)};
    if (!publish_partials(blk, partials, pstride, vals, 3, sync, &last)) return;
    const int nb = blk.n;
    int err = 0;
    double tot[3];
    collect_slots<PNT, 3, 2u>(partials, pstride, nb, red, &err, tot);
    const double rho = tot[0], max_b = tot[1], nfl = tot[2];
    err = __syncthreads_or(err);
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
        ps->n_active = na;
        ps->done = !(max_b <= DBL_MAX) ? PCG_BREAKDOWN
                   : (max_b == 0.0)    ? PCG_CONVERGED
                   : (max_iters <= 0)  ? PCG_MAX_ITERS
                                       : PCG_RUNNING;
        ps->sync_error = err;
        ps->from_slots = r_form;
        if (err) ps->done = PCG_BREAKDOWN;
    }
    reset_arrivals(sync);
}

template <typename T, typename V>
__global__ __launch_bounds__(PNT) void k_rhs(Geo g, const uint32_t* __restrict__ tile_list,
                                             const uint32_t* __restrict__ d_nactive,
                                             const uint32_t* __restrict__ count,
                                             const T* __restrict__ u, const T* __restrict__ v,
                                             const T* __restrict__ w, T scale,
                                             uint8_t* __restrict__ diag, V* __restrict__ b,
                                             V* __restrict__ z, V* __restrict__ x,
                                             V* __restrict__ s0, V* __restrict__ s1,
                                             double* __restrict__ partials, int64_t pstride,
                                             PcgState* __restrict__ ps, double tol, int max_iters,
                                             int r_form)
{
    rhs_body<T, V>(plain_blk(), g, tile_list, d_nactive, count, u, v, w, scale, diag, b, z, x, s0, s1,
                   partials, pstride, ps, tol, max_iters, r_form);
}

template <typename T, typename V>
__global__ __launch_bounds__(PNT) void kb_rhs(const RhsArgs<T, V>* __restrict__ tab,
                                              const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk blk, const RhsArgs<T, V>& a) {
        rhs_body<T, V>(blk, a.g, as_global(a.tile_list), as_global(a.d_nactive), as_global(a.count), as_global(a.u), as_global(a.v), as_global(a.w), (T)a.scale, as_global(a.diag), as_global(a.b), as_global(a.z),
                       as_global(a.x), as_global(a.s0), as_global(a.s1), as_global(a.partials), a.pstride, as_global(a.ps), a.tol, a.max_iters, a.r_form);
    });
}

template <typename T, typename V>
void launch_b_rhs(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL((kb_rhs<T, V>), dim3(L.blocks), dim3(PNT), 0, st, (const RhsArgs<T, V>*)L.args, L.first,
                       L.ns);
}
template void launch_b_rhs<float, float>(const BatchLaunch&, hipStream_t);
template void launch_b_rhs<double, double>(const BatchLaunch&, hipStream_t);

template <typename T, typename V>
void launch_rhs(const Geo& g, int groups, const uint32_t* tile_list, const uint32_t* d_nactive,
                const uint32_t* count, const T* u, const T* v, const T* w, double scale, uint8_t* diag,
                V* b, V* z, V* x, V* s0, V* s1, double* partials, int64_t pstride, PcgState* st_dev,
                double tol, int max_iters, int r_form, hipStream_t st)
{
    hipLaunchKernelGGL((k_rhs<T, V>), dim3((unsigned)groups), dim3(PNT), 0, st, g, tile_list, d_nactive,
                       count, u, v, w, (T)scale, diag, b, z, x, s0, s1, partials, pstride, st_dev,
                       tol, max_iters, r_form);
}

template void launch_rhs<float, float>(const Geo&, int, const uint32_t*, const uint32_t*,
                                       const uint32_t*, const float*, const float*, const float*,
                                       double, uint8_t*, float*, float*, float*, float*, float*,
                                       double*, int64_t, PcgState*, double, int, int, hipStream_t);
template void launch_rhs<double, double>(const Geo&, int, const uint32_t*, const uint32_t*,
                                         const uint32_t*, const double*, const double*, const double*,
                                         double, uint8_t*, double*, double*, double*, double*,
                                         double*, double*, int64_t, PcgState*, double, int, int,
                                         hipStream_t);

// ---------------------------------------------------------------------------
// The two iteration kernels run a bounded number of 256-thread workgroups
// (at most PCG_MAX_GROUPS); each walks a contiguous range of active tiles, so
// that the workgroups of one XCD cover one spatial chunk of the tile list and
// share its halos in L2. Thread t owns the x-adjacent cell pair (2t, 2t + 1)
// of the current tile, read and written with one wide access per vector, and
// stages one entry of the face halos: waves 0 and 1 the -x and +x faces (one
// cell per lane), waves 2 and 3 the y and z faces (two adjacent cells per
// lane). Every halo lane reads one aligned cell pair of the neighbouring
// tile, so all lanes issue the same loads. LDS is double-buffered and the
// tiles two ahead are loaded into registers before the current tile's
// stencil is evaluated, so loads overlap arithmetic and one barrier per tile
// suffices.
// ---------------------------------------------------------------------------

constexpr int PCG_NT = 256;

// LDS image of one tile: its 512 cells, the -x and +x halos (one value in
// every even slot of 128), then the -y, +y, -z and +z halos (64 values each)
constexpr int LX_M = TILE_CELLS;
constexpr int LX_P = LX_M + 128;
constexpr int LY_M = LX_P + 128;
constexpr int LY_P = LY_M + 64;
constexpr int LZ_M = LY_P + 64;
constexpr int LZ_P = LZ_M + 64;
constexpr int STAGE2 = LZ_P + 64;

// Tiles whose loads are in flight while a direction-kernel tile is
// evaluated (even). Each costs about ten VGPRs in FP32 and eighteen in FP64;
// the kernel must stay within 128 VGPRs so that four workgroups fit on a CU.
// Four or six measured no faster than two at 256^3.
#ifndef FLIPMI_PCG_AHEAD_DIR
#define FLIPMI_PCG_AHEAD_DIR 2
#endif
template <typename V>
constexpr int pcg_ahead_dir = sizeof(V) == 4 ? FLIPMI_PCG_AHEAD_DIR : 2;
static_assert(FLIPMI_PCG_AHEAD_DIR >= 2 && FLIPMI_PCG_AHEAD_DIR % 2 == 0, "tiles go in pairs");

template <typename V>
struct alignas(2 * sizeof(V)) Pair {
    V a, b;
};

template <typename V>
__device__ inline Pair<V> ld2(const V* __restrict__ p, int64_t i)
{
    return *(const Pair<V>*)(p + i);
}

template <typename V>
__device__ inline void st2(V* __restrict__ p, int64_t i, V a, V b)
{
    *(Pair<V>*)(p + i) = Pair<V>{a, b};
}

// The halo entry a thread stages: face f of the tile (-x +x -y +y -z +z),
// the even local index of the cell pair it reads in the neighbouring tile,
// whether it keeps the pair's second cell (x faces keep one cell) and its
// LDS slot. The faces of a wave's two half-waves (f_lo for lanes 0-31, f_hi
// for lanes 32-63; equal in waves 0 and 1) are wave-uniform, so the
// neighbour slots are read with scalar loads, which complete apart from the
// vector loads of the data.
struct HaloLane {
    int f, f_lo, f_hi, src, dst;
    int hx, hy, hz;  // position of the staged halo cell relative to the tile's first cell
    bool hi, upper;
};

__device__ inline HaloLane halo_lane(int tid)
{
    HaloLane h;
    if (tid < 128) {  // x faces: lane m stages cell (x, m & 7, m >> 3)
        const int m = tid & 63, a = m & 7, b = m >> 3;
        h.f = tid >> 6;
        const int li = (h.f == 0 ? 7 : 0) + 8 * a + 64 * b;
        h.src = li & ~1;
        h.hi = (li & 1) != 0;
        h.dst = (h.f == 0 ? LX_M : LX_P) + 2 * (a + 8 * b);
        h.hx = h.f == 0 ? -1 : TILE;
        h.hy = a;
        h.hz = b;
    } else if (tid < 192) {  // y faces: lane m stages cells (2 (m & 3) + {0, 1}, y, m >> 2)
        const int m = tid & 31, x = 2 * (m & 3), zz = m >> 2;
        h.f = tid < 160 ? 2 : 3;
        h.src = x + 8 * (h.f == 2 ? 7 : 0) + 64 * zz;
        h.dst = (h.f == 2 ? LY_M : LY_P) + x + 8 * zz;
        h.hx = x;
        h.hy = h.f == 2 ? -1 : TILE;
        h.hz = zz;
        h.hi = false;
    } else {  // z faces: lane m stages cells (2 (m & 3) + {0, 1}, m >> 2, z)
        const int m = tid & 31, x = 2 * (m & 3), yy = m >> 2;
        h.f = tid < 224 ? 4 : 5;
        h.src = x + 8 * yy + 64 * (h.f == 4 ? 7 : 0);
        h.dst = (h.f == 4 ? LZ_M : LZ_P) + x + 8 * yy;
        h.hx = x;
        h.hy = yy;
        h.hz = h.f == 4 ? -1 : TILE;
        h.hi = false;
    }
    h.f_lo = __builtin_amdgcn_readfirstlane(h.f);
    h.f_hi = __builtin_amdgcn_readlane(h.f, 32);
    h.upper = (tid & 63) >= 32;
    return h;
}

// Neighbour sums of the cell pair (2t, 2t + 1) from the staged tile; c0, c1
// are the pair's own staged values. Same summation order for every cell:
// ((x- + x+) + (y- + y+)) + (z- + z+).
template <typename V>
__device__ inline void pair_neighbour_sums(const V* st, int t, V c0, V c1, V& n0, V& n1)
{
    const int l0 = 2 * t;
    const int lx = l0 & 7, ly = (l0 >> 3) & 7, lz = l0 >> 6;
    const V xm = st[lx > 0 ? l0 - 1 : LX_M + 2 * (ly + 8 * lz)];
    const V xp = st[lx < 6 ? l0 + 2 : LX_P + 2 * (ly + 8 * lz)];
    const Pair<V> ym = *(const Pair<V>*)(st + (ly > 0 ? l0 - 8 : LY_M + lx + 8 * lz));
    const Pair<V> yp = *(const Pair<V>*)(st + (ly < 7 ? l0 + 8 : LY_P + lx + 8 * lz));
    const Pair<V> zm = *(const Pair<V>*)(st + (lz > 0 ? l0 - 64 : LZ_M + lx + 8 * ly));
    const Pair<V> zp = *(const Pair<V>*)(st + (lz < 7 ? l0 + 64 : LZ_P + lx + 8 * ly));
    n0 = ((xm + c1) + (ym.a + yp.a)) + (zm.a + zp.a);
    n1 = ((c0 + xp) + (ym.b + yp.b)) + (zm.b + zp.b);
}

// Values of one tile that a thread stages: its cell pair and its halo pair,
// loaded into registers two tiles ahead of their use. Every load is
// unconditional (a missing neighbour or a past-the-end tile reads a valid
// address of the workgroup's own range and is masked where it is consumed),
// so no control-flow merge makes the compiler wait for the loads early.
template <typename V>
struct DirRegs {
    Pair<V> z, s, hz, hs;
    uint32_t d;  // the pair's two diagonal bytes
    bool m;      // the halo's neighbour tile exists
};

template <typename V>
__device__ inline void dir_fetch(DirRegs<V>& r, const V* __restrict__ z, const V* __restrict__ s_old,
                                 const uint8_t* __restrict__ diag, int slot, int32_t nslot, int tid,
                                 int hsrc)
{
    const int64_t e = (int64_t)slot * TILE_CELLS + 2 * tid;
    const int64_t h = nslot >= 0 ? (int64_t)nslot * TILE_CELLS + hsrc : e;
    r.z = ld2(z, e);
    r.s = ld2(s_old, e);
    r.d = *(const uint16_t*)(diag + e);
    r.hz = ld2(z, h);
    r.hs = ld2(s_old, h);
    r.m = nslot >= 0;
}

// neighbour slot across this lane's halo face of tile `slot`
__device__ inline int32_t next_nbr(const int32_t* __restrict__ nbr, int slot, const HaloLane& hl)
{
    const int32_t a = nbr[(int64_t)slot * 6 + hl.f_lo];
    const int32_t b = nbr[(int64_t)slot * 6 + hl.f_hi];
    return hl.upper ? b : a;
}

// One tile of the direction kernel: stage the tile in LDS, then store it,
// issue the loads AH tiles ahead and evaluate the stencil. The barrier
// orders LDS only, so those loads stay in flight across the next tiles'
// barriers.
template <typename V, int AH>
__device__ inline double dir_tile(V* st, DirRegs<V>& cur, V beta, int t, int tlast, int32_t& nn,
                                  const int32_t* __restrict__ nbr, const uint8_t* __restrict__ diag,
                                  const V* __restrict__ z, const V* __restrict__ s_old, V* __restrict__ s_new,
                                  V* __restrict__ q_out, int tid, const HaloLane& hl)
{
    const V sc0 = fma(beta, cur.s.a, cur.z.a), sc1 = fma(beta, cur.s.b, cur.z.b);
    const V hv0 = fma(beta, cur.hs.a, cur.hz.a), hv1 = fma(beta, cur.hs.b, cur.hz.b);
    const V h0 = cur.m ? (hl.hi ? hv1 : hv0) : V(0);
    const V h1 = cur.m ? hv1 : V(0);
    const int d0 = (int)(cur.d & 0xFFu), d1 = (int)(cur.d >> 8);
    st2(st, 2 * tid, sc0, sc1);
    st2(st, hl.dst, h0, h1);  // x faces: the second slot is padding
    lds_barrier();
    st2(s_new, (int64_t)t * TILE_CELLS + 2 * tid, sc0, sc1);
    const int32_t nn3 = next_nbr(nbr, min(t + AH + 1, tlast), hl);
    V n0, n1;
    pair_neighbour_sums(st, tid, sc0, sc1, n0, n1);
    const V q0 = d0 ? fma((V)d0, sc0, -n0) : V(0);
    const V q1 = d1 ? fma((V)d1, sc1, -n1) : V(0);
    if (q_out) st2(q_out, (int64_t)t * TILE_CELLS + 2 * tid, q0, q1);
    const double dot = (double)sc0 * (double)q0 + (double)sc1 * (double)q1;
    // The loads AH tiles ahead go out once nothing computed from cur's old
    // values is live (the compiler computes s in place of the loaded z), so
    // they can take cur's registers: a copy between registers at the loop's
    // back edge would wait for the loads.
    __builtin_amdgcn_sched_barrier(0);
    dir_fetch(cur, z, s_old, diag, min(t + AH, tlast), nn, tid, hl.src);
    nn = nn3;
    // keep the next tile's LDS stores (which wait for its loads) after this
    // tile's work
    __builtin_amdgcn_sched_barrier(0);
    return dot;
}

// direction kernel: s = z + beta s_old, q = A s, sigma = s.q; q is stored
// when q_out is set (the multigrid solve's update reads it)
template <typename V>
__device__ __forceinline__ void pcg_direction_body(Blk blk, int na_hint, const int32_t* __restrict__ nbr,
                                                   const uint8_t* __restrict__ diag,
                                                   const V* __restrict__ z, const V* __restrict__ s_old,
                                                   V* __restrict__ s_new, V* __restrict__ q_out,
                                                   double* __restrict__ pslots, PcgState* __restrict__ ps)
{
    __shared__ alignas(16) V stg[2][STAGE2];
    __shared__ double red[2 * (PCG_NT / WAVE)];
    const int tid = threadIdx.x;
    const HaloLane hl = halo_lane(tid);
    // With the active-tile count known (na_hint >= 0) the first tiles' loads
    // go out before the solver state arrives; a workgroup without tiles loads
    // a valid tile it does not use.
    const int na = na_hint >= 0 ? na_hint : ps->n_active;
    int t0, t1;
    tile_range(blk, na, t0, t1);
    const int tlast = t0 < t1 ? t1 - 1 : max(min(t0, na - 1), 0);
    constexpr int AH = pcg_ahead_dir<V>;
    DirRegs<V> R[AH];
    int32_t nn = next_nbr(nbr, min(t0, tlast), hl);
#pragma unroll
    for (int j = 0; j < AH; ++j) {
        dir_fetch(R[j], z, s_old, diag, min(t0 + j, tlast), nn, tid, hl.src);
        nn = next_nbr(nbr, min(t0 + j + 1, tlast), hl);
    }
    // complete the previous update's reduction (the slots' addresses do not
    // depend on the state, so their loads go out at once) and test its residual
    const SumMax rm = reduce_slots_all<PCG_NT>(slot_rho(pslots, blk.n), slot_max(pslots, blk.n), blk.n, red);
    if (ps->done != PCG_RUNNING) return;
    const int k = ps->iter;
    const double ps_rho = ps->rho, max_b = ps->max_b, rho_prev = ps->rho_prev;
    // k = 0: the solve's start, from the RHS (or, after a preconditioner
    // application, from its slots)
    const bool slots = k > 0 || ps->from_slots != 0;
    const double rho = slots ? rm.sum : ps_rho;
    const double maxr = slots ? rm.mx : max_b;
    const double beta_d = k > 0 ? rho / rho_prev : 0.0;
    const int state = !(maxr <= DBL_MAX) || !(fabs(rho) <= DBL_MAX) ? PCG_BREAKDOWN
                      : maxr <= ps->tol * max_b                   ? PCG_CONVERGED
                      : k >= ps->max_iters                          ? PCG_MAX_ITERS
                                                                    : PCG_RUNNING;
    if (blk.id == 0 && tid == 0) {
        ps->kd = k;
        ps->max_r = maxr;
        ps->rho = rho;
        ps->beta = beta_d;
        if (state != PCG_RUNNING) ps->done = state;
    }
    if (state != PCG_RUNNING) return;
    const V beta = (V)beta_d;
    double acc = 0.0;
    if (t0 < t1) {
        // Tiles go in pairs, both halves unconditional: a branch around the
        // second half would make the compiler wait for every outstanding
        // load at the loop head. With an odd count the last pair's second
        // half is the last tile again, from the values fetched before its
        // update: it stores what the first half stored and its sum is dropped.
        // The loop body covers AH tiles so that every register set keeps its
        // name (a copy between sets would wait for the copied loads), and has
        // no branch inside (a merge of paths with different loads in flight
        // makes the compiler wait for nearly all of them); the pairs left
        // over, fewer than AH / 2, follow the loop.
        auto pair = [&](DirRegs<V>& ra, DirRegs<V>& rb, int t) {
            acc += dir_tile<V, AH>(stg[0], ra, beta, t, tlast, nn, nbr, diag, z, s_old, s_new, q_out, tid, hl);
            const bool real = t + 1 < t1;
            const double v = dir_tile<V, AH>(stg[1], rb, beta, real ? t + 1 : tlast, tlast, nn, nbr, diag, z,
                                             s_old, s_new, q_out, tid, hl);
            acc += real ? v : 0.0;
        };
        const int pairs = (t1 - t0 + 1) >> 1;
        int t = t0;
        for (int q = 0; q < pairs / (AH / 2); ++q) {
#pragma unroll
            for (int r = 0; r < AH; r += 2, t += 2) pair(R[r], R[r + 1], t);
        }
#pragma unroll
        for (int r = 0; r + 2 < AH; r += 2, t += 2)
            if (r / 2 < pairs % (AH / 2)) pair(R[r], R[r + 1], t);
    }
    const double part = block_sum<PCG_NT>(acc, red);
    if (tid == 0) slot_sig(pslots, blk.n)[blk.id] = part;  // completed by U_k
}

template <typename V>
__global__ __launch_bounds__(PCG_NT) void k_pcg_direction(int na_hint, const int32_t* __restrict__ nbr,
                                                          const uint8_t* __restrict__ diag,
                                                          const V* __restrict__ z,
                                                          const V* __restrict__ s_old,
                                                          V* __restrict__ s_new, V* __restrict__ q_out,
                                                          double* __restrict__ pslots,
                                                          PcgState* __restrict__ ps)
{
    pcg_direction_body<V>(plain_blk(), na_hint, nbr, diag, z, s_old, s_new, q_out, pslots, ps);
}

template <typename V>
__global__ __launch_bounds__(PCG_NT) void kb_pcg_direction(const DirArgs<V>* __restrict__ tab,
                                                           const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk blk, const DirArgs<V>& a) {
        pcg_direction_body<V>(blk, a.na_hint, as_global(a.nbr), as_global(a.diag), as_global(a.z), as_global(a.s_old),
                              as_global(a.s_new), a.q ? as_global(a.q) : nullptr, as_global(a.pslots),
                              as_global(a.ps));
    });
}

template <typename V>
void launch_b_pcg_direction(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_pcg_direction<V>, dim3(L.blocks), dim3(PCG_NT), 0, st, (const DirArgs<V>*)L.args,
                       L.first, L.ns);
}
template void launch_b_pcg_direction<float>(const BatchLaunch&, hipStream_t);
template void launch_b_pcg_direction<double>(const BatchLaunch&, hipStream_t);

template <typename V>
void launch_pcg_direction(int groups, int na_hint, const int32_t* tile_nbr, const uint8_t* diag, const V* z,
                          const V* s_old, V* s_new, V* q_out, double* pslots, PcgState* st_dev,
                          hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop)
{
    if (ev_start)
        hipExtLaunchKernelGGL(k_pcg_direction<V>, dim3((unsigned)groups), dim3(PCG_NT), 0, st, ev_start, ev_stop,
                              0, na_hint, tile_nbr, diag, z, s_old, s_new, q_out, pslots, st_dev);
    else
        hipLaunchKernelGGL(k_pcg_direction<V>, dim3((unsigned)groups), dim3(PCG_NT), 0, st, na_hint, tile_nbr, diag,
                           z, s_old, s_new, q_out, pslots, st_dev);
}

template void launch_pcg_direction<float>(int, int, const int32_t*, const uint8_t*, const float*,
                                          const float*, float*, float*, double*, PcgState*, hipStream_t, hipEvent_t,
                                          hipEvent_t);
template void launch_pcg_direction<double>(int, int, const int32_t*, const uint8_t*, const double*,
                                           const double*, double*, double*, double*, PcgState*,
                                           hipStream_t, hipEvent_t, hipEvent_t);

// ---------------------------------------------------------------------------
// Multigrid V-cycle, fine level (FLIP_FLAG_MULTIGRID): the two kernels that
// touch the solver's tile layout, built like the direction kernel (cell pair
// per thread, one staged halo pair per lane, LDS-only barriers, the tiles two
// ahead in registers, unconditional tile pairs). The V-cycle and its coarse
// levels are described with the coarse kernels; here:
//   down: u = w r / n;  t = r - A u = (1 - w) r + sum of u over the fluid
//         neighbours;  level-1 b = (sum of t over the 2x2x2 children) / 2
//   up:   y = w r / n + x1(parent);  z = y + w (r - A y) / n, with the
//         partial sums r . z and max |r| for the next direction kernel.
// A pair of x-adjacent cells (2t, 2t + 1) has one parent, and so has the
// halo pair of a y or z face; an x-face halo lane keeps one cell.
// ---------------------------------------------------------------------------

template <typename V>
struct MgRegs {
    Pair<V> r, hr;   // the pair's and the halo pair's r
    uint32_t d, hd;  // their n_c bytes
    V e, he;         // up: level-1 solution at the pair's and the halo cell's parent
    uint32_t tile;   // grid index of the tile these values belong to
    bool m;          // the halo's neighbour tile exists
};

__device__ inline int mg_clamp(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

// tile index of the active tile in `slot` (scalar)
__device__ inline uint32_t next_tile(const uint32_t* __restrict__ tile_list, int slot) { return tile_list[slot]; }

template <typename V, bool UP>
__device__ inline void mg_fetch(MgRegs<V>& q, const V* __restrict__ r, const uint8_t* __restrict__ diag,
                                const V* __restrict__ cx, const Geo& g, const MgLevel& c, int slot, int32_t nslot,
                                uint32_t tile, int tid, const HaloLane& hl)
{
    const int64_t e = (int64_t)slot * TILE_CELLS + 2 * tid;
    const int64_t h = nslot >= 0 ? (int64_t)nslot * TILE_CELLS + hl.src : e;
    q.r = ld2(r, e);
    q.hr = ld2(r, h);
    q.d = *(const uint16_t*)(diag + e);
    q.hd = *(const uint16_t*)(diag + h);
    q.m = nslot >= 0;
    q.tile = tile;
    if (UP) {
        const int ti = (int)(tile % (uint32_t)g.tx), tj = (int)((tile / (uint32_t)g.tx) % (uint32_t)g.ty);
        const int tk = (int)(tile / ((uint32_t)g.tx * (uint32_t)g.ty));
        const int l0 = 2 * tid;
        const int gi = TILE * ti + (l0 & 7), gj = TILE * tj + ((l0 >> 3) & 7), gk = TILE * tk + (l0 >> 6);
        // coordinates past the domain (cells of a partial tile, a missing
        // neighbour) are clamped: their values are not used
        q.e = cx[mg_clamp(gi >> 1, c.nx) + (int64_t)c.nx * (mg_clamp(gj >> 1, c.ny) + (int64_t)c.ny * mg_clamp(gk >> 1, c.nz))];
        const int hi_ = TILE * ti + hl.hx, hj = TILE * tj + hl.hy, hk = TILE * tk + hl.hz;
        q.he = cx[mg_clamp(hi_ >> 1, c.nx) + (int64_t)c.nx * (mg_clamp(hj >> 1, c.ny) + (int64_t)c.ny * mg_clamp(hk >> 1, c.nz))];
    }
}

template <typename V>
__device__ inline V mg_recip(int d)
{
    return smoother_recip<V>(d);
}

// The down kernel's work on one tile from the pair's r and x0 = w r / n (u0,
// u1) and the halo lane's x0 (h0, h1): writes level-1 b for the tile's
// 4x4x4 parents (those inside level 1). fetch(slot, nbr slot, tile) loads
// the tile two ahead once this tile's values are no longer needed.
template <typename V, typename Fetch>
__device__ inline void mg_down_stage(V* st, V* psum, V r0, V r1, V u0, V u1, V h0, V h1, int d0, int d1,
                                     uint32_t tile_cur, int t, int tlast, int32_t& nn, uint32_t& tn,
                                     const int32_t* __restrict__ nbr, const uint32_t* __restrict__ tile_list,
                                     const Geo& g, const MgLevel& c, V* __restrict__ cb, int tid, const HaloLane& hl,
                                     Fetch&& fetch)
{
    const V w = V(6) / V(7);
    st2(st, 2 * tid, u0, u1);
    st2(st, hl.dst, h0, h1);
    lds_barrier();
    const int32_t nn3 = next_nbr(nbr, min(t + 3, tlast), hl);
    const uint32_t tn3 = next_tile(tile_list, min(t + 3, tlast));
    V n0, n1;
    pair_neighbour_sums(st, tid, u0, u1, n0, n1);
    const V t0v = d0 ? (r0 - w * r0) + n0 : V(0);
    const V t1v = d1 ? (r1 - w * r1) + n1 : V(0);
    psum[tid] = t0v + t1v;
    lds_barrier();
    if (tid < 64) {
        // parent p of the tile's 4x4x4 block: its children are the x-pairs
        // px + 4 y + 32 z for y in {2py, 2py+1}, z in {2pz, 2pz+1}
        const int px = tid & 3, py = (tid >> 2) & 3, pz = tid >> 4;
        const int b0 = px + 4 * (2 * py) + 32 * (2 * pz);
        const V sum = (psum[b0] + psum[b0 + 4]) + (psum[b0 + 32] + psum[b0 + 36]);
        const int ti = (int)(tile_cur % (uint32_t)g.tx), tj = (int)((tile_cur / (uint32_t)g.tx) % (uint32_t)g.ty);
        const int tk = (int)(tile_cur / ((uint32_t)g.tx * (uint32_t)g.ty));
        const int ci = 4 * ti + px, cj = 4 * tj + py, ck = 4 * tk + pz;
        if (ci < c.nx && cj < c.ny && ck < c.nz) cb[ci + (int64_t)c.nx * (cj + (int64_t)c.ny * ck)] = V(0.5) * sum;
    }
    // nn and tn belong to tile t + 2 (loaded one tile ahead, like nn)
    __builtin_amdgcn_sched_barrier(0);
    fetch(min(t + 2, tlast), nn, tn);
    nn = nn3;
    tn = tn3;
    __builtin_amdgcn_sched_barrier(0);
}

// one tile of the down kernel
template <typename V>
__device__ inline void mg_down_tile(V* st, V* psum, MgRegs<V>& cur, int t, int tlast, int32_t& nn, uint32_t& tn,
                                    const int32_t* __restrict__ nbr, const uint32_t* __restrict__ tile_list,
                                    const uint8_t* __restrict__ diag, const V* __restrict__ r, const Geo& g,
                                    const MgLevel& c, V* __restrict__ cb, int tid, const HaloLane& hl)
{
    const V w = V(6) / V(7);
    const int d0 = (int)(cur.d & 0xFFu), d1 = (int)(cur.d >> 8);
    const int hd0 = (int)(cur.hd & 0xFFu), hd1 = (int)(cur.hd >> 8);
    const V r0 = cur.r.a, r1 = cur.r.b;
    const V u0 = w * r0 * mg_recip<V>(d0), u1 = w * r1 * mg_recip<V>(d1);
    const V hu0 = w * cur.hr.a * mg_recip<V>(hd0), hu1 = w * cur.hr.b * mg_recip<V>(hd1);
    const V h0 = cur.m ? (hl.hi ? hu1 : hu0) : V(0);
    const V h1 = cur.m ? hu1 : V(0);
    mg_down_stage<V>(st, psum, r0, r1, u0, u1, h0, h1, d0, d1, cur.tile, t, tlast, nn, tn, nbr, tile_list, g, c, cb,
                     tid, hl, [&](int slot, int32_t ns, uint32_t tl) {
                         mg_fetch<V, false>(cur, r, diag, nullptr, g, c, slot, ns, tl, tid, hl);
                     });
}

template <typename V>
__device__ inline void mg_up_tile(V* st, MgRegs<V>& cur, int t, int tlast, int32_t& nn, uint32_t& tn,
                                  const int32_t* __restrict__ nbr, const uint32_t* __restrict__ tile_list,
                                  const uint8_t* __restrict__ diag, const V* __restrict__ r, const V* __restrict__ cx,
                                  const Geo& g, const MgLevel& c, V* __restrict__ z, int tid, const HaloLane& hl,
                                  double& rz, double& rmax)
{
    const V w = V(6) / V(7);
    const int d0 = (int)(cur.d & 0xFFu), d1 = (int)(cur.d >> 8);
    const int hd0 = (int)(cur.hd & 0xFFu), hd1 = (int)(cur.hd >> 8);
    const V r0 = cur.r.a, r1 = cur.r.b;
    const V i0 = mg_recip<V>(d0), i1 = mg_recip<V>(d1);
    const V y0 = d0 ? w * r0 * i0 + cur.e : V(0), y1 = d1 ? w * r1 * i1 + cur.e : V(0);
    const V hy0 = hd0 ? w * cur.hr.a * mg_recip<V>(hd0) + cur.he : V(0);
    const V hy1 = hd1 ? w * cur.hr.b * mg_recip<V>(hd1) + cur.he : V(0);
    const V h0 = cur.m ? (hl.hi ? hy1 : hy0) : V(0);
    const V h1 = cur.m ? hy1 : V(0);
    st2(st, 2 * tid, y0, y1);
    st2(st, hl.dst, h0, h1);
    lds_barrier();
    const int32_t nn3 = next_nbr(nbr, min(t + 3, tlast), hl);
    const uint32_t tn3 = next_tile(tile_list, min(t + 3, tlast));
    V n0, n1;
    pair_neighbour_sums(st, tid, y0, y1, n0, n1);
    const V z0 = d0 ? y0 + w * ((r0 - (V)d0 * y0) + n0) * i0 : V(0);
    const V z1 = d1 ? y1 + w * ((r1 - (V)d1 * y1) + n1) * i1 : V(0);
    st2(z, (int64_t)t * TILE_CELLS + 2 * tid, z0, z1);
    rz += (double)r0 * (double)z0 + (double)r1 * (double)z1;
    rmax = fmax(rmax, fmax(finite_or_inf(fabs((double)r0)), finite_or_inf(fabs((double)r1))));
    __builtin_amdgcn_sched_barrier(0);
    mg_fetch<V, true>(cur, r, diag, cx, g, c, min(t + 2, tlast), nn, tn, tid, hl);
    nn = nn3;
    tn = tn3;
    __builtin_amdgcn_sched_barrier(0);
}

template <typename V, bool UP>
__device__ __forceinline__ void mg_fine_body(Blk blk, int na_hint, const Geo& g,
                                             const uint32_t* __restrict__ tile_list, const int32_t* __restrict__ nbr,
                                             const uint8_t* __restrict__ diag, const V* __restrict__ r,
                                             const MgLevel& c, V* __restrict__ z, double* __restrict__ pslots,
                                             const PcgState* __restrict__ ps)
{
    __shared__ alignas(16) V stg[2][STAGE2];
    __shared__ V psum[2][PCG_NT];
    __shared__ double red[2 * (PCG_NT / WAVE)];
    const int tid = threadIdx.x;
    const HaloLane hl = halo_lane(tid);
    const int na = na_hint >= 0 ? na_hint : ps->n_active;
    int t0, t1;
    tile_range(blk, na, t0, t1);
    if (ps->done != PCG_RUNNING || na == 0) return;
    const int tlast = t0 < t1 ? t1 - 1 : max(min(t0, na - 1), 0);
    const V* const cx = (const V*)c.x;
    V* const cb = (V*)c.b;
    MgRegs<V> A, B;
    // nn and tn: neighbour slot and tile index of the next tile to fetch
    int32_t nn = next_nbr(nbr, min(t0, tlast), hl);
    uint32_t tn = next_tile(tile_list, min(t0, tlast));
    mg_fetch<V, UP>(A, r, diag, cx, g, c, min(t0, tlast), nn, tn, tid, hl);
    nn = next_nbr(nbr, min(t0 + 1, tlast), hl);
    tn = next_tile(tile_list, min(t0 + 1, tlast));
    mg_fetch<V, UP>(B, r, diag, cx, g, c, min(t0 + 1, tlast), nn, tn, tid, hl);
    nn = next_nbr(nbr, min(t0 + 2, tlast), hl);
    tn = next_tile(tile_list, min(t0 + 2, tlast));
    double rz = 0.0, rmax = 0.0;
    // unconditional tile pairs, as in the direction kernel; an odd count
    // repeats the last tile, which rewrites the same values (its sums dropped)
    for (int t = t0; t < t1; t += 2) {
        const bool real = t + 1 < t1;
        if (UP) {
            mg_up_tile<V>(stg[0], A, t, tlast, nn, tn, nbr, tile_list, diag, r, cx, g, c, z, tid, hl, rz, rmax);
            double rz2 = 0.0, rmax2 = 0.0;
            mg_up_tile<V>(stg[1], B, real ? t + 1 : tlast, tlast, nn, tn, nbr, tile_list, diag, r, cx, g, c, z, tid,
                          hl, rz2, rmax2);
            rz += real ? rz2 : 0.0;
            rmax = real ? fmax(rmax, rmax2) : rmax;
        } else {
            mg_down_tile<V>(stg[0], psum[0], A, t, tlast, nn, tn, nbr, tile_list, diag, r, g, c, cb, tid, hl);
            mg_down_tile<V>(stg[1], psum[1], B, real ? t + 1 : tlast, tlast, nn, tn, nbr, tile_list, diag, r, g, c,
                            cb, tid, hl);
        }
    }
    if (!UP) return;
    const double prz = block_sum<PCG_NT>(rz, red);
    const double pmx = block_max<PCG_NT>(rmax, red);
    if (tid == 0) {  // completed by the next direction kernel
        slot_rho(pslots, blk.n)[blk.id] = prz;
        slot_max(pslots, blk.n)[blk.id] = pmx;
    }
}

template <typename V, bool UP>
__global__ __launch_bounds__(PCG_NT) void k_mg_fine(int na_hint, Geo g, const uint32_t* __restrict__ tile_list,
                                                    const int32_t* __restrict__ nbr, const uint8_t* __restrict__ diag,
                                                    const V* __restrict__ r, MgLevel c, V* __restrict__ z,
                                                    double* __restrict__ pslots, const PcgState* __restrict__ ps)
{
    mg_fine_body<V, UP>(plain_blk(), na_hint, g, tile_list, nbr, diag, r, c, z, pslots, ps);
}

template <typename V, bool UP>
__global__ __launch_bounds__(PCG_NT) void kb_mg_fine(const MgFineArgs<V>* __restrict__ tab,
                                                     const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk blk, const MgFineArgs<V>& a) {
        MgLevel c = a.c;
        c.b = as_global(c.b);
        c.x = as_global(c.x);
        mg_fine_body<V, UP>(blk, a.na_hint, a.g, as_global(a.tile_list), as_global(a.nbr), as_global(a.diag),
                            as_global(a.r), c, as_global(a.z), as_global(a.pslots), as_global(a.ps));
    });
}

template <typename V>
void launch_b_mg_fine(bool up, const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    auto kern = up ? kb_mg_fine<V, true> : kb_mg_fine<V, false>;
    hipLaunchKernelGGL(kern, dim3(L.blocks), dim3(PCG_NT), 0, st, (const MgFineArgs<V>*)L.args, L.first, L.ns);
}
template void launch_b_mg_fine<float>(bool, const BatchLaunch&, hipStream_t);
template void launch_b_mg_fine<double>(bool, const BatchLaunch&, hipStream_t);

template <typename V>
void launch_mg_fine(bool up, int groups, int na_hint, const Geo& g, const uint32_t* tile_list,
                    const int32_t* tile_nbr, const uint8_t* diag, const V* r, const MgLevel& c, V* z,
                    double* pslots, const PcgState* ps, hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop)
{
    auto kern = up ? k_mg_fine<V, true> : k_mg_fine<V, false>;
    if (ev_start)
        hipExtLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(PCG_NT), 0, st, ev_start, ev_stop, 0, na_hint, g,
                              tile_list, tile_nbr, diag, r, c, z, pslots, ps);
    else
        hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(PCG_NT), 0, st, na_hint, g, tile_list, tile_nbr, diag,
                           r, c, z, pslots, ps);
}
template void launch_mg_fine<float>(bool, int, int, const Geo&, const uint32_t*, const int32_t*, const uint8_t*,
                                    const float*, const MgLevel&, float*, double*, const PcgState*, hipStream_t,
                                    hipEvent_t, hipEvent_t);
template void launch_mg_fine<double>(bool, int, int, const Geo&, const uint32_t*, const int32_t*, const uint8_t*,
                                     const double*, const MgLevel&, double*, double*, const PcgState*, hipStream_t,
                                     hipEvent_t, hipEvent_t);

template <typename V>
struct UpdRegs {
    Pair<V> s, x, z, h;
    uint32_t d;  // the pair's two diagonal bytes
    bool m;      // the halo's neighbour tile exists
};

template <typename V>
__device__ inline void upd_fetch(UpdRegs<V>& r, const V* __restrict__ s, const V* __restrict__ x,
                                 const V* __restrict__ z, const uint8_t* __restrict__ diag, int slot,
                                 int32_t nslot, int tid, int hsrc)
{
    const int64_t e = (int64_t)slot * TILE_CELLS + 2 * tid;
    const int64_t h = nslot >= 0 ? (int64_t)nslot * TILE_CELLS + hsrc : e;
    r.s = ld2(s, e);
    r.x = ld2(x, e);
    r.z = ld2(z, e);
    r.d = *(const uint16_t*)(diag + e);
    r.h = ld2(s, h);
    r.m = nslot >= 0;
}

// x += alpha s; r = n z - alpha q; z = r / n for one cell (n = 0: not fluid,
// x and z stay 0); accumulates r.z and max|r|. With RF the stored vector is
// r itself (r -= alpha q; a preconditioner application follows, which also
// forms the sums).
template <typename V, bool RF>
__device__ inline void upd_cell(int d, V sc, V xc, V zc, V nsum, V alpha, V& xn, V& zn, double& rz,
                                double& rmax)
{
    const V q = fma((V)d, sc, -nsum);  // same rounding as the direction kernel
    xn = fma(alpha, sc, xc);
    if (RF) {
        zn = d ? fma(-alpha, q, zc) : V(0);
        return;
    }
    const V r = d ? fma((V)d, zc, -alpha * q) : V(0);
    zn = d ? r / (V)d : V(0);
    rz += (double)r * (double)zn;
    rmax = fmax(rmax, finite_or_inf(fabs((double)r)));
}

template <typename V, bool RF>
__device__ inline void upd_tile(V* st, UpdRegs<V>& cur, V alpha, int t, int tlast, int32_t& nn,
                                const int32_t* __restrict__ nbr, const uint8_t* __restrict__ diag,
                                const V* __restrict__ s, V* __restrict__ x, V* __restrict__ z, int tid,
                                const HaloLane& hl, double& rz, double& rmax)
{
    const Pair<V> sc = cur.s, xc = cur.x, zc = cur.z;
    const V h0 = cur.m ? (hl.hi ? cur.h.b : cur.h.a) : V(0);
    const V h1 = cur.m ? cur.h.b : V(0);
    const int d0 = (int)(cur.d & 0xFFu), d1 = (int)(cur.d >> 8);
    st2(st, 2 * tid, sc.a, sc.b);
    st2(st, hl.dst, h0, h1);  // x faces: the second slot is padding
    lds_barrier();
    const int32_t nn3 = next_nbr(nbr, min(t + 3, tlast), hl);
    upd_fetch(cur, s, x, z, diag, min(t + 2, tlast), nn, tid, hl.src);
    nn = nn3;
    V n0, n1;
    pair_neighbour_sums(st, tid, sc.a, sc.b, n0, n1);
    V x0, x1, z0, z1;
    upd_cell<V, RF>(d0, sc.a, xc.a, zc.a, n0, alpha, x0, z0, rz, rmax);
    upd_cell<V, RF>(d1, sc.b, xc.b, zc.b, n1, alpha, x1, z1, rz, rmax);
    const int64_t e = (int64_t)t * TILE_CELLS + 2 * tid;
    st2(x, e, x0, x1);
    st2(z, e, z0, z1);
    __builtin_amdgcn_sched_barrier(0);  // see dir_tile
}

// update kernel: x += alpha s; r = n z - alpha A s; z = r / n; r.z; max|r|
template <typename V, bool RF>
__device__ __forceinline__ void pcg_update_body(Blk blk, int na_hint, const int32_t* __restrict__ nbr,
                                                const uint8_t* __restrict__ diag, const V* __restrict__ s,
                                                V* __restrict__ x, V* __restrict__ z,
                                                double* __restrict__ pslots, PcgState* __restrict__ ps)
{
    __shared__ alignas(16) V stg[2][STAGE2];
    __shared__ double red[2 * (PCG_NT / WAVE)];
    const int tid = threadIdx.x;
    const HaloLane hl = halo_lane(tid);
    const int na = na_hint >= 0 ? na_hint : ps->n_active;  // as in the direction kernel
    int t0, t1;
    tile_range(blk, na, t0, t1);
    const int tlast = t0 < t1 ? t1 - 1 : max(min(t0, na - 1), 0);
    UpdRegs<V> A, B;
    int32_t nn = next_nbr(nbr, min(t0, tlast), hl);
    upd_fetch(A, s, x, z, diag, min(t0, tlast), nn, tid, hl.src);
    nn = next_nbr(nbr, min(t0 + 1, tlast), hl);
    upd_fetch(B, s, x, z, diag, min(t0 + 1, tlast), nn, tid, hl.src);
    nn = next_nbr(nbr, min(t0 + 2, tlast), hl);
    // complete the direction kernel's reduction: alpha = rho / s.q
    const double sigma = reduce_slots_all<PCG_NT>(slot_sig(pslots, blk.n), blk.n, red);
    if (ps->done != PCG_RUNNING) return;
    const double rho = ps->rho;
    const bool bad = !(sigma > 0.0) || !(sigma <= DBL_MAX);
    const double alpha_d = rho / sigma;
    if (blk.id == 0 && tid == 0) {
        if (bad) ps->done = PCG_BREAKDOWN;
        ps->alpha = alpha_d;
        ps->rho_prev = rho;
        ps->iter = ps->kd + 1;
    }
    if (bad) return;
    const V alpha = (V)alpha_d;
    double rz = 0.0, rmax = 0.0;
    {
        // tiles in unconditional pairs, as in the direction kernel
        for (int t = t0; t < t1; t += 2) {
            upd_tile<V, RF>(stg[0], A, alpha, t, tlast, nn, nbr, diag, s, x, z, tid, hl, rz, rmax);
            const bool real = t + 1 < t1;
            double rz2 = 0.0, rmax2 = 0.0;
            upd_tile<V, RF>(stg[1], B, alpha, real ? t + 1 : tlast, tlast, nn, nbr, diag, s, x, z, tid, hl, rz2,
                            rmax2);
            rz += real ? rz2 : 0.0;
            rmax = real ? fmax(rmax, rmax2) : rmax;
        }
    }
    if (RF) return;  // the preconditioner application forms the sums
    const double prz = block_sum<PCG_NT>(rz, red);
    const double pmx = block_max<PCG_NT>(rmax, red);
    if (tid == 0) {  // completed by D_{k+1}
        slot_rho(pslots, blk.n)[blk.id] = prz;
        slot_max(pslots, blk.n)[blk.id] = pmx;
    }
}

template <typename V, bool RF>
__global__ __launch_bounds__(PCG_NT) void k_pcg_update(int na_hint, const int32_t* __restrict__ nbr,
                                                       const uint8_t* __restrict__ diag,
                                                       const V* __restrict__ s, V* __restrict__ x,
                                                       V* __restrict__ z, double* __restrict__ pslots,
                                                       PcgState* __restrict__ ps)
{
    pcg_update_body<V, RF>(plain_blk(), na_hint, nbr, diag, s, x, z, pslots, ps);
}

template <typename V, bool RF>
__global__ __launch_bounds__(PCG_NT) void kb_pcg_update(const UpdArgs<V>* __restrict__ tab,
                                                        const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk blk, const UpdArgs<V>& a) {
        pcg_update_body<V, RF>(blk, a.na_hint, as_global(a.nbr), as_global(a.diag), as_global(a.s), as_global(a.x), as_global(a.z), as_global(a.pslots), as_global(a.ps));
    });
}

template <typename V>
void launch_b_pcg_update(bool r_form, const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    auto kern = r_form ? kb_pcg_update<V, true> : kb_pcg_update<V, false>;
    hipLaunchKernelGGL(kern, dim3(L.blocks), dim3(PCG_NT), 0, st, (const UpdArgs<V>*)L.args, L.first, L.ns);
}
template void launch_b_pcg_update<float>(bool, const BatchLaunch&, hipStream_t);
template void launch_b_pcg_update<double>(bool, const BatchLaunch&, hipStream_t);

template <typename V>
void launch_pcg_update(int groups, int na_hint, const int32_t* tile_nbr, const uint8_t* diag, const V* s, V* x,
                       V* z, double* pslots, PcgState* st_dev, bool r_form, hipStream_t st,
                       hipEvent_t ev_start, hipEvent_t ev_stop)
{
    auto kern = r_form ? k_pcg_update<V, true> : k_pcg_update<V, false>;
    if (ev_start)
        hipExtLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(PCG_NT), 0, st, ev_start, ev_stop, 0, na_hint,
                              tile_nbr, diag, s, x, z, pslots, st_dev);
    else
        hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(PCG_NT), 0, st, na_hint, tile_nbr, diag, s, x, z,
                           pslots, st_dev);
}

template void launch_pcg_update<float>(int, int, const int32_t*, const uint8_t*, const float*, float*,
                                       float*, double*, PcgState*, bool, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_pcg_update<double>(int, int, const int32_t*, const uint8_t*, const double*, double*,
                                        double*, double*, PcgState*, bool, hipStream_t, hipEvent_t, hipEvent_t);

// ---------------------------------------------------------------------------
// The multigrid solve's update and the fine level's down kernel in one pass.
// The update leaves r' = r - alpha q (q = A s, stored by the direction
// kernel) and the down kernel's first read is r' with its face halo, so one
// kernel updates x and r and restricts r' to level 1. r' on the halo is
// formed from the neighbour tile's r and q by the same operations as that
// tile's own workgroup uses, and q is the value the update kernel would
// recompute (the same fma on the same staged s), so every value written is
// the one the two kernels write apart. The halo reads need the neighbour's r
// unchanged while the kernel runs, so r' goes to another vector (r_out): the
// caller alternates two vectors between r and the V-cycle's z.
// ---------------------------------------------------------------------------

template <typename V>
struct UdRegs {
    Pair<V> r, hr, q, hq, x, s;  // the pair's and the halo pair's r and q; the pair's x and s
    uint32_t d, hd;              // n_c bytes of the pair and of the halo pair
    uint32_t tile;               // grid index of the tile
    bool m;                      // the halo's neighbour tile exists
};

template <typename V>
__device__ inline void ud_fetch(UdRegs<V>& u, const V* __restrict__ r, const V* __restrict__ q,
                                const V* __restrict__ x, const V* __restrict__ s, const uint8_t* __restrict__ diag,
                                int slot, int32_t nslot, uint32_t tile, int tid, const HaloLane& hl)
{
    const int64_t e = (int64_t)slot * TILE_CELLS + 2 * tid;
    const int64_t h = nslot >= 0 ? (int64_t)nslot * TILE_CELLS + hl.src : e;
    u.r = ld2(r, e);
    u.q = ld2(q, e);
    u.x = ld2(x, e);
    u.s = ld2(s, e);
    u.d = *(const uint16_t*)(diag + e);
    u.hr = ld2(r, h);
    u.hq = ld2(q, h);
    u.hd = *(const uint16_t*)(diag + h);
    u.m = nslot >= 0;
    u.tile = tile;
}

template <typename V>
__device__ inline void ud_tile(V* st, V* psum, UdRegs<V>& cur, V alpha, int t, int tlast, int32_t& nn, uint32_t& tn,
                               const int32_t* __restrict__ nbr, const uint32_t* __restrict__ tile_list,
                               const uint8_t* __restrict__ diag, const V* __restrict__ s, const V* __restrict__ q,
                               V* __restrict__ x, const V* __restrict__ r, V* __restrict__ r_out, const Geo& g,
                               const MgLevel& c, V* __restrict__ cb, int tid, const HaloLane& hl)
{
    const V w = V(6) / V(7);
    const int d0 = (int)(cur.d & 0xFFu), d1 = (int)(cur.d >> 8);
    const int hd0 = (int)(cur.hd & 0xFFu), hd1 = (int)(cur.hd >> 8);
    // the update in residual form (upd_cell)
    const V x0 = fma(alpha, cur.s.a, cur.x.a), x1 = fma(alpha, cur.s.b, cur.x.b);
    const V r0 = d0 ? fma(-alpha, cur.q.a, cur.r.a) : V(0);
    const V r1 = d1 ? fma(-alpha, cur.q.b, cur.r.b) : V(0);
    const V hr0 = hd0 ? fma(-alpha, cur.hq.a, cur.hr.a) : V(0);
    const V hr1 = hd1 ? fma(-alpha, cur.hq.b, cur.hr.b) : V(0);
    const int64_t e = (int64_t)t * TILE_CELLS + 2 * tid;
    st2(x, e, x0, x1);
    st2(r_out, e, r0, r1);
    // the down kernel on r' (mg_down_tile)
    const V u0 = w * r0 * mg_recip<V>(d0), u1 = w * r1 * mg_recip<V>(d1);
    const V hu0 = w * hr0 * mg_recip<V>(hd0), hu1 = w * hr1 * mg_recip<V>(hd1);
    const V h0 = cur.m ? (hl.hi ? hu1 : hu0) : V(0);
    const V h1 = cur.m ? hu1 : V(0);
    mg_down_stage<V>(st, psum, r0, r1, u0, u1, h0, h1, d0, d1, cur.tile, t, tlast, nn, tn, nbr, tile_list, g, c, cb,
                     tid, hl, [&](int slot, int32_t ns, uint32_t tl) {
                         ud_fetch<V>(cur, r, q, x, s, diag, slot, ns, tl, tid, hl);
                     });
}

// x += alpha s; r_out = r - alpha q; level-1 b = R (r_out - A w r_out / n) / 2
template <typename V>
__device__ __forceinline__ void pcg_update_down_body(Blk blk, int na_hint, const Geo& g,
                                                     const uint32_t* __restrict__ tile_list,
                                                     const int32_t* __restrict__ nbr, const uint8_t* __restrict__ diag,
                                                     const V* __restrict__ s, const V* __restrict__ q,
                                                     V* __restrict__ x, const V* __restrict__ r,
                                                     V* __restrict__ r_out, const MgLevel& c,
                                                     double* __restrict__ pslots, PcgState* __restrict__ ps)
{
    __shared__ alignas(16) V stg[2][STAGE2];
    __shared__ V psum[2][PCG_NT];
    __shared__ double red[2 * (PCG_NT / WAVE)];
    const int tid = threadIdx.x;
    const HaloLane hl = halo_lane(tid);
    const int na = na_hint >= 0 ? na_hint : ps->n_active;
    int t0, t1;
    tile_range(blk, na, t0, t1);
    const int tlast = t0 < t1 ? t1 - 1 : max(min(t0, na - 1), 0);
    V* const cb = (V*)c.b;
    UdRegs<V> A, B;
    int32_t nn = next_nbr(nbr, min(t0, tlast), hl);
    uint32_t tn = next_tile(tile_list, min(t0, tlast));
    ud_fetch<V>(A, r, q, x, s, diag, min(t0, tlast), nn, tn, tid, hl);
    nn = next_nbr(nbr, min(t0 + 1, tlast), hl);
    tn = next_tile(tile_list, min(t0 + 1, tlast));
    ud_fetch<V>(B, r, q, x, s, diag, min(t0 + 1, tlast), nn, tn, tid, hl);
    nn = next_nbr(nbr, min(t0 + 2, tlast), hl);
    tn = next_tile(tile_list, min(t0 + 2, tlast));
    // complete the direction kernel's reduction: alpha = rho / s.q (as in
    // the update kernel)
    const double sigma = reduce_slots_all<PCG_NT>(slot_sig(pslots, blk.n), blk.n, red);
    if (ps->done != PCG_RUNNING) return;
    const double rho = ps->rho;
    const bool bad = !(sigma > 0.0) || !(sigma <= DBL_MAX);
    const double alpha_d = rho / sigma;
    if (blk.id == 0 && tid == 0) {
        if (bad) ps->done = PCG_BREAKDOWN;
        ps->alpha = alpha_d;
        ps->rho_prev = rho;
        ps->iter = ps->kd + 1;
    }
    if (bad || na == 0) return;
    const V alpha = (V)alpha_d;
    // unconditional tile pairs; an odd count repeats the last tile, which
    // rewrites the same values
    for (int t = t0; t < t1; t += 2) {
        const bool real = t + 1 < t1;
        ud_tile<V>(stg[0], psum[0], A, alpha, t, tlast, nn, tn, nbr, tile_list, diag, s, q, x, r, r_out, g, c, cb,
                   tid, hl);
        ud_tile<V>(stg[1], psum[1], B, alpha, real ? t + 1 : tlast, tlast, nn, tn, nbr, tile_list, diag, s, q, x, r,
                   r_out, g, c, cb, tid, hl);
    }
}

template <typename V>
__global__ __launch_bounds__(PCG_NT) void k_pcg_update_down(int na_hint, Geo g, const uint32_t* __restrict__ tile_list,
                                                            const int32_t* __restrict__ nbr,
                                                            const uint8_t* __restrict__ diag, const V* __restrict__ s,
                                                            const V* __restrict__ q, V* __restrict__ x,
                                                            const V* __restrict__ r, V* __restrict__ r_out, MgLevel c,
                                                            double* __restrict__ pslots, PcgState* __restrict__ ps)
{
    pcg_update_down_body<V>(plain_blk(), na_hint, g, tile_list, nbr, diag, s, q, x, r, r_out, c, pslots, ps);
}

template <typename V>
__global__ __launch_bounds__(PCG_NT) void kb_pcg_update_down(const UpdDownArgs<V>* __restrict__ tab,
                                                             const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk blk, const UpdDownArgs<V>& a) {
        MgLevel c = a.c;
        c.b = as_global(c.b);
        pcg_update_down_body<V>(blk, a.na_hint, a.g, as_global(a.tile_list), as_global(a.nbr), as_global(a.diag),
                                as_global(a.s), as_global(a.q), as_global(a.x), as_global(a.r),
                                as_global(a.r_out), c, as_global(a.pslots), as_global(a.ps));
    });
}

template <typename V>
void launch_b_pcg_update_down(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_pcg_update_down<V>, dim3(L.blocks), dim3(PCG_NT), 0, st, (const UpdDownArgs<V>*)L.args,
                       L.first, L.ns);
}
template void launch_b_pcg_update_down<float>(const BatchLaunch&, hipStream_t);
template void launch_b_pcg_update_down<double>(const BatchLaunch&, hipStream_t);

template <typename V>
void launch_pcg_update_down(int groups, int na_hint, const Geo& g, const uint32_t* tile_list,
                            const int32_t* tile_nbr, const uint8_t* diag, const V* s, const V* q, V* x,
                            const V* r, V* r_out, const MgLevel& c, double* pslots, PcgState* st_dev,
                            hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop)
{
    if (ev_start)
        hipExtLaunchKernelGGL(k_pcg_update_down<V>, dim3((unsigned)groups), dim3(PCG_NT), 0, st, ev_start, ev_stop,
                              0, na_hint, g, tile_list, tile_nbr, diag, s, q, x, r, r_out, c, pslots, st_dev);
    else
        hipLaunchKernelGGL(k_pcg_update_down<V>, dim3((unsigned)groups), dim3(PCG_NT), 0, st, na_hint, g, tile_list,
                           tile_nbr, diag, s, q, x, r, r_out, c, pslots, st_dev);
}
template void launch_pcg_update_down<float>(int, int, const Geo&, const uint32_t*, const int32_t*, const uint8_t*,
                                            const float*, const float*, float*, const float*, float*, const MgLevel&,
                                            double*, PcgState*, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_pcg_update_down<double>(int, int, const Geo&, const uint32_t*, const int32_t*,
                                             const uint8_t*, const double*, const double*, double*, const double*,
                                             double*, const MgLevel&, double*, PcgState*, hipStream_t, hipEvent_t,
                                             hipEvent_t);

// ---------------------------------------------------------------------------
// Mixed precision (FLIP_MIXED): FP32 inner Jacobi-PCG (FP32 vectors and
// stencil, FP64 reductions, the kernels above) inside an outer iterative
// refinement whose right-hand side, solution and residual are FP64.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(PNT) void k_rhs_mixed(Geo g, const uint32_t* __restrict__ tile_list,
                                                   const uint32_t* __restrict__ d_nactive,
                                                   const uint32_t* __restrict__ count,
                                                   const float* __restrict__ u,
                                                   const float* __restrict__ v,
                                                   const float* __restrict__ w, double scale,
                                                   uint8_t* __restrict__ diag,
                                                   double* __restrict__ b64,
                                                   double* __restrict__ x64, float* __restrict__ z,
                                                   float* __restrict__ x, float* __restrict__ s0,
                                                   float* __restrict__ s1,
                                                   double* __restrict__ partials, int64_t pstride,
                                                   PcgState* __restrict__ ps, double tol,
                                                   int max_iters, double ir_tol, int max_outer, int r_form)
{
    __shared__ double red[PNT / WAVE];
    __shared__ bool last;
    unsigned* const sync = pcg_sync(ps);
    const Blk blk = plain_blk();
    const int na = (int)*d_nactive;
    int t0, t1;
    tile_range(blk, na, t0, t1);
    const int l = threadIdx.x;
    double rz = 0.0, mb = 0.0, nf = 0.0;
    for (int slot = t0; slot < t1; ++slot) {
        const uint32_t t = tile_list[slot];
        const int ti = (int)(t % g.tx), tj = (int)((t / g.tx) % g.ty), tk = (int)(t / ((uint32_t)g.tx * g.ty));
        const int i = ti * TILE + (l & 7), j = tj * TILE + ((l >> 3) & 7), k = tk * TILE + (l >> 6);
        int d = 0;
        double bd = 0.0;
        if (i < g.nx && j < g.ny && k < g.nz) {
            const int64_t c = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
            if (count[c] > 0) {
                d = (i > 0) + (i < g.nx - 1) + (j > 0) + (j < g.ny - 1) + (k > 0) + (k < g.nz - 1);
                const int64_t fu = i + (int64_t)(g.nx + 1) * (j + (int64_t)g.ny * k);
                const int64_t fv = i + (int64_t)g.nx * (j + (int64_t)(g.ny + 1) * k);
                const int64_t fw = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
                // face differences of float samples are exact in double
                const double div = ((double)u[fu + 1] - (double)u[fu]) + ((double)v[fv + g.nx] - (double)v[fv]) +
                                   ((double)w[fw + (int64_t)g.nx * g.ny] - (double)w[fw]);
                bd = scale * div;
            }
        }
        const int64_t e = (int64_t)slot * TILE_CELLS + l;
        // the first inner solve starts from z = b / n, or from r = b when a
        // preconditioner application follows (multigrid)
        const float zq = r_form ? (float)bd : (d ? (float)(bd / d) : 0.0f);
        diag[e] = (uint8_t)d;
        b64[e] = bd;
        x64[e] = 0.0;
        z[e] = zq;
        x[e] = 0.0f;
        s0[e] = 0.0f;
        s1[e] = 0.0f;
        rz += (double)d * (double)zq * (double)zq;
        mb = fmax(mb, finite_or_inf(fabs(bd)));
        nf += d ? 1.0 : 0.0;
    }
    const double vals[3] = {block_sum<PNT>(rz, red), block_max<PNT>(mb, red), block_sum<PNT>(nf, red)};
    if (!publish_partials(blk, partials, pstride, vals, 3, sync, &last)) return;
    const int nb = blk.n;
    int err = 0;
    double tot[3];
    collect_slots<PNT, 3, 2u>(partials, pstride, nb, red, &err, tot);
    const double rho = tot[0], max_b = tot[1], nfl = tot[2];
    err = __syncthreads_or(err);
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
        ps->n_active = na;
        ps->max_b0 = max_b;
        ps->ir_tol = ir_tol;
        ps->max_r64 = max_b;
        ps->outer = 0;
        ps->max_outer = max_outer;
        ps->outer_done = (max_b == 0.0) ? 1 : 0;
        ps->from_slots = r_form;
        ps->done = !(max_b <= DBL_MAX) ? PCG_BREAKDOWN
                   : (max_b == 0.0)    ? PCG_CONVERGED
                   : (max_iters <= 0)  ? PCG_MAX_ITERS
                                       : PCG_RUNNING;
        ps->sync_error = err;
        if (err) ps->done = PCG_BREAKDOWN;
    }
    reset_arrivals(sync);
}

void launch_rhs_mixed(const Geo& g, int groups, const uint32_t* tile_list, const uint32_t* d_nactive,
                      const uint32_t* count, const float* u, const float* v, const float* w,
                      double scale, uint8_t* diag, double* b64, double* x64, float* z, float* x,
                      float* s0, float* s1, double* partials, int64_t pstride, PcgState* st_dev,
                      double tol, int max_iters, double ir_tol, int max_outer, int r_form, hipStream_t st)
{
    hipLaunchKernelGGL(k_rhs_mixed, dim3((unsigned)groups), dim3(PNT), 0, st, g, tile_list, d_nactive,
                       count, u, v, w, scale, diag, b64, x64, z, x, s0, s1, partials, pstride, st_dev,
                       tol, max_iters, ir_tol, max_outer, r_form);
}

// One refinement, 512 threads per workgroup, one tile at a time. The updated
// FP64 solution of the tile and its face halos is staged in LDS; the solution
// is double-buffered (x64_in -> x64_out, x_in -> x_out) because other
// workgroups read this tile's values as their halo.
//
// The inner solve restarts from the new residual (s = 0). Continuing the
// FP32 iteration with its search direction instead (a residual replacement)
// took more than twice the iterations on the drop scene: the FP32 recursion
// drifts from the true residual by about 1e-4 of max|b| by the time of a
// refinement, so the kept direction no longer fits the replaced residual.
__global__ __launch_bounds__(PNT) void k_ir_update(const int32_t* __restrict__ nbr,
                                                   const uint8_t* __restrict__ diag,
                                                   const double* __restrict__ b64,
                                                   const double* __restrict__ x64_in,
                                                   double* __restrict__ x64_out,
                                                   const float* __restrict__ x_in,
                                                   float* __restrict__ x_out, float* __restrict__ z,
                                                   float* __restrict__ s0, float* __restrict__ s1,
                                                   double* __restrict__ partials, int64_t pstride,
                                                   PcgState* __restrict__ ps, int r_form)
{
    __shared__ double stg[STAGE];
    __shared__ double red[PNT / WAVE];
    __shared__ bool last;
    unsigned* const sync = pcg_sync(ps);
    const Blk blk = plain_blk();
    int t0, t1;
    tile_range(blk, ps->n_active, t0, t1);
    const int l = threadIdx.x;
    double rz = 0.0, mr = 0.0;
    for (int slot = t0; slot < t1; ++slot) {
        const int64_t e = (int64_t)slot * TILE_CELLS + l;
        const double xn = x64_in[e] + (double)x_in[e];
        stg[l] = xn;
        if (l < HALO) {
            const int f = l >> 6;
            const int32_t ns = nbr[(int64_t)slot * 6 + f];
            double hv = 0.0;
            if (ns >= 0) {
                const int64_t en = (int64_t)ns * TILE_CELLS + halo_source(f, l & 63);
                hv = x64_in[en] + (double)x_in[en];
            }
            stg[TILE_CELLS + l] = hv;
        }
        __syncthreads();
        const int d = diag[e];
        double r = 0.0;
        float zq = 0.0f;
        if (d) {
            r = b64[e] - fma((double)d, xn, -neighbour_sum(stg, l));
            zq = r_form ? (float)r : (float)(r / d);
        }
        x64_out[e] = xn;
        x_out[e] = 0.0f;
        z[e] = zq;
        s0[e] = 0.0f;
        s1[e] = 0.0f;
        mr = fmax(mr, finite_or_inf(fabs(r)));
        rz += (double)d * (double)zq * (double)zq;
        __syncthreads();
    }
    const double vals[2] = {block_sum<PNT>(rz, red), block_max<PNT>(mr, red)};
    if (!publish_partials(blk, partials, pstride, vals, 2, sync, &last)) return;
    int err = 0;
    double tot[2];
    collect_slots<PNT, 2, 2u>(partials, pstride, blk.n, red, &err, tot);
    const double rho = tot[0], max_r = tot[1];
    err = __syncthreads_or(err);
    if (threadIdx.x == 0) {
        const int outer = ps->outer + 1;
        ps->outer = outer;
        ps->max_r64 = max_r;
        if (err || !(max_r <= DBL_MAX)) {
            ps->done = PCG_BREAKDOWN;
            ps->outer_done = 2;
            if (err) ps->sync_error = 1;
        } else if (max_r <= ps->ir_tol * ps->max_b0) {
            ps->done = PCG_CONVERGED;
            ps->outer_done = 1;
        } else if (outer >= ps->max_outer) {
            ps->done = PCG_MAX_ITERS;
            ps->outer_done = 2;
        } else {
            // restart the inner solve on the new residual
            ps->done = PCG_RUNNING;
            ps->iter = 0;
            ps->max_b = max_r;
            ps->max_r = max_r;
            ps->rho = rho;
            ps->alpha = 0.0;
            ps->beta = 0.0;
        }
    }
    reset_arrivals(sync);
}

void launch_ir_update(int groups, const int32_t* tile_nbr, const uint8_t* diag, const double* b64,
                      const double* x64_in, double* x64_out, const float* x_in, float* x_out,
                      float* z, float* s0, float* s1, double* partials, int64_t pstride,
                      PcgState* st_dev, int r_form, hipStream_t st)
{
    hipLaunchKernelGGL(k_ir_update, dim3((unsigned)groups), dim3(PNT), 0, st, tile_nbr, diag, b64,
                       x64_in, x64_out, x_in, x_out, z, s0, s1, partials, pstride, st_dev, r_form);
}

// ---------------------------------------------------------------------------
// projection, Eq. (5): u = u* - (dt / (rho dx)) (p+ - p-) on every non-wall
// face touching a fluid cell; p = 0 in air
// ---------------------------------------------------------------------------

// Projection (Eq. (5)) of all three components in one pass: thread (i, j, k)
// updates the u, v and w faces at that index that exist. A face between two
// cells of the domain with a fluid cell on either side takes
// star - (dt / (rho dx)) (p+ - p-), the pressure of an air cell being 0 and
// the difference and its scaling formed in the solution's precision, rounded
// to the face precision once (mixed: the FP64 solution's difference is not
// cut to FP32 before it cancels); every other face keeps its star value
// (the six walls hold 0 from the force step). The fluid status and pressure
// of cell (i, j, k) are looked up once for its three faces, with those of its
// three lower neighbours. Workgroups of 64 x 4 threads cover x-contiguous
// rows of faces: blocks of 64 indices in x, 4 in y and 1 in z, x fastest.
constexpr int PRJ_BX = 64, PRJ_BY = 4;

__host__ __device__ inline int64_t project3_blocks(const Geo& g)
{
    return (int64_t)((g.nx + PRJ_BX) / PRJ_BX) * ((g.ny + PRJ_BY) / PRJ_BY) * (g.nz + 1);
}

template <typename T, typename V>
__device__ __forceinline__ void project3_body(Blk blk, const Geo& g, const uint8_t* __restrict__ diag,
                                              const int32_t* __restrict__ tile_slot, const V* __restrict__ p,
                                              const T* __restrict__ su, const T* __restrict__ sv,
                                              const T* __restrict__ sw, T* __restrict__ ou, T* __restrict__ ov,
                                              T* __restrict__ ow, V scale)
{
    const int nbx = (g.nx + PRJ_BX) / PRJ_BX, nby = (g.ny + PRJ_BY) / PRJ_BY;
    const int bx = blk.id % nbx, by = (blk.id / nbx) % nby, k = blk.id / (nbx * nby);
    const int i = bx * PRJ_BX + (int)(threadIdx.x % PRJ_BX), j = by * PRJ_BY + (int)(threadIdx.x / PRJ_BX);
    if (i > g.nx || j > g.ny || k > g.nz) return;
    const bool in_c = i < g.nx && j < g.ny && k < g.nz;
    // faces that exist at this index, and those between two cells of the domain
    const bool has_u = j < g.ny && k < g.nz, has_v = i < g.nx && k < g.nz, has_w = i < g.nx && j < g.ny;
    const bool int_u = has_u && i > 0 && i < g.nx, int_v = has_v && j > 0 && j < g.ny;
    const bool int_w = has_w && k > 0 && k < g.nz;
    const int64_t fu = i + (int64_t)(g.nx + 1) * (j + (int64_t)g.ny * k);
    const int64_t fv = i + (int64_t)g.nx * (j + (int64_t)(g.ny + 1) * k);
    const int64_t fw = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
    T o_u = has_u ? su[fu] : T(0), o_v = has_v ? sv[fv] : T(0), o_w = has_w ? sw[fw] : T(0);
    // Fluid status and pressure of this cell and its three lower neighbours,
    // from the tile layout: a fluid cell of an active tile has a nonzero n_c
    // byte (every cell of a grid with more than one cell has a neighbour; a
    // one-cell grid has no interior face), every other cell is not fluid and
    // holds p = 0. The four lookups go out at once, at coordinates clamped
    // into the grid (a lookup whose face does not need it is masked below):
    // two rounds of loads instead of a chain of four lookups.
    const int ic = min(i, g.nx - 1), jc = min(j, g.ny - 1), kc = min(k, g.nz - 1);
    const int ci[4] = {ic, max(i - 1, 0), ic, ic}, cj[4] = {jc, jc, max(j - 1, 0), jc};
    const int ck[4] = {kc, kc, kc, max(k - 1, 0)};
    int32_t sl[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) sl[q] = tile_slot[(ci[q] >> 3) + g.tx * ((cj[q] >> 3) + g.ty * (ck[q] >> 3))];
    bool fl[4];
    V pv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t e = (int64_t)(sl[q] >= 0 ? sl[q] : 0) * TILE_CELLS + (ci[q] & 7) + 8 * (cj[q] & 7) +
                          64 * (ck[q] & 7);
        const V pr = p[e];
        fl[q] = sl[q] >= 0 && diag[e] > 0;
        pv[q] = fl[q] ? pr : V(0);
    }
    const bool fc = (int_u || int_v || int_w) && in_c && fl[0];
    const bool fx = int_u && fl[1], fy = int_v && fl[2], fz = int_w && fl[3];
    const V vc = pv[0], vx = pv[1], vy = pv[2], vz = pv[3];
    const V pp = fc ? vc : V(0);
    if (int_u && (fc || fx)) o_u = o_u - (T)(scale * (pp - (fx ? vx : V(0))));
    if (int_v && (fc || fy)) o_v = o_v - (T)(scale * (pp - (fy ? vy : V(0))));
    if (int_w && (fc || fz)) o_w = o_w - (T)(scale * (pp - (fz ? vz : V(0))));
    if (has_u) ou[fu] = o_u;
    if (has_v) ov[fv] = o_v;
    if (has_w) ow[fw] = o_w;
}

template <typename T, typename V>
__global__ __launch_bounds__(PRJ_BX * PRJ_BY) void k_project3(Geo g, const uint8_t* __restrict__ diag,
                                                              const int32_t* __restrict__ tile_slot,
                                                              const V* __restrict__ p, const T* __restrict__ su,
                                                              const T* __restrict__ sv, const T* __restrict__ sw,
                                                              T* __restrict__ ou, T* __restrict__ ov,
                                                              T* __restrict__ ow, V scale)
{
    project3_body<T, V>(plain_blk(), g, diag, tile_slot, p, su, sv, sw, ou, ov, ow, scale);
}

template <typename T, typename V>
__global__ __launch_bounds__(PRJ_BX * PRJ_BY) void kb_project3(const ProjectArgs<T, V>* __restrict__ tab,
                                                               const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk blk, const ProjectArgs<T, V>& a) {
        project3_body<T, V>(blk, a.g, as_global(a.diag), as_global(a.tile_slot), as_global(a.p),
                            as_global(a.star[0]), as_global(a.star[1]), as_global(a.star[2]), as_global(a.out[0]),
                            as_global(a.out[1]), as_global(a.out[2]), a.scale);
    });
}

int64_t project_blocks(const Geo& g) { return project3_blocks(g); }

template <typename T, typename V>
void launch_b_project3(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL((kb_project3<T, V>), dim3(L.blocks), dim3(PRJ_BX * PRJ_BY), 0, st,
                       (const ProjectArgs<T, V>*)L.args, L.first, L.ns);
}
template void launch_b_project3<float, float>(const BatchLaunch&, hipStream_t);
template void launch_b_project3<double, double>(const BatchLaunch&, hipStream_t);

// one thread per scene: copy the solver state a host poll needs
__global__ __launch_bounds__(64) void kb_summary(const SummaryArgs* __restrict__ tab,
                                                 const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk blk, const SummaryArgs& a) {
        if (threadIdx.x != 0) return;
        const PcgState* ps = as_global(a.ps);
        SolveSummary o;
        o.max_b = ps->max_b;
        o.max_r = ps->max_r;
        o.iter = ps->iter;
        o.done = ps->done;
        o.nfluid = ps->nfluid;
        o.n_active = ps->n_active;
        o.sync_error = ps->sync_error;
        o.pad_ = 0;
        *as_global(a.out) = o;
    });
}

void launch_b_summary(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_summary, dim3(L.blocks), dim3(64), 0, st, (const SummaryArgs*)L.args, L.first, L.ns);
}

template <typename T, typename V>
void launch_project3(const Geo& g, const uint8_t* diag, const int32_t* tile_slot, const V* p, T* const star[3],
                     T* const out[3], V scale, hipStream_t st)
{
    hipLaunchKernelGGL((k_project3<T, V>), dim3((unsigned)project3_blocks(g)), dim3(PRJ_BX * PRJ_BY), 0, st, g,
                       diag, tile_slot, p, star[0], star[1], star[2], out[0], out[1], out[2], scale);
}
template void launch_project3<float, float>(const Geo&, const uint8_t*, const int32_t*, const float*,
                                            float* const[3], float* const[3], float, hipStream_t);
template void launch_project3<double, double>(const Geo&, const uint8_t*, const int32_t*, const double*,
                                              double* const[3], double* const[3], double, hipStream_t);
template void launch_project3<float, double>(const Geo&, const uint8_t*, const int32_t*, const double*,
                                             float* const[3], float* const[3], double, hipStream_t);


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

// ---------------------------------------------------------------------------
// Red-black Gauss-Seidel (FLIP_FLAG_RED_BLACK_GS): the paper's GPU pressure
// solver (Sec. 3.2.3). The cells are split by the parity of i + j + k; every
// neighbour of a cell has the other parity, so one colour is updated in
// parallel from the other's values, p_c = (b_c + sum of p over the fluid
// neighbours) / n_c, in two passes per iteration (red, then black). Air
// neighbours hold 0; cells outside the box are not counted in n_c and add
// nothing. One workgroup per active tile, one cell of the colour per thread.
// A tile's origin is a multiple of 8, so local and global parity agree.
// ---------------------------------------------------------------------------

namespace {

// value of p at local cell l of slot `slot` shifted one cell along direction
// f (0..5: -x +x -y +y -z +z), from the neighbouring tile when it leaves the
// tile (0 when that tile is not active)
template <typename V>
__device__ inline V gs_neighbour(const V* __restrict__ p, const int32_t* __restrict__ nbr, int slot, int lx, int ly,
                                 int lz, int f)
{
    int x = lx, y = ly, z = lz, s = slot;
    const int d = (f & 1) ? 1 : -1;
    int* c = f < 2 ? &x : (f < 4 ? &y : &z);
    *c += d;
    if (*c < 0 || *c > 7) {
        s = nbr[(int64_t)slot * 6 + f];
        *c &= 7;
    }
    return s >= 0 ? p[(int64_t)s * TILE_CELLS + x + 8 * y + 64 * z] : V(0);
}

template <typename V>
__device__ inline V gs_nsum(const V* __restrict__ p, const int32_t* __restrict__ nbr, int slot, int lx, int ly, int lz)
{
    return ((gs_neighbour(p, nbr, slot, lx, ly, lz, 0) + gs_neighbour(p, nbr, slot, lx, ly, lz, 1)) +
            (gs_neighbour(p, nbr, slot, lx, ly, lz, 2) + gs_neighbour(p, nbr, slot, lx, ly, lz, 3))) +
           (gs_neighbour(p, nbr, slot, lx, ly, lz, 4) + gs_neighbour(p, nbr, slot, lx, ly, lz, 5));
}

template <typename V>
__device__ inline double gs_nsum_f64(const V* __restrict__ p, const int32_t* __restrict__ nbr, int slot, int lx, int ly,
                                     int lz)
{
    double v[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) v[f] = (double)gs_neighbour(p, nbr, slot, lx, ly, lz, f);
    return ((v[0] + v[1]) + (v[2] + v[3])) + (v[4] + v[5]);
}

}  // namespace

template <typename V, int COLOR>
__global__ __launch_bounds__(256) void k_gs_sweep(const int32_t* __restrict__ nbr, const uint8_t* __restrict__ diag,
                                                  const V* __restrict__ b, V* __restrict__ p)
{
    const int slot = blockIdx.x, t = threadIdx.x;
    // thread t: x-row t / 4 of the tile, the (t % 4)-th cell of the colour in it
    const int ly = (t >> 2) & 7, lz = t >> 5;
    const int lx = 2 * (t & 3) + ((ly + lz + COLOR) & 1);
    const int64_t e = (int64_t)slot * TILE_CELLS + lx + 8 * ly + 64 * lz;
    const int d = diag[e];
    if (d == 0) return;
    p[e] = (b[e] + gs_nsum(p, nbr, slot, lx, ly, lz)) / (V)d;
}

// max |b - A p| over the fluid cells (in FP64), folded into *rmax (the bits
// of a non-negative double order like unsigned integers; *rmax starts at 0)
template <typename V>
__global__ __launch_bounds__(256) void k_gs_residual(const int32_t* __restrict__ nbr,
                                                     const uint8_t* __restrict__ diag, const V* __restrict__ b,
                                                     const V* __restrict__ p, unsigned long long* __restrict__ rmax)
{
    __shared__ double red[256 / WAVE];
    const int slot = blockIdx.x, t = threadIdx.x;
    double m = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int l = t + 256 * h;
        const int lx = l & 7, ly = (l >> 3) & 7, lz = l >> 6;
        const int64_t e = (int64_t)slot * TILE_CELLS + l;
        const int d = diag[e];
        if (d) {
            // evaluated in FP64: in FP32 the rounding of this expression alone
            // is of the order of the tolerances in use
            const double r = (double)b[e] - ((double)d * (double)p[e] - gs_nsum_f64(p, nbr, slot, lx, ly, lz));
            m = fmax(m, finite_or_inf(fabs(r)));
        }
    }
    m = block_max<256>(m, red);
    if (t == 0) atomicMax(rmax, (unsigned long long)__double_as_longlong(m));
}

template <typename V>
void launch_gs_sweeps(int n_active, int iters, const int32_t* nbr, const uint8_t* diag, const V* b, V* p,
                      hipStream_t st)
{
    if (n_active <= 0) return;
    for (int i = 0; i < iters; ++i) {
        hipLaunchKernelGGL((k_gs_sweep<V, 0>), dim3((unsigned)n_active), dim3(256), 0, st, nbr, diag, b, p);
        hipLaunchKernelGGL((k_gs_sweep<V, 1>), dim3((unsigned)n_active), dim3(256), 0, st, nbr, diag, b, p);
    }
}

template <typename V>
void launch_gs_residual(int n_active, const int32_t* nbr, const uint8_t* diag, const V* b, const V* p,
                        unsigned long long* rmax, hipStream_t st)
{
    launch_fill_u64((uint64_t*)rmax, 1, 0ull, st);
    if (n_active <= 0) return;
    hipLaunchKernelGGL(k_gs_residual<V>, dim3((unsigned)n_active), dim3(256), 0, st, nbr, diag, b, p, rmax);
}

template void launch_gs_sweeps<float>(int, int, const int32_t*, const uint8_t*, const float*, float*, hipStream_t);
template void launch_gs_sweeps<double>(int, int, const int32_t*, const uint8_t*, const double*, double*,
                                       hipStream_t);
template void launch_gs_residual<float>(int, const int32_t*, const uint8_t*, const float*, const float*,
                                        unsigned long long*, hipStream_t);
template void launch_gs_residual<double>(int, const int32_t*, const uint8_t*, const double*, const double*,
                                         unsigned long long*, hipStream_t);

}  // namespace flipmi
