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
//   bottom:         x = 0, then 10 sweeps x += w (b - A x) / n
//   up, level l:    y = x0 + P x_{l+1};  x_l = y + w (b - A y) / n
// The levels below level 1 take two sweeps on each side instead of one
// (down: x1 = x0 + w (b - A x0) / n, t = b - A x1; up: y = x1 + P x_{l+1},
// then two sweeps), which costs their latency-bound kernels little and
// takes the 256^3 drop scene from 24 to about 21 iterations.
// Between the fine grid and level 1, P copies a coarse value to its fluid
// children and R sums the children; between dense levels P is cell-centred
// trilinear and R its transpose (described with those kernels). Both R have
// a total weight of 8 per coarse cell, and the coarse equation is scaled by
// 1/2: the coarse stencil at twice the spacing, h^2 scaling. One pre- and
// one post-sweep with the same smoother, a fixed number of bottom sweeps and
// R = P^T make the cycle a fixed symmetric positive definite operator, as CG
// needs. Level 0 reads r and writes z; the fine up-kernel also forms the
// partial sums r . z and max |r| that the next direction kernel completes.
//
// Every kernel reads the solver state and exits when the solve is over (the
// dense-level kernels issue their loads first, so the two waits overlap).
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

// (a dense level has far fewer than 2^31 cells: 32-bit index arithmetic)
__device__ inline int level_index(const MgLevel& L, int i, int j, int k) { return i + L.nx * (j + L.ny * k); }

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

// ---- transfers between dense levels ----------------------------------------------
//
// Between dense levels the prolongation is cell-centred trilinear: along each
// axis a fine cell takes 3/4 of its parent and 1/4 of the parent's neighbour
// on the cell's side (even child: below, odd child: above), that neighbour
// clamped into the coarse box (at a wall the cell takes its parent whole).
// The restriction is its transpose, which per axis gives coarse cell c
//   3/4 of each child 2c, 2c + 1 (1 for child 2c when c = 0 and for child
//   2c + 1 when c is the last cell, where the prolongation clamped) and
//   1/4 of the nearer children 2c - 1 and 2c + 2 of its two neighbours.
// Between the fine grid and level 1 the tile-layout kernels keep the
// piecewise-constant pair (P copies the parent, R sums the children).

template <typename V>
__device__ inline V recip_nc(int d)
{
    return smoother_recip<V>(d);
}

// weight of fine cell 2c - 1 + k (k = 0..3) in coarse cell c, on an axis of n coarse cells
template <typename V>
__device__ inline V restrict_weight(int k, int c, int n)
{
    if (k == 0 || k == 3) return V(0.25);
    return ((k == 1 && c == 0) || (k == 2 && c == n - 1)) ? V(1) : V(0.75);
}

// A box of NX x NY x NZ cells walked by NT threads a column at a time: a
// thread keeps one (x, y) column (its index arithmetic done once) and steps
// through z, P threads sharing a column when NT holds several copies of the
// NX * NY columns.
template <int NX, int NY, int NZ, int NT>
struct Cols {
    static constexpr int C = NX * NY;  // columns
    static constexpr int P = NT / C;   // threads per column
    static constexpr int J = (NZ + P - 1) / P;  // z steps per thread
    static_assert(P >= 1, "a thread per column at least");
};

// ---- down: dense level f to level c ---------------------------------------------

// One workgroup per 8 x 4 x 4 block of level-c cells. Their restriction reads
// t = b - A x0 (x0 = w b / n) on the children plus one fine cell around them
// (18 x 10 x 10, the t region), and t there reads x0 one cell further out
// (20 x 12 x 12, the u region): b and n of the u region are loaded once
// (every load issued unconditionally: clamped address, masked value), x0 and
// t are formed in LDS, and the restriction runs along x, then y, then z.
constexpr int MGD_CX = 8, MGD_CY = 4, MGD_CZ = 4;
constexpr int MGD_TX = 2 * MGD_CX + 2, MGD_TY = 2 * MGD_CY + 2, MGD_TZ = 2 * MGD_CZ + 2;
constexpr int MGD_UX = MGD_TX + 2, MGD_UY = MGD_TY + 2, MGD_UZ = MGD_TZ + 2;
constexpr int MGD_T = MGD_TX * MGD_TY * MGD_TZ;  // 1800
constexpr int MGD_U = MGD_UX * MGD_UY * MGD_UZ;  // 2880
static_assert(MGD_TZ * MGD_TY * MGD_CX + MGD_TZ * MGD_CY * MGD_CX <= MGD_U, "x and y passes fit the b buffer");

// workgroups of a restriction to level c: one per 8 x 4 x 4 block of c, x fastest
__host__ __device__ inline int mg_down_blocks_x(const MgLevel& c) { return (c.nx + MGD_CX - 1) / MGD_CX; }
__host__ __device__ inline int mg_down_blocks_y(const MgLevel& c) { return (c.ny + MGD_CY - 1) / MGD_CY; }
__host__ __device__ inline int64_t mg_down_blocks(const MgLevel& c)
{
    return (int64_t)mg_down_blocks_x(c) * mg_down_blocks_y(c) * ((c.nz + MGD_CZ - 1) / MGD_CZ);
}

// The restriction of t (on the t region, in ts) to the block's coarse
// cells, along x, then y, then z, with the two intermediate passes in the
// scratch area w (at least (TZ TY + TZ CY) CX values); writes c.b = R t / 2.
template <typename V, int NT>
__device__ __forceinline__ void mg_restrict_block(const V* ts, V* w, int cx0, int cy0, int cz0, const MgLevel& c)
{
    const int tid = threadIdx.x;
    V* const rx = w;                                  // [TZ][TY][CX]
    V* const ry = w + MGD_TZ * MGD_TY * MGD_CX;       // [TZ][CY][CX]
    for (int q = tid; q < MGD_TZ * MGD_TY * MGD_CX; q += NT) {
        const int i = q % MGD_CX, row = q / MGD_CX;   // row = ly + TY lz
        const int C = cx0 + i;
        const V* t = ts + row * MGD_TX + 2 * i;
        rx[q] = (restrict_weight<V>(0, C, c.nx) * t[0] + restrict_weight<V>(1, C, c.nx) * t[1]) +
                (restrict_weight<V>(2, C, c.nx) * t[2] + restrict_weight<V>(3, C, c.nx) * t[3]);
    }
    __syncthreads();
    for (int q = tid; q < MGD_TZ * MGD_CY * MGD_CX; q += NT) {
        const int i = q % MGD_CX, j = (q / MGD_CX) % MGD_CY, lz = q / (MGD_CX * MGD_CY);
        const int C = cy0 + j;
        const V* t = rx + (lz * MGD_TY + 2 * j) * MGD_CX + i;
        ry[q] = (restrict_weight<V>(0, C, c.ny) * t[0] + restrict_weight<V>(1, C, c.ny) * t[MGD_CX]) +
                (restrict_weight<V>(2, C, c.ny) * t[2 * MGD_CX] + restrict_weight<V>(3, C, c.ny) * t[3 * MGD_CX]);
    }
    __syncthreads();
    if (tid < MGD_CX * MGD_CY * MGD_CZ) {
        const int i = tid % MGD_CX, j = (tid / MGD_CX) % MGD_CY, k = tid / (MGD_CX * MGD_CY);
        const int ci = cx0 + i, cj = cy0 + j, ck = cz0 + k;
        constexpr int S = MGD_CY * MGD_CX;
        const V* t = ry + (2 * k) * S + j * MGD_CX + i;
        const V v = (restrict_weight<V>(0, ck, c.nz) * t[0] + restrict_weight<V>(1, ck, c.nz) * t[S]) +
                    (restrict_weight<V>(2, ck, c.nz) * t[2 * S] + restrict_weight<V>(3, ck, c.nz) * t[3 * S]);
        if (ci < c.nx && cj < c.ny && ck < c.nz) ((V*)c.b)[level_index(c, ci, cj, ck)] = V(0.5) * v;
    }
}

// NT threads per workgroup: 512, or 1024 on the small levels, where a
// launch has few workgroups and the time is the chain of each thread's
// serial work (the values are the same either way; batched launches use
// MG_BATCH_NT)
template <typename V, int NT>
__device__ __forceinline__ void mg_down_body(Blk blk, const MgLevel& f, const MgLevel& c,
                                             const PcgState* __restrict__ ps)
{
    using CU = Cols<MGD_UX, MGD_UY, MGD_UZ, NT>;
    using CT = Cols<MGD_TX, MGD_TY, MGD_TZ, NT>;
    __shared__ V us[MGD_U];       // x0 on the u region
    __shared__ V bs[MGD_U];       // b on the u region; later the x and y passes
    __shared__ uint8_t ds[MGD_U];  // n (0: not fluid or outside the level)
    __shared__ V ts[MGD_T];
    const int tid = threadIdx.x;
    const int gbx = mg_down_blocks_x(c), gby = mg_down_blocks_y(c);
    const int bid = c.dlist ? (int)c.dlist[blk.id] : blk.id;  // plain launches: the listed blocks
    const int cx0 = (bid % gbx) * MGD_CX, cy0 = ((bid / gbx) % gby) * MGD_CY;
    const int cz0 = (bid / (gbx * gby)) * MGD_CZ;
    const int ox = 2 * cx0 - 2, oy = 2 * cy0 - 2, oz = 2 * cz0 - 2;  // u region origin on level f
    const V* const fb = (const V*)f.b;
    // this thread's column of the u region
    const int ucol = tid % CU::C, uzg = tid / CU::C;
    const bool uact = tid < CU::C * CU::P;
    const int ugx = ox + ucol % MGD_UX, ugy = oy + ucol / MGD_UX;
    const bool uxy = ugx >= 0 && ugx < f.nx && ugy >= 0 && ugy < f.ny;
    const int ubase = min(max(ugx, 0), f.nx - 1) + f.nx * min(max(ugy, 0), f.ny - 1);
    const int sxy = f.nx * f.ny;
    V bv[CU::J];
    int dv[CU::J];
    bool iv[CU::J];
#pragma unroll
    for (int m = 0; m < CU::J; ++m) {
        const int lz = uzg + CU::P * m, gz = oz + lz;
        iv[m] = uact && lz < MGD_UZ && uxy && gz >= 0 && gz < f.nz;
        const int e = ubase + sxy * min(max(gz, 0), f.nz - 1);
        dv[m] = f.d[e];
        bv[m] = fb[e];
    }
    if (ps->done != PCG_RUNNING) return;
    const V w = mg_omega<V>();
#pragma unroll
    for (int m = 0; m < CU::J; ++m) {
        const int lz = uzg + CU::P * m;
        if (uact && lz < MGD_UZ) {
            const int q = ucol + CU::C * lz;
            const int d = iv[m] ? dv[m] : 0;
            us[q] = d ? w * bv[m] * recip_nc<V>(d) : V(0);
            bs[q] = bv[m];
            ds[q] = (uint8_t)d;
        }
    }
    __syncthreads();
    // t = b - A x0 = (1 - w) b + (sum of x0 over the neighbours) on the t region
    constexpr int SY = MGD_UX, SZ = MGD_UX * MGD_UY;
    if (tid < CT::C * CT::P) {
        const int tcol = tid % CT::C;
        const int ub = (tcol % MGD_TX + 1) + SY * (tcol / MGD_TX + 1);
        for (int lz = tid / CT::C; lz < MGD_TZ; lz += CT::P) {
            const int u = ub + SZ * (lz + 1);
            const V nsum = ((us[u - 1] + us[u + 1]) + (us[u - SY] + us[u + SY])) + (us[u - SZ] + us[u + SZ]);
            ts[tcol + CT::C * lz] = ds[u] ? (V(1) - w) * bs[u] + nsum : V(0);
        }
    }
    __syncthreads();
    mg_restrict_block<V, NT>(ts, bs, cx0, cy0, cz0, c);
}

template <typename V, int NT>
__global__ __launch_bounds__(NT) void k_mg_down(MgLevel f, MgLevel c, const PcgState* __restrict__ ps)
{
    mg_down_body<V, NT>(plain_blk(), f, c, ps);
}

template <typename V>
__global__ __launch_bounds__(MG_BATCH_NT) void kb_mg_down(const MgPairArgs* __restrict__ tab,
                                                  const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const MgPairArgs& a) {
        mg_down_body<V, MG_BATCH_NT>(b, glob(a.f), glob(a.c), as_global(a.ps));
    });
}

// ---- down with two sweeps (the levels below level 1) ------------------------------
//
// The same blocks; two damped-Jacobi sweeps from zero before the restriction:
// x0 = w b / n, x1 = x0 + w (b - A x0) / n, t = b - A x1. t on the t region
// reads x1 one cell further out (the v region, 20 x 12 x 12), and x1 there
// reads x0, b and n one more cell out (the u region, 22 x 14 x 14).
constexpr int MGD2_VX = MGD_TX + 2, MGD2_VY = MGD_TY + 2, MGD2_VZ = MGD_TZ + 2;
constexpr int MGD2_UX = MGD_TX + 4, MGD2_UY = MGD_TY + 4, MGD2_UZ = MGD_TZ + 4;
constexpr int MGD2_V = MGD2_VX * MGD2_VY * MGD2_VZ;  // 2880
constexpr int MGD2_U = MGD2_UX * MGD2_UY * MGD2_UZ;  // 4312
static_assert(MGD_TZ * MGD_TY * MGD_CX + MGD_TZ * MGD_CY * MGD_CX <= MGD2_U, "x and y passes fit the b buffer");

template <typename V, int NT>
__device__ __forceinline__ void mg_down2_body(Blk blk, const MgLevel& f, const MgLevel& c,
                                              const PcgState* __restrict__ ps)
{
    using CU = Cols<MGD2_UX, MGD2_UY, MGD2_UZ, NT>;
    using CV = Cols<MGD2_VX, MGD2_VY, MGD2_VZ, NT>;
    using CT = Cols<MGD_TX, MGD_TY, MGD_TZ, NT>;
    __shared__ V us[MGD2_U];       // x0 on the u region
    __shared__ V bs[MGD2_U];       // b on the u region; later the x and y passes
    __shared__ uint8_t ds[MGD2_U];  // n (0: not fluid or outside the level)
    __shared__ V vs[MGD2_V];       // x1 on the v region
    __shared__ V ts[MGD_T];
    const int tid = threadIdx.x;
    const int gbx = mg_down_blocks_x(c), gby = mg_down_blocks_y(c);
    const int bid = c.dlist ? (int)c.dlist[blk.id] : blk.id;  // plain launches: the listed blocks
    const int cx0 = (bid % gbx) * MGD_CX, cy0 = ((bid / gbx) % gby) * MGD_CY;
    const int cz0 = (bid / (gbx * gby)) * MGD_CZ;
    const int ox = 2 * cx0 - 3, oy = 2 * cy0 - 3, oz = 2 * cz0 - 3;  // u region origin on level f
    const V* const fb = (const V*)f.b;
    const int ucol = tid % CU::C, uzg = tid / CU::C;
    const bool uact = tid < CU::C * CU::P;
    const int ugx = ox + ucol % MGD2_UX, ugy = oy + ucol / MGD2_UX;
    const bool uxy = ugx >= 0 && ugx < f.nx && ugy >= 0 && ugy < f.ny;
    const int ubase = min(max(ugx, 0), f.nx - 1) + f.nx * min(max(ugy, 0), f.ny - 1);
    const int sxy = f.nx * f.ny;
    V bv[CU::J];
    int dv[CU::J];
    bool iv[CU::J];
#pragma unroll
    for (int m = 0; m < CU::J; ++m) {
        const int lz = uzg + CU::P * m, gz = oz + lz;
        iv[m] = uact && lz < MGD2_UZ && uxy && gz >= 0 && gz < f.nz;
        const int e = ubase + sxy * min(max(gz, 0), f.nz - 1);
        dv[m] = f.d[e];
        bv[m] = fb[e];
    }
    if (ps->done != PCG_RUNNING) return;
    const V w = mg_omega<V>();
#pragma unroll
    for (int m = 0; m < CU::J; ++m) {
        const int lz = uzg + CU::P * m;
        if (uact && lz < MGD2_UZ) {
            const int q = ucol + CU::C * lz;
            const int d = iv[m] ? dv[m] : 0;
            us[q] = d ? w * bv[m] * recip_nc<V>(d) : V(0);
            bs[q] = bv[m];
            ds[q] = (uint8_t)d;
        }
    }
    __syncthreads();
    constexpr int SY = MGD2_UX, SZ = MGD2_UX * MGD2_UY;
    if (tid < CV::C * CV::P) {
        const int vcol = tid % CV::C;
        const int ub = (vcol % MGD2_VX + 1) + SY * (vcol / MGD2_VX + 1);
        for (int lz = tid / CV::C; lz < MGD2_VZ; lz += CV::P) {
            const int u = ub + SZ * (lz + 1);
            const int d = ds[u];
            const V x0 = us[u];
            const V nsum = ((us[u - 1] + us[u + 1]) + (us[u - SY] + us[u + SY])) + (us[u - SZ] + us[u + SZ]);
            vs[vcol + CV::C * lz] = d ? x0 + w * ((bs[u] - (V)d * x0) + nsum) * recip_nc<V>(d) : V(0);
        }
    }
    __syncthreads();
    constexpr int VY = MGD2_VX, VZ = MGD2_VX * MGD2_VY;
    if (tid < CT::C * CT::P) {
        const int tcol = tid % CT::C;
        const int tx = tcol % MGD_TX, ty = tcol / MGD_TX;
        const int vb = (tx + 1) + VY * (ty + 1), ub = (tx + 2) + SY * (ty + 2);
        for (int lz = tid / CT::C; lz < MGD_TZ; lz += CT::P) {
            const int v = vb + VZ * (lz + 1), u = ub + SZ * (lz + 2);
            const int d = ds[u];
            const V x1 = vs[v];
            const V nsum = ((vs[v - 1] + vs[v + 1]) + (vs[v - VY] + vs[v + VY])) + (vs[v - VZ] + vs[v + VZ]);
            ts[tcol + CT::C * lz] = d ? (bs[u] - (V)d * x1) + nsum : V(0);
        }
    }
    __syncthreads();
    mg_restrict_block<V, NT>(ts, bs, cx0, cy0, cz0, c);
}

template <typename V, int NT>
__global__ __launch_bounds__(NT) void k_mg_down2(MgLevel f, MgLevel c, const PcgState* __restrict__ ps)
{
    mg_down2_body<V, NT>(plain_blk(), f, c, ps);
}

template <typename V>
__global__ __launch_bounds__(MG_BATCH_NT2) void kb_mg_down2(const MgPairArgs* __restrict__ tab,
                                                   const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const MgPairArgs& a) {
        mg_down2_body<V, MG_BATCH_NT2>(b, glob(a.f), glob(a.c), as_global(a.ps));
    });
}

// ---- bottom: the coarsest level (at most 8^3 cells), one workgroup -------------

template <typename V>
__device__ __forceinline__ void mg_bottom_body(const MgLevel& L, const PcgState* __restrict__ ps)
{
    __shared__ V xs[2][512];
    const int q = threadIdx.x;
    const int n = level_count(L);
    const bool own = q < n;
    const int i = q % L.nx, j = (q / L.nx) % L.ny, k = q / (L.nx * L.ny);
    const int qc = own ? q : 0;
    const int dl = L.d[qc];
    const V bl = ((const V*)L.b)[qc];
    if (ps->done != PCG_RUNNING) return;
    const int d = own ? dl : 0;
    const V b = own ? bl : V(0);
    const V w = mg_omega<V>();
    const V wr = w * recip_nc<V>(d);
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
            xn = x[q] + (b - (V)d * x[q] + nsum) * wr;
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
    batch_for_each(tab, first, ns, [&](Blk b, const MgPairArgs& a) {  // the coarsest level is f
        mg_bottom_body<V>(glob(a.f), as_global(a.ps));
    });
}

// ---- up: dense level f from level c --------------------------------------------

// One workgroup per 16 x 8 x 8 block of level-f cells. The smoothing sweep
// reads y = x0 + P x_c on the block plus one cell around it (18 x 10 x 10, the
// y region), and P there reads the parents of those cells and the parents'
// neighbours (12 x 8 x 8 level-c cells, loaded clamped into the level, which
// is the prolongation's clamp). y is formed in LDS, then each thread updates
// four cells of the block.
constexpr int MGU_FX = 16, MGU_FY = 8, MGU_FZ = 8;
constexpr int MGU_YX = MGU_FX + 2, MGU_YY = MGU_FY + 2, MGU_YZ = MGU_FZ + 2;
constexpr int MGU_CX = MGU_FX / 2 + 4, MGU_CY = MGU_FY / 2 + 4, MGU_CZ = MGU_FZ / 2 + 4;
constexpr int MGU_Y = MGU_YX * MGU_YY * MGU_YZ;  // 1800
constexpr int MGU_C = MGU_CX * MGU_CY * MGU_CZ;  // 768

__host__ __device__ inline int mg_up_blocks_x(const MgLevel& f) { return (f.nx + MGU_FX - 1) / MGU_FX; }
__host__ __device__ inline int mg_up_blocks_y(const MgLevel& f) { return (f.ny + MGU_FY - 1) / MGU_FY; }
__host__ __device__ inline int64_t mg_up_blocks(const MgLevel& f)
{
    return (int64_t)mg_up_blocks_x(f) * mg_up_blocks_y(f) * ((f.nz + MGU_FZ - 1) / MGU_FZ);
}

template <typename V, int NT>
__device__ __forceinline__ void mg_up_body(Blk blk, const MgLevel& f, const MgLevel& c,
                                           const PcgState* __restrict__ ps)
{
    using CC = Cols<MGU_CX, MGU_CY, MGU_CZ, NT>;
    using CY = Cols<MGU_YX, MGU_YY, MGU_YZ, NT>;
    using CF = Cols<MGU_FX, MGU_FY, MGU_FZ, NT>;
    __shared__ V xs[MGU_C];
    __shared__ V ys[MGU_Y];
    __shared__ V bs[MGU_Y];
    __shared__ uint8_t ds[MGU_Y];
    const int tid = threadIdx.x;
    const int gbx = mg_up_blocks_x(f), gby = mg_up_blocks_y(f);
    const int bid = f.ulist ? (int)f.ulist[blk.id] : blk.id;  // plain launches: the listed blocks
    const int fx0 = (bid % gbx) * MGU_FX, fy0 = ((bid / gbx) % gby) * MGU_FY;
    const int fz0 = (bid / (gbx * gby)) * MGU_FZ;
    // coarse region origin: the parent of the y region's first cell, minus one
    const int px0 = fx0 / 2 - 2, py0 = fy0 / 2 - 2, pz0 = fz0 / 2 - 2;
    const V* const cx = (const V*)c.x;
    const V* const fb = (const V*)f.b;
    // coarse region, a column per thread (loaded clamped into level c)
    const int ccol = tid % CC::C, czg = tid / CC::C;
    const bool cact = tid < CC::C * CC::P;
    const int cbase = min(max(px0 + ccol % MGU_CX, 0), c.nx - 1) + c.nx * min(max(py0 + ccol / MGU_CX, 0), c.ny - 1);
    V xv[CC::J];
#pragma unroll
    for (int m = 0; m < CC::J; ++m) {
        const int k = pz0 + czg + CC::P * m;
        xv[m] = cx[cbase + c.nx * c.ny * min(max(k, 0), c.nz - 1)];
    }
    // y region, a column per thread
    const int ycol = tid % CY::C, yzg = tid / CY::C;
    const bool yact = tid < CY::C * CY::P;
    const int ylx = ycol % MGU_YX, yly = ycol / MGU_YX;
    const int gx = fx0 - 1 + ylx, gy = fy0 - 1 + yly;
    const bool yxy = gx >= 0 && gx < f.nx && gy >= 0 && gy < f.ny;
    const int ybase = min(max(gx, 0), f.nx - 1) + f.nx * min(max(gy, 0), f.ny - 1);
    const int sxy = f.nx * f.ny;
    V bv[CY::J];
    int dv[CY::J];
    bool iv[CY::J];
#pragma unroll
    for (int m = 0; m < CY::J; ++m) {
        const int lz = yzg + CY::P * m, gz = fz0 - 1 + lz;
        iv[m] = yact && lz < MGU_YZ && yxy && gz >= 0 && gz < f.nz;
        const int e = ybase + sxy * min(max(gz, 0), f.nz - 1);
        dv[m] = f.d[e];
        bv[m] = fb[e];
    }
    if (ps->done != PCG_RUNNING) return;
#pragma unroll
    for (int m = 0; m < CC::J; ++m) {
        const int lz = czg + CC::P * m;
        if (cact && lz < MGU_CZ) xs[ccol + CC::C * lz] = xv[m];
    }
    __syncthreads();
    const V w = mg_omega<V>();
    constexpr int CS = MGU_CX * MGU_CY;
    // parent and the parent's neighbour on this column's side in x and y
    // (region coordinates; the region holds clamped values)
    const int ax = (gx >> 1) - px0, ay = (gy >> 1) - py0;
    const int sx = (gx & 1) ? 1 : -1, sy = (gy & 1) ? MGU_CX : -MGU_CX;
#pragma unroll
    for (int m = 0; m < CY::J; ++m) {
        const int lz = yzg + CY::P * m;
        if (!yact || lz >= MGU_YZ) break;
        const int q = ycol + CY::C * lz;
        const int gz = fz0 - 1 + lz;
        const int d = iv[m] ? dv[m] : 0;
        V y = V(0);
        if (d) {
            const int az = (gz >> 1) - pz0, sz = (gz & 1) ? CS : -CS;
            const V* p = xs + ax + MGU_CX * ay + CS * az;
            const V x00 = V(0.75) * p[0] + V(0.25) * p[sx];
            const V x10 = V(0.75) * p[sy] + V(0.25) * p[sy + sx];
            const V x01 = V(0.75) * p[sz] + V(0.25) * p[sz + sx];
            const V x11 = V(0.75) * p[sz + sy] + V(0.25) * p[sz + sy + sx];
            const V y0 = V(0.75) * x00 + V(0.25) * x10, y1 = V(0.75) * x01 + V(0.25) * x11;
            y = w * bv[m] * recip_nc<V>(d) + (V(0.75) * y0 + V(0.25) * y1);
        }
        ys[q] = y;
        bs[q] = bv[m];
        ds[q] = (uint8_t)d;
    }
    __syncthreads();
    constexpr int SY = MGU_YX, SZ = MGU_YX * MGU_YY;
    const int fcol = tid % CF::C, fzg = tid / CF::C;
    const int lx = fcol % MGU_FX, ly = fcol / MGU_FX;
    const int i = fx0 + lx, j = fy0 + ly;
    const int ub = (lx + 1) + SY * (ly + 1);
    if (tid < CF::C * CF::P && i < f.nx && j < f.ny) {
#pragma unroll
        for (int m = 0; m < CF::J; ++m) {
            const int lz = fzg + CF::P * m, k = fz0 + lz;
            if (lz >= MGU_FZ || k >= f.nz) break;
            const int u = ub + SZ * (lz + 1);
            const int d = ds[u];
            const V yc = ys[u];
            const V nsum = ((ys[u - 1] + ys[u + 1]) + (ys[u - SY] + ys[u + SY])) + (ys[u - SZ] + ys[u + SZ]);
            ((V*)f.x)[level_index(f, i, j, k)] = d ? yc + w * ((bs[u] - (V)d * yc) + nsum) * recip_nc<V>(d) : V(0);
        }
    }
}

template <typename V, int NT>
__global__ __launch_bounds__(NT) void k_mg_up(MgLevel f, MgLevel c, const PcgState* __restrict__ ps)
{
    mg_up_body<V, NT>(plain_blk(), f, c, ps);
}

template <typename V>
__global__ __launch_bounds__(MG_BATCH_NT) void kb_mg_up(const MgPairArgs* __restrict__ tab,
                                                const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const MgPairArgs& a) {
        mg_up_body<V, MG_BATCH_NT>(b, glob(a.f), glob(a.c), as_global(a.ps));
    });
}

// ---- up with two sweeps (the levels below level 1) ----------------------------------
//
// The same blocks; the down kernel's two sweeps recomputed, the correction
// added, then two sweeps: y0 = x1 + P x_c, y1 = y0 + w (b - A y0) / n,
// x = y1 + w (b - A y1) / n. x on the block reads y1 one cell around it (the
// y region, 18 x 10 x 10), y1 there reads y0 one more cell out (the z region,
// 20 x 12 x 12, whose parents and their neighbours are the same 12 x 8 x 8
// coarse cells), and x1 on the z region reads x0, b and n one more cell out
// (the b region, 22 x 14 x 14).
constexpr int MGU2_ZX = MGU_FX + 4, MGU2_ZY = MGU_FY + 4, MGU2_ZZ = MGU_FZ + 4;
constexpr int MGU2_BX = MGU_FX + 6, MGU2_BY = MGU_FY + 6, MGU2_BZ = MGU_FZ + 6;
constexpr int MGU2_Z = MGU2_ZX * MGU2_ZY * MGU2_ZZ;  // 2880
constexpr int MGU2_B = MGU2_BX * MGU2_BY * MGU2_BZ;  // 4312

template <typename V, int NT>
__device__ __forceinline__ void mg_up2_body(Blk blk, const MgLevel& f, const MgLevel& c,
                                            const PcgState* __restrict__ ps)
{
    using CC = Cols<MGU_CX, MGU_CY, MGU_CZ, NT>;
    using CB = Cols<MGU2_BX, MGU2_BY, MGU2_BZ, NT>;
    using CZ = Cols<MGU2_ZX, MGU2_ZY, MGU2_ZZ, NT>;
    using CY = Cols<MGU_YX, MGU_YY, MGU_YZ, NT>;
    using CF = Cols<MGU_FX, MGU_FY, MGU_FZ, NT>;
    __shared__ V xs[MGU_C];         // x_c on the coarse region
    __shared__ V us[MGU2_B];        // x0 on the b region
    __shared__ V bs[MGU2_B];        // b on the b region
    __shared__ uint8_t ds[MGU2_B];  // n (0: not fluid or outside the level)
    __shared__ V zs[MGU2_Z];        // y0 on the z region
    __shared__ V ys[MGU_Y];         // y1 on the y region
    const int tid = threadIdx.x;
    const int gbx = mg_up_blocks_x(f), gby = mg_up_blocks_y(f);
    const int bid = f.ulist ? (int)f.ulist[blk.id] : blk.id;  // plain launches: the listed blocks
    const int fx0 = (bid % gbx) * MGU_FX, fy0 = ((bid / gbx) % gby) * MGU_FY;
    const int fz0 = (bid / (gbx * gby)) * MGU_FZ;
    const int px0 = fx0 / 2 - 2, py0 = fy0 / 2 - 2, pz0 = fz0 / 2 - 2;
    const V* const cx = (const V*)c.x;
    const V* const fb = (const V*)f.b;
    const int ccol = tid % CC::C, czg = tid / CC::C;
    const bool cact = tid < CC::C * CC::P;
    const int cbase = min(max(px0 + ccol % MGU_CX, 0), c.nx - 1) + c.nx * min(max(py0 + ccol / MGU_CX, 0), c.ny - 1);
    V xv[CC::J];
#pragma unroll
    for (int m = 0; m < CC::J; ++m) {
        const int k = pz0 + czg + CC::P * m;
        xv[m] = cx[cbase + c.nx * c.ny * min(max(k, 0), c.nz - 1)];
    }
    // b region (origin three cells below the block), a column per thread
    const int bcol = tid % CB::C, bzg = tid / CB::C;
    const bool bact = tid < CB::C * CB::P;
    const int bgx = fx0 - 3 + bcol % MGU2_BX, bgy = fy0 - 3 + bcol / MGU2_BX;
    const bool bxy = bgx >= 0 && bgx < f.nx && bgy >= 0 && bgy < f.ny;
    const int bbase = min(max(bgx, 0), f.nx - 1) + f.nx * min(max(bgy, 0), f.ny - 1);
    const int sxy = f.nx * f.ny;
    V bv[CB::J];
    int dv[CB::J];
    bool iv[CB::J];
#pragma unroll
    for (int m = 0; m < CB::J; ++m) {
        const int lz = bzg + CB::P * m, gz = fz0 - 3 + lz;
        iv[m] = bact && lz < MGU2_BZ && bxy && gz >= 0 && gz < f.nz;
        const int e = bbase + sxy * min(max(gz, 0), f.nz - 1);
        dv[m] = f.d[e];
        bv[m] = fb[e];
    }
    if (ps->done != PCG_RUNNING) return;
    const V w = mg_omega<V>();
#pragma unroll
    for (int m = 0; m < CC::J; ++m) {
        const int lz = czg + CC::P * m;
        if (cact && lz < MGU_CZ) xs[ccol + CC::C * lz] = xv[m];
    }
#pragma unroll
    for (int m = 0; m < CB::J; ++m) {
        const int lz = bzg + CB::P * m;
        if (bact && lz < MGU2_BZ) {
            const int q = bcol + CB::C * lz;
            const int d = iv[m] ? dv[m] : 0;
            us[q] = d ? w * bv[m] * recip_nc<V>(d) : V(0);
            bs[q] = bv[m];
            ds[q] = (uint8_t)d;
        }
    }
    __syncthreads();
    constexpr int BY = MGU2_BX, BZ = MGU2_BX * MGU2_BY;
    constexpr int CS = MGU_CX * MGU_CY;
    // y0 = x1 + P x_c on the z region (origin two cells below the block)
    if (tid < CZ::C * CZ::P) {
        const int zcol = tid % CZ::C;
        const int lx = zcol % MGU2_ZX, ly = zcol / MGU2_ZX;
        const int gx = fx0 - 2 + lx, gy = fy0 - 2 + ly;
        const int ax = (gx >> 1) - px0, ay = (gy >> 1) - py0;
        const int sx = (gx & 1) ? 1 : -1, sy = (gy & 1) ? MGU_CX : -MGU_CX;
        const int ub = (lx + 1) + BY * (ly + 1);
        for (int lz = tid / CZ::C; lz < MGU2_ZZ; lz += CZ::P) {
            const int u = ub + BZ * (lz + 1);
            const int d = ds[u];
            V y = V(0);
            if (d) {
                const V x0 = us[u];
                const V nsum = ((us[u - 1] + us[u + 1]) + (us[u - BY] + us[u + BY])) + (us[u - BZ] + us[u + BZ]);
                const V x1 = x0 + w * ((bs[u] - (V)d * x0) + nsum) * recip_nc<V>(d);
                const int gz = fz0 - 2 + lz;
                const int az = (gz >> 1) - pz0, sz = (gz & 1) ? CS : -CS;
                const V* p = xs + ax + MGU_CX * ay + CS * az;
                const V x00 = V(0.75) * p[0] + V(0.25) * p[sx];
                const V x10 = V(0.75) * p[sy] + V(0.25) * p[sy + sx];
                const V x01 = V(0.75) * p[sz] + V(0.25) * p[sz + sx];
                const V x11 = V(0.75) * p[sz + sy] + V(0.25) * p[sz + sy + sx];
                const V y0 = V(0.75) * x00 + V(0.25) * x10, y1 = V(0.75) * x01 + V(0.25) * x11;
                y = x1 + (V(0.75) * y0 + V(0.25) * y1);
            }
            zs[zcol + CZ::C * lz] = y;
        }
    }
    __syncthreads();
    // y1 on the y region (origin one cell below the block)
    constexpr int ZY = MGU2_ZX, ZZ = MGU2_ZX * MGU2_ZY;
    if (tid < CY::C * CY::P) {
        const int ycol = tid % CY::C;
        const int lx = ycol % MGU_YX, ly = ycol / MGU_YX;
        const int zb = (lx + 1) + ZY * (ly + 1), ub = (lx + 2) + BY * (ly + 2);
        for (int lz = tid / CY::C; lz < MGU_YZ; lz += CY::P) {
            const int z = zb + ZZ * (lz + 1), u = ub + BZ * (lz + 2);
            const int d = ds[u];
            const V yc = zs[z];
            const V nsum = ((zs[z - 1] + zs[z + 1]) + (zs[z - ZY] + zs[z + ZY])) + (zs[z - ZZ] + zs[z + ZZ]);
            ys[ycol + CY::C * lz] = d ? yc + w * ((bs[u] - (V)d * yc) + nsum) * recip_nc<V>(d) : V(0);
        }
    }
    __syncthreads();
    constexpr int SY = MGU_YX, SZ = MGU_YX * MGU_YY;
    const int fcol = tid % CF::C, fzg = tid / CF::C;
    const int lx = fcol % MGU_FX, ly = fcol / MGU_FX;
    const int i = fx0 + lx, j = fy0 + ly;
    const int yb = (lx + 1) + SY * (ly + 1), ub = (lx + 3) + BY * (ly + 3);
    if (tid < CF::C * CF::P && i < f.nx && j < f.ny) {
#pragma unroll
        for (int m = 0; m < CF::J; ++m) {
            const int lz = fzg + CF::P * m, k = fz0 + lz;
            if (lz >= MGU_FZ || k >= f.nz) break;
            const int y = yb + SZ * (lz + 1), u = ub + BZ * (lz + 3);
            const int d = ds[u];
            const V yc = ys[y];
            const V nsum = ((ys[y - 1] + ys[y + 1]) + (ys[y - SY] + ys[y + SY])) + (ys[y - SZ] + ys[y + SZ]);
            ((V*)f.x)[level_index(f, i, j, k)] = d ? yc + w * ((bs[u] - (V)d * yc) + nsum) * recip_nc<V>(d) : V(0);
        }
    }
}

template <typename V, int NT>
__global__ __launch_bounds__(NT) void k_mg_up2(MgLevel f, MgLevel c, const PcgState* __restrict__ ps)
{
    mg_up2_body<V, NT>(plain_blk(), f, c, ps);
}

template <typename V>
__global__ __launch_bounds__(MG_BATCH_NT2) void kb_mg_up2(const MgPairArgs* __restrict__ tab,
                                                 const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const MgPairArgs& a) {
        mg_up2_body<V, MG_BATCH_NT2>(b, glob(a.f), glob(a.c), as_global(a.ps));
    });
}

// ---- cell types of the coarse levels -----------------------------------------
//
// One wave per restriction block of level c (8 x 4 x 4 cells, two per lane):
// the wave writes the cells' types and, for the plain launches, lists the
// block when it holds a fluid cell, and lists the prolongation block
// (16 x 8 x 8) that contains it the first time one of its restriction blocks
// is listed.
constexpr int MGT_WAVES = 4;  // waves (restriction blocks) per workgroup

__host__ __device__ inline int64_t mg_types_groups(const MgLevel& c)
{
    return (mg_down_blocks(c) + MGT_WAVES - 1) / MGT_WAVES;
}

template <typename Fluid>
__device__ __forceinline__ void mg_types_block(Blk b, const MgLevel& c, Fluid is_fluid)
{
    const int lane = threadIdx.x & 63;
    const int64_t db = (int64_t)b.id * MGT_WAVES + (threadIdx.x >> 6);
    const int nbx = mg_down_blocks_x(c), nby = mg_down_blocks_y(c);
    const bool live = db < mg_down_blocks(c);
    const int bx = (int)(db % nbx), by = (int)((db / nbx) % nby), bz = (int)(db / ((int64_t)nbx * nby));
    bool any = false;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e = lane + 64 * h;  // x fastest within the block
        const int i = bx * MGD_CX + (e & 7), j = by * MGD_CY + ((e >> 3) & 3), k = bz * MGD_CZ + (e >> 5);
        if (!live || i >= c.nx || j >= c.ny || k >= c.nz) continue;
        const bool fluid = is_fluid(i, j, k);
        c.d[level_index(c, i, j, k)] = fluid ? (uint8_t)level_nc(c, i, j, k) : (uint8_t)0;
        any = any || fluid;
    }
    if (!c.dlist) return;  // uniform: batched launches list nothing
    if (__ballot(any) != 0 && lane == 0) {
        c.dlist[atomicAdd(c.cnt, 1u)] = (uint32_t)db;
        const int ub = (bx * MGD_CX) / MGU_FX +
                       mg_up_blocks_x(c) * ((by * MGD_CY) / MGU_FY + mg_up_blocks_y(c) * ((bz * MGD_CZ) / MGU_FZ));
        if (atomicOr(&c.uflag[ub], 1u) == 0u) c.ulist[atomicAdd(c.cnt + 1, 1u)] = (uint32_t)ub;
    }
}

// level 1 from the fine grid's n_c (tile layout): fluid when a child is.
// The 2x2x2 children of a level-1 cell lie in one 8^3 tile (even offsets),
// where they are four x-adjacent byte pairs; cells of an active tile outside
// the domain hold n_c = 0, and an inactive tile holds no fluid cell.
__device__ __forceinline__ void mg_types_fine_body(Blk b, const Geo& g, const int32_t* __restrict__ tile_slot,
                                                   const uint8_t* __restrict__ diag, const MgLevel& c)
{
    mg_types_block(b, c, [&](int i, int j, int k) {
        const int gi = 2 * i, gj = 2 * j, gk = 2 * k;
        const int32_t s = tile_slot[(gi >> 3) + (int64_t)g.tx * ((gj >> 3) + (int64_t)g.ty * (gk >> 3))];
        if (s < 0) return false;
        const uint8_t* d = diag + (int64_t)s * TILE_CELLS + (gi & 7) + 8 * (gj & 7) + 64 * (gk & 7);
        const uint16_t p00 = *(const uint16_t*)d, p10 = *(const uint16_t*)(d + 8);
        const uint16_t p01 = *(const uint16_t*)(d + 64), p11 = *(const uint16_t*)(d + 72);
        return ((p00 | p10) | (p01 | p11)) != 0;
    });
}

__global__ __launch_bounds__(64 * MGT_WAVES) void k_mg_types_fine(Geo g, const int32_t* __restrict__ tile_slot,
                                                                 const uint8_t* __restrict__ diag, MgLevel c)
{
    mg_types_fine_body(plain_blk(), g, tile_slot, diag, c);
}

__global__ __launch_bounds__(64 * MGT_WAVES) void kb_mg_types_fine(const MgTypesFineArgs* __restrict__ tab,
                                                                  const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const MgTypesFineArgs& a) {
        mg_types_fine_body(b, a.g, as_global(a.tile_slot), as_global(a.diag), glob(a.c));
    });
}

// level c from level f: fluid when a child is
__device__ __forceinline__ void mg_types_body(Blk b, const MgLevel& f, const MgLevel& c)
{
    mg_types_block(b, c, [&](int i, int j, int k) {
        bool fluid = false;
        for (int o = 0; o < 8; ++o) {
            const int fi = 2 * i + (o & 1), fj = 2 * j + ((o >> 1) & 1), fk = 2 * k + (o >> 2);
            if (fi < f.nx && fj < f.ny && fk < f.nz && f.d[level_index(f, fi, fj, fk)] > 0) fluid = true;
        }
        return fluid;
    });
}

__global__ __launch_bounds__(64 * MGT_WAVES) void k_mg_types(MgLevel f, MgLevel c)
{
    mg_types_body(plain_blk(), f, c);
}

__global__ __launch_bounds__(64 * MGT_WAVES) void kb_mg_types(const MgPairArgs* __restrict__ tab,
                                                             const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const MgPairArgs& a) {
        mg_types_body(b, glob(a.f), glob(a.c));
    });
}

// ---- launchers -----------------------------------------------------------------

namespace {
inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }
}  // namespace

void launch_mg_types_fine(const Geo& g, const int32_t* tile_slot, const uint8_t* diag, const MgLevel& c,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_mg_types_fine, dim3((unsigned)mg_types_groups(c)), dim3(64 * MGT_WAVES), 0, st, g,
                       tile_slot, diag, c);
}

void launch_mg_types(const MgLevel& f, const MgLevel& c, hipStream_t st)
{
    hipLaunchKernelGGL(k_mg_types, dim3((unsigned)mg_types_groups(c)), dim3(64 * MGT_WAVES), 0, st, f, c);
}

template <typename V>
void launch_mg_coarse(const MgLevel* lv, int nlev, const PcgState* ps, hipStream_t st)
{
    // launches of fewer than 512 workgroups (the levels below 128^3 cells at
    // 256^3) run 1024-thread workgroups, larger ones 512 (256 threads for
    // all: 1.69 ms per step for the coarse levels at 256^3; 1024 for the
    // small ones: 1.44; 512 for the 128^3 level: 1.32, where 1024 was slower)
    // (the shape is chosen by the level's whole block count). Launches of
    // 512 workgroups or more run the listed blocks only; the smaller ones run
    // every block: there the list's extra dependent load cost more (about
    // 0.2 us per launch) than the few air blocks it saved.
    constexpr int64_t SMALL = 512;
    for (int l = 0; l + 1 < nlev; ++l) {
        MgLevel c = lv[l + 1];
        const int64_t nb = mg_down_blocks(c);
        if (nb < SMALL) c.dlist = nullptr;
        const int64_t grid = c.dlist ? c.nd : nb;
        if (grid <= 0) continue;
        auto kern = mg_two_sweeps(l) ? (nb < SMALL ? k_mg_down2<V, 1024> : k_mg_down2<V, 512>)
                                     : (nb < SMALL ? k_mg_down<V, 1024> : k_mg_down<V, 512>);
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(nb < SMALL ? 1024 : 512), 0, st, lv[l], c, ps);
    }
    hipLaunchKernelGGL(k_mg_bottom<V>, dim3(1), dim3(512), 0, st, lv[nlev - 1], ps);
    for (int l = nlev - 2; l >= 0; --l) {
        MgLevel f = lv[l];
        const int64_t nb = mg_up_blocks(f);
        if (nb < SMALL) f.ulist = nullptr;
        const int64_t grid = f.ulist ? f.nu : nb;
        if (grid <= 0) continue;
        auto kern = mg_two_sweeps(l) ? (nb < SMALL ? k_mg_up2<V, 1024> : k_mg_up2<V, 512>)
                                     : (nb < SMALL ? k_mg_up<V, 1024> : k_mg_up<V, 512>);
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(nb < SMALL ? 1024 : 512), 0, st, f, lv[l + 1], ps);
    }
}

template void launch_mg_coarse<float>(const MgLevel*, int, const PcgState*, hipStream_t);
template void launch_mg_coarse<double>(const MgLevel*, int, const PcgState*, hipStream_t);

// ---- batched launchers (grids: see mg_batch_blocks) ------------------------------

int64_t mg_blocks(int kind, const MgLevel& f, const MgLevel& c)
{
    switch (kind) {
    case MG_B_TYPES: return mg_types_groups(c);
    case MG_B_DOWN: return mg_down_blocks(c);
    case MG_B_BOTTOM: return 1;
    default: return mg_up_blocks(f);  // MG_B_UP
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
void launch_b_mg_level(int kind, bool two_sweeps, const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    const MgPairArgs* a = (const MgPairArgs*)L.args;
    if (kind == MG_B_DOWN)
        hipLaunchKernelGGL(two_sweeps ? kb_mg_down2<V> : kb_mg_down<V>, dim3(L.blocks),
                           dim3(two_sweeps ? MG_BATCH_NT2 : MG_BATCH_NT), 0, st, a, L.first, L.ns);
    else if (kind == MG_B_BOTTOM)
        hipLaunchKernelGGL(kb_mg_bottom<V>, dim3(L.blocks), dim3(512), 0, st, a, L.first, L.ns);
    else
        hipLaunchKernelGGL(two_sweeps ? kb_mg_up2<V> : kb_mg_up<V>, dim3(L.blocks),
                           dim3(two_sweeps ? MG_BATCH_NT2 : MG_BATCH_NT), 0, st, a, L.first, L.ns);
}
template void launch_b_mg_level<float>(int, bool, const BatchLaunch&, hipStream_t);
template void launch_b_mg_level<double>(int, bool, const BatchLaunch&, hipStream_t);

}  // namespace flipmi
