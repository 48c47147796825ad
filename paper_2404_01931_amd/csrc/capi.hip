// C ABI of libflipmi: configuration, workspace carving, seeding, the step
// sequence and readback. See include/flip.h for the contract of each call.
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/flip.h"
#include "batch.h"
#include "common.h"
#include "handle.h"

using namespace flipmi;

// Scratch of flip_surface_mesh_noalloc: the marching-cubes edge flags, vertex
// numbers, per-cube counts and scan words live here instead of in a caller
// workspace. Every device the library runs on holds its own copy for the life
// of the process; host code reaches it only through the device address looked
// up at flip_init (the array's name is not a device address on the host).
constexpr size_t MC_SCRATCH_BYTES = (size_t)64 << 20;
static_assert(MC_SCRATCH_BYTES == FLIP_MESH_SCRATCH_MAX_BYTES, "header and library agree on the limit");
static __device__ __align__(256) unsigned char scratch[MC_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch[SCRATCH_MAX_DEVICES] = {};

// Looks up (once per device, with that device current) and returns the device
// address of this device's `scratch`.
flip_status scratch_setup(int dev)
{
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return FLIP_E_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev]) return FLIP_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FLIP_E_HIP;
    g_scratch[dev] = p;
    return FLIP_OK;
}

void* scratch_of(int dev)
{
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[dev];
}

constexpr size_t ALIGN = 256;
constexpr int TIMED_PCG_EVERY = 8;  // with kernel timing on, one PCG iteration in 8 is bracketed
constexpr int EVENT_PAIRS = 2048;
constexpr int MAX_REFINEMENTS = 20;  // FLIP_MIXED: outer refinements per step

size_t align_up(size_t v) { return (v + ALIGN - 1) & ~(ALIGN - 1); }

// Computes the workspace layout; with base == nullptr it only sums sizes.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <typename P>
    P* take(size_t bytes)
    {
        size_t o = off;
        off = align_up(off + (bytes ? bytes : 1));
        return base ? (P*)(base + o) : nullptr;
    }
};


// ---------------------------------------------------------------------------
// seeding (paper Sec. 3.1.2): sub^3 jittered subcells per cell whose centre is
// inside a region. Jitter: SplitMix64 output sequence (Steele, Lea & Flood
// 2014) of `seed`, element 3 * (sub^3 * cell + subcell) + axis, top 53 bits.
// ---------------------------------------------------------------------------

uint64_t splitmix_element(uint64_t seed, uint64_t index)
{
    uint64_t z = seed + (index + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double jitter(uint64_t seed, uint64_t index)
{
    return (double)(splitmix_element(seed, index) >> 11) * 0x1.0p-53;
}

const flip_region* region_of_centre(const flip_config& c, int i, int j, int k)
{
#pragma clang fp contract(off)
    const double p[3] = {(i + 0.5) * c.dx, (j + 0.5) * c.dx, (k + 0.5) * c.dx};
    for (uint32_t r = 0; r < c.n_regions; ++r) {
        const flip_region& g = c.regions[r];
        if (g.kind == FLIP_REGION_BOX) {
            bool in = true;
            for (int a = 0; a < 3; ++a) in = in && (g.lo[a] <= p[a] && p[a] < g.hi[a]);
            if (in) return &g;
        } else {
            double d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double d = p[a] - g.center[a];
                const double dd = d * d;
                d2 = d2 + dd;
            }
            if (d2 < g.radius * g.radius) return &g;
        }
    }
    return nullptr;
}

int64_t seeded_count(const flip_config& c)
{
    const int64_t per = (int64_t)c.subcells_per_axis * c.subcells_per_axis * c.subcells_per_axis;
    int64_t n = 0;
    for (int k = 0; k < c.nz; ++k)
        for (int j = 0; j < c.ny; ++j)
            for (int i = 0; i < c.nx; ++i)
                if (region_of_centre(c, i, j, k)) n += per;
    return n;
}

template <typename T>
void seed_particles(const flip_config& c, std::vector<T>& pos, std::vector<T>& vel, int64_t n)
{
#pragma clang fp contract(off)
    const int sub = c.subcells_per_axis;
    const int64_t per = (int64_t)sub * sub * sub;
    int64_t q = 0;
    for (int k = 0; k < c.nz; ++k)
        for (int j = 0; j < c.ny; ++j)
            for (int i = 0; i < c.nx; ++i) {
                const flip_region* r = region_of_centre(c, i, j, k);
                if (!r) continue;
                const uint64_t cell = (uint64_t)i + (uint64_t)c.nx * ((uint64_t)j + (uint64_t)c.ny * k);
                for (int sz = 0; sz < sub; ++sz)
                    for (int sy = 0; sy < sub; ++sy)
                        for (int sx = 0; sx < sub; ++sx) {
                            const uint64_t s = (uint64_t)sx + (uint64_t)sub * ((uint64_t)sy + (uint64_t)sub * sz);
                            const uint64_t base = 3u * (per * cell + s);
                            const double x = (((double)sx + jitter(c.seed, base + 0)) / sub + i) * c.dx;
                            const double y = (((double)sy + jitter(c.seed, base + 1)) / sub + j) * c.dx;
                            const double z = (((double)sz + jitter(c.seed, base + 2)) / sub + k) * c.dx;
                            pos[q] = (T)x;
                            pos[n + q] = (T)y;
                            pos[2 * n + q] = (T)z;
                            for (int a = 0; a < 3; ++a) vel[a * n + q] = (T)r->vel[a];
                            ++q;
                        }
            }
}

}  // namespace


namespace {

size_t real_bytes(int prec) { return prec == FLIP_FP64 ? 8 : 4; }

flip_status validate(const flip_config* c)
{
    if (!c) return FLIP_E_INVALID;
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return FLIP_E_INVALID;
    if ((int64_t)c->nx * c->ny * c->nz >= (int64_t)1 << 31) return FLIP_E_INVALID;
    if (!(c->dx > 0.0) || !std::isfinite(c->dx)) return FLIP_E_INVALID;
    if (!(c->dt > 0.0) || !std::isfinite(c->dt)) return FLIP_E_INVALID;
    if (!(c->density > 0.0) || !std::isfinite(c->density)) return FLIP_E_INVALID;
    if (!(c->flip_ratio >= 0.0 && c->flip_ratio <= 1.0)) return FLIP_E_INVALID;
    if (!(c->pcg_tol >= 0.0) || !std::isfinite(c->pcg_tol)) return FLIP_E_INVALID;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(c->gravity[a])) return FLIP_E_INVALID;
    if (c->precision != FLIP_FP32 && c->precision != FLIP_FP64 && c->precision != FLIP_MIXED)
        return FLIP_E_INVALID;
    if (c->precision == FLIP_MIXED && (!(c->ir_tol > 0.0) || !std::isfinite(c->ir_tol))) return FLIP_E_INVALID;
    if ((c->flags & FLIP_FLAG_RED_BLACK_GS) && (c->precision == FLIP_MIXED || (c->flags & FLIP_FLAG_MULTIGRID)))
        return FLIP_E_INVALID;
    if ((c->flags & FLIP_FLAG_ADAPTIVE_DT) && (!(c->cfl > 0.0) || !std::isfinite(c->cfl))) return FLIP_E_INVALID;
    if ((c->flags & FLIP_FLAG_RESEED) && (c->subcells_per_axis < 1 || c->subcells_per_axis > 16))
        return FLIP_E_INVALID;
    if (c->particle_capacity >= ((int64_t)1 << 31)) return FLIP_E_INVALID;
    if (c->pos0) {
        if (c->n_particles < 0 || c->n_particles >= ((int64_t)1 << 31) || !c->vel0) return FLIP_E_INVALID;
    } else {
        if (c->n_regions > 0 && !c->regions) return FLIP_E_INVALID;
        if (c->n_regions > 4096) return FLIP_E_INVALID;
        if (c->subcells_per_axis < 1 || c->subcells_per_axis > 16) return FLIP_E_INVALID;
        for (uint32_t r = 0; r < c->n_regions; ++r)
            if (c->regions[r].kind != FLIP_REGION_BOX && c->regions[r].kind != FLIP_REGION_SPHERE)
                return FLIP_E_INVALID;
    }
    return FLIP_OK;
}

flip_status particle_count(const flip_config* c, int64_t* n)
{
    if (c->pos0) {
        *n = c->n_particles;
        return FLIP_OK;
    }
    int64_t m = seeded_count(*c);
    if (m >= ((int64_t)1 << 31)) return FLIP_E_INVALID;
    *n = m;
    return FLIP_OK;
}

Geo make_geo(const flip_config* c)
{
    Geo g;
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    g.tx = (c->nx + TILE - 1) / TILE;
    g.ty = (c->ny + TILE - 1) / TILE;
    g.tz = (c->nz + TILE - 1) / TILE;
    g.dx = c->dx;
    g.inv_dx = 1.0 / c->dx;
    int e = 0;
    g.dyadic = std::frexp(c->dx, &e) == 0.5 && e > -120 && e < 120;
    return g;
}

Sizes make_sizes(const flip_config* c, int64_t n)
{
    Sizes s;
    s.n = n;
    s.pcap = std::max<int64_t>(n, c->particle_capacity);
    s.C = (int64_t)c->nx * c->ny * c->nz;
    Geo g = make_geo(c);
    s.T = tiles_of(g);
    s.cap = s.T * TILE_CELLS;
    s.F[0] = (int64_t)(c->nx + 1) * c->ny * c->nz;
    s.F[1] = (int64_t)c->nx * (c->ny + 1) * c->nz;
    s.F[2] = (int64_t)c->nx * c->ny * (c->nz + 1);
    s.rb = real_bytes(c->precision);
    return s;
}

// Persistent workgroups of the solver kernels: one per PCG_TILES_PER_GROUP
// grid tiles, at least one, at most PCG_MAX_GROUPS. A function of the grid
// alone, so a scene's reductions run in the same order alone and in a batch.
int solver_groups(int64_t tiles)
{
    const int64_t g = (tiles + PCG_TILES_PER_GROUP - 1) / PCG_TILES_PER_GROUP;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, PCG_MAX_GROUPS));
}

// One layout for both sizing and carving.
void carve(flip_handle* h, Carver& cv)
{
    const Sizes& s = h->sz;
    const size_t rb = s.rb;
    for (int q = 0; q < 2; ++q) {
        h->pos[q] = cv.take<void>((3 * s.pcap + PARTICLE_PAD) * rb);
        h->vel[q] = cv.take<void>((3 * s.pcap + PARTICLE_PAD) * rb);
        h->id[q] = cv.take<uint32_t>(4 * s.pcap);
    }
    h->key = cv.take<uint32_t>(4 * s.pcap);
    h->rank = cv.take<uint32_t>(4 * s.pcap);
    h->perm = cv.take<uint32_t>(4 * s.pcap);
    h->count = cv.take<uint32_t>(4 * s.C);
    h->count_next = cv.take<uint32_t>(4 * s.C);
    h->start = cv.take<uint32_t>(4 * s.C);
    h->scan_tmp = cv.take<uint32_t>(4 * scan_tmp_words(s.C > s.T ? s.C : s.T));
    h->tile_flag = cv.take<uint32_t>(4 * s.T);
    h->tile_next = cv.take<uint32_t>(4 * s.T);
    h->tile_excl = cv.take<uint32_t>(4 * s.T);
    h->tile_list = cv.take<uint32_t>(4 * s.T);
    h->tile_slot = cv.take<int32_t>(4 * s.T);
    h->tile_nbr = cv.take<int32_t>(24 * s.T);
    h->d_nactive = cv.take<uint32_t>(4);
    for (int a = 0; a < 3; ++a) {
        h->f_old[a] = cv.take<void>(s.F[a] * rb);
        h->f_star[a] = cv.take<void>(s.F[a] * rb);
        h->f_new[a] = cv.take<void>(s.F[a] * rb);
    }
    h->diag = cv.take<uint8_t>(s.cap);
    h->b = cv.take<void>(s.cap * rb);
    h->z = cv.take<void>(s.cap * rb);
    h->xin[0] = cv.take<void>(s.cap * rb);
    h->s[0] = cv.take<void>(s.cap * rb);
    h->s[1] = cv.take<void>(s.cap * rb);
    h->nmg = 0;
    if (h->cfg.flags & FLIP_FLAG_MULTIGRID) {
        // z = M r, then the coarse levels: every axis halved (ceil) until
        // none has more than MG_BOTTOM_SIDE cells
        h->mgz = cv.take<void>(s.cap * rb);
        if (mg_fused_update(rb)) h->q = cv.take<void>(s.cap * rb);
        int nx = h->cfg.nx, ny = h->cfg.ny, nz = h->cfg.nz;
        do {
            nx = (nx + 1) / 2;
            ny = (ny + 1) / 2;
            nz = (nz + 1) / 2;
            const int64_t cells = (int64_t)nx * ny * nz;
            MgLevel& L = h->mg[h->nmg++];
            L = MgLevel{};
            L.nx = nx;
            L.ny = ny;
            L.nz = nz;
            L.b = cv.take<void>(cells * rb);
            L.d = cv.take<uint8_t>(cells);
        } while ((nx > MG_BOTTOM_SIDE || ny > MG_BOTTOM_SIDE || nz > MG_BOTTOM_SIDE) && h->nmg < MG_MAX_LEVELS);
        // cleared at every step, in one range: the solutions x (air cells
        // hold 0; the blocks a plain launch skips are not written), the
        // block marks and the block counts
        const size_t zero_from = cv.off;
        for (int l = 0; l < h->nmg; ++l) {
            MgLevel& L = h->mg[l];
            L.x = cv.take<void>((int64_t)L.nx * L.ny * L.nz * rb);
        }
        for (int l = 0; l < h->nmg; ++l) {
            MgLevel& L = h->mg[l];
            L.uflag = cv.take<uint32_t>(4 * mg_blocks(MG_B_UP, L, L));
        }
        h->mg_cnt = cv.take<uint32_t>(4 * 2 * MG_MAX_LEVELS);
        h->mg_zero = cv.base ? cv.base + zero_from : nullptr;
        h->mg_zero_bytes = cv.off - zero_from;
        for (int l = 0; l < h->nmg; ++l) {
            MgLevel& L = h->mg[l];
            L.dlist = cv.take<uint32_t>(4 * mg_blocks(MG_B_DOWN, L, L));
            L.ulist = cv.take<uint32_t>(4 * mg_blocks(MG_B_UP, L, L));
            L.cnt = h->mg_cnt ? h->mg_cnt + 2 * l : nullptr;
        }
    }
    if (h->prec == FLIP_MIXED) {
        h->xin[1] = cv.take<void>(s.cap * rb);
        h->b64 = cv.take<double>(s.cap * 8);
        h->x64[0] = cv.take<double>(s.cap * 8);
        h->x64[1] = cv.take<double>(s.cap * 8);
    }
    h->partials = cv.take<double>(3 * sizeof(double) * solver_groups(s.T));
    h->pslots = cv.take<double>(PCG_SLOT_SETS * sizeof(double) * solver_groups(s.T));
    h->ps = cv.take<PcgState>(PCG_STATE_BYTES + SYNC_BYTES);
    h->gs_rmax = cv.take<unsigned long long>(8);
    h->diagw = cv.take<DiagWords>(sizeof(DiagWords));
    h->diag_part = cv.take<double>(8 * DIAG_ENERGY_BLOCKS);
    h->d_reseeded = cv.take<uint32_t>(4);
    h->staging = cv.take<void>(8 * s.C);
}


// ---- kernel timing (FLIP_FLAG_KERNEL_TIMING) --------------------------------

int timer_begin(flip_handle* h, int kind, hipStream_t st, int pcg_iter = -1)
{
    if (!(h->cfg.flags & FLIP_FLAG_KERNEL_TIMING) || h->ev_used + 1 >= (int)h->ev.size()) return -1;
    const int q = h->ev_used;
    h->ev_used += 2;
    h->ev_kind[q / 2] = kind;
    h->ev_iter[q / 2] = pcg_iter;
    (void)hipEventRecord(h->ev[q], st);
    return q;
}

void timer_end(flip_handle* h, int q, hipStream_t st)
{
    if (q >= 0) (void)hipEventRecord(h->ev[q + 1], st);
}

// An event pair for a launch that records its own start and end (the solver
// kernels: their launches are short, so the dispatch latency that separate
// event records would include matters). Returns the pair's first index or -1.
int timer_pair(flip_handle* h, int kind, int pcg_iter)
{
    if (!(h->cfg.flags & FLIP_FLAG_KERNEL_TIMING) || h->ev_used + 1 >= (int)h->ev.size()) return -1;
    const int q = h->ev_used;
    h->ev_used += 2;
    h->ev_kind[q / 2] = kind;
    h->ev_iter[q / 2] = pcg_iter;
    return q;
}

flip_status timer_collect(flip_handle* h, hipStream_t st)
{
    if (h->ev_used == 0) return FLIP_OK;
    HIP_TRY(hipStreamSynchronize(st));
    for (int q = 0; q < h->ev_used; q += 2) {
        if (h->ev_kind[q / 2] < 0) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev[q], h->ev[q + 1]) == hipSuccess) {
            h->stats.kernel_ms[h->ev_kind[q / 2]] += ms;
            h->stats.kernel_launches[h->ev_kind[q / 2]] += 1;
        }
    }
    h->ev_used = 0;
    return FLIP_OK;
}

// ---- one step -----------------------------------------------------------------

// Launch PCG iterations in chunks until the device-side state says the current
// (inner) solve is over; returns the state read at the end. Iteration k is
// D_k then U_k; the direction kernel tests convergence of the residual the
// update before it left, so the sequence is D_0, then (U_k, D_{k+1}) pairs,
// and every chunk ends with a test.
template <typename V>
flip_status pcg_loop(flip_handle* h, V* x, int max_iters, hipStream_t st, PcgState* out)
{
    // Chunk sizes: each host test idles the GPU for a round trip, and each
    // iteration launched past convergence still costs its launches (two with
    // Jacobi, a dozen with the V-cycle), so the multigrid solve starts with
    // the previous step's count and then tests every two iterations, the
    // Jacobi solve with two fewer than before and then every eight.
    const bool mg_solve = h->nmg > 0;
    int chunk = h->prev_iters > 2 ? (mg_solve ? h->prev_iters : h->prev_iters - 2) : 16;
    const int next_chunk = mg_solve ? 2 : 8;
    int launched = 0;
    const int first_sample = h->ev_used / 2;
    // FLIP_FLAG_MULTIGRID: r lives in rvec(k) before update k and the last
    // V-cycle's z = M r in zvec(k); a V-cycle runs before every direction
    // kernel. With FP32 vectors the update kernel also does the V-cycle's
    // fine down kernel (launch_pcg_update_down), so `precondition` then
    // starts at level 1, and it writes the new r to the vector that held z:
    // h->z and h->mgz trade places at every update. In FP64, r stays in h->z
    // and z in h->mgz. Without multigrid r / n lives in h->z.
    const bool mg = h->nmg > 0;
    const bool fused = mg && mg_fused_update(sizeof(V));
    auto rvec = [&](int k) { return (V*)(fused && (k & 1) ? h->mgz : h->z); };
    auto zvec = [&](int k) { return (V*)(fused && (k & 1) ? h->z : h->mgz); };
    auto direction = [&](int k) {
        const int sc = h->scur;
        const int q = (k % TIMED_PCG_EVERY) == 0 ? timer_pair(h, FLIP_KERNEL_PCG_DIRECTION, k) : -1;
        launch_pcg_direction<V>(h->groups, h->na, h->tile_nbr, h->diag, mg ? zvec(k) : (const V*)h->z,
                                (const V*)h->s[sc], (V*)h->s[sc ^ 1], fused ? (V*)h->q : nullptr, h->pslots, h->ps,
                                st, q >= 0 ? h->ev[q] : nullptr, q >= 0 ? h->ev[q + 1] : nullptr);
    };
    auto precondition = [&](int k, bool fine_down) {
        if (!mg) return;
        const bool timed = (k % TIMED_PCG_EVERY) == 0;
        int q = -1;
        if (fine_down) {
            q = timed ? timer_pair(h, FLIP_KERNEL_MG_DOWN_FINE, k) : -1;
            launch_mg_fine<V>(false, h->groups, h->na, h->geo, h->tile_list, h->tile_nbr, h->diag, rvec(k),
                              h->mg[0], nullptr, nullptr, h->ps, st, q >= 0 ? h->ev[q] : nullptr,
                              q >= 0 ? h->ev[q + 1] : nullptr);
        }
        q = timed ? timer_begin(h, FLIP_KERNEL_MG_COARSE, st, k) : -1;
        launch_mg_coarse<V>(h->mg, h->nmg, h->ps, st);
        timer_end(h, q, st);
        q = timed ? timer_pair(h, FLIP_KERNEL_MG_UP_FINE, k) : -1;
        launch_mg_fine<V>(true, h->groups, h->na, h->geo, h->tile_list, h->tile_nbr, h->diag, rvec(k), h->mg[0],
                          zvec(k), h->pslots, h->ps, st, q >= 0 ? h->ev[q] : nullptr,
                          q >= 0 ? h->ev[q + 1] : nullptr);
    };
    precondition(0, true);
    direction(0);
    for (;;) {
        for (int it = 0; it < chunk; ++it) {
            const int k = launched + it;
            const int sc = h->scur;
            const int q = (k % TIMED_PCG_EVERY) == 0 ? timer_pair(h, FLIP_KERNEL_PCG_UPDATE, k) : -1;
            if (fused)
                launch_pcg_update_down<V>(h->groups, h->na, h->geo, h->tile_list, h->tile_nbr, h->diag,
                                          (const V*)h->s[sc ^ 1], (const V*)h->q, x, rvec(k), rvec(k + 1),
                                          h->mg[0], h->pslots, h->ps, st, q >= 0 ? h->ev[q] : nullptr,
                                          q >= 0 ? h->ev[q + 1] : nullptr);
            else
                launch_pcg_update<V>(h->groups, h->na, h->tile_nbr, h->diag, (const V*)h->s[sc ^ 1], x, (V*)h->z,
                                     h->pslots, h->ps, mg, st, q >= 0 ? h->ev[q] : nullptr,
                                     q >= 0 ? h->ev[q + 1] : nullptr);
            h->scur = sc ^ 1;
            precondition(k + 1, !fused);
            direction(k + 1);
        }
        launched += chunk;
        HIP_TRY(hipMemcpyAsync(h->h_ps, h->ps, sizeof(PcgState), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (h->h_ps->done != PCG_RUNNING || launched > max_iters + 8) break;
        chunk = next_chunk;
    }
    *out = *h->h_ps;
    h->prev_iters = out->iter;
    // timed launches at or past the final iteration found the solve over and did no work
    for (int q = first_sample; q < h->ev_used / 2; ++q)
        if (h->ev_iter[q] >= out->iter) h->ev_kind[q] = -1;
    return FLIP_OK;
}

// Red-black Gauss-Seidel solve (FLIP_FLAG_RED_BLACK_GS, Sec. 3.2.3) from the
// state the right-hand-side kernel left (p = 0, max |b|, tolerance): chunks of
// GS_CHECK_EVERY iterations, each followed by the residual max |b - A p| over
// the fluid cells, until it meets the tolerance or the cap.
constexpr int GS_CHECK_EVERY = 32;

int gs_iter_cap(const flip_config& c)
{
    const int64_t n = std::max(c.nx, std::max(c.ny, c.nz));
    return c.pcg_max_iters > 0 ? c.pcg_max_iters : (int)std::min<int64_t>(50 * n * n, 1 << 30);
}

template <typename V>
flip_status gs_loop(flip_handle* h, V* p, int max_iters, hipStream_t st, PcgState* state)
{
    unsigned long long* rmax = h->gs_rmax;
    const double target = state->tol * state->max_b;
    int iters = 0;
    double max_r = 0.0;
    for (;;) {
        const int chunk = std::min(GS_CHECK_EVERY, max_iters - iters);
        launch_gs_sweeps<V>(h->na, chunk, h->tile_nbr, h->diag, (const V*)h->b, p, st);
        launch_gs_residual<V>(h->na, h->tile_nbr, h->diag, (const V*)h->b, p, rmax, st);
        iters += chunk;
        HIP_TRY(hipMemcpyAsync(&h->h_ps->max_r, rmax, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        max_r = h->h_ps->max_r;
        if (!(max_r <= DBL_MAX)) {
            state->done = PCG_BREAKDOWN;
            break;
        }
        if (max_r <= target) {
            state->done = PCG_CONVERGED;
            break;
        }
        if (iters >= max_iters) {
            state->done = PCG_MAX_ITERS;
            break;
        }
    }
    state->iter = iters;
    state->max_r = max_r;
    return FLIP_OK;
}

// binning of the particles' current positions alone (keys, counts, starts,
// the stable sort): the space hash for work outside a step
template <typename T>
void rebin(flip_handle* h, hipStream_t st)
{
    const Geo& g = h->geo;
    const Sizes& s = h->sz;
    const int64_t n = s.n;
    const int nxt = h->cur ^ 1;
    h->keys_ready = false;  // the sort moves the particles
    launch_fill_u32(h->count, s.C, 0u, st);
    launch_bin_keys<T>(g, (const T*)h->pos[h->cur], n, h->key, h->rank, h->count, st);
    launch_exclusive_scan_u32(h->count, h->start, s.C, h->scan_tmp, st);
    launch_bin_scatter(h->key, h->rank, h->start, n, h->perm, st);
    launch_bin_gather<T>(h->perm, h->key, h->start, h->count, n, (const T*)h->pos[h->cur],
                         (const T*)h->vel[h->cur], h->id[h->cur], (T*)h->pos[nxt], (T*)h->vel[nxt], h->id[nxt],
                         st);
    h->cur = nxt;
}

template <typename T, bool MIXED>
flip_status run_step(flip_handle* h, hipStream_t st)
{
    const Geo& g = h->geo;
    const Sizes& s = h->sz;
    int64_t n = s.n;
    const int nxt = h->cur ^ 1;
    const flip_config& c = h->cfg;

    // 0. the step's dt: fixed, or the CFL rule of Sec. 3.1.4 on the particles'
    // speeds at the step's start
    double dt = c.dt;
    if (c.flags & FLIP_FLAG_ADAPTIVE_DT) {
        launch_max_speed2<T>((const T*)h->vel[h->cur], n, h->gs_rmax, st);
        HIP_TRY(hipMemcpyAsync(&h->h_ps->max_r, h->gs_rmax, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const double umax = std::sqrt(h->h_ps->max_r);
        if (umax > 0.0) dt = std::min(c.dt, c.cfl * c.dx / umax);
    }
    h->stats.dt = dt;

    // 1. binning
    int tq = timer_begin(h, FLIP_KERNEL_BIN_KEYS, st);
    if (h->keys_ready) {
        // the previous step's grid-to-particle binned the positions it wrote
        // (keys, provisional ranks, counts and tile flags)
        HIP_TRY(hipMemcpyAsync(h->count, h->count_next, 4 * s.C, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(h->tile_flag, h->tile_next, 4 * s.T, hipMemcpyDeviceToDevice, st));
    } else {
        launch_fill_u32(h->count, s.C, 0u, st);
        launch_fill_u32(h->tile_flag, s.T, 0u, st);
        launch_bin_keys<T>(g, (const T*)h->pos[h->cur], n, h->key, h->rank, h->count, st, h->tile_flag);
    }
    h->keys_ready = false;
    timer_end(h, tq, st);
    tq = timer_begin(h, FLIP_KERNEL_BIN_SCAN, st);
    launch_exclusive_scan_u32(h->count, h->start, s.C, h->scan_tmp, st);
    timer_end(h, tq, st);
    tq = timer_begin(h, FLIP_KERNEL_BIN_SCATTER, st);
    launch_bin_scatter(h->key, h->rank, h->start, n, h->perm, st);
    timer_end(h, tq, st);
    h->stats.n_reseeded = 0;
    if (c.flags & FLIP_FLAG_RESEED) {
        // Sec. 3.1.2: refill sparse fluid cells. The new total sets the
        // particle arrays' stride, so it is read back before the move.
        uint32_t* add = (uint32_t*)h->staging;
        uint32_t* off = add + s.C;
        const int sub = c.subcells_per_axis;
        tq = timer_begin(h, FLIP_KERNEL_BIN_GATHER, st);
        launch_reseed_plan(h->count, s.C, (uint32_t)(sub * sub * sub), add, st);
        launch_exclusive_scan_u32(add, off, s.C, h->scan_tmp, st);
        launch_reseed_total(add, off, s.C, h->d_reseeded, st);
        HIP_TRY(hipMemcpyAsync(h->h_words, h->d_reseeded, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const int64_t added = h->h_words[0];
        if (n + added > s.pcap) {  // nothing moved yet
            timer_end(h, tq, st);
            (void)timer_collect(h, st);
            return FLIP_E_WORKSPACE;
        }
        launch_reseed_move<T>(g, sub, c.seed, (uint64_t)h->stats.steps, h->perm, h->key, h->start, h->count,
                              add, off, n, n + added, (const T*)h->pos[h->cur], (const T*)h->vel[h->cur],
                              h->id[h->cur], (T*)h->pos[nxt], (T*)h->vel[nxt], h->id[nxt], st);
        timer_end(h, tq, st);
        n += added;
        h->sz.n = n;
        h->stats.n_particles = n;
        h->stats.n_reseeded = added;
    } else {
        tq = timer_begin(h, FLIP_KERNEL_BIN_GATHER, st);
        launch_bin_gather<T>(h->perm, h->key, h->start, h->count, n, (const T*)h->pos[h->cur],
                             (const T*)h->vel[h->cur], h->id[h->cur], (T*)h->pos[nxt], (T*)h->vel[nxt],
                             h->id[nxt], st);
        timer_end(h, tq, st);
    }
    h->cur = nxt;
    tq = timer_begin(h, FLIP_KERNEL_TILES, st);
    launch_tiles(g, h->count, h->tile_flag, h->tile_excl, h->tile_slot, h->tile_list, h->tile_nbr,
                 h->d_nactive, h->scan_tmp, st, true);
    timer_end(h, tq, st);

    // 2. particle-to-grid, gravity, walls
    const T* pos = (const T*)h->pos[h->cur];
    const T* vel = (const T*)h->vel[h->cur];
    const bool grav = !(c.flags & FLIP_FLAG_NO_GRAVITY);
    {
        const T gdt[3] = {(T)(grav ? c.gravity[0] * dt : 0.0), (T)(grav ? c.gravity[1] * dt : 0.0),
                          (T)(grav ? c.gravity[2] * dt : 0.0)};
        T* const old[3] = {(T*)h->f_old[0], (T*)h->f_old[1], (T*)h->f_old[2]};
        T* const star[3] = {(T*)h->f_star[0], (T*)h->f_star[1], (T*)h->f_star[2]};
        tq = timer_begin(h, FLIP_KERNEL_P2G, st);
        launch_p2g<T>(g, pos, vel, n, h->start, h->count, h->tile_flag, gdt, old, star, st);
        timer_end(h, tq, st);
    }

    // 3. right-hand side and solver start
    PcgState ps_host{};
    flip_status ret = FLIP_OK;
    const bool project = !(c.flags & FLIP_FLAG_NO_PROJECTION);
    const int max_iters = solve_iter_cap(c);
    const double scale_b = -c.density * c.dx / dt;
    h->scur = 0;
    h->xi = 0;
    // the solver kernels read the active-tile count from device memory: no
    // host round trip between binning and the solve
    const int G = h->groups;
    tq = timer_begin(h, FLIP_KERNEL_RHS, st);
    if (MIXED)
        launch_rhs_mixed(g, G, h->tile_list, h->d_nactive, h->count, (const float*)h->f_star[0],
                         (const float*)h->f_star[1], (const float*)h->f_star[2], scale_b, h->diag,
                         h->b64, h->x64[0], (float*)h->z, (float*)h->xin[0], (float*)h->s[0],
                         (float*)h->s[1], h->partials, G, h->ps, project ? c.pcg_tol : 0.0,
                         project ? max_iters : 0, c.ir_tol, MAX_REFINEMENTS, h->nmg > 0 ? 1 : 0, st);
    else
        launch_rhs<T, T>(g, G, h->tile_list, h->d_nactive, h->count, (const T*)h->f_star[0],
                         (const T*)h->f_star[1], (const T*)h->f_star[2], scale_b, h->diag, (T*)h->b,
                         (T*)h->z, (T*)h->xin[0], (T*)h->s[0], (T*)h->s[1], h->partials, G, h->ps,
                         project ? c.pcg_tol : 0.0, project ? max_iters : 0, h->nmg > 0 ? 1 : 0, st);
    timer_end(h, tq, st);
    // cell types of the multigrid levels, from this step's fluid cells, and
    // the blocks of each level that hold a fluid cell
    if (h->nmg > 0 && project) {
        launch_fill_bytes_zero(h->mg_zero, (int64_t)h->mg_zero_bytes, st);
        launch_mg_types_fine(g, h->tile_slot, h->diag, h->mg[0], st);
        for (int l = 0; l + 1 < h->nmg; ++l) launch_mg_types(h->mg[l], h->mg[l + 1], st);
        HIP_TRY(hipMemcpyAsync(h->h_mgcnt, h->mg_cnt, 4 * 2 * h->nmg, hipMemcpyDeviceToHost, st));
    }

    // 4. PCG (FP32 inner solves inside FP64 refinement when MIXED). One read
    // of the solver state after its start gives the active-tile count (the
    // iteration kernels then issue their first loads without waiting for the
    // state) and skips the loop when the start already decided the solve.
    HIP_TRY(hipMemcpyAsync(h->h_ps, h->ps, sizeof(PcgState), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&h->h_diag->nonfinite, &h->diagw->nonfinite, sizeof(uint32_t), hipMemcpyDeviceToHost,
                           st));
    HIP_TRY(hipStreamSynchronize(st));
    ps_host = *h->h_ps;
    h->na = ps_host.n_active;
    if (h->nmg > 0 && project)
        for (int l = 0; l < h->nmg; ++l) {
            h->mg[l].nd = (int)h->h_mgcnt[2 * l];
            h->mg[l].nu = (int)h->h_mgcnt[2 * l + 1];
        }
    // particle state that an earlier step's grid-to-particle left non-finite
    const bool nonfinite_before = h->h_diag->nonfinite != 0;
    int iters = 0, refinements = 0;
    const bool gs = (c.flags & FLIP_FLAG_RED_BLACK_GS) != 0;
    if (project && gs) {
        if (ps_host.done == PCG_RUNNING) {
            flip_status r = gs_loop<T>(h, (T*)h->xin[0], gs_iter_cap(c), st, &ps_host);
            if (r != FLIP_OK) return r;
            iters = ps_host.iter;
        }
    }
    if (project) {
        while (!gs && ps_host.done == PCG_RUNNING) {
            flip_status r = pcg_loop<T>(h, (T*)h->xin[h->xi], max_iters, st, &ps_host);
            if (r != FLIP_OK) return r;
            iters += ps_host.iter;
            if (!MIXED || ps_host.done == PCG_BREAKDOWN || ps_host.outer_done != 0) break;
            const int xi = h->xi;
            launch_ir_update(G, h->tile_nbr, h->diag, h->b64, h->x64[xi], h->x64[xi ^ 1],
                             (const float*)h->xin[xi], (float*)h->xin[xi ^ 1], (float*)h->z,
                             (float*)h->s[0], (float*)h->s[1], h->partials, G, h->ps, h->nmg > 0 ? 1 : 0, st);
            h->xi = xi ^ 1;
            h->scur = 0;
            ++refinements;
            HIP_TRY(hipMemcpyAsync(h->h_ps, h->ps, sizeof(PcgState), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            ps_host = *h->h_ps;
            if (ps_host.outer_done != 0) break;
        }
        if (MIXED) {
            if (ps_host.outer_done != 1) ret = (ps_host.done == PCG_BREAKDOWN)
                                                  ? (ps_host.sync_error ? FLIP_E_HIP : FLIP_E_NONFINITE)
                                                  : FLIP_E_NOT_CONVERGED;
        } else {
            if (ps_host.done == PCG_MAX_ITERS || ps_host.done == PCG_RUNNING) ret = FLIP_E_NOT_CONVERGED;
            if (ps_host.done == PCG_BREAKDOWN) ret = ps_host.sync_error ? FLIP_E_HIP : FLIP_E_NONFINITE;
        }
        // 5. projection with the solution (FP64 when MIXED)
        const T scale = (T)(dt / (c.density * c.dx));
        T* const star[3] = {(T*)h->f_star[0], (T*)h->f_star[1], (T*)h->f_star[2]};
        T* const fnew[3] = {(T*)h->f_new[0], (T*)h->f_new[1], (T*)h->f_new[2]};
        tq = timer_begin(h, FLIP_KERNEL_PROJECT, st);
        if (MIXED)
            launch_project3<float, double>(g, h->diag, h->tile_slot, h->x64[h->xi], (float* const*)star,
                                           (float* const*)fnew, dt / (c.density * c.dx), st);
        else
            launch_project3<T, T>(g, h->diag, h->tile_slot, (const T*)h->xin[h->xi], star, fnew, scale, st);
        timer_end(h, tq, st);
    } else {
        for (int a = 0; a < 3; ++a)
            HIP_TRY(hipMemcpyAsync(h->f_new[a], h->f_star[a], s.F[a] * sizeof(T),
                                   hipMemcpyDeviceToDevice, st));
    }

    // 6. grid-to-particle, blend, advect, clamp; it also bins the positions
    // it writes for the next step (keys, provisional ranks, counts, tile flags)
    tq = timer_begin(h, FLIP_KERNEL_G2P, st);
    launch_fill_u32(h->count_next, s.C, 0u, st);
    launch_fill_u32(h->tile_next, s.T, 0u, st);
    launch_g2p<T>(g, n, h->start, h->count, (T*)h->pos[h->cur], (T*)h->vel[h->cur], (const T*)h->f_new[0],
                  (const T*)h->f_new[1], (const T*)h->f_new[2], (const T*)h->f_old[0],
                  (const T*)h->f_old[1], (const T*)h->f_old[2], (T)c.flip_ratio, (T)dt,
                  (c.flags & FLIP_FLAG_ADVECT_PARTICLE_VEL) ? 1 : 0, &h->diagw->nonfinite, st,
                  h->key, h->rank, h->count_next, h->tile_next);
    timer_end(h, tq, st);

    // 7. diagnostics, in FP64: the solve's true residual, the divergence the
    // projection left, the particles' energy and largest speed
    if (c.flags & FLIP_FLAG_DIAGNOSTICS) {
        DiagWords* dw = h->diagw;
        if (project && ps_host.n_active > 0) {
            if (MIXED)
                launch_gs_residual<double>(ps_host.n_active, h->tile_nbr, h->diag, h->b64, h->x64[h->xi], &dw->rmax,
                                           st);
            else
                launch_gs_residual<T>(ps_host.n_active, h->tile_nbr, h->diag, (const T*)h->b,
                                      (const T*)h->xin[h->xi], &dw->rmax, st);
        } else {
            launch_fill_u64((uint64_t*)&dw->rmax, 1, 0ull, st);
        }
        const T* fn[3] = {(const T*)h->f_new[0], (const T*)h->f_new[1], (const T*)h->f_new[2]};
        const T* fs[3] = {(const T*)h->f_star[0], (const T*)h->f_star[1], (const T*)h->f_star[2]};
        launch_div_max<T>(g, h->count, fn, fs, nullptr, dw->div_max, st);
        launch_particle_energy<T>((const T*)h->vel[h->cur], n, h->diag_part, &dw->energy, &dw->speed2, st);
        h->diag_dt = dt;
        h->diag_valid = true;
    }
    if (hipGetLastError() != hipSuccess) return FLIP_E_HIP;
    h->keys_ready = true;

    if (nonfinite_before && ret == FLIP_OK) ret = FLIP_E_NONFINITE;
    const bool solved = ps_host.n_active > 0 && project;
    const int status = MIXED ? (ps_host.outer_done == 1 ? 0 : (ps_host.done == PCG_BREAKDOWN ? 2 : 1))
                             : (ps_host.done == PCG_CONVERGED ? 0 : (ps_host.done == PCG_BREAKDOWN ? 2 : 1));
    record_step(h, solved, status, ps_host.n_active, ps_host.nfluid, MIXED ? ps_host.max_b0 : ps_host.max_b,
                MIXED ? ps_host.max_r64 : ps_host.max_r, iters, refinements, ret);
    flip_status tr = timer_collect(h, st);
    return ret != FLIP_OK ? ret : tr;
}

}  // namespace

namespace flipmi {

int solve_iter_cap(const flip_config& c)
{
    return c.pcg_max_iters > 0 ? c.pcg_max_iters : 20 * std::max(c.nx, std::max(c.ny, c.nz));
}

void record_step(flip_handle* h, bool solved, int status, int n_active, int nfluid, double max_b,
                 double max_r, int iters, int refinements, flip_status ret)
{
    flip_step_stats& S = h->stats;
    S.steps += 1;
    S.n_fluid_cells = nfluid;
    S.n_active_tiles = n_active;
    S.pcg_iterations = iters;
    S.refinements = refinements;
    S.pcg_status = solved ? status : 0;
    S.max_b = max_b;
    S.max_r = max_r;
    S.pcg_iterations_total += iters;
    S.pcg_cell_iterations_total += (int64_t)iters * nfluid;
    if (ret != FLIP_OK && S.latched_status == 0) S.latched_status = ret;
}

}  // namespace flipmi

extern "C" {

const char* flip_status_string(flip_status s)
{
    switch (s) {
        case FLIP_OK: return "ok";
        case FLIP_E_INVALID: return "invalid argument";
        case FLIP_E_WORKSPACE: return "workspace missing, too small or misaligned";
        case FLIP_E_HIP: return "HIP runtime error";
        case FLIP_E_NOT_CONVERGED: return "PCG did not converge within pcg_max_iters";
        case FLIP_E_NONFINITE: return "non-finite values (solver breakdown or non-finite particle state)";
        case FLIP_E_STATE: return "invalid state";
    }
    return "unknown status";
}

flip_status flip_workspace_bytes(const flip_config* cfg, size_t* out_bytes)
{
    if (!out_bytes) return FLIP_E_INVALID;
    flip_status v = validate(cfg);
    if (v != FLIP_OK) return v;
    int64_t n = 0;
    v = particle_count(cfg, &n);
    if (v != FLIP_OK) return v;
    flip_handle tmp;
    tmp.cfg = *cfg;
    tmp.prec = cfg->precision;
    tmp.sz = make_sizes(cfg, n);
    Carver cv(nullptr);
    carve(&tmp, cv);
    *out_bytes = cv.off;
    return FLIP_OK;
}

flip_status flip_init(const flip_config* cfg, void* d_ws, size_t ws_bytes, void* hip_stream,
                      flip_handle** out)
{
    if (!out) return FLIP_E_INVALID;
    *out = nullptr;
    flip_status v = validate(cfg);
    if (v != FLIP_OK) return v;
    int64_t n = 0;
    v = particle_count(cfg, &n);
    if (v != FLIP_OK) return v;
    const double L[3] = {cfg->nx * cfg->dx, cfg->ny * cfg->dx, cfg->nz * cfg->dx};
    if (cfg->pos0) {
        for (int a = 0; a < 3; ++a)
            for (int64_t p = 0; p < n; ++p) {
                const double q = cfg->pos0[a * n + p], w = cfg->vel0[a * n + p];
                if (!(q >= 0.0 && q <= L[a]) || !std::isfinite(w)) return FLIP_E_INVALID;
            }
    }
    flip_handle* h = new (std::nothrow) flip_handle();
    if (!h) return FLIP_E_INVALID;
    h->cfg = *cfg;
    h->prec = cfg->precision;
    h->geo = make_geo(cfg);
    h->sz = make_sizes(cfg, n);
    h->groups = solver_groups(h->sz.T);
    Carver dry(nullptr);
    carve(h, dry);
    if (!d_ws || ws_bytes < dry.off || ((uintptr_t)d_ws & (ALIGN - 1))) {
        delete h;
        return FLIP_E_WORKSPACE;
    }
    // set-up of the no-allocation entry points' device scratch on this device
    if (hipGetDevice(&h->device) != hipSuccess || scratch_setup(h->device) != FLIP_OK) {
        delete h;
        return FLIP_E_HIP;
    }
    Carver cv(d_ws);
    carve(h, cv);
    hipStream_t st = (hipStream_t)hip_stream;
    h->last_stream = st;

    // particles on the host, then one upload
    const size_t rb = h->sz.rb;
    std::vector<uint32_t> ids((size_t)n);
    for (int64_t p = 0; p < n; ++p) ids[p] = (uint32_t)p;
    flip_status rc = FLIP_OK;
    auto upload = [&](auto tag) -> flip_status {
        using T = decltype(tag);
        std::vector<T> pos((size_t)(3 * n)), vel((size_t)(3 * n));
        if (cfg->pos0) {
            for (int64_t q = 0; q < 3 * n; ++q) {
                pos[q] = (T)cfg->pos0[q];
                vel[q] = (T)cfg->vel0[q];
            }
        } else {
            seed_particles<T>(*cfg, pos, vel, n);
        }
        if (n > 0) {
            HIP_TRY(hipMemcpyAsync(h->pos[0], pos.data(), 3 * n * rb, hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(h->vel[0], vel.data(), 3 * n * rb, hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(h->id[0], ids.data(), 4 * n, hipMemcpyHostToDevice, st));
        }
        HIP_TRY(hipStreamSynchronize(st));
        return FLIP_OK;
    };
    rc = (h->prec == FLIP_FP64) ? upload(double{}) : upload(float{});
    if (rc != FLIP_OK) {
        delete h;
        return rc;
    }
    h->cfg.regions = nullptr;
    h->cfg.n_regions = 0;
    h->cfg.pos0 = nullptr;
    h->cfg.vel0 = nullptr;

    // grid state readable before the first step
    const Sizes& s = h->sz;
    launch_fill_u32(h->count, s.C, 0u, st);
    launch_fill_u32(h->start, s.C, 0u, st);
    launch_fill_u32((uint32_t*)h->tile_slot, s.T, 0xFFFFFFFFu, st);
    for (int a = 0; a < 3; ++a) {
        launch_fill_bytes_zero(h->f_old[a], s.F[a] * rb, st);
        launch_fill_bytes_zero(h->f_star[a], s.F[a] * rb, st);
        launch_fill_bytes_zero(h->f_new[a], s.F[a] * rb, st);
    }
    launch_fill_bytes_zero(h->diag, s.cap, st);
    launch_fill_bytes_zero(h->ps, PCG_STATE_BYTES + SYNC_BYTES, st);
    launch_fill_bytes_zero(h->diagw, sizeof(DiagWords), st);
    launch_fill_u64((uint64_t*)h->partials, 3 * h->groups, SLOT_EMPTY_BITS, st);
    if (hipHostMalloc((void**)&h->h_ps, sizeof(PcgState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h->h_words, 2 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h->h_mgcnt, 4 * 2 * MG_MAX_LEVELS, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h->h_diag, sizeof(DiagWords), hipHostMallocDefault) != hipSuccess) {
        flip_destroy(h);
        return FLIP_E_HIP;
    }
    if (cfg->flags & FLIP_FLAG_KERNEL_TIMING) {
        h->ev.resize(2 * EVENT_PAIRS);
        h->ev_kind.resize(EVENT_PAIRS);
        h->ev_iter.resize(EVENT_PAIRS);
        for (auto& e : h->ev)
            if (hipEventCreate(&e) != hipSuccess) {
                flip_destroy(h);
                return FLIP_E_HIP;
            }
    }
    if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) {
        flip_destroy(h);
        return FLIP_E_HIP;
    }
    h->stats.n_particles = n;
    *out = h;
    return FLIP_OK;
}

flip_status flip_step(flip_handle* h, int nsteps, void* hip_stream)
{
    if (!h || nsteps < 0) return FLIP_E_INVALID;
    hipStream_t st = (hipStream_t)hip_stream;
    h->last_stream = st;
    flip_status first = FLIP_OK;
    for (int k = 0; k < nsteps; ++k) {
        flip_status r = (h->prec == FLIP_FP64)     ? run_step<double, false>(h, st)
                        : (h->prec == FLIP_MIXED) ? run_step<float, true>(h, st)
                                                  : run_step<float, false>(h, st);
        if (r == FLIP_E_HIP) return r;
        if (r != FLIP_OK && first == FLIP_OK) first = r;
    }
    return first;
}

flip_status flip_field_bytes(const flip_handle* h, int field, size_t* out_bytes)
{
    if (!h || !out_bytes) return FLIP_E_INVALID;
    const Sizes& s = h->sz;
    switch (field) {
        case FLIP_FIELD_POS:
        case FLIP_FIELD_VEL: *out_bytes = 3 * s.n * s.rb; break;
        case FLIP_FIELD_ID: *out_bytes = 4 * s.n; break;
        case FLIP_FIELD_CELL_COUNT:
        case FLIP_FIELD_CELL_START: *out_bytes = 4 * s.C; break;
        case FLIP_FIELD_FLAGS: *out_bytes = s.C; break;
        case FLIP_FIELD_U_OLD:
        case FLIP_FIELD_U_STAR:
        case FLIP_FIELD_U_NEW: *out_bytes = (s.F[0] + s.F[1] + s.F[2]) * s.rb; break;
        case FLIP_FIELD_RHS:
        case FLIP_FIELD_PRESSURE: *out_bytes = s.C * (h->prec == FLIP_MIXED ? 8 : s.rb); break;
        case FLIP_FIELD_DIV: *out_bytes = s.C * 8; break;
        default: return FLIP_E_INVALID;
    }
    return FLIP_OK;
}

flip_status flip_readback(flip_handle* h, int field, void* dst, size_t dst_bytes, int dst_is_device,
                          void* hip_stream)
{
    if (!h || !dst) return FLIP_E_INVALID;
    size_t need = 0;
    flip_status v = flip_field_bytes(h, field, &need);
    if (v != FLIP_OK) return v;
    if (dst_bytes < need) return FLIP_E_INVALID;
    hipStream_t st = (hipStream_t)hip_stream;
    const hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const Sizes& s = h->sz;
    char* d = (char*)dst;
    switch (field) {
        case FLIP_FIELD_POS: HIP_TRY(hipMemcpyAsync(d, h->pos[h->cur], need, kind, st)); break;
        case FLIP_FIELD_VEL: HIP_TRY(hipMemcpyAsync(d, h->vel[h->cur], need, kind, st)); break;
        case FLIP_FIELD_ID: HIP_TRY(hipMemcpyAsync(d, h->id[h->cur], need, kind, st)); break;
        case FLIP_FIELD_CELL_COUNT: HIP_TRY(hipMemcpyAsync(d, h->count, need, kind, st)); break;
        case FLIP_FIELD_CELL_START: HIP_TRY(hipMemcpyAsync(d, h->start, need, kind, st)); break;
        case FLIP_FIELD_FLAGS:
            launch_flags_from_count(h->count, s.C, (uint8_t*)h->staging, st);
            HIP_TRY(hipMemcpyAsync(d, h->staging, need, kind, st));
            break;
        case FLIP_FIELD_U_OLD:
        case FLIP_FIELD_U_STAR:
        case FLIP_FIELD_U_NEW: {
            void* const* f = field == FLIP_FIELD_U_OLD ? h->f_old : (field == FLIP_FIELD_U_STAR ? h->f_star : h->f_new);
            size_t off = 0;
            for (int a = 0; a < 3; ++a) {
                HIP_TRY(hipMemcpyAsync(d + off, f[a], s.F[a] * s.rb, kind, st));
                off += s.F[a] * s.rb;
            }
            break;
        }
        case FLIP_FIELD_RHS:
        case FLIP_FIELD_PRESSURE: {
            const void* src = field == FLIP_FIELD_RHS ? h->b : h->xin[h->xi];
            if (h->prec == FLIP_MIXED)
                launch_densify<double, double>(h->geo, h->tile_slot, h->diag,
                                               field == FLIP_FIELD_RHS ? h->b64 : h->x64[h->xi],
                                               (double*)h->staging, st);
            else if (h->prec == FLIP_FP64)
                launch_densify<double, double>(h->geo, h->tile_slot, h->diag, (const double*)src,
                                               (double*)h->staging, st);
            else
                launch_densify<float, float>(h->geo, h->tile_slot, h->diag, (const float*)src,
                                             (float*)h->staging, st);
            HIP_TRY(hipMemcpyAsync(d, h->staging, need, kind, st));
            break;
        }
        case FLIP_FIELD_DIV: {
            if (h->prec == FLIP_FP64) {
                const double* fn[3] = {(const double*)h->f_new[0], (const double*)h->f_new[1],
                                       (const double*)h->f_new[2]};
                launch_div_max<double>(h->geo, h->count, fn, fn, (double*)h->staging, nullptr, st);
            } else {
                const float* fn[3] = {(const float*)h->f_new[0], (const float*)h->f_new[1],
                                      (const float*)h->f_new[2]};
                launch_div_max<float>(h->geo, h->count, fn, fn, (double*)h->staging, nullptr, st);
            }
            HIP_TRY(hipMemcpyAsync(d, h->staging, need, kind, st));
            break;
        }
        default: return FLIP_E_INVALID;
    }
    if (hipGetLastError() != hipSuccess) return FLIP_E_HIP;
    if (!dst_is_device) HIP_TRY(hipStreamSynchronize(st));
    return FLIP_OK;
}

flip_status flip_surface_field_bytes(const flip_handle* h, int refine, size_t* out_bytes)
{
    if (!h || !out_bytes || refine < 1 || refine > 16) return FLIP_E_INVALID;
    const flip_config& c = h->cfg;
    *out_bytes = (size_t)(c.nx * refine + 1) * (c.ny * refine + 1) * (c.nz * refine + 1) * h->sz.rb;
    return FLIP_OK;
}

flip_status flip_surface_field(flip_handle* h, double radius, double search_radius, int refine, void* d_phi,
                               size_t phi_bytes, void* hip_stream)
{
    if (!h || !d_phi) return FLIP_E_INVALID;
    if (!(radius > 0.0) || !std::isfinite(radius) || !(search_radius > 0.0) || !std::isfinite(search_radius))
        return FLIP_E_INVALID;
    size_t need = 0;
    flip_status v = flip_surface_field_bytes(h, refine, &need);
    if (v != FLIP_OK) return v;
    if (phi_bytes < need) return FLIP_E_INVALID;
    hipStream_t st = (hipStream_t)hip_stream;
    h->last_stream = st;
    if (h->prec == FLIP_FP64) {
        rebin<double>(h, st);
        launch_surface_field<double>(h->geo, refine, radius, search_radius, h->start, h->count,
                                     (const double*)h->pos[h->cur], h->sz.n, (double*)d_phi, st);
    } else {
        rebin<float>(h, st);
        launch_surface_field<float>(h->geo, refine, radius, search_radius, h->start, h->count,
                                    (const float*)h->pos[h->cur], h->sz.n, (float*)d_phi, st);
    }
    if (hipGetLastError() != hipSuccess) return FLIP_E_HIP;
    return FLIP_OK;
}

namespace {

// the mesh scratch of a sampling grid, carved from the caller's workspace
size_t mc_carve(const flip_config& c, int refine, void* base, McTable** tab, McWork* w)
{
    const int64_t nc = (int64_t)(c.nx * refine + 1) * (c.ny * refine + 1) * (c.nz * refine + 1);
    const int64_t ncube = (int64_t)(c.nx * refine) * (c.ny * refine) * (c.nz * refine);
    Carver cv(base);
    *tab = cv.take<McTable>(sizeof(McTable));
    w->flag = cv.take<uint32_t>(4 * 3 * nc);
    w->vidx = cv.take<uint32_t>(4 * 3 * nc);
    w->cnt = cv.take<uint32_t>(4 * ncube);
    w->toff = cv.take<uint32_t>(4 * ncube);
    w->scan_tmp = cv.take<uint32_t>(4 * scan_tmp_words(std::max<int64_t>(3 * nc, ncube)));
    w->totals = cv.take<uint32_t>(8);
    return cv.off;
}

}  // namespace

flip_status flip_surface_mesh_workspace_bytes(const flip_handle* h, int refine, size_t* out_bytes)
{
    if (!h || !out_bytes || refine < 1 || refine > 16) return FLIP_E_INVALID;
    const flip_config& c = h->cfg;
    if ((int64_t)(c.nx * refine + 1) * (c.ny * refine + 1) * (c.nz * refine + 1) * 3 >= ((int64_t)1 << 31))
        return FLIP_E_INVALID;
    McTable* tab;
    McWork w;
    *out_bytes = mc_carve(c, refine, nullptr, &tab, &w);
    return FLIP_OK;
}

namespace {

// marching cubes with its scratch at d_work (checked by the caller)
flip_status mesh_body(flip_handle* h, const void* d_phi, int refine, void* d_work, void* d_vertices,
                      void* d_normals, int64_t max_vertices, int32_t* d_triangles, int64_t max_triangles,
                      int64_t* n_vertices, int64_t* n_triangles, void* hip_stream)
{
    const bool count_only = !d_vertices && !d_normals && !d_triangles;
    if (!count_only && (!d_vertices || !d_normals || !d_triangles)) return FLIP_E_INVALID;
    hipStream_t st = (hipStream_t)hip_stream;
    h->last_stream = st;
    McTable* tab;
    McWork w;
    mc_carve(h->cfg, refine, d_work, &tab, &w);
    const flip_config& c = h->cfg;
    const int cx = c.nx * refine + 1, cy = c.ny * refine + 1, cz = c.nz * refine + 1;
    HIP_TRY(hipMemcpyAsync(tab, &mc_table(), sizeof(McTable), hipMemcpyHostToDevice, st));
    const bool fp64 = h->prec == FLIP_FP64;
    if (fp64) launch_mc_count<double>((const double*)d_phi, cx, cy, cz, tab, w, st);
    else launch_mc_count<float>((const float*)d_phi, cx, cy, cz, tab, w, st);
    HIP_TRY(hipMemcpyAsync(h->h_words, w.totals, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hipGetLastError() != hipSuccess) return FLIP_E_HIP;
    const int64_t nv = h->h_words[0], nt = h->h_words[1];
    *n_vertices = nv;
    *n_triangles = nt;
    if (count_only) return FLIP_OK;
    if (nv > max_vertices || nt > max_triangles) return FLIP_E_WORKSPACE;
    const double hs = c.dx / refine;
    if (fp64)
        launch_mc_emit<double>((const double*)d_phi, cx, cy, cz, hs, tab, w, nv, nt, (double*)d_vertices,
                               (double*)d_normals, d_triangles, st);
    else
        launch_mc_emit<float>((const float*)d_phi, cx, cy, cz, hs, tab, w, nv, nt, (float*)d_vertices,
                              (float*)d_normals, d_triangles, st);
    if (hipGetLastError() != hipSuccess) return FLIP_E_HIP;
    return FLIP_OK;
}

}  // namespace

flip_status flip_surface_mesh(flip_handle* h, const void* d_phi, int refine, void* d_work, size_t work_bytes,
                              void* d_vertices, void* d_normals, int64_t max_vertices, int32_t* d_triangles,
                              int64_t max_triangles, int64_t* n_vertices, int64_t* n_triangles, void* hip_stream)
{
    if (!h || !d_phi || !d_work || !n_vertices || !n_triangles) return FLIP_E_INVALID;
    size_t need = 0;
    flip_status v = flip_surface_mesh_workspace_bytes(h, refine, &need);
    if (v != FLIP_OK) return v;
    if (work_bytes < need || ((uintptr_t)d_work & (ALIGN - 1))) return FLIP_E_WORKSPACE;
    return mesh_body(h, d_phi, refine, d_work, d_vertices, d_normals, max_vertices, d_triangles, max_triangles,
                     n_vertices, n_triangles, hip_stream);
}

flip_status flip_surface_mesh_noalloc(flip_handle* h, const void* d_phi, int refine, void* d_vertices,
                                      void* d_normals, int64_t max_vertices, int32_t* d_triangles,
                                      int64_t max_triangles, int64_t* n_vertices, int64_t* n_triangles,
                                      void* hip_stream)
{
    if (!h || !d_phi || !n_vertices || !n_triangles) return FLIP_E_INVALID;
    size_t need = 0;
    flip_status v = flip_surface_mesh_workspace_bytes(h, refine, &need);
    if (v != FLIP_OK) return v;
    if (need > MC_SCRATCH_BYTES) return FLIP_E_WORKSPACE;
    void* work = scratch_of(h->device);
    if (!work) return FLIP_E_HIP;
    return mesh_body(h, d_phi, refine, work, d_vertices, d_normals, max_vertices, d_triangles, max_triangles,
                     n_vertices, n_triangles, hip_stream);
}

flip_status flip_stats(flip_handle* h, flip_step_stats* out)
{
    if (!h || !out) return FLIP_E_INVALID;
    hipStream_t st = h->last_stream;
    HIP_TRY(hipMemcpyAsync(h->h_diag, h->diagw, sizeof(DiagWords), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const DiagWords& d = *h->h_diag;
    flip_step_stats& S = h->stats;
    if (d.nonfinite) {
        S.nonfinite = 1;
        if (S.latched_status == 0) S.latched_status = FLIP_E_NONFINITE;
    }
    if (h->diag_valid) {
        const double rmax = __builtin_bit_cast(double, d.rmax);
        const double dn = __builtin_bit_cast(double, d.div_max[0]);
        const double ds = __builtin_bit_cast(double, d.div_max[1]);
        S.true_residual = S.max_b > 0.0 ? rmax / S.max_b : 0.0;
        S.div_ratio = ds > 0.0 ? dn / ds : 0.0;
        S.kinetic_energy = d.energy;
        S.max_speed = std::sqrt(__builtin_bit_cast(double, d.speed2));
        S.cfl_number = S.max_speed * h->diag_dt / h->cfg.dx;
    }
    *out = S;
    return FLIP_OK;
}

void flip_destroy(flip_handle* h)
{
    if (!h) return;
    if (h->last_stream) (void)hipStreamSynchronize(h->last_stream);
    for (auto& e : h->ev)
        if (e) (void)hipEventDestroy(e);
    if (h->h_ps) (void)hipHostFree(h->h_ps);
    if (h->h_words) (void)hipHostFree(h->h_words);
    if (h->h_mgcnt) (void)hipHostFree(h->h_mgcnt);
    if (h->h_diag) (void)hipHostFree(h->h_diag);
    delete h;
}

}  // extern "C"
