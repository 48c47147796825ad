// Internal declarations shared by the library's translation units (not public).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flipmi {

// PCG vectors live in 8x8x8 tiles of cells; only tiles holding a fluid cell
// are stored ("active" tiles). Inside a tile, cells are x-fastest.
constexpr int TILE = 8;
constexpr int TILE_CELLS = TILE * TILE * TILE;

// Grid geometry passed by value to every kernel.
struct Geo {
    int nx, ny, nz;     // cells per axis
    int tx, ty, tz;     // tiles per axis (ceil(n / 8))
    double dx, inv_dx;
    // 1 when dx is a power of two: then x / dx of an FP32 coordinate is exact
    // in FP32, and so is its offset from the binned cell (kernels use FP32
    // sample coordinates instead of FP64 ones, with identical results)
    int dyadic;
};

// Solver state shared between the kernels of one solve. The start kernels
// (right-hand side, refinement) complete their reductions in their last
// workgroup, which writes the state.
//
// Iteration k is a direction kernel D_k then an update kernel U_k. Each
// kernel's grid reduction is completed by the kernel after it: every
// workgroup stores its partial sums (plain stores; the kernel boundary makes
// them visible) and every workgroup of the next kernel sums all of them in
// the same fixed order, so all take the same decision. D_k completes U_{k-1}'s
// reduction (r.z, max|r|) and decides convergence; U_k completes D_k's
// (s.q). A field read inside a kernel is never written by another workgroup
// of the same kernel: D reads iter and rho_prev and writes rho, kd, max_r,
// beta (and done when the solve ends); U reads rho and kd and writes
// rho_prev, iter, alpha (and done on a breakdown).
struct PcgState {
    double rho;        // r . z of the current residual
    double alpha;      // step length of the current iteration
    double beta;       // direction update factor for the next iteration
    double max_b;      // max |b| over fluid cells (the inner solve's start)
    double max_r;      // max |r| at the last convergence test
    double tol;        // relative tolerance
    int iter;          // completed updates (written by U)
    int max_iters;
    int done;          // 0 running, 1 converged, 2 max iterations, 3 breakdown
    int nfluid;        // fluid cells of this solve
    int from_slots;    // 1: D_0 also takes r . z and max|r| from the slots (a
                       // preconditioner application ran between the start and D_0)
    int n_active;      // active tiles
    int sync_error;    // a partial result never became visible (reduction aborted)
    int pad_;
    // mixed precision: outer iterative refinement in FP64 around FP32 inner solves
    double max_b0;     // max |b| of the FP64 right-hand side
    double ir_tol;     // outer tolerance relative to max_b0
    double max_r64;    // max |b - A x| of the FP64 solution after the last refinement
    int outer;         // refinements done
    int outer_done;    // 0 running, 1 converged, 2 out of refinements
    int max_outer;
    int kd;            // iteration of the last direction kernel (written by D)
    double rho_prev;   // r . z of the iteration before (written by U)
};

enum { PCG_RUNNING = 0, PCG_CONVERGED = 1, PCG_MAX_ITERS = 2, PCG_BREAKDOWN = 3 };

// The solver state is followed in device memory by the workgroup arrival
// counters of the grid reductions (SYNC_BYTES, zero between kernels).
constexpr int PCG_STATE_BYTES = 256;
constexpr int SYNC_BYTES = 9 * 32 * 4;
static_assert(sizeof(PcgState) <= PCG_STATE_BYTES, "solver state outgrew its slot");
__host__ __device__ inline unsigned* pcg_sync(PcgState* ps)
{
    return (unsigned*)((char*)ps + PCG_STATE_BYTES);
}

// Upper bound on the workgroups of one PCG iteration kernel (4 per CU; a
// sweep over 256..16384 on the 256^3 drop scene found 1024 fastest). A build
// may set another bound with -DFLIPMI_PCG_GROUPS=n.
#ifndef FLIPMI_PCG_GROUPS
#define FLIPMI_PCG_GROUPS 1024
#endif
constexpr int PCG_MAX_GROUPS = FLIPMI_PCG_GROUPS;

// Grid tiles per solver workgroup below that bound. Only a part of a scene's
// tiles hold fluid, and every workgroup of an iteration kernel also reads the
// partial sums of all workgroups of the kernel before it, so small scenes
// (and batches of them) run with a few active tiles per workgroup rather
// than one workgroup per grid tile.
#ifndef FLIPMI_PCG_TILES_PER_GROUP
#define FLIPMI_PCG_TILES_PER_GROUP 16
#endif
constexpr int PCG_TILES_PER_GROUP = FLIPMI_PCG_TILES_PER_GROUP;

// Slots of the iteration kernels' partial sums, per solve: s.q, r.z and
// max|r|, one double per workgroup each.
constexpr int PCG_SLOT_SETS = 3;
__host__ __device__ inline double* slot_sig(double* s, int) { return s; }
__host__ __device__ inline double* slot_rho(double* s, int g) { return s + (int64_t)g; }
__host__ __device__ inline double* slot_max(double* s, int g) { return s + 2 * (int64_t)g; }

// Reduction slots hold this pattern when empty (see device_util.h).
constexpr uint64_t SLOT_EMPTY_BITS = 0x7FF4DEADBEEF0001ull;

inline int64_t tiles_of(const Geo& g) { return (int64_t)g.tx * g.ty * g.tz; }

// Elements of slack after each particle state array (x|y|z or u|v|w): the
// particle-to-grid kernel reads eight consecutive particles from any start.
constexpr int PARTICLE_PAD = 8;

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files, explicit instantiations for float
// and double). All are asynchronous on `st`.
// ---------------------------------------------------------------------------

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
void launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t st);
void launch_fill_bytes_zero(void* p, int64_t bytes, hipStream_t st);

// tile_flag (optional, cleared by the caller): set for every 8^3 tile that
// receives a particle, the flags launch_tiles would otherwise derive from count
template <typename T>
void launch_bin_keys(const Geo& g, const T* pos, int64_t n, uint32_t* key, uint32_t* rank,
                     uint32_t* count, hipStream_t st, uint32_t* tile_flag = nullptr);
// exclusive scan of n u32 values; tmp needs scan_tmp_words(n) u32 words
int64_t scan_tmp_words(int64_t n);
void launch_exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp,
                               hipStream_t st);
void launch_bin_scatter(const uint32_t* key, const uint32_t* rank, const uint32_t* start,
                        int64_t n, uint32_t* perm, hipStream_t st);
template <typename T>
void launch_bin_gather(const uint32_t* perm, const uint32_t* key, const uint32_t* start,
                       const uint32_t* count, int64_t n, const T* pos_in, const T* vel_in,
                       const uint32_t* id_in, T* pos_out, T* vel_out, uint32_t* id_out,
                       hipStream_t st);

// reseeding (Sec. 3.1.2): add[c] = new particles of cell c (target - count
// for 0 < count < target); total = off[C-1] + add[C-1] with off the exclusive
// scan of add; move = the spread gather of the binned particles into n_out
// slots, then the new particles, and count/start of the refilled cells
void launch_reseed_plan(const uint32_t* count, int64_t C, uint32_t target, uint32_t* add, hipStream_t st);
void launch_reseed_total(const uint32_t* add, const uint32_t* off, int64_t C, uint32_t* total, hipStream_t st);
template <typename T>
void launch_reseed_move(const Geo& g, int sub, uint64_t seed, uint64_t step, const uint32_t* perm,
                        const uint32_t* key, uint32_t* start, uint32_t* count, const uint32_t* add,
                        const uint32_t* off, int64_t n, int64_t n_out, const T* pos_in, const T* vel_in,
                        const uint32_t* id_in, T* pos_out, T* vel_out, uint32_t* id_out, hipStream_t st);

// surface scalar field (Sec. 3.3.1) at the (n*refine+1)^3 sampling corners,
// from binned particles
template <typename T>
void launch_surface_field(const Geo& g, int refine, double radius, double search, const uint32_t* start,
                          const uint32_t* count, const T* pos, int64_t n, T* phi, hipStream_t st);

// marching cubes (Sec. 3.3.2): the case table (triangles per configuration as
// local-edge triples) and the scratch arrays of one mesh extraction
constexpr int MC_MAX_TRI = 12;
struct McTable {
    uint8_t ntri[256];
    int8_t edge[256][3 * MC_MAX_TRI];
};
const McTable& mc_table();  // built once on the host
struct McWork {
    uint32_t* flag;      // 3 per corner: the edge crosses phi = 0
    uint32_t* vidx;      // 3 per corner: vertex index of the edge (exclusive scan of flag)
    uint32_t* cnt;       // per cube: triangles
    uint32_t* toff;      // per cube: first triangle (exclusive scan of cnt)
    uint32_t* scan_tmp;  // scan_tmp_words(max(3 corners, cubes))
    uint32_t* totals;    // [vertices, triangles]
};
template <typename T>
void launch_mc_count(const T* phi, int cx, int cy, int cz, const McTable* tab, const McWork& w, hipStream_t st);
template <typename T>
void launch_mc_emit(const T* phi, int cx, int cy, int cz, double h, const McTable* tab, const McWork& w,
                    int64_t nv, int64_t nt, T* verts, T* normals, int32_t* tris, hipStream_t st);

// tiles: flags -> scan -> compaction -> neighbour table; writes the active
// count to *d_nactive (flags_set: the binning already set the flags)
void launch_tiles(const Geo& g, const uint32_t* count, uint32_t* tile_flag, uint32_t* tile_excl,
                  int32_t* tile_slot, uint32_t* tile_list, int32_t* tile_nbr, uint32_t* d_nactive,
                  uint32_t* scan_tmp, hipStream_t st, bool flags_set = false);

// red-black Gauss-Seidel (FLIP_FLAG_RED_BLACK_GS): `iters` iterations (a red
// and a black pass each) over the n_active tiles, and max |b - A p| over the
// fluid cells into *rmax (as the bits of a non-negative double)
template <typename V>
void launch_gs_sweeps(int n_active, int iters, const int32_t* nbr, const uint8_t* diag, const V* b, V* p,
                      hipStream_t st);
template <typename V>
void launch_gs_residual(int n_active, const int32_t* nbr, const uint8_t* diag, const V* b, const V* p,
                        unsigned long long* rmax, hipStream_t st);

// FLIP_FLAG_ADAPTIVE_DT: max over particles of (u^2 + v^2) + w^2 (FP64) into
// *out, as the bits of a non-negative double
template <typename T>
void launch_max_speed2(const T* vel, int64_t n, unsigned long long* out, hipStream_t st);

// particle-to-grid for all faces, with gravity (gdt = g * dt per axis) and walls;
// p2g_blocks: its workgroup count (one per 10^3 block of cells, P2G_NT threads)
constexpr int P2G_NT = 192;
int64_t p2g_blocks(const Geo& g);
template <typename T>
void launch_p2g(const Geo& g, const T* pos, const T* vel, int64_t n, const uint32_t* start,
                const uint32_t* count, const uint32_t* tile_flag, const T gdt[3], T* const old[3],
                T* const star[3], hipStream_t st);

// right-hand side, solver start, and the two kernels of one PCG iteration.
// All run `groups` persistent workgroups that split the active tiles among
// themselves; the active-tile count is read from device memory (d_nactive for
// the start kernels, the solver state afterwards), so nothing depends on the
// host knowing it. `partials` holds 3 * pstride doubles, pstride >= groups;
// the iteration kernels' `pslots` hold PCG_SLOT_SETS * groups doubles.
template <typename T, typename V>
void launch_rhs(const Geo& g, int groups, const uint32_t* tile_list, const uint32_t* d_nactive,
                const uint32_t* count, const T* u, const T* v, const T* w, double scale, uint8_t* diag,
                V* b, V* z, V* x, V* s0, V* s1, double* partials, int64_t pstride, PcgState* st_dev,
                double tol, int max_iters, int r_form, hipStream_t st);
// na_hint: the active-tile count when the host knows it (its loads then start
// before the solver state is read), else -1. With ev_start/ev_stop non-null
// the launch records the kernel's own start and end in those events
// (dispatch latency excluded).
// q_out: where the direction kernel stores q = A s (the multigrid solve), or null
template <typename V>
void launch_pcg_direction(int groups, int na_hint, const int32_t* tile_nbr, const uint8_t* diag, const V* z,
                          const V* s_old, V* s_new, V* q_out, double* pslots, PcgState* st_dev,
                          hipStream_t st, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
template <typename V>
void launch_pcg_update(int groups, int na_hint, const int32_t* tile_nbr, const uint8_t* diag, const V* s, V* x,
                       V* z, double* pslots, PcgState* st_dev, bool r_form, hipStream_t st,
                       hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// mixed precision: right-hand side in FP64 (b64), FP64 solution x64 = 0 and the
// start of the first FP32 inner solve (z = b64 / n rounded, x = 0, s = 0)
void launch_rhs_mixed(const Geo& g, int groups, const uint32_t* tile_list, const uint32_t* d_nactive,
                      const uint32_t* count, const float* u, const float* v, const float* w,
                      double scale, uint8_t* diag, double* b64, double* x64, float* z, float* x,
                      float* s0, float* s1, double* partials, int64_t pstride, PcgState* st_dev,
                      double tol, int max_iters, double ir_tol, int max_outer, int r_form, hipStream_t st);
// one refinement: x64_out = x64_in + x_in; r64 = b64 - A x64_out; unless
// converged, the inner FP32 solve restarts on r64 (z = r64 / n rounded,
// x_out = 0, s = 0)
void launch_ir_update(int groups, const int32_t* tile_nbr, const uint8_t* diag, const double* b64,
                      const double* x64_in, double* x64_out, const float* x_in, float* x_out,
                      float* z, float* s0, float* s1, double* partials, int64_t pstride,
                      PcgState* st_dev, int r_form, hipStream_t st);

// ---- multigrid preconditioner (FLIP_FLAG_MULTIGRID) --------------------------
// One coarse level, dense with i fastest: right-hand side b and solution x of
// its correction equation (the real type of the solve), and n_c of its fluid
// cells (0 elsewhere).
struct MgLevel {
    int nx, ny, nz;
    void* b;
    void* x;
    uint8_t* d;
    // Active blocks of the plain launches (null in batched launches, which run
    // every block): the blocks of the restriction into this level (8 x 4 x 4
    // cells) and of the prolongation into it (16 x 8 x 8) that hold a fluid
    // cell, listed by the cell-type kernel; a block of air cells only would
    // write values no later kernel reads (b) or zeros the step already holds (x).
    uint32_t* uflag;  // per prolongation block: 1 once listed
    uint32_t* dlist;  // listed restriction blocks, in no particular order
    uint32_t* ulist;  // listed prolongation blocks
    uint32_t* cnt;    // [0] restriction blocks listed, [1] prolongation blocks listed
    int nd, nu;       // the counts, read back by the host before the solve
};
constexpr int MG_MAX_LEVELS = 32;
constexpr int MG_BOTTOM_SIDE = 8;      // coarsen until every axis has at most 8 cells
constexpr int MG_BOTTOM_SWEEPS = 10;   // Jacobi sweeps on the coarsest level
// Smoothing sweeps before and after the coarse-grid correction on a dense
// level: one on the first dense level (level 1), two on every level below
// it down to the coarsest. Indices are those of the dense levels (0 = level
// 1); the fine level has one sweep.
constexpr int MG_TWO_SWEEPS_FROM = 1;
inline bool mg_two_sweeps(int dense_index) { return dense_index >= MG_TWO_SWEEPS_FROM; }
// whether a multigrid solve with solver vectors of `vector_bytes` bytes runs
// the fused update (launch_pcg_update_down): FP32 vectors (the FP32 path and
// the mixed path's inner solves), not FP64
inline bool mg_fused_update(size_t vector_bytes) { return vector_bytes == 4; }
// cell types of the first coarse level from the fine n_c, and of each next one
void launch_mg_types_fine(const Geo& g, const int32_t* tile_slot, const uint8_t* diag, const MgLevel& c,
                          hipStream_t st);
void launch_mg_types(const MgLevel& f, const MgLevel& c, hipStream_t st);
// the fine-level kernels of the V-cycle (up = false: smoothing and
// restriction of r into lv0.b; up = true: prolongation of lv0.x, smoothing
// into z and the partial sums r . z, max |r| in pslots)
// A V-cycle is launch_mg_fine(down), launch_mg_coarse, launch_mg_fine(up).
// With ev_start/ev_stop non-null a fine launch records its own start and end.
template <typename V>
void launch_mg_fine(bool up, int groups, int na_hint, const Geo& g, const uint32_t* tile_list,
                    const int32_t* tile_nbr, const uint8_t* diag, const V* r, const MgLevel& lv0, V* z,
                    double* pslots, const PcgState* ps, hipStream_t st, hipEvent_t ev_start = nullptr,
                    hipEvent_t ev_stop = nullptr);
// the coarse part of a V-cycle over levels lv[0..nlev): restrictions down to
// the coarsest level, its sweeps, prolongations and smoothing back up to lv[0]
template <typename V>
void launch_mg_coarse(const MgLevel* lv, int nlev, const PcgState* ps, hipStream_t st);
// the multigrid solve's update (residual form) fused with the fine level's
// down kernel: x += alpha s, r_out = r - alpha q (q from the direction
// kernel), level-1 b from r_out, as launch_pcg_update then
// launch_mg_fine(down). r_out must not be r (the kernel reads r's halos
// while it writes r_out). Used with FP32 solver vectors (mg_fused_update);
// in FP64 the extra q vector costs the direction kernel more than the
// fusion saves.
template <typename V>
void launch_pcg_update_down(int groups, int na_hint, const Geo& g, const uint32_t* tile_list,
                            const int32_t* tile_nbr, const uint8_t* diag, const V* s, const V* q, V* x,
                            const V* r, V* r_out, const MgLevel& c, double* pslots, PcgState* st_dev,
                            hipStream_t st, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);

// projection (Eq. (5)) of the three velocity components, one launch
template <typename T, typename V>
void launch_project3(const Geo& g, const uint8_t* diag, const int32_t* tile_slot, const V* p, T* const star[3],
                     T* const out[3], V scale, hipStream_t st);

// grid-to-particle: one workgroup per tile; start/count is the cell hash of
// the binned particles. With key_out (optional) it also bins the positions it
// writes, as launch_bin_keys would: key, provisional rank, counts into
// count_next and tile flags into tile_next (both cleared by the caller)
template <typename T>
void launch_g2p(const Geo& g, int64_t n, const uint32_t* start, const uint32_t* count, T* pos, T* vel,
                const T* u_new, const T* v_new, const T* w_new, const T* u_old, const T* v_old,
                const T* w_old, T alpha, T dt, int advect_particle_vel, uint32_t* nonfinite, hipStream_t st,
                uint32_t* key_out = nullptr, uint32_t* rank_out = nullptr, uint32_t* count_next = nullptr,
                uint32_t* tile_next = nullptr);

template <typename V, typename O>
void launch_densify(const Geo& g, const int32_t* tile_slot, const uint8_t* diag, const V* src,
                    O* dst, hipStream_t st);
void launch_flags_from_count(const uint32_t* count, int64_t ncells, uint8_t* flags,
                             hipStream_t st);

// ---- per-step diagnostics (FLIP_FLAG_DIAGNOSTICS), evaluated in FP64 ----

// Device words of a handle's diagnostics: maxima as bits of non-negative
// doubles, the energy sum, and the latch of non-finite particle state that
// grid-to-particle sets (never cleared).
struct DiagWords {
    unsigned long long rmax;      // max |b - A p| over fluid cells
    unsigned long long div_max[2];// max |div u_new|, max |div u*| over fluid cells
    unsigned long long speed2;    // max |v|^2 over the particles
    double energy;                // 1/2 sum |v|^2 over the particles
    uint32_t nonfinite;           // 1 once a particle's state was not finite
    uint32_t pad_;
};
constexpr int DIAG_ENERGY_BLOCKS = 512;  // workgroups (and partials) of the energy sum

// the divergence of f_new per cell (over dx, 0 off fluid) into div_out when
// non-null, and max |div| of f_new and f_star over fluid cells into
// maxbits[0..1] when non-null
template <typename T>
void launch_div_max(const Geo& g, const uint32_t* count, const T* const f_new[3], const T* const f_star[3],
                    double* div_out, unsigned long long* maxbits, hipStream_t st);
// 1/2 sum |v|^2 into *energy (part: DIAG_ENERGY_BLOCKS doubles of scratch) and
// max |v|^2 into *speed2
template <typename T>
void launch_particle_energy(const T* vel, int64_t n, double* part, double* energy, unsigned long long* speed2,
                            hipStream_t st);
}  // namespace flipmi
