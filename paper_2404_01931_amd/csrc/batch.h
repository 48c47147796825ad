// Batched launches (internal): one launch runs the same kernel for several
// scenes. Each scene contributes the grid its plain launch would use; the
// grids are concatenated and every workgroup finds its scene in a table of
// first-workgroup offsets. The per-scene arguments are the plain launch's
// arguments, stored as one struct per scene in device memory.
#pragma once

#include "common.h"

namespace flipmi {

// Device tables of one batched launch: args[ns] (struct per scene) and
// first[ns + 1] (first[0] = 0, first[ns] = blocks).
struct BatchLaunch {
    const void* args = nullptr;
    const uint32_t* first = nullptr;
    int ns = 0;
    uint32_t blocks = 0;
};

// workgroups of the plain launches (the batched ones concatenate them)
constexpr int ELEM_NT = 256;        // one thread per element
constexpr int SCAN_NT = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_NT * SCAN_ITEMS;
inline uint32_t elem_blocks(int64_t n) { return (uint32_t)((n + ELEM_NT - 1) / ELEM_NT); }
inline uint32_t scan_blocks(int64_t n) { return (uint32_t)((n + SCAN_TILE - 1) / SCAN_TILE); }

// ---- arguments, one struct per kernel --------------------------------------

struct FillU32Args {
    uint32_t* p;
    int64_t n;
    uint32_t v;
};

template <typename T>
struct BinKeysArgs {
    Geo g;
    const T *px, *py, *pz;
    int64_t n;
    uint32_t *key, *rank, *count;
};

struct ScanTotalsArgs {
    const uint32_t* in;
    int64_t n;
    uint32_t* totals;
};

struct ScanTotalsScanArgs {
    uint32_t* totals;
    int64_t nb;
};

struct ScanApplyArgs {
    const uint32_t* in;
    uint32_t* out;
    int64_t n;
    const uint32_t* offsets;
};

struct ScatterArgs {
    const uint32_t *key, *rank, *start;
    int64_t n;
    uint32_t* perm;
};

template <typename T>
struct GatherArgs {
    const uint32_t *perm, *key, *start, *count;
    int64_t n;
    const T *pos_in, *vel_in;
    const uint32_t* id_in;
    T *pos_out, *vel_out;
    uint32_t* id_out;
};

struct TileFlagsArgs {
    Geo g;
    const uint32_t* count;
    uint32_t* tile_flag;
};

struct TileCompactArgs {
    Geo g;
    const uint32_t *flag, *excl;
    int32_t* tile_slot;
    uint32_t* tile_list;
    int32_t* tile_nbr;
    uint32_t* d_nactive;
};

template <typename T>
struct P2GArgs {
    Geo g;
    int64_t n;
    const T *px, *py, *pz, *vx, *vy, *vz;
    const uint32_t *start, *count;
    const uint32_t* tile_flag;  // the binning's 8^3 tiles holding a particle
    T gdt[3];
    T* old[3];
    T* star[3];
};

template <typename T, typename V>
struct RhsArgs {
    Geo g;
    const uint32_t *tile_list, *d_nactive, *count;
    const T *u, *v, *w;
    double scale;
    uint8_t* diag;
    V *b, *z, *x, *s0, *s1;
    double* partials;
    int64_t pstride;
    PcgState* ps;
    double tol;
    int max_iters;
    int r_form;  // 1: start in residual form (a preconditioner application follows)
};

template <typename V>
struct DirArgs {
    int na_hint;  // -1: the active-tile count is read from the solver state
    const int32_t* nbr;
    const uint8_t* diag;
    const V *z, *s_old;
    V* s_new;
    V* q;  // q = A s_new for the multigrid update, or null
    double* pslots;
    PcgState* ps;
};

template <typename V>
struct UpdArgs {
    int na_hint;  // -1: as in DirArgs
    const int32_t* nbr;
    const uint8_t* diag;
    const V* s;
    V *x, *z;
    double* pslots;
    PcgState* ps;
};

// the multigrid solve's update fused with the fine level's down kernel
template <typename V>
struct UpdDownArgs {
    int na_hint;  // -1: as in DirArgs
    Geo g;
    const uint32_t* tile_list;
    const int32_t* nbr;
    const uint8_t* diag;
    const V *s, *q;
    V* x;
    const V* r;
    V* r_out;
    MgLevel c;
    double* pslots;
    PcgState* ps;
};

template <typename T, typename V>
struct ProjectArgs {
    Geo g;
    const uint8_t* diag;
    const int32_t* tile_slot;
    const V* p;
    const T* star[3];
    T* out[3];
    V scale;
};

template <typename T>
struct G2PArgs {
    Geo g;
    int64_t n;
    const uint32_t *start, *count;
    T *px, *py, *pz, *vx, *vy, *vz;
    const T *un, *vn, *wn, *uo, *vo, *wo;
    T alpha, dt, skin, Lx, Ly, Lz;
    int advect_particle_vel;
    uint32_t* nonfinite;  // the scene's latch of non-finite particle state
};

// multigrid V-cycle (FLIP_FLAG_MULTIGRID)
struct MgTypesFineArgs {
    Geo g;
    const int32_t* tile_slot;
    const uint8_t* diag;
    MgLevel c;
};

// a coarse level and the one below it: cell types, restriction (f -> c),
// prolongation (c -> f); the coarsest level's sweeps use f alone
struct MgPairArgs {
    MgLevel f, c;
    const PcgState* ps;
};

template <typename V>
struct MgFineArgs {
    int na_hint;
    Geo g;
    const uint32_t* tile_list;
    const int32_t* nbr;
    const uint8_t* diag;
    const V* r;
    MgLevel c;
    V* z;
    double* pslots;
    const PcgState* ps;
};

enum { MG_B_TYPES = 0, MG_B_DOWN = 1, MG_B_BOTTOM = 2, MG_B_UP = 3 };
// threads per workgroup of the batched dense-level kernels (MG_B_DOWN, MG_B_UP):
// a serving batch's scenes are 32^3 to 96^3, all their dense levels small; on
// the serving stream 512 measured 1% above 256 and 1024
constexpr int MG_BATCH_NT = 512;
// the same for the two-sweep levels, whose regions have more columns (22 x 14
// of b and n: with 512 threads one thread per column walks all 14 planes)
constexpr int MG_BATCH_NT2 = 1024;
// workgroups of one scene's plain launch of a coarse kernel of that kind
int64_t mg_blocks(int kind, const MgLevel& f, const MgLevel& c);

// Per-scene summary of the solver state after a batched step, gathered into
// one array so the host reads every scene's state with one copy.
struct SolveSummary {
    double max_b, max_r;
    int iter, done, nfluid, n_active, sync_error, pad_;
};

struct SummaryArgs {
    const PcgState* ps;
    SolveSummary* out;
};

// ---- batched launchers (asynchronous on st; nothing is launched when
// L.blocks == 0) --------------------------------------------------------------

void launch_b_fill_u32(const BatchLaunch& L, hipStream_t st);
template <typename T>
void launch_b_bin_keys(const BatchLaunch& L, hipStream_t st);
void launch_b_scan_totals(const BatchLaunch& L, hipStream_t st);
void launch_b_scan_totals_scan(const BatchLaunch& L, hipStream_t st);
void launch_b_scan_apply(const BatchLaunch& L, hipStream_t st);
void launch_b_bin_scatter(const BatchLaunch& L, hipStream_t st);
template <typename T>
void launch_b_bin_gather(const BatchLaunch& L, hipStream_t st);
void launch_b_tile_flags(const BatchLaunch& L, hipStream_t st);
void launch_b_tile_compact(const BatchLaunch& L, hipStream_t st);
template <typename T>
void launch_b_p2g(const BatchLaunch& L, hipStream_t st);
template <typename T, typename V>
void launch_b_rhs(const BatchLaunch& L, hipStream_t st);
template <typename V>
void launch_b_pcg_direction(const BatchLaunch& L, hipStream_t st);
template <typename V>
void launch_b_pcg_update(bool r_form, const BatchLaunch& L, hipStream_t st);
template <typename V>
void launch_b_pcg_update_down(const BatchLaunch& L, hipStream_t st);
// the projection of the three components (one launch; project_blocks
// workgroups per scene)
int64_t project_blocks(const Geo& g);
template <typename T, typename V>
void launch_b_project3(const BatchLaunch& L, hipStream_t st);
template <typename T>
void launch_b_g2p(const BatchLaunch& L, hipStream_t st);
void launch_b_summary(const BatchLaunch& L, hipStream_t st);
void launch_b_mg_types_fine(const BatchLaunch& L, hipStream_t st);
void launch_b_mg_types(const BatchLaunch& L, hipStream_t st);
template <typename V>
void launch_b_mg_level(int kind, bool two_sweeps, const BatchLaunch& L, hipStream_t st);
template <typename V>
void launch_b_mg_fine(bool up, const BatchLaunch& L, hipStream_t st);

}  // namespace flipmi
