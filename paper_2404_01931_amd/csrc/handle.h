// The library's handle and the pieces of the step shared by the plain and
// the batched step (internal).
#pragma once

#include <vector>

#include "../../include/flip.h"
#include "common.h"

namespace flipmi {

struct Sizes {
    int64_t n = 0, C = 0, T = 0, cap = 0, F[3] = {0, 0, 0};
    int64_t pcap = 0;  // particle slots of the workspace (>= n; reseeding adds particles)
    size_t rb = 4;  // bytes of the real type
};

#define HIP_TRY(call)                              \
    do {                                           \
        if ((call) != hipSuccess) return FLIP_E_HIP; \
    } while (0)

}  // namespace flipmi

struct flip_handle {
    flip_config cfg;  // copy; region / array pointers cleared after init
    int prec = FLIP_FP32;
    flipmi::Geo geo{};
    flipmi::Sizes sz;
    // particles (double-buffered)
    void* pos[2] = {nullptr, nullptr};
    void* vel[2] = {nullptr, nullptr};
    uint32_t* id[2] = {nullptr, nullptr};
    uint32_t *key = nullptr, *rank = nullptr, *perm = nullptr;
    // cells
    uint32_t *count = nullptr, *start = nullptr, *scan_tmp = nullptr;
    // the next step's cell counts and 8^3 tile flags, accumulated by a plain
    // step's grid-to-particle as it writes the positions (with key and rank);
    // keys_ready says they belong to the current positions
    uint32_t *count_next = nullptr, *tile_next = nullptr;
    bool keys_ready = false;
    // tiles
    uint32_t *tile_flag = nullptr, *tile_excl = nullptr, *tile_list = nullptr, *d_nactive = nullptr;
    int32_t *tile_slot = nullptr, *tile_nbr = nullptr;
    // faces
    void* f_old[3] = {};
    void* f_star[3] = {};
    void* f_new[3] = {};
    // solver (compact tile storage)
    uint8_t* diag = nullptr;
    void *b = nullptr, *z = nullptr, *xin[2] = {nullptr, nullptr}, *s[2] = {nullptr, nullptr};
    double* b64 = nullptr;                     // FLIP_MIXED only
    double* x64[2] = {nullptr, nullptr};       // FLIP_MIXED only
    int xi = 0;                                // current solution buffer
    int scur = 0;                              // current direction buffer
    void* mgz = nullptr;                       // FLIP_FLAG_MULTIGRID: z = M r
    void* q = nullptr;                         // FLIP_FLAG_MULTIGRID, FP32 vectors: q = A s from the direction kernel
    flipmi::MgLevel mg[flipmi::MG_MAX_LEVELS] = {};  // coarse levels below the fine grid
    int nmg = 0;
    uint32_t* mg_cnt = nullptr;     // block counts of every level (2 per level)
    char* mg_zero = nullptr;        // the range cleared at each step (solutions, block marks, counts)
    size_t mg_zero_bytes = 0;
    double* partials = nullptr;  // reduction slots of the start kernels (EMPTY when idle)
    double* pslots = nullptr;    // partial sums of the iteration kernels
    unsigned long long* gs_rmax = nullptr;  // FLIP_FLAG_RED_BLACK_GS: residual max (double bits)
    uint32_t* d_reseeded = nullptr;         // FLIP_FLAG_RESEED: new particles of the step
    flipmi::PcgState* ps = nullptr;
    flipmi::DiagWords* diagw = nullptr;  // diagnostics and the non-finite latch
    double* diag_part = nullptr;          // partial sums of the energy (DIAG_ENERGY_BLOCKS)
    void* staging = nullptr;
    // host side
    int cur = 0;
    int groups = 1;  // persistent workgroups of the solver kernels
    int na = -1;     // active tiles of the current solve, once read back
    int prev_iters = 0;
    flipmi::PcgState* h_ps = nullptr;
    uint32_t* h_words = nullptr;  // pinned landing of small readbacks (2 words)
    uint32_t* h_mgcnt = nullptr;  // pinned landing of the multigrid block counts
    flipmi::DiagWords* h_diag = nullptr;  // pinned landing of the diagnostics
    double diag_dt = 0.0;                 // dt of the step the diagnostics describe
    bool diag_valid = false;              // diagnostics enqueued since init
    hipStream_t last_stream = nullptr;
    int device = -1;  // the HIP device current at flip_init
    flip_step_stats stats{};
    // kernel timing
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;
    std::vector<int> ev_iter;  // PCG iteration of a timed solver launch, -1 otherwise
    int ev_used = 0;
};

namespace flipmi {

// Per-step bookkeeping after the solve (stats, latched status), shared by the
// plain and the batched step. `solved`: a projection ran; `status`: 0
// converged, 1 not converged, 2 breakdown.
void record_step(flip_handle* h, bool solved, int status, int n_active, int nfluid, double max_b,
                 double max_r, int iters, int refinements, flip_status ret);

// iteration cap of one solve
int solve_iter_cap(const flip_config& c);

}  // namespace flipmi
