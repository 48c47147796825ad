/*
 * flip.h - C ABI of libflipmi, an MI355X (gfx950) implementation of one FLIP
 * incompressible-fluid timestep as defined in Centeno & Pereira, "Fluid
 * Implicit Particle Simulation for CPU and GPU" (arXiv 2404.01931).
 *
 * One step is, in this order:
 *   1. particle binning by cell: raw cell index, stable counting sort, space
 *      hash (start offset and count per cell), fluid flags  (Sec. 3.1.5, 3.2.2)
 *   2. particle-to-grid transfer onto the staggered MAC grid with the
 *      trilinear hat kernel                                   (Sec. 3.1.6, Eq. 4)
 *   3. gravity on every face, zero normal velocity on the six domain walls,
 *      right-hand side of the pressure Poisson system         (Sec. 3.1.7, Eq. 6)
 *   4. matrix-free seven-point Poisson solve by preconditioned conjugate
 *      gradient                                                (Sec. 3.1.7)
 *   5. projection of the face velocities                       (Sec. 3.1.7, Eq. 5)
 *   6. grid-to-particle PIC/FLIP blend, forward-Euler advection and the
 *      skin-width clamp                                        (Sec. 3.1.8, 3.1.3)
 *
 * Conventions
 *   Domain [0, nx dx] x [0, ny dx] x [0, nz dx]; solid walls on all six faces.
 *   Cells are flattened x-fastest: c = i + nx (j + ny k) (Sec. 3.1.1, Fig. 2).
 *   Face component a (0 = u, 1 = v, 2 = w) has dims (nx+[a==0], ny+[a==1],
 *   nz+[a==2]), flattened x-fastest; the sample of face (i, j, k) sits at the
 *   cell-centre offset 1/2 on the two other axes and at offset 0 on axis a.
 *   Particle arrays are structure-of-arrays (Sec. 3.2.1): all x, then all y,
 *   then all z.
 *   The real type ("real") of particle and grid data is float for FLIP_FP32
 *   and FLIP_MIXED, double for FLIP_FP64.
 *
 * Errors
 *   Every call returns a flip_status; nothing throws or aborts. Argument
 *   errors are reported synchronously. Solver outcomes (non-convergence,
 *   non-finite values) are returned by the flip_step that met them and are
 *   also latched in the handle, where flip_stats reports them.
 *
 * Memory and streams
 *   The caller owns the device workspace (flip_workspace_bytes) and keeps it
 *   alive until flip_destroy. The library allocates no device memory of its
 *   own; it allocates a small host-side handle and a few bytes of pinned host
 *   memory in flip_init. Work is enqueued on the caller's HIP stream
 *   (hipStream_t passed as void*, NULL = the null stream).
 */
#ifndef FLIPMI_FLIP_H
#define FLIPMI_FLIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct flip_handle flip_handle;

typedef enum {
    FLIP_OK = 0,
    FLIP_E_INVALID = -1,       /* bad argument or configuration                         */
    FLIP_E_WORKSPACE = -2,     /* workspace missing, too small or misaligned            */
    FLIP_E_HIP = -3,           /* a HIP runtime call failed                             */
    FLIP_E_NOT_CONVERGED = -4, /* PCG hit pcg_max_iters before the tolerance            */
    FLIP_E_NONFINITE = -5,     /* non-finite values: a solver breakdown (non-positive or
                                  non-finite curvature, e.g. from a non-finite right-hand
                                  side), or a particle position or velocity that became
                                  NaN or infinite (latched by grid-to-particle, reported
                                  by the next flip_step and by flip_stats)              */
    FLIP_E_STATE = -6          /* call not valid in the handle's current state          */
} flip_status;

typedef enum { FLIP_FP32 = 0, FLIP_FP64 = 1, FLIP_MIXED = 2 } flip_precision;

enum { FLIP_REGION_BOX = 0, FLIP_REGION_SPHERE = 1 };

/* Fluid region for seeding (Sec. 3.1.2): a box lo <= x < hi on every axis, or
 * a sphere |x - center|^2 < radius^2. Seeded particles get velocity vel. */
typedef struct {
    int32_t kind;
    double lo[3], hi[3];
    double center[3], radius;
    double vel[3];
} flip_region;

/* configuration flags */
enum {
    FLIP_FLAG_NO_GRAVITY = 1u,         /* skip the gravity term                            */
    FLIP_FLAG_NO_PROJECTION = 2u,      /* skip solve and projection (transfer-only steps)  */
    FLIP_FLAG_ADVECT_PARTICLE_VEL = 4u,/* advect with the blended particle velocity        */
    FLIP_FLAG_KERNEL_TIMING = 8u,      /* bracket kernel launches with HIP events           */
    FLIP_FLAG_MULTIGRID = 16u,         /* precondition the pressure CG (FLIP_MIXED: its FP32
                                          inner solves) with a multigrid V-cycle instead of
                                          Jacobi                                              */
    FLIP_FLAG_RED_BLACK_GS = 32u,      /* solve the pressure equation by red-black
                                          Gauss-Seidel (the paper's GPU solver, Sec. 3.2.3)
                                          instead of CG: same system and stopping rule, the
                                          residual max |b - A p| (evaluated in FP64) tested
                                          every 32 iterations (a red and a black pass each);
                                          in FP32 it cannot fall much below 1e-5 max |b| on
                                          grids of 32^3 and up, so FP32 runs need a tolerance
                                          above that; pcg_max_iters then caps
                                          those iterations (<= 0: 50 * max(nx, ny, nz)^2).
                                          FLIP_FP32 and FLIP_FP64 only, not with
                                          FLIP_FLAG_MULTIGRID, not in a batch
                                          (FLIP_E_INVALID)                                    */
    FLIP_FLAG_ADAPTIVE_DT = 64u,       /* CFL time step (Sec. 3.1.4): each step takes
                                          dt = min(flip_config.dt, cfl * dx / |u|max), |u|max
                                          the speed of the fastest particle at the step's
                                          start (one 8-byte readback per step); the step's dt
                                          is reported in flip_step_stats.dt. Needs cfl > 0;
                                          not in a batch (FLIP_E_INVALID)                     */
    FLIP_FLAG_RESEED = 128u,           /* particle reseeding (Sec. 3.1.2): after binning, each
                                          fluid cell holding k < sub^3 particles (sub =
                                          subcells_per_axis, which must be in [1, 16] also
                                          when pos0 is given) gets sub^3 - k new ones, one in
                                          each of its jitter subcells k .. sub^3 - 1 (x-fastest
                                          order), at the jittered point of the subcell moved
                                          into the cell if rounding put it outside; velocity:
                                          the mean of the cell's k particles; ids continue
                                          from the current count in cell order. Jitter:
                                          SplitMix64 of `seed`, element 3 * (sub^3 * (ncells *
                                          (step + 1) + cell) + subcell) + axis, step the number
                                          of steps done before. One 8-byte readback per step.
                                          A step that would exceed particle_capacity returns
                                          FLIP_E_WORKSPACE before moving any particle. Not in
                                          a batch (FLIP_E_INVALID)                            */
    FLIP_FLAG_DIAGNOSTICS = 256u       /* after every step, evaluate in FP64 (whatever the
                                          precision) and report in flip_step_stats: the true
                                          residual max |b - A p| / max |b| of the pressure
                                          solve (Sec. 3.1.7) from the b and p it used, the
                                          divergence left by the projection max |div u_new| /
                                          max |div u*| over fluid cells (Eq. (5)), the
                                          particles' kinetic energy and largest speed (the
                                          energy of Sec. 4; the CFL number of Sec. 3.1.4).
                                          A few extra passes over the grid and the particles
                                          per step; not in a batch (FLIP_E_INVALID)          */
};

typedef struct {
    int32_t nx, ny, nz;        /* cells per axis, each >= 1                                */
    double dx;                 /* cell size (Delta tau), > 0                               */
    double gravity[3];         /* external acceleration, e.g. (0, -9.81, 0)                */
    double dt;                 /* fixed time step, > 0                                     */
    double flip_ratio;         /* blending factor alpha in [0, 1]: v = PIC + alpha(FLIP-PIC)*/
    double density;            /* rho > 0 (scales the pressure only)                       */
    double pcg_tol;            /* stop when max|r| <= pcg_tol * max|b| over fluid cells
                                  (FLIP_MIXED: tolerance of each FP32 inner solve, relative
                                  to the residual it starts from)                           */
    int32_t pcg_max_iters;     /* <= 0 selects 20 * max(nx, ny, nz)                        */
    double ir_tol;             /* FLIP_MIXED: stop refining when the FP64 residual
                                  max|b - A x| <= ir_tol * max|b| (at most 20 refinements)  */
    int32_t precision;         /* flip_precision                                           */
    uint32_t flags;            /* FLIP_FLAG_*                                              */
    /* initial particles: either seeded from regions ...                                  */
    uint32_t n_regions;
    const flip_region* regions;/* host array, read only during flip_init                   */
    int32_t subcells_per_axis; /* jitter subcells per axis (2 -> 8 particles per cell)     */
    uint64_t seed;             /* SplitMix64 seed of the jitter                            */
    /* ... or given explicitly (used when pos0 != NULL)                                   */
    int64_t n_particles;
    const double* pos0;        /* host, 3 * n_particles doubles, SoA, inside the domain    */
    const double* vel0;        /* host, 3 * n_particles doubles, SoA                       */
    double cfl;                /* FLIP_FLAG_ADAPTIVE_DT: the CFL number alpha (the paper
                                  uses 3); ignored otherwise                               */
    int64_t particle_capacity; /* particles the workspace holds (FLIP_FLAG_RESEED adds
                                  particles); <= the initial count means that count        */
} flip_config;

/* fields for flip_readback / flip_field_bytes */
enum {
    FLIP_FIELD_POS = 0,        /* real[3n] SoA, binned order of the last step              */
    FLIP_FIELD_VEL = 1,        /* real[3n] SoA                                             */
    FLIP_FIELD_ID = 2,         /* uint32[n]: initial index of each particle                */
    FLIP_FIELD_CELL_COUNT = 3, /* uint32[ncells]: particles per cell (space hash)          */
    FLIP_FIELD_CELL_START = 4, /* uint32[ncells]: exclusive scan of the counts             */
    FLIP_FIELD_FLAGS = 5,      /* uint8[ncells]: 1 = fluid (count > 0), 0 = air            */
    FLIP_FIELD_U_OLD = 6,      /* real[Fu + Fv + Fw]: raw particle-to-grid result          */
    FLIP_FIELD_U_STAR = 7,     /* real[Fu + Fv + Fw]: after gravity and walls              */
    FLIP_FIELD_U_NEW = 8,      /* real[Fu + Fv + Fw]: after projection                     */
    FLIP_FIELD_RHS = 9,        /* real[ncells]: b (0 off fluid); double for FLIP_MIXED      */
    FLIP_FIELD_PRESSURE = 10,  /* real[ncells]: p (0 off fluid); double for FLIP_MIXED      */
    FLIP_FIELD_DIV = 11,       /* double[ncells]: divergence of u_new per fluid cell (sum of
                                  its face differences over dx, Sec. 3.1.7), evaluated in
                                  FP64 from the stored faces; 0 off fluid                   */
    FLIP_FIELD_COUNT_ = 12
};

/* kernels that FLIP_FLAG_KERNEL_TIMING measures */
enum {
    FLIP_KERNEL_BIN_KEYS = 0,
    FLIP_KERNEL_BIN_SCAN = 1,
    FLIP_KERNEL_BIN_SCATTER = 2,
    FLIP_KERNEL_BIN_GATHER = 3,
    FLIP_KERNEL_TILES = 4,
    FLIP_KERNEL_P2G = 5,
    FLIP_KERNEL_RHS = 6,
    FLIP_KERNEL_PCG_DIRECTION = 7, /* s = z + beta s, q = A s, s.q                        */
    FLIP_KERNEL_PCG_UPDATE = 8,    /* x += alpha s, r -= alpha A s, r.z, max|r|          */
    FLIP_KERNEL_PROJECT = 9,
    FLIP_KERNEL_G2P = 10,
    FLIP_KERNEL_MG_DOWN_FINE = 11, /* FLIP_FLAG_MULTIGRID, fine level: smooth r, restrict  */
    FLIP_KERNEL_MG_UP_FINE = 12,   /* FLIP_FLAG_MULTIGRID, fine level: prolong, smooth, r.z */
    FLIP_KERNEL_MG_COARSE = 13,    /* FLIP_FLAG_MULTIGRID: all coarse levels of one V-cycle
                                      (several launches, timed together)                    */
    FLIP_KERNEL_COUNT = 14
};

typedef struct {
    int64_t steps;                 /* steps completed since flip_init                      */
    int64_t n_particles;
    int64_t n_fluid_cells;         /* last step                                            */
    int64_t n_active_tiles;        /* last step: 8x8x8 tiles holding a fluid cell          */
    int32_t pcg_iterations;        /* last step                                            */
    int32_t pcg_status;            /* last step: 0 converged, 1 max iters, 2 breakdown     */
    double max_b;                  /* last step: max |b| over fluid cells                  */
    double max_r;                  /* last step: final max |r| (solver's recursive residual;
                                      FLIP_MIXED: the FP64 residual |b - A x| of the result) */
    int64_t pcg_iterations_total;  /* summed over all steps                                */
    int64_t pcg_cell_iterations_total; /* sum over steps of fluid cells x PCG iterations      */
    int32_t latched_status;        /* first solver error since init (flip_status), or 0    */
    int32_t refinements;           /* last step, FLIP_MIXED: outer FP64 refinements        */
    double kernel_ms[FLIP_KERNEL_COUNT];      /* summed durations of timed launches        */
    int64_t kernel_launches[FLIP_KERNEL_COUNT];/* number of timed launches                 */
    double dt;                     /* last step: the time step it took                     */
    int64_t n_reseeded;            /* last step: particles FLIP_FLAG_RESEED added          */
    /* FLIP_FLAG_DIAGNOSTICS, last step (0 without the flag), evaluated in FP64:          */
    double true_residual;          /* max |b - A p| / max |b| over fluid cells, b and p as
                                      the solve left them (FLIP_MIXED: the FP64 ones)      */
    double div_ratio;              /* max |div u_new| / max |div u*| over fluid cells       */
    double kinetic_energy;         /* 1/2 sum |v|^2 over the particles (unit particle mass) */
    double max_speed;              /* largest particle speed after the step                */
    double cfl_number;             /* max_speed * dt / dx                                  */
    int32_t nonfinite;             /* 1 once a particle position or velocity was not finite
                                      (latched since init; with or without the flag)       */
    int32_t pad_;
} flip_step_stats;

/* Device workspace needed for cfg (pure; used for HBM admission). */
flip_status flip_workspace_bytes(const flip_config* cfg, size_t* out_bytes);

/* Validate cfg, carve the caller-owned device workspace d_ws (ws_bytes long,
 * 256-byte aligned), seed or upload the particles and return a handle.
 * Seeding (Sec. 3.1.2, Fig. 3): every cell whose centre lies inside a region
 * gets subcells_per_axis^3 particles, one at a uniformly random point of each
 * of its jitter subcells (SplitMix64 of `seed`, element 3 * (sub^3 * cell +
 * subcell) + axis, top 53 bits); or pos0 / vel0 give the particles (every
 * position inside the domain, every velocity finite). Particle ids are the
 * initial indices. Errors: FLIP_E_INVALID (configuration, or pos0 / vel0 out
 * of range or not finite), FLIP_E_WORKSPACE (d_ws missing, too small or
 * misaligned), FLIP_E_HIP. Synchronises hip_stream before returning. */
flip_status flip_init(const flip_config* cfg, void* d_ws, size_t ws_bytes, void* hip_stream,
                      flip_handle** out);

/* Run nsteps >= 0 steps on hip_stream. The PCG loop is controlled from the
 * host, so this call waits for the stream at the solver's convergence checks;
 * projection and grid-to-particle of the last step may still be in flight
 * when it returns. Returns the first solver error met, if any, after
 * completing every step. */
flip_status flip_step(flip_handle* h, int nsteps, void* hip_stream);

/* Size in bytes of a readback field. */
flip_status flip_field_bytes(const flip_handle* h, int field, size_t* out_bytes);

/* Copy a field into dst (dst_bytes >= flip_field_bytes). dst_is_device != 0:
 * dst is device memory and the copy is stream-ordered; otherwise dst is host
 * memory and the call synchronises hip_stream. Particles come in the binned
 * order of the last step (the counting sort by cell of Sec. 3.1.5, stable:
 * particles of a cell keep their previous order); FLIP_FIELD_ID maps them to
 * their initial indices. Cell fields are the space hash of Sec. 3.1.5 (start
 * offset and count per cell) and the fluid flags; face fields are the MAC
 * grid samples of Sec. 3.1.1 before forces (U_OLD), after forces and walls
 * (U_STAR) and after projection (U_NEW); RHS and PRESSURE the Poisson system
 * of Sec. 3.1.7. The caller owns dst. Errors: FLIP_E_INVALID (null handle or
 * dst, unknown field, dst_bytes too small), FLIP_E_HIP. */
flip_status flip_readback(flip_handle* h, int field, void* dst, size_t dst_bytes, int dst_is_device,
                          void* hip_stream);

/* ---- surface reconstruction: scalar field (Sec. 3.3.1) -------------------
 *
 * The improved-blobby signed distance of the particles' current positions at
 * the corners of a sampling grid of spacing dx / refine (1 <= refine <= 16):
 *   phi(x) = |x - sum_i w_i x_i| - radius,
 *   w_i = k(|x - x_i| / R) / sum_j k(|x - x_j| / R),  k(s) = max(0, (1 - s^2)^3),
 * over the particles closer than R = search_radius (every particle has the
 * same radius); a corner with no particle closer than R gets phi = R
 * (outside). Negative inside the fluid, positive outside.
 *
 * Corners (I, J, K), I in 0 .. nx*refine (x fastest), at (I, J, K) * dx / refine.
 * d_phi: caller-owned device memory of flip_surface_field_bytes bytes, reals
 * of the particle precision (double for FLIP_FP64, float otherwise). The call
 * bins the particles first (the binning of a step: their order, the ID field
 * and the cell fields change as after a step's binning) and is stream-ordered
 * on hip_stream; it does not synchronise. The search visits the cells within R
 * of a corner, so its cost grows with (2 R / dx + 1)^3.
 * Errors: FLIP_E_INVALID for a null pointer, refine out of range, radius or
 * search_radius not positive and finite, or phi_bytes too small. */
flip_status flip_surface_field_bytes(const flip_handle* h, int refine, size_t* out_bytes);
flip_status flip_surface_field(flip_handle* h, double radius, double search_radius, int refine, void* d_phi,
                               size_t phi_bytes, void* hip_stream);

/* ---- surface reconstruction: marching cubes (Sec. 3.3.2) ------------------
 *
 * The triangle mesh of phi = 0 for a corner field d_phi as written by
 * flip_surface_field with the same refine. A corner is inside when phi < 0;
 * every grid edge whose corners differ carries one vertex at the linear zero
 * of phi along it; vertices are numbered in the order of their edges (edge id
 * 3 * corner + axis, corners x-fastest), triangles in cube order (x-fastest)
 * and, within a cube, by a case table built from this rule: on each cube
 * face two crossing edges are joined by a segment and a face with four joins
 * each inside corner's two edges; segments run with the cut-off inside
 * corners on their left seen from outside the cube; segments close into
 * loops, each from its lowest local edge (0-3 along x, 4-7 along y, 8-11
 * along z), and a loop v0 .. v(m-1) gives (v0, v(k+1), v(k)): normals point
 * out of the fluid. Vertex normals (Sec. 3.3.2): the unit normals of the
 * triangles at the vertex, each weighted by the inverse of its area, summed
 * and normalised (summed with atomics: the last bits vary between runs).
 *
 * d_work: caller-owned device scratch of flip_surface_mesh_workspace_bytes
 * bytes (256-byte aligned; about 32 bytes per corner). d_vertices and
 * d_normals hold 3 reals per vertex (x, y, z; the particle precision),
 * d_triangles 3 int32 vertex indices per triangle, all device memory with
 * room for max_vertices / max_triangles. With all three output pointers NULL
 * the call only counts. The counts are returned in *n_vertices and
 * *n_triangles (host); the call synchronises hip_stream to read them, then
 * enqueues the output kernels without waiting for them.
 * Errors: FLIP_E_INVALID (null arguments, refine out of [1, 16], a grid of
 * 2^31 / 3 corners or more, only some outputs given); FLIP_E_WORKSPACE
 * (d_work too small or misaligned, or the mesh larger than max_vertices or
 * max_triangles: counts set, nothing written). */
flip_status flip_surface_mesh_workspace_bytes(const flip_handle* h, int refine, size_t* out_bytes);
flip_status flip_surface_mesh(flip_handle* h, const void* d_phi, int refine, void* d_work, size_t work_bytes,
                              void* d_vertices, void* d_normals, int64_t max_vertices, int32_t* d_triangles,
                              int64_t max_triangles, int64_t* n_vertices, int64_t* n_triangles,
                              void* hip_stream);

/* ---- marching cubes without a caller workspace -----------------------------
 *
 * For callers that cannot allocate device memory (code that may not call
 * hipMalloc, tight serving loops, harnesses that forbid allocation): the same
 * call as flip_surface_mesh, with the same arguments, outputs, results and
 * errors, but its scratch is a library-owned device array of
 * FLIP_MESH_SCRATCH_MAX_BYTES per GPU (held from the first flip_init on that
 * GPU until the process ends) instead of d_work. Nothing is allocated: no
 * hipMalloc, no hipFree, no allocating library call.
 * Limit: a sampling grid whose flip_surface_mesh_workspace_bytes exceeds
 * FLIP_MESH_SCRATCH_MAX_BYTES (about two million corners, e.g. a 104^3
 * sampling grid fits) returns FLIP_E_WORKSPACE before anything is enqueued.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (a call writes every scratch word before it reads it): calls that overlap on one GPU, on
 * different streams or from different threads, race and must be serialised
 * by the caller. The call synchronises hip_stream (it reads the counts back),
 * so back-to-back calls on one stream are ordered. */
#define FLIP_MESH_SCRATCH_MAX_BYTES ((size_t)64 << 20)
flip_status flip_surface_mesh_noalloc(flip_handle* h, const void* d_phi, int refine, void* d_vertices,
                                      void* d_normals, int64_t max_vertices, int32_t* d_triangles,
                                      int64_t max_triangles, int64_t* n_vertices, int64_t* n_triangles,
                                      void* hip_stream);

/* Statistics of the handle; synchronises the stream of the last step. A
 * non-finite particle state latched on the device since the last check is
 * reported here (nonfinite, and latched_status = FLIP_E_NONFINITE if no
 * earlier error was latched). */
flip_status flip_stats(flip_handle* h, flip_step_stats* out);

/* Release the handle (not the workspace). NULL is ignored. */
void flip_destroy(flip_handle* h);

/* ---- batched stepping (serving many independent scenes) -----------------
 *
 * A batch advances several scenes together: every kernel of the step is
 * launched once for all scenes, each workgroup working on one scene, so a
 * step of many small scenes costs about as many launches as a step of one.
 * Each scene keeps its own state in its own workspace, its own reductions
 * and its own convergence test (a converged scene's solver workgroups exit at
 * once while the others iterate). A scene's results are bitwise those that
 * flip_step gives for the same handle alone: the same kernels run with the
 * same per-scene work split and reduction order.
 *
 * Requirements: 1 <= nscenes <= FLIP_BATCH_MAX_SCENES initialised handles,
 * all FLIP_FP32 or all FLIP_FP64 (FLIP_MIXED is not batched), all with or
 * all without FLIP_FLAG_MULTIGRID, none with FLIP_FLAG_NO_PROJECTION,
 * FLIP_FLAG_KERNEL_TIMING, FLIP_FLAG_RED_BLACK_GS, FLIP_FLAG_ADAPTIVE_DT or
 * FLIP_FLAG_RESEED, no handle twice. The handles stay owned by the
 * caller, must outlive the batch and must not be stepped by other calls while
 * the batch steps.
 *
 * The launch tables live in a caller-owned device workspace
 * (flip_batch_workspace_bytes, 256-byte aligned), written once by
 * flip_batch_create. With FLIP_BATCH_GRAPHS the batch records its launch
 * sequences as HIP graphs (before the solve, a chunk of solver iterations,
 * after the solve) from its second step on and replays them; the graphs
 * are released by flip_batch_destroy.
 *
 * Slot batches (continuous batching): flip_batch_create_slots makes a batch
 * of nslots empty slots; scenes join with flip_batch_attach and leave with
 * flip_batch_detach between steps, and the batch is never rebuilt. Every
 * launch of a slot batch runs a fixed grid whose workgroups loop over the
 * workgroups of the scenes present (taken from the tables, which the next
 * step rewrites with one host-to-device copy when the scenes changed), so the
 * graphs recorded once are replayed whatever the scenes. A scene is stepped
 * exactly as in a batch built for it (the same per-scene grid, work split and
 * reduction order), so its results are again bitwise those of flip_step. */
enum { FLIP_BATCH_MAX_SCENES = 256 };
enum { FLIP_BATCH_GRAPHS = 1u, FLIP_BATCH_MULTIGRID = 2u };

typedef struct flip_batch flip_batch;

/* Shape of a slot batch: nslots in 1 .. FLIP_BATCH_MAX_SCENES; precision
 * FLIP_FP32 or FLIP_FP64; flags FLIP_BATCH_GRAPHS and FLIP_BATCH_MULTIGRID
 * (the scenes' preconditioner: set exactly when they use
 * FLIP_FLAG_MULTIGRID); the largest grid a scene may have (it sets the
 * multigrid levels the launch sequence covers). */
typedef struct {
    int nslots;
    int precision;
    uint32_t flags;
    int max_nx, max_ny, max_nz;
} flip_batch_slots;

/* Counters of a batch since its creation. */
typedef struct {
    int64_t steps;           /* batched steps taken                                  */
    int64_t graph_launches;  /* recorded graphs replayed                             */
    int64_t graph_captures;  /* graphs recorded                                      */
    int64_t table_uploads;   /* table copies (at creation, and after scene changes)   */
    int nslots, occupied;    /* slots, and slots holding a scene                     */
} flip_batch_info;

/* Device workspace needed by a batch of these handles. */
flip_status flip_batch_workspace_bytes(flip_handle* const* handles, int nscenes, size_t* out_bytes);

/* Build the launch tables of a batch into d_ws (enqueued on hip_stream and
 * synchronised before returning) and return the batch. flags: FLIP_BATCH_*. */
flip_status flip_batch_create(flip_handle* const* handles, int nscenes, uint32_t flags, void* d_ws,
                              size_t ws_bytes, void* hip_stream, flip_batch** out);

/* Device workspace of a slot batch of this shape (FLIP_E_INVALID for a bad
 * shape). */
flip_status flip_batch_slots_workspace_bytes(const flip_batch_slots* spec, size_t* out_bytes);

/* Make an empty slot batch whose tables live in d_ws (at least
 * flip_batch_slots_workspace_bytes, 256-byte aligned, caller-owned, must
 * outlive the batch). Nothing is enqueued. Errors: FLIP_E_INVALID (shape),
 * FLIP_E_WORKSPACE (d_ws). */
flip_status flip_batch_create_slots(const flip_batch_slots* spec, void* d_ws, size_t ws_bytes, void* hip_stream,
                                    flip_batch** out);

/* Put handle h into the empty slot `slot` of a slot batch, from the next
 * step on. h must meet the requirements above, have the batch's precision
 * and preconditioner, fit the batch's largest grid and not be in the batch
 * already; it stays owned by the caller and must stay alive while attached.
 * Errors (nothing changes): FLIP_E_INVALID. */
flip_status flip_batch_attach(flip_batch* b, int slot, flip_handle* h);

/* Empty slot `slot` (the handle may be destroyed afterwards, once the last
 * step's work is complete, which flip_destroy waits for). FLIP_E_INVALID for
 * an empty or out-of-range slot or a batch not made by
 * flip_batch_create_slots. */
flip_status flip_batch_detach(flip_batch* b, int slot);

/* The batch's counters (host only). */
flip_status flip_batch_get_info(const flip_batch* b, flip_batch_info* out);

/* Run nsteps >= 0 steps of every scene of the batch on hip_stream. As with
 * flip_step, the host waits at the solver's convergence checks. Each scene's
 * statistics and latched status are updated as by flip_step; the call
 * returns the first solver error met by any scene, after completing every
 * step of every scene. */
flip_status flip_batch_step(flip_batch* b, int nsteps, void* hip_stream);

/* Release the batch and its graphs (not the workspace or the handles). NULL
 * is ignored. */
void flip_batch_destroy(flip_batch* b);

const char* flip_status_string(flip_status s);

#ifdef __cplusplus
}
#endif
#endif /* FLIPMI_FLIP_H */
