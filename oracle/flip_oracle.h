/*
 * FP64 CPU oracle for one FLIP timestep (arXiv 2404.01931).
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg. Independent of the GPU library: no shared
 * code, headers, tables or helpers.
 *
 * Conventions
 *   grid      nx * ny * nz cells of side dx; domain [0, nx dx] x [0, ny dx] x
 *             [0, nz dx]; solid walls on the six domain faces.
 *   cells     flattened x-fastest: c = i + nx (j + ny k).
 *   faces     component a in {0,1,2} (u, v, w); array dims are the cell dims
 *             with one extra entry on axis a, flattened x-fastest.
 *   particles structure-of-arrays, double precision.
 * All arrays are caller-owned; the oracle allocates only temporaries.
 */
#ifndef FLIP_ORACLE_H
#define FLIP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, ny, nz;
    double dx;
} orc_grid;

enum { ORC_REGION_BOX = 0, ORC_REGION_SPHERE = 1 };

typedef struct {
    int kind;
    double lo[3], hi[3];      /* box: lo <= x < hi on every axis      */
    double center[3], radius; /* sphere: |x - center|^2 < radius^2    */
    double vel[3];            /* initial velocity of seeded particles */
} orc_region;

enum { ORC_PRECOND_MIC0 = 0, ORC_PRECOND_JACOBI = 1 };
enum { ORC_ADVECT_PARTICLE_VEL = 4u };

int64_t orc_face_count(const orc_grid* g, int a);
double orc_uniform01(uint64_t seed, uint64_t counter);

/* Seeding; returns the particle count. With px == NULL only counts. */
int64_t orc_seed(const orc_grid* g, const orc_region* regs, int nreg, int sub, uint64_t seed,
                 double* px, double* py, double* pz, double* vx, double* vy, double* vz);

void orc_cell_keys(const orc_grid* g, int64_t n, const double* px, const double* py,
                   const double* pz, uint32_t* key);
/* perm[slot] = index of the particle that moves to `slot` (stable sort by key) */
void orc_bin(const orc_grid* g, int64_t n, const double* px, const double* py, const double* pz,
             uint32_t* key, uint32_t* count, uint32_t* start, int64_t* perm);
void orc_fluid_flags(const orc_grid* g, const uint32_t* count, uint8_t* fluid);

void orc_p2g(const orc_grid* g, int a, int64_t n, const double* px, const double* py,
             const double* pz, const double* vel, double* out, double* weight_out);
void orc_forces_walls(const orc_grid* g, int a, double accel, double dt, double* f_in_out);
void orc_divergence(const orc_grid* g, const double* u, const double* v, const double* w,
                    double* div);
void orc_rhs(const orc_grid* g, const uint8_t* fluid, const double* u, const double* v,
             const double* w, double density, double dt, double* b);
void orc_apply_A(const orc_grid* g, const uint8_t* fluid, const double* x, double* y);
int orc_pcg(const orc_grid* g, const uint8_t* fluid, const double* b, double* p, double tol,
            int max_iters, int precond, int* iters_out, double* max_r_out, double* max_b_out);
void orc_project(const orc_grid* g, int a, const uint8_t* fluid, const double* p, double density,
                 double dt, const double* star, double* out);
double orc_interp(const orc_grid* g, int a, const double* f, double x, double y, double z);
void orc_g2p_advect(const orc_grid* g, int64_t n, double* px, double* py, double* pz,
                    double* vx, double* vy, double* vz, const double* const unew[3],
                    const double* const uold[3], double flip_ratio, double dt, unsigned flags);
/* CFL time step (Sec. 3.1.4): the fastest particle's speed |u|max, and
   dt = min(dt_max, alpha dx / |u|max) (dt_max when every particle is at rest) */
double orc_cfl_dt(int64_t n, const double* vx, const double* vy, const double* vz, double dx, double alpha,
                  double dt_max);
/* Reseeding (Sec. 3.1.2): new particles for every fluid cell holding fewer
   than sub^3 binned particles (count/start of the binning, velocities in
   binned order); returns their number, written in cell order when px_new is
   not NULL. Readings at the definition. */
int64_t orc_reseed(const orc_grid* g, int sub, uint64_t seed, int64_t step, int round_fp32,
                   const uint32_t* count, const uint32_t* start, const double* vx, const double* vy,
                   const double* vz, double* px_new, double* py_new, double* pz_new, double* vx_new,
                   double* vy_new, double* vz_new, uint32_t* cell_new);
/* Surface scalar field (Sec. 3.3.1): improved-blobby signed distance at the
   (nx*refine+1) x (ny*refine+1) x (nz*refine+1) corners of the sampling grid,
   x fastest; phi = search where no particle is closer than search. */
void orc_surface_field(const orc_grid* g, int refine, double radius, double search, int64_t n,
                       const double* px, const double* py, const double* pz, double* phi);
/* Marching cubes (Sec. 3.3.2) on the corner field phi of the sampling grid:
   vertices (3 doubles each), unit vertex normals, triangles (3 vertex indices
   each); counts only when verts == NULL. Returns the triangle count, the
   vertex count in *nv. The triangulation rule is stated at the definition. */
int64_t orc_surface_mesh(const orc_grid* g, int refine, const double* phi, double* verts, double* normals,
                         int64_t* tris, int64_t* nv);
/* the triangles of one cube configuration (bit q set: corner q inside) as
   local-edge triples; returns their number */
int orc_mc_case_triangles(unsigned inside, int* tri_edges);

#ifdef __cplusplus
}
#endif
#endif
