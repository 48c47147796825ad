/*
 * FP64 CPU oracle for one FLIP timestep (Centeno & Pereira, "Fluid Implicit
 * Particle Simulation for CPU and GPU", arXiv 2404.01931).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain, obviously-correct
 * reference that the GPU library is checked against. Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it. It shares
 * no code, header, table or helper with the GPU library, and the GPU library
 * never calls it.
 *
 * Every stage is a direct transcription of the definition it follows, in
 * double precision, with no blocking, fusion or reordering:
 *   seeding            paper Sec. 3.1.2 (jittered subcells, Fig. 3)
 *   binning            paper Sec. 3.1.5 (raw cell index, sort, space hash,
 *                      Fig. 4) and Sec. 3.2.2 (exclusive scan with identity)
 *   particle-to-grid   paper Sec. 3.1.6, Eq. (4a), (4b) and the normalised
 *                      weighted sum that follows them
 *   forces / walls     paper Sec. 2.1.1 Eq. (1) (gravity), Sec. 3.1.7 (solid
 *                      walls, free surface p = 0)
 *   right-hand side    paper Sec. 3.1.7, Eq. (6) by central differences
 *   operator           paper Sec. 3.1.7 (seven-point Laplacian, symmetric)
 *   solve              paper Sec. 3.1.7 (PCG on the CPU); preconditioner
 *                      MIC(0) as in Bridson's book (paper ref. [5]) or Jacobi
 *   projection         paper Sec. 3.1.7, Eq. (5)
 *   grid-to-particle   paper Sec. 3.1.8 (trilinear interpolation of the new
 *                      field and of the change, PIC/FLIP blend)
 *   advection / clamp  paper Sec. 3.1.3 (forward Euler, skin-width clamp)
 *   CFL time step      paper Sec. 3.1.4 (dt <= alpha dx / fastest speed)
 *   reseeding          paper Sec. 3.1.2, closing paragraph (refill sparse
 *                      fluid cells up to the seeding density)
 *   surface field      paper Sec. 3.3.1 (improved-blobby signed distance at
 *                      the corners of a sampling grid)
 *   surface mesh       paper Sec. 3.3.2 (marching cubes, inverse-area
 *                      weighted vertex normals)
 *
 * Readings of points the paper leaves open are stated where they are used.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "flip_oracle.h"

/* ------------------------------------------------------------------------ */
/* Indexing. Cells are flattened x-fastest (paper Sec. 3.1.1, Fig. 2).      */
/* Face arrays of component a have one extra entry along axis a.            */
/* ------------------------------------------------------------------------ */

static int64_t n_cells(const orc_grid* g) { return (int64_t)g->nx * g->ny * g->nz; }

static int64_t cell_index(const orc_grid* g, int i, int j, int k)
{
    return i + (int64_t)g->nx * (j + (int64_t)g->ny * k);
}

static void face_dims(const orc_grid* g, int a, int d[3])
{
    d[0] = g->nx + (a == 0);
    d[1] = g->ny + (a == 1);
    d[2] = g->nz + (a == 2);
}

static int64_t face_index(const int d[3], int i, int j, int k)
{
    return i + (int64_t)d[0] * (j + (int64_t)d[1] * k);
}

int64_t orc_face_count(const orc_grid* g, int a)
{
    int d[3];
    face_dims(g, a, d);
    return (int64_t)d[0] * d[1] * d[2];
}

/* ------------------------------------------------------------------------ */
/* Seeding (paper Sec. 3.1.2): a cell whose centre lies inside the fluid    */
/* region gets sub^3 subcells, each with one particle at a uniformly random */
/* point of the subcell. Random numbers: the SplitMix64 output sequence     */
/* (Steele, Lea & Flood, OOPSLA 2014), element number `counter` of the      */
/* sequence started at `seed`, top 53 bits scaled to [0, 1).                */
/* ------------------------------------------------------------------------ */

static uint64_t splitmix64_element(uint64_t seed, uint64_t counter)
{
    uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double orc_uniform01(uint64_t seed, uint64_t counter)
{
    return (double)(splitmix64_element(seed, counter) >> 11) * 0x1.0p-53;
}

static int region_contains(const orc_region* r, const double x[3])
{
    if (r->kind == ORC_REGION_BOX) {
        for (int a = 0; a < 3; ++a)
            if (!(r->lo[a] <= x[a] && x[a] < r->hi[a])) return 0;
        return 1;
    }
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double d = x[a] - r->center[a];
        d2 += d * d;
    }
    return d2 < r->radius * r->radius;
}

int64_t orc_seed(const orc_grid* g, const orc_region* regs, int nreg, int sub,
                 uint64_t seed, double* px, double* py, double* pz,
                 double* vx, double* vy, double* vz)
{
    int64_t n = 0;
    const int64_t per_cell = (int64_t)sub * sub * sub;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                double centre[3] = {(i + 0.5) * g->dx, (j + 0.5) * g->dx, (k + 0.5) * g->dx};
                const orc_region* hit = NULL;
                for (int r = 0; r < nreg && !hit; ++r)
                    if (region_contains(&regs[r], centre)) hit = &regs[r];
                if (!hit) continue;
                int64_t lin = cell_index(g, i, j, k);
                for (int sz = 0; sz < sub; ++sz)
                    for (int sy = 0; sy < sub; ++sy)
                        for (int sx = 0; sx < sub; ++sx) {
                            if (px) {
                                int64_t s = sx + (int64_t)sub * (sy + (int64_t)sub * sz);
                                uint64_t ctr = 3u * (uint64_t)(per_cell * lin + s);
                                double xi = orc_uniform01(seed, ctr + 0);
                                double yi = orc_uniform01(seed, ctr + 1);
                                double zi = orc_uniform01(seed, ctr + 2);
                                px[n] = ((sx + xi) / sub + i) * g->dx;
                                py[n] = ((sy + yi) / sub + j) * g->dx;
                                pz[n] = ((sz + zi) / sub + k) * g->dx;
                                vx[n] = hit->vel[0];
                                vy[n] = hit->vel[1];
                                vz[n] = hit->vel[2];
                            }
                            ++n;
                        }
            }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Binning (paper Sec. 3.1.5, Fig. 4; Sec. 3.2.2).                          */
/* The raw cell index of a particle is the floor of the exact quotient      */
/* x / dx on each axis (clamped into the grid). The floor is taken on the   */
/* real number x / dx, not on its rounded value: the candidate q is         */
/* corrected until q*dx <= x < (q+1)*dx, each comparison made exactly with  */
/* a fused multiply-add whose sign equals the sign of the exact difference. */
/* ------------------------------------------------------------------------ */

static int exact_floor_div(double x, double dx, int n)
{
    double q = floor(x / dx);
    while (fma(q, dx, -x) > 0.0) q -= 1.0;          /* q*dx > x     */
    while (fma(q + 1.0, dx, -x) <= 0.0) q += 1.0;   /* (q+1)*dx <= x */
    if (q < 0.0) q = 0.0;
    if (q > n - 1) q = n - 1;
    return (int)q;
}

void orc_cell_keys(const orc_grid* g, int64_t n, const double* px, const double* py,
                   const double* pz, uint32_t* key)
{
    for (int64_t p = 0; p < n; ++p) {
        int i = exact_floor_div(px[p], g->dx, g->nx);
        int j = exact_floor_div(py[p], g->dx, g->ny);
        int k = exact_floor_div(pz[p], g->dx, g->nz);
        key[p] = (uint32_t)cell_index(g, i, j, k);
    }
}

void orc_bin(const orc_grid* g, int64_t n, const double* px, const double* py,
             const double* pz, uint32_t* key, uint32_t* count, uint32_t* start,
             int64_t* perm)
{
    const int64_t C = n_cells(g);
    orc_cell_keys(g, n, px, py, pz, key);
    memset(count, 0, sizeof(uint32_t) * (size_t)C);
    for (int64_t p = 0; p < n; ++p) count[key[p]]++;
    /* all-prefix-sums with identity 0: start[c] = count[0] + ... + count[c-1] */
    uint32_t run = 0;
    for (int64_t c = 0; c < C; ++c) {
        start[c] = run;
        run += count[c];
    }
    /* stable counting sort: particles of one cell keep their current order */
    uint32_t* fill = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)C);
    memcpy(fill, start, sizeof(uint32_t) * (size_t)C);
    for (int64_t p = 0; p < n; ++p) perm[fill[key[p]]++] = p;
    free(fill);
}

void orc_fluid_flags(const orc_grid* g, const uint32_t* count, uint8_t* fluid)
{
    const int64_t C = n_cells(g);
    for (int64_t c = 0; c < C; ++c) fluid[c] = count[c] > 0 ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Particle-to-grid (paper Sec. 3.1.6, Eq. (4)).                            */
/* Face sample points: component a sits at the cell-centre offset (1/2)     */
/* on the two other axes and at offset 0 on axis a (MAC grid, Sec. 3.1.1).  */
/* For each face: q_f = sum_P q_P k(x_P - x_f) / sum_P k(x_P - x_f), with   */
/* k the trilinear hat; a face no particle reaches gets 0.                  */
/* The sums are accumulated particle by particle over the faces the         */
/* particle reaches; addition order does not change the definition.         */
/* ------------------------------------------------------------------------ */

/* The two sample planes of one axis that bracket a particle's coordinate   */
/* x, given the particle's cell c on that axis (the binning's exact floor): */
/* plane lo at (lo + off) dx and plane lo + 1 one spacing above, off = 0 on  */
/* the component's own axis (samples on cell faces, lo = c) and 1/2 on the  */
/* two others (samples at cell-centre height, lo = c - 1 below the centre   */
/* of the cell, else c). Between the two planes the hat of Eq. (4b) is      */
/* 1 - |x / dx - (lo + off)| for plane lo, which equals the distance from x */
/* to the other plane over dx: ((lo + 1 + off) dx - x) / dx, and likewise   */
/* (x - (lo + off) dx) / dx for plane lo + 1. Each distance is x minus the  */
/* exact product plane * dx, rounded once (fma), so a weight is zero        */
/* exactly when the particle lies on the other plane, never by cancellation */
/* (the hat of a tiny distance is 1 - r with r rounded near 1). max(0, .)   */
/* keeps the support at a domain edge that rounding of n dx moved. Returns  */
/* lo; w[0] is the weight of plane lo, w[1] that of plane lo + 1.           */
static int bracket(double x, int c, double off, double dx, double w[2])
{
    int lo = c;
    if (off != 0.0 && fma(-((double)c + 0.5), dx, x) < 0.0) lo = c - 1;
    const double below = fma(-((double)lo + off), dx, x);     /* x - plane lo     */
    const double above = fma((double)lo + 1.0 + off, dx, -x); /* plane lo + 1 - x */
    w[0] = above > 0.0 ? above / dx : 0.0;
    w[1] = below > 0.0 ? below / dx : 0.0;
    return lo;
}

void orc_p2g(const orc_grid* g, int a, int64_t n, const double* px, const double* py,
             const double* pz, const double* vel, double* out, double* weight_out)
{
    int d[3];
    face_dims(g, a, d);
    const int nc[3] = {g->nx, g->ny, g->nz};
    const int64_t F = (int64_t)d[0] * d[1] * d[2];
    double* W = (double*)calloc((size_t)F, sizeof(double));
    double* M = (double*)calloc((size_t)F, sizeof(double));
    for (int64_t p = 0; p < n; ++p) {
        const double x[3] = {px[p], py[p], pz[p]};
        /* the hat has support |r| < 1: only the two sample planes that     */
        /* bracket the particle on each axis can receive a non-zero weight  */
        int base[3];
        double w[3][2];
        for (int ax = 0; ax < 3; ++ax)
            base[ax] = bracket(x[ax], exact_floor_div(x[ax], g->dx, nc[ax]), (ax == a) ? 0.0 : 0.5, g->dx, w[ax]);
        for (int dk = 0; dk <= 1; ++dk)
            for (int dj = 0; dj <= 1; ++dj)
                for (int di = 0; di <= 1; ++di) {
                    int fi = base[0] + di, fj = base[1] + dj, fk = base[2] + dk;
                    if (fi < 0 || fi >= d[0] || fj < 0 || fj >= d[1] || fk < 0 || fk >= d[2])
                        continue;
                    double k = w[0][di] * w[1][dj] * w[2][dk];
                    int64_t f = face_index(d, fi, fj, fk);
                    W[f] += k;
                    M[f] += vel[p] * k;
                }
    }
    for (int64_t f = 0; f < F; ++f) {
        out[f] = W[f] > 0.0 ? M[f] / W[f] : 0.0;
        if (weight_out) weight_out[f] = W[f];
    }
    free(W);
    free(M);
}

/* ------------------------------------------------------------------------ */
/* External force and solid walls. Gravity is added to every face sample of */
/* its component (force step of the splitting, paper Sec. 2.1.3); the       */
/* normal velocity on the six domain faces is then set to zero (solid-wall  */
/* condition, paper Sec. 3.1.7).                                            */
/* ------------------------------------------------------------------------ */

void orc_forces_walls(const orc_grid* g, int a, double accel, double dt, double* f_in_out)
{
    int d[3];
    face_dims(g, a, d);
    for (int k = 0; k < d[2]; ++k)
        for (int j = 0; j < d[1]; ++j)
            for (int i = 0; i < d[0]; ++i) {
                int64_t f = face_index(d, i, j, k);
                f_in_out[f] += accel * dt;
                int idx = (a == 0) ? i : (a == 1) ? j : k;
                int lim = (a == 0) ? g->nx : (a == 1) ? g->ny : g->nz;
                if (idx == 0 || idx == lim) f_in_out[f] = 0.0;
            }
}

/* ------------------------------------------------------------------------ */
/* Discrete divergence by central differences (paper Eq. (6)), per cell:    */
/* div_c = [(u_{i+1}-u_i) + (v_{j+1}-v_j) + (w_{k+1}-w_k)] / dx.            */
/* ------------------------------------------------------------------------ */

static double face_sum_difference(const orc_grid* g, const double* u, const double* v,
                                  const double* w, int i, int j, int k)
{
    int du[3], dv[3], dw[3];
    face_dims(g, 0, du);
    face_dims(g, 1, dv);
    face_dims(g, 2, dw);
    return (u[face_index(du, i + 1, j, k)] - u[face_index(du, i, j, k)]) +
           (v[face_index(dv, i, j + 1, k)] - v[face_index(dv, i, j, k)]) +
           (w[face_index(dw, i, j, k + 1)] - w[face_index(dw, i, j, k)]);
}

void orc_divergence(const orc_grid* g, const double* u, const double* v, const double* w,
                    double* div)
{
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i)
                div[cell_index(g, i, j, k)] = face_sum_difference(g, u, v, w, i, j, k) / g->dx;
}

/* ------------------------------------------------------------------------ */
/* Right-hand side of A p = b (paper Sec. 3.1.7). Multiplying the discrete  */
/* Poisson equation by dx^2 rho / dt gives integer stencil coefficients and */
/* b_c = -(rho dx / dt) * [sum of face differences] on fluid cells.         */
/* ------------------------------------------------------------------------ */

void orc_rhs(const orc_grid* g, const uint8_t* fluid, const double* u, const double* v,
             const double* w, double density, double dt, double* b)
{
    const double scale = -density * g->dx / dt;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                int64_t c = cell_index(g, i, j, k);
                b[c] = fluid[c] ? scale * face_sum_difference(g, u, v, w, i, j, k) : 0.0;
            }
}

/* ------------------------------------------------------------------------ */
/* Seven-point operator (paper Sec. 3.1.7), restricted to fluid cells:      */
/* (A p)_c = n_c p_c - sum over fluid neighbours p_nb, where n_c counts the */
/* neighbours inside the domain (fluid or air; air carries p = 0, the free- */
/* surface condition) and neighbours across a solid wall are left out.      */
/* Non-fluid rows are zero.                                                 */
/* ------------------------------------------------------------------------ */

static const int NB[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};

static int in_domain(const orc_grid* g, int i, int j, int k)
{
    return i >= 0 && i < g->nx && j >= 0 && j < g->ny && k >= 0 && k < g->nz;
}

static int neighbour_count(const orc_grid* g, int i, int j, int k)
{
    int n = 0;
    for (int t = 0; t < 6; ++t) n += in_domain(g, i + NB[t][0], j + NB[t][1], k + NB[t][2]);
    return n;
}

void orc_apply_A(const orc_grid* g, const uint8_t* fluid, const double* x, double* y)
{
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                int64_t c = cell_index(g, i, j, k);
                if (!fluid[c]) {
                    y[c] = 0.0;
                    continue;
                }
                double acc = neighbour_count(g, i, j, k) * x[c];
                for (int t = 0; t < 6; ++t) {
                    int ii = i + NB[t][0], jj = j + NB[t][1], kk = k + NB[t][2];
                    if (!in_domain(g, ii, jj, kk)) continue;
                    int64_t nb = cell_index(g, ii, jj, kk);
                    if (fluid[nb]) acc -= x[nb];
                }
                y[c] = acc;
            }
}

/* ------------------------------------------------------------------------ */
/* Preconditioners.                                                         */
/* Jacobi: z = r / n_c.                                                     */
/* MIC(0): modified incomplete Cholesky with zero fill-in, A ~ L L^T with   */
/* L's sparsity that of A's lower triangle in x-fastest order. The diagonal */
/* factor of each cell is built from its already-factored -x, -y, -z        */
/* neighbours; the "modified" part adds tau times the fill-in that plain    */
/* IC(0) would drop back onto the diagonal, and a pivot falling below      */
/* sigma * n_c is replaced by n_c (tau = 0.97, sigma = 0.25, the values     */
/* Bridson's book uses).                                                    */
/* ------------------------------------------------------------------------ */

/* coupling of cell (i,j,k) to its +axis neighbour: -1 if both are fluid    */
static double offdiag(const orc_grid* g, const uint8_t* fluid, int i, int j, int k, int axis)
{
    int ii = i + (axis == 0), jj = j + (axis == 1), kk = k + (axis == 2);
    if (!in_domain(g, i, j, k) || !in_domain(g, ii, jj, kk)) return 0.0;
    if (!fluid[cell_index(g, i, j, k)] || !fluid[cell_index(g, ii, jj, kk)]) return 0.0;
    return -1.0;
}

static double precon_at(const orc_grid* g, const double* pc, int i, int j, int k)
{
    return in_domain(g, i, j, k) ? pc[cell_index(g, i, j, k)] : 0.0;
}

static void mic0_factor(const orc_grid* g, const uint8_t* fluid, double* pc)
{
    const double tau = 0.97, sigma = 0.25;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                int64_t c = cell_index(g, i, j, k);
                pc[c] = 0.0;
                if (!fluid[c]) continue;
                double diag = neighbour_count(g, i, j, k);
                double ax_m = offdiag(g, fluid, i - 1, j, k, 0);   /* (i-1) <-> i */
                double ay_m = offdiag(g, fluid, i, j - 1, k, 1);
                double az_m = offdiag(g, fluid, i, j, k - 1, 2);
                double p_xm = precon_at(g, pc, i - 1, j, k);
                double p_ym = precon_at(g, pc, i, j - 1, k);
                double p_zm = precon_at(g, pc, i, j, k - 1);
                double e = diag - (ax_m * p_xm) * (ax_m * p_xm) - (ay_m * p_ym) * (ay_m * p_ym) -
                           (az_m * p_zm) * (az_m * p_zm);
                double fill =
                    ax_m * (offdiag(g, fluid, i - 1, j, k, 1) + offdiag(g, fluid, i - 1, j, k, 2)) * p_xm * p_xm +
                    ay_m * (offdiag(g, fluid, i, j - 1, k, 0) + offdiag(g, fluid, i, j - 1, k, 2)) * p_ym * p_ym +
                    az_m * (offdiag(g, fluid, i, j, k - 1, 0) + offdiag(g, fluid, i, j, k - 1, 1)) * p_zm * p_zm;
                e -= tau * fill;
                if (e < sigma * diag) e = diag;
                pc[c] = 1.0 / sqrt(e);
            }
}

static void mic0_apply(const orc_grid* g, const uint8_t* fluid, const double* pc,
                       const double* r, double* tmp, double* z)
{
    /* solve L q = r (forward, increasing index) */
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                int64_t c = cell_index(g, i, j, k);
                tmp[c] = 0.0;
                if (!fluid[c]) continue;
                double t = r[c];
                if (i > 0) t -= offdiag(g, fluid, i - 1, j, k, 0) * pc[cell_index(g, i - 1, j, k)] * tmp[cell_index(g, i - 1, j, k)];
                if (j > 0) t -= offdiag(g, fluid, i, j - 1, k, 1) * pc[cell_index(g, i, j - 1, k)] * tmp[cell_index(g, i, j - 1, k)];
                if (k > 0) t -= offdiag(g, fluid, i, j, k - 1, 2) * pc[cell_index(g, i, j, k - 1)] * tmp[cell_index(g, i, j, k - 1)];
                tmp[c] = t * pc[c];
            }
    /* solve L^T z = q (backward, decreasing index) */
    for (int k = g->nz - 1; k >= 0; --k)
        for (int j = g->ny - 1; j >= 0; --j)
            for (int i = g->nx - 1; i >= 0; --i) {
                int64_t c = cell_index(g, i, j, k);
                z[c] = 0.0;
                if (!fluid[c]) continue;
                double t = tmp[c];
                if (i + 1 < g->nx) t -= offdiag(g, fluid, i, j, k, 0) * pc[c] * z[cell_index(g, i + 1, j, k)];
                if (j + 1 < g->ny) t -= offdiag(g, fluid, i, j, k, 1) * pc[c] * z[cell_index(g, i, j + 1, k)];
                if (k + 1 < g->nz) t -= offdiag(g, fluid, i, j, k, 2) * pc[c] * z[cell_index(g, i, j, k + 1)];
                z[c] = t * pc[c];
            }
}

static void jacobi_apply(const orc_grid* g, const uint8_t* fluid, const double* r, double* z)
{
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                int64_t c = cell_index(g, i, j, k);
                z[c] = fluid[c] ? r[c] / neighbour_count(g, i, j, k) : 0.0;
            }
}

static double dot_fluid(int64_t C, const uint8_t* fluid, const double* a, const double* b)
{
    double s = 0.0;
    for (int64_t c = 0; c < C; ++c)
        if (fluid[c]) s += a[c] * b[c];
    return s;
}

static double maxabs_fluid(int64_t C, const uint8_t* fluid, const double* a)
{
    double m = 0.0;
    for (int64_t c = 0; c < C; ++c)
        if (fluid[c] && fabs(a[c]) > m) m = fabs(a[c]);
    return m;
}

/* ------------------------------------------------------------------------ */
/* Preconditioned conjugate gradient (paper Sec. 3.1.7, CPU solver).        */
/* Starts from p = 0. Stops when max|r| <= tol * max|b| over fluid cells    */
/* (r the recursively updated residual). Returns 0 on convergence, 1 when   */
/* max_iters is reached first, 2 on a breakdown (non-positive or non-finite */
/* curvature).                                                              */
/* ------------------------------------------------------------------------ */

int orc_pcg(const orc_grid* g, const uint8_t* fluid, const double* b, double* p, double tol,
            int max_iters, int precond, int* iters_out, double* max_r_out, double* max_b_out)
{
    const int64_t C = n_cells(g);
    double* r = (double*)malloc(sizeof(double) * (size_t)C);
    double* z = (double*)malloc(sizeof(double) * (size_t)C);
    double* s = (double*)malloc(sizeof(double) * (size_t)C);
    double* q = (double*)malloc(sizeof(double) * (size_t)C);
    double* tmp = (double*)malloc(sizeof(double) * (size_t)C);
    double* pc = NULL;
    int status = 1, it = 0;

    for (int64_t c = 0; c < C; ++c) {
        p[c] = 0.0;
        r[c] = fluid[c] ? b[c] : 0.0;
    }
    double max_b = maxabs_fluid(C, fluid, r);
    double max_r = max_b;
    if (max_b == 0.0) {
        status = 0;
        goto done;
    }
    if (precond == ORC_PRECOND_MIC0) {
        pc = (double*)malloc(sizeof(double) * (size_t)C);
        mic0_factor(g, fluid, pc);
        mic0_apply(g, fluid, pc, r, tmp, z);
    } else {
        jacobi_apply(g, fluid, r, z);
    }
    memcpy(s, z, sizeof(double) * (size_t)C);
    double rho = dot_fluid(C, fluid, r, z);
    for (it = 1; it <= max_iters; ++it) {
        orc_apply_A(g, fluid, s, q);
        double sq = dot_fluid(C, fluid, s, q);
        if (!(sq > 0.0) || !isfinite(sq)) {
            status = 2;
            break;
        }
        double alpha = rho / sq;
        for (int64_t c = 0; c < C; ++c) {
            if (!fluid[c]) continue;
            p[c] += alpha * s[c];
            r[c] -= alpha * q[c];
        }
        max_r = maxabs_fluid(C, fluid, r);
        if (max_r <= tol * max_b) {
            status = 0;
            break;
        }
        if (precond == ORC_PRECOND_MIC0)
            mic0_apply(g, fluid, pc, r, tmp, z);
        else
            jacobi_apply(g, fluid, r, z);
        double rho_new = dot_fluid(C, fluid, r, z);
        double beta = rho_new / rho;
        rho = rho_new;
        for (int64_t c = 0; c < C; ++c) s[c] = fluid[c] ? z[c] + beta * s[c] : 0.0;
    }
    if (it > max_iters) it = max_iters;
done:
    if (iters_out) *iters_out = it;
    if (max_r_out) *max_r_out = max_r;
    if (max_b_out) *max_b_out = max_b;
    free(r);
    free(z);
    free(s);
    free(q);
    free(tmp);
    free(pc);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Projection (paper Sec. 3.1.7, Eq. (5)): every face that is not a domain  */
/* wall and touches at least one fluid cell gets                            */
/*   u_f = u*_f - (dt / rho) (p_plus - p_minus) / dx,                       */
/* with p = 0 in air cells (free surface). Wall faces and faces between two */
/* air cells keep u*.                                                       */
/* ------------------------------------------------------------------------ */

void orc_project(const orc_grid* g, int a, const uint8_t* fluid, const double* p, double density,
                 double dt, const double* star, double* out)
{
    int d[3];
    face_dims(g, a, d);
    const double scale = dt / (density * g->dx);
    for (int k = 0; k < d[2]; ++k)
        for (int j = 0; j < d[1]; ++j)
            for (int i = 0; i < d[0]; ++i) {
                int64_t f = face_index(d, i, j, k);
                out[f] = star[f];
                int idx = (a == 0) ? i : (a == 1) ? j : k;
                int lim = (a == 0) ? g->nx : (a == 1) ? g->ny : g->nz;
                if (idx == 0 || idx == lim) continue;
                int64_t cp = cell_index(g, i, j, k);
                int64_t cm = cell_index(g, i - (a == 0), j - (a == 1), k - (a == 2));
                if (!fluid[cp] && !fluid[cm]) continue;
                double pp = fluid[cp] ? p[cp] : 0.0;
                double pm = fluid[cm] ? p[cm] : 0.0;
                out[f] = star[f] - scale * (pp - pm);
            }
}

/* ------------------------------------------------------------------------ */
/* Grid-to-particle and advection (paper Sec. 3.1.8 and Sec. 3.1.3).        */
/* Trilinear interpolation of a face field at a particle: the eight sample  */
/* points around it, indices clamped to the valid range at the domain edge, */
/* blended by nested linear interpolations a + t (b - a) along x, y, z.     */
/* PIC = interp(u_new); change = interp(u_new - u_old); FLIP = v + change;  */
/* v <- PIC + alpha (FLIP - PIC). Forward Euler moves the particle with the */
/* grid velocity PIC (or with the blended velocity when the flag asks for   */
/* it), then each coordinate is clamped into [s, L - s] with s = dx/1000.   */
/* ------------------------------------------------------------------------ */

static double lerp(double a, double b, double t) { return a + t * (b - a); }

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

double orc_interp(const orc_grid* g, int a, const double* f, double x, double y, double z)
{
    int d[3];
    face_dims(g, a, d);
    const double pos[3] = {x, y, z};
    int i0[3], i1[3];
    double t[3];
    for (int ax = 0; ax < 3; ++ax) {
        double gc = pos[ax] / g->dx - ((ax == a) ? 0.0 : 0.5);
        double fl = floor(gc);
        t[ax] = gc - fl;
        i0[ax] = clampi((int)fl, 0, d[ax] - 1);
        i1[ax] = clampi((int)fl + 1, 0, d[ax] - 1);
    }
#define F(I, J, K) f[face_index(d, (I), (J), (K))]
    double c00 = lerp(F(i0[0], i0[1], i0[2]), F(i1[0], i0[1], i0[2]), t[0]);
    double c10 = lerp(F(i0[0], i1[1], i0[2]), F(i1[0], i1[1], i0[2]), t[0]);
    double c01 = lerp(F(i0[0], i0[1], i1[2]), F(i1[0], i0[1], i1[2]), t[0]);
    double c11 = lerp(F(i0[0], i1[1], i1[2]), F(i1[0], i1[1], i1[2]), t[0]);
#undef F
    double c0 = lerp(c00, c10, t[1]);
    double c1 = lerp(c01, c11, t[1]);
    return lerp(c0, c1, t[2]);
}

void orc_g2p_advect(const orc_grid* g, int64_t n, double* px, double* py, double* pz,
                    double* vx, double* vy, double* vz, const double* const unew[3],
                    const double* const uold[3], double flip_ratio, double dt, unsigned flags)
{
    double* delta[3];
    for (int a = 0; a < 3; ++a) {
        int64_t F = orc_face_count(g, a);
        delta[a] = (double*)malloc(sizeof(double) * (size_t)F);
        for (int64_t f = 0; f < F; ++f) delta[a][f] = unew[a][f] - uold[a][f];
    }
    const double skin = 1e-3 * g->dx;
    const double L[3] = {g->nx * g->dx, g->ny * g->dx, g->nz * g->dx};
    for (int64_t p = 0; p < n; ++p) {
        double* pos[3] = {&px[p], &py[p], &pz[p]};
        double* vel[3] = {&vx[p], &vy[p], &vz[p]};
        double pic[3], vnew[3];
        for (int a = 0; a < 3; ++a) {
            pic[a] = orc_interp(g, a, unew[a], px[p], py[p], pz[p]);
            double change = orc_interp(g, a, delta[a], px[p], py[p], pz[p]);
            double flip = *vel[a] + change;
            vnew[a] = pic[a] + flip_ratio * (flip - pic[a]);
        }
        for (int a = 0; a < 3; ++a) {
            double adv = (flags & ORC_ADVECT_PARTICLE_VEL) ? vnew[a] : pic[a];
            double x = *pos[a] + dt * adv;
            if (x < skin) x = skin;
            if (x > L[a] - skin) x = L[a] - skin;
            *pos[a] = x;
            *vel[a] = vnew[a];
        }
    }
    for (int a = 0; a < 3; ++a) free(delta[a]);
}

/* Sec. 3.1.4: dt <= alpha dx / |u|, with |u| the speed of the fastest particle. */
double orc_cfl_dt(int64_t n, const double* vx, const double* vy, const double* vz, double dx, double alpha,
                  double dt_max)
{
    double umax = 0.0;
    for (int64_t p = 0; p < n; ++p) {
        const double speed = sqrt((vx[p] * vx[p] + vy[p] * vy[p]) + vz[p] * vz[p]);
        if (speed > umax) umax = speed;
    }
    if (umax == 0.0) return dt_max;
    const double dt = alpha * dx / umax;
    return dt < dt_max ? dt : dt_max;
}

/* ------------------------------------------------------------------------ */
/* Reseeding (paper Sec. 3.1.2, closing paragraph): a fluid cell holding     */
/* fewer particles than the seeding density asks for (sub^3 per cell) is     */
/* refilled up to that number. The paper gives no further detail; readings:  */
/*  - a cell with k particles, 0 < k < sub^3, gets sub^3 - k new particles,  */
/*    one in each of its jitter subcells k .. sub^3 - 1 (x-fastest order),   */
/*    at the same jittered point rule as the initial seeding;                */
/*  - the jitter is element 3 (sub^3 (C (step + 1) + cell) + subcell) + axis */
/*    of the seed's SplitMix64 sequence (C cells), so no step reuses the     */
/*    numbers of the initial seeding or of another step;                     */
/*  - a point that rounding (FP64, or FP32 when round_fp32) puts outside its */
/*    cell, by the exact floor of the binning, is moved one representable    */
/*    value at a time back into the cell;                                    */
/*  - its velocity is the mean of the k particles already in the cell        */
/*    (summed in FP64 in their binned order, then divided by k);             */
/*  - cells with no particle (air) and cells at or above the density are     */
/*    left alone.                                                            */
/* count/start describe the binned particles, whose velocities vx, vy, vz    */
/* are given in binned order. With px_new == NULL only the number of new     */
/* particles is returned. New particles come out in cell order.              */
/* ------------------------------------------------------------------------ */

static double move_into_cell(double x, int i, double dx, int n, int round_fp32)
{
    if (round_fp32) {
        float f = (float)x;
        while (exact_floor_div((double)f, dx, n) < i) f = nextafterf(f, INFINITY);
        while (exact_floor_div((double)f, dx, n) > i) f = nextafterf(f, -INFINITY);
        return (double)f;
    }
    while (exact_floor_div(x, dx, n) < i) x = nextafter(x, INFINITY);
    while (exact_floor_div(x, dx, n) > i) x = nextafter(x, -INFINITY);
    return x;
}

int64_t orc_reseed(const orc_grid* g, int sub, uint64_t seed, int64_t step, int round_fp32,
                   const uint32_t* count, const uint32_t* start, const double* vx, const double* vy,
                   const double* vz, double* px_new, double* py_new, double* pz_new, double* vx_new,
                   double* vy_new, double* vz_new, uint32_t* cell_new)
{
    const int64_t C = n_cells(g);
    const int64_t per_cell = (int64_t)sub * sub * sub;
    int64_t m = 0;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                const int64_t c = cell_index(g, i, j, k);
                const int64_t have = count[c];
                if (have == 0 || have >= per_cell) continue;
                double mean[3] = {0.0, 0.0, 0.0};
                if (px_new) {
                    const double* v[3] = {vx, vy, vz};
                    for (int a = 0; a < 3; ++a) {
                        double sum = 0.0;
                        for (int64_t q = 0; q < have; ++q) sum += v[a][start[c] + q];
                        mean[a] = sum / (double)have;
                        if (round_fp32) mean[a] = (double)(float)mean[a];
                    }
                }
                for (int64_t s = have; s < per_cell; ++s) {
                    if (px_new) {
                        const int sx = (int)(s % sub), sy = (int)((s / sub) % sub), sz = (int)(s / ((int64_t)sub * sub));
                        const uint64_t ctr = 3u * (uint64_t)(per_cell * (C * (step + 1) + c) + s);
                        const double x = ((sx + orc_uniform01(seed, ctr + 0)) / sub + i) * g->dx;
                        const double y = ((sy + orc_uniform01(seed, ctr + 1)) / sub + j) * g->dx;
                        const double z = ((sz + orc_uniform01(seed, ctr + 2)) / sub + k) * g->dx;
                        px_new[m] = move_into_cell(x, i, g->dx, g->nx, round_fp32);
                        py_new[m] = move_into_cell(y, j, g->dx, g->ny, round_fp32);
                        pz_new[m] = move_into_cell(z, k, g->dx, g->nz, round_fp32);
                        vx_new[m] = mean[0];
                        vy_new[m] = mean[1];
                        vz_new[m] = mean[2];
                        cell_new[m] = (uint32_t)c;
                    }
                    ++m;
                }
            }
    return m;
}

/* ------------------------------------------------------------------------ */
/* Surface reconstruction, scalar field (paper Sec. 3.3.1): at every corner  */
/* x of the sampling grid (spacing dx / refine, corners 0 .. n*refine per    */
/* axis) the improved-blobby distance                                        */
/*   phi(x) = | x - sum_i w_i x_i | - sum_i w_i r_i,                         */
/*   w_i = k(|x - x_i| / R) / sum_j k(|x - x_j| / R),  k(s) = max(0,(1-s^2)^3) */
/* over the particles closer than the search radius R, every particle with   */
/* the same radius r. Reading: a corner with no particle closer than R is    */
/* outside and gets phi = R. Written as the definition: every corner against */
/* every particle (the O(m n) form the paper starts from).                   */
/* ------------------------------------------------------------------------ */

static double blobby_kernel(double s)
{
    const double t = 1.0 - s * s;
    return t > 0.0 ? t * t * t : 0.0;
}

void orc_surface_field(const orc_grid* g, int refine, double radius, double search, int64_t n,
                       const double* px, const double* py, const double* pz, double* phi)
{
    const int cx = g->nx * refine + 1, cy = g->ny * refine + 1, cz = g->nz * refine + 1;
    double* kv = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int K = 0; K < cz; ++K)
        for (int J = 0; J < cy; ++J)
            for (int I = 0; I < cx; ++I) {
                const double x[3] = {(double)I * g->dx / refine, (double)J * g->dx / refine,
                                     (double)K * g->dx / refine};
                double ksum = 0.0;
                for (int64_t p = 0; p < n; ++p) {
                    const double d[3] = {x[0] - px[p], x[1] - py[p], x[2] - pz[p]};
                    const double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                    kv[p] = dist < search ? blobby_kernel(dist / search) : 0.0;
                    ksum += kv[p];
                }
                double out = search;
                if (ksum > 0.0) {
                    double xbar[3] = {0.0, 0.0, 0.0}, rbar = 0.0;
                    for (int64_t p = 0; p < n; ++p) {
                        if (kv[p] == 0.0) continue;
                        const double w = kv[p] / ksum;
                        xbar[0] += w * px[p];
                        xbar[1] += w * py[p];
                        xbar[2] += w * pz[p];
                        rbar += w * radius;
                    }
                    const double e[3] = {x[0] - xbar[0], x[1] - xbar[1], x[2] - xbar[2]};
                    out = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]) - rbar;
                }
                phi[I + (int64_t)cx * (J + (int64_t)cy * K)] = out;
            }
    free(kv);
}

/* ------------------------------------------------------------------------ */
/* Marching cubes (paper Sec. 3.3.2). A corner is inside when phi < 0. Each   */
/* grid edge whose two corners differ carries one vertex, at the linearly     */
/* interpolated zero of phi; vertices are numbered in the order of their      */
/* edges, edge id 3 * corner + axis (corner x-fastest, the edge running from  */
/* it in +axis). The paper gives no case table; the triangles of a cube follow */
/* from this rule, applied to each cube directly:                             */
/*  - on each of the cube's six faces, a face with two crossing edges gets a  */
/*    segment joining them; a face with four gets, for each of its inside     */
/*    corners, a segment joining that corner's two edges (inside corners are  */
/*    kept apart);                                                            */
/*  - each segment runs so that the inside corners it cuts off lie on its     */
/*    left seen from outside the cube: (Q - P) x (m - P) . n > 0 for the      */
/*    points P -> Q at the edge midpoints of the unit cube, m the mean of     */
/*    those corners and n the face's outward normal;                          */
/*  - the segments close into loops, each taken from its lowest local edge;   */
/*    local edges: 0-3 along x at (y, z) = (0,0), (1,0), (0,1), (1,1); 4-7    */
/*    along y at (x, z); 8-11 along z at (x, y);                              */
/*  - a loop v0, v1, ..., v(m-1) gives the triangles (v0, v(k+1), v(k)),      */
/*    k = 1 .. m-2, whose normals then point out of the fluid.                */
/* Cubes are taken x-fastest, loops in order of their first edge.             */
/* Vertex normals: the unit normals of the triangles at a vertex, each        */
/* weighted by the inverse of the triangle's area, summed and normalised      */
/* (degenerate triangles skipped; a vertex with none keeps (0, 0, 0)).        */
/* ------------------------------------------------------------------------ */

/* local edge -> its two corners (corner = cx + 2 cy + 4 cz) */
static void mc_edge_corners(int e, int* a, int* b)
{
    const int axis = e / 4, q = e % 4;
    int c0[3];
    if (axis == 0) { c0[0] = 0; c0[1] = q & 1; c0[2] = q >> 1; }
    else if (axis == 1) { c0[0] = q & 1; c0[1] = 0; c0[2] = q >> 1; }
    else { c0[0] = q & 1; c0[1] = q >> 1; c0[2] = 0; }
    *a = c0[0] + 2 * c0[1] + 4 * c0[2];
    c0[axis] = 1;
    *b = c0[0] + 2 * c0[1] + 4 * c0[2];
}

static int mc_edge_of(int a, int b)
{
    for (int e = 0; e < 12; ++e) {
        int p, q;
        mc_edge_corners(e, &p, &q);
        if ((p == a && q == b) || (p == b && q == a)) return e;
    }
    return -1;
}

/* triangles of one cube as local-edge triples; returns their number */
static int mc_cube_triangles(unsigned inside, int tri[][3])
{
    int next[12];
    for (int e = 0; e < 12; ++e) next[e] = -1;
    for (int axis = 0; axis < 3; ++axis)
        for (int side = 0; side < 2; ++side) {
            /* the face's corners in cyclic order */
            const int u = (axis + 1) % 3, v = (axis + 2) % 3;
            int cyc[4];
            const int uv[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
            for (int t = 0; t < 4; ++t) {
                int c[3];
                c[axis] = side;
                c[u] = uv[t][0];
                c[v] = uv[t][1];
                cyc[t] = c[0] + 2 * c[1] + 4 * c[2];
            }
            int ncross = 0;
            for (int t = 0; t < 4; ++t)
                ncross += ((inside >> cyc[t]) & 1) != ((inside >> cyc[(t + 1) % 4]) & 1);
            /* segments: (edge, edge, cut-off corners as a bit set) */
            int seg[2][2], cut[2], nseg = 0;
            if (ncross == 2) {
                int ends[2], k = 0;
                for (int t = 0; t < 4; ++t)
                    if (((inside >> cyc[t]) & 1) != ((inside >> cyc[(t + 1) % 4]) & 1))
                        ends[k++] = mc_edge_of(cyc[t], cyc[(t + 1) % 4]);
                seg[0][0] = ends[0];
                seg[0][1] = ends[1];
                cut[0] = 0;
                for (int t = 0; t < 4; ++t)
                    if ((inside >> cyc[t]) & 1) cut[0] |= 1 << cyc[t];
                nseg = 1;
            } else if (ncross == 4) {
                for (int t = 0; t < 4; ++t)
                    if ((inside >> cyc[t]) & 1) {
                        seg[nseg][0] = mc_edge_of(cyc[(t + 3) % 4], cyc[t]);
                        seg[nseg][1] = mc_edge_of(cyc[t], cyc[(t + 1) % 4]);
                        cut[nseg] = 1 << cyc[t];
                        ++nseg;
                    }
            }
            double n[3] = {0.0, 0.0, 0.0};
            n[axis] = side ? 1.0 : -1.0;
            for (int s = 0; s < nseg; ++s) {
                double P[3], Q[3], m[3] = {0.0, 0.0, 0.0};
                int a, b, cnt = 0;
                mc_edge_corners(seg[s][0], &a, &b);
                for (int d = 0; d < 3; ++d) P[d] = 0.5 * (((a >> d) & 1) + ((b >> d) & 1));
                mc_edge_corners(seg[s][1], &a, &b);
                for (int d = 0; d < 3; ++d) Q[d] = 0.5 * (((a >> d) & 1) + ((b >> d) & 1));
                for (int c = 0; c < 8; ++c)
                    if ((cut[s] >> c) & 1) {
                        for (int d = 0; d < 3; ++d) m[d] += (c >> d) & 1;
                        ++cnt;
                    }
                for (int d = 0; d < 3; ++d) m[d] /= cnt;
                const double dq[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
                const double dm[3] = {m[0] - P[0], m[1] - P[1], m[2] - P[2]};
                const double cr[3] = {dq[1] * dm[2] - dq[2] * dm[1], dq[2] * dm[0] - dq[0] * dm[2],
                                      dq[0] * dm[1] - dq[1] * dm[0]};
                const double side_test = cr[0] * n[0] + cr[1] * n[1] + cr[2] * n[2];
                if (side_test > 0) next[seg[s][0]] = seg[s][1];
                else next[seg[s][1]] = seg[s][0];
            }
        }
    int ntri = 0, seen[12] = {0};
    for (int e = 0; e < 12; ++e) {
        if (next[e] < 0 || seen[e]) continue;
        int loop[12], m = 0, v = e;
        do {
            seen[v] = 1;
            loop[m++] = v;
            v = next[v];
        } while (v != e && v >= 0 && m < 12);
        for (int k = 1; k + 1 < m; ++k) {
            tri[ntri][0] = loop[0];
            tri[ntri][1] = loop[k + 1];
            tri[ntri][2] = loop[k];
            ++ntri;
        }
    }
    return ntri;
}

int orc_mc_case_triangles(unsigned inside, int* tri_edges)
{
    int tri[16][3];
    const int nt = mc_cube_triangles(inside & 255u, tri);
    if (tri_edges)
        for (int t = 0; t < nt; ++t)
            for (int k = 0; k < 3; ++k) tri_edges[3 * t + k] = tri[t][k];
    return nt;
}

/* phi on corners (cx = nx*refine+1 ...), spacing h = dx / refine. Returns the
   vertex count through *nv and the triangle count; with verts == NULL only
   counts. */
int64_t orc_surface_mesh(const orc_grid* g, int refine, const double* phi, double* verts, double* normals,
                         int64_t* tris, int64_t* nv)
{
    const int cx = g->nx * refine + 1, cy = g->ny * refine + 1, cz = g->nz * refine + 1;
    const int64_t ncorner = (int64_t)cx * cy * cz;
    const double h = g->dx / refine;
    int64_t* vid = (int64_t*)malloc(sizeof(int64_t) * (size_t)(3 * ncorner));
    int64_t nvert = 0;
    for (int64_t c = 0; c < ncorner; ++c) {
        const int I = (int)(c % cx), J = (int)((c / cx) % cy), K = (int)(c / ((int64_t)cx * cy));
        const int ijk[3] = {I, J, K}, lim[3] = {cx, cy, cz};
        for (int a = 0; a < 3; ++a) {
            vid[3 * c + a] = -1;
            if (ijk[a] + 1 >= lim[a]) continue;
            const int64_t step = a == 0 ? 1 : (a == 1 ? cx : (int64_t)cx * cy);
            const double f0 = phi[c], f1 = phi[c + step];
            if ((f0 < 0.0) == (f1 < 0.0)) continue;
            if (verts) {
                const double t = f0 / (f0 - f1);
                for (int d = 0; d < 3; ++d) verts[3 * nvert + d] = ijk[d] * h;
                verts[3 * nvert + a] = (ijk[a] + t) * h;
            }
            vid[3 * c + a] = nvert++;
        }
    }
    int64_t ntri = 0;
    for (int K = 0; K + 1 < cz; ++K)
        for (int J = 0; J + 1 < cy; ++J)
            for (int I = 0; I + 1 < cx; ++I) {
                unsigned inside = 0;
                for (int q = 0; q < 8; ++q) {
                    const int64_t c = (I + (q & 1)) + (int64_t)cx * ((J + ((q >> 1) & 1)) + (int64_t)cy * (K + (q >> 2)));
                    if (phi[c] < 0.0) inside |= 1u << q;
                }
                int tri[16][3];
                const int nt = mc_cube_triangles(inside, tri);
                for (int t = 0; t < nt; ++t) {
                    if (tris)
                        for (int k = 0; k < 3; ++k) {
                            int a, b;
                            mc_edge_corners(tri[t][k], &a, &b);
                            const int64_t c = (I + (a & 1)) + (int64_t)cx * ((J + ((a >> 1) & 1)) + (int64_t)cy * (K + (a >> 2)));
                            tris[3 * ntri + k] = vid[3 * c + tri[t][k] / 4];
                        }
                    ++ntri;
                }
            }
    if (verts && normals) {
        for (int64_t v = 0; v < 3 * nvert; ++v) normals[v] = 0.0;
        for (int64_t t = 0; t < ntri; ++t) {
            const double* A = verts + 3 * tris[3 * t];
            const double* B = verts + 3 * tris[3 * t + 1];
            const double* C = verts + 3 * tris[3 * t + 2];
            const double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
            const double w[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
            const double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
            const double len = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
            if (!(len > 0.0)) continue;
            const double area = 0.5 * len;
            for (int k = 0; k < 3; ++k)
                for (int d = 0; d < 3; ++d) normals[3 * tris[3 * t + k] + d] += (cr[d] / len) / area;
        }
        for (int64_t v = 0; v < nvert; ++v) {
            double* nn = normals + 3 * v;
            const double len = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
            if (len > 0.0)
                for (int d = 0; d < 3; ++d) nn[d] /= len;
        }
    }
    free(vid);
    *nv = nvert;
    return ntri;
}
