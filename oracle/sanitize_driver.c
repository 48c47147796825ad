/*
 * Exercise every entry point of the FP64 oracle on small inputs, for a build
 * under AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure:
 * run by the test suite on the CPU). It composes whole steps the way the
 * Python module does (bin, particle-to-grid, gravity and walls, right-hand
 * side, PCG with both preconditioners, projection, grid-to-particle), plus the
 * CFL rule, reseeding, the surface field and marching cubes, on a ragged grid,
 * with an empty particle set and with particles on the domain's faces.
 * Exit status 0 when every consistency check holds; the sanitizers abort on
 * the first memory or undefined-behaviour error.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "flip_oracle.h"

static int failures = 0;

#define CHECK(cond)                                                            \
    do {                                                                       \
        if (!(cond)) {                                                         \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                        \
        }                                                                      \
    } while (0)

static double* dalloc(int64_t n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

/* one step of the method on particles p (3 x n SoA) and velocities v */
static void one_step(const orc_grid* g, int64_t n, double* p, double* v, int precond, unsigned flags)
{
    const int64_t C = (int64_t)g->nx * g->ny * g->nz;
    uint32_t* key = (uint32_t*)calloc((size_t)(n > 0 ? n : 1), 4);
    uint32_t* count = (uint32_t*)calloc((size_t)C, 4);
    uint32_t* start = (uint32_t*)calloc((size_t)C, 4);
    int64_t* perm = (int64_t*)calloc((size_t)(n > 0 ? n : 1), 8);
    uint8_t* fluid = (uint8_t*)calloc((size_t)C, 1);
    orc_bin(g, n, p, p + n, p + 2 * n, key, count, start, perm);
    int64_t total = 0;
    for (int64_t c = 0; c < C; ++c) total += count[c];
    CHECK(total == n);
    /* move the particles into binned order */
    double* q = dalloc(3 * n);
    double* w = dalloc(3 * n);
    for (int64_t s = 0; s < n; ++s)
        for (int a = 0; a < 3; ++a) {
            q[a * n + s] = p[a * n + perm[s]];
            w[a * n + s] = v[a * n + perm[s]];
        }
    memcpy(p, q, sizeof(double) * (size_t)(3 * n));
    memcpy(v, w, sizeof(double) * (size_t)(3 * n));
    orc_fluid_flags(g, count, fluid);
    double *old[3], *star[3], *nw[3], *wt[3];
    for (int a = 0; a < 3; ++a) {
        const int64_t F = orc_face_count(g, a);
        old[a] = dalloc(F);
        star[a] = dalloc(F);
        nw[a] = dalloc(F);
        wt[a] = dalloc(F);
        orc_p2g(g, a, n, p, p + n, p + 2 * n, v + a * n, old[a], wt[a]);
        memcpy(star[a], old[a], sizeof(double) * (size_t)F);
        orc_forces_walls(g, a, a == 1 ? -9.81 : 0.0, 1.0 / 240, star[a]);
    }
    double* b = dalloc(C);
    double* x = dalloc(C);
    double* div = dalloc(C);
    double* Ax = dalloc(C);
    orc_rhs(g, fluid, star[0], star[1], star[2], 1.0, 1.0 / 240, b);
    orc_divergence(g, star[0], star[1], star[2], div);
    int iters = 0;
    double max_r = 0.0, max_b = 0.0;
    const int st = orc_pcg(g, fluid, b, x, 1e-10, 10000, precond, &iters, &max_r, &max_b);
    CHECK(st == 0);
    orc_apply_A(g, fluid, x, Ax);
    for (int64_t c = 0; c < C; ++c)
        if (fluid[c]) CHECK(Ax[c] - b[c] <= 1e-8 * (max_b > 0 ? max_b : 1.0) && b[c] - Ax[c] <= 1e-8 * (max_b > 0 ? max_b : 1.0));
    for (int a = 0; a < 3; ++a) orc_project(g, a, fluid, x, 1.0, 1.0 / 240, star[a], nw[a]);
    const double* un[3] = {nw[0], nw[1], nw[2]};
    const double* uo[3] = {old[0], old[1], old[2]};
    orc_g2p_advect(g, n, p, p + n, p + 2 * n, v, v + n, v + 2 * n, un, uo, 0.95, 1.0 / 240, flags);
    const double L[3] = {g->nx * g->dx, g->ny * g->dx, g->nz * g->dx};
    for (int a = 0; a < 3; ++a)
        for (int64_t s = 0; s < n; ++s) CHECK(p[a * n + s] > 0.0 && p[a * n + s] < L[a]);
    /* interpolation at and beyond the domain's corners clamps its indices */
    (void)orc_interp(g, 0, nw[0], 0.0, 0.0, 0.0);
    (void)orc_interp(g, 1, nw[1], L[0], L[1], L[2]);
    (void)orc_cfl_dt(n, v, v + n, v + 2 * n, g->dx, 3.0, 1.0 / 240);
    /* reseeding: count first, then write */
    const int64_t m = orc_reseed(g, 2, 7, 0, 1, count, start, v, v + n, v + 2 * n, NULL, NULL, NULL, NULL, NULL,
                                 NULL, NULL);
    double* rp = dalloc(3 * m);
    double* rv = dalloc(3 * m);
    uint32_t* rc = (uint32_t*)calloc((size_t)(m > 0 ? m : 1), 4);
    CHECK(orc_reseed(g, 2, 7, 0, 1, count, start, v, v + n, v + 2 * n, rp, rp + m, rp + 2 * m, rv, rv + m,
                     rv + 2 * m, rc) == m);
    for (int a = 0; a < 3; ++a) {
        free(old[a]);
        free(star[a]);
        free(nw[a]);
        free(wt[a]);
    }
    free(rp);
    free(rv);
    free(rc);
    free(b);
    free(x);
    free(div);
    free(Ax);
    free(q);
    free(w);
    free(key);
    free(count);
    free(start);
    free(perm);
    free(fluid);
}

static void surface(const orc_grid* g, int64_t n, const double* p, int refine)
{
    const int64_t nc = (int64_t)(g->nx * refine + 1) * (g->ny * refine + 1) * (g->nz * refine + 1);
    double* phi = dalloc(nc);
    orc_surface_field(g, refine, 0.5 * g->dx, 2.0 * g->dx, n, p, p + n, p + 2 * n, phi);
    int64_t nv = 0;
    const int64_t nt = orc_surface_mesh(g, refine, phi, NULL, NULL, NULL, &nv);
    double* verts = dalloc(3 * nv);
    double* normals = dalloc(3 * nv);
    int64_t* tris = (int64_t*)calloc((size_t)(3 * nt > 0 ? 3 * nt : 1), 8);
    int64_t nv2 = 0;
    CHECK(orc_surface_mesh(g, refine, phi, verts, normals, tris, &nv2) == nt);
    CHECK(nv2 == nv);
    for (int64_t t = 0; t < 3 * nt; ++t) CHECK(tris[t] >= 0 && tris[t] < nv);
    free(phi);
    free(verts);
    free(normals);
    free(tris);
}

int main(void)
{
    /* every marching-cubes configuration */
    int tri[48];
    for (unsigned c = 0; c < 256; ++c) {
        const int nt = orc_mc_case_triangles(c, tri);
        CHECK(nt >= 0 && nt <= 16);
        for (int k = 0; k < 3 * nt; ++k) CHECK(tri[k] >= 0 && tri[k] < 12);
    }
    CHECK(orc_uniform01(1234567, 0) >= 0.0 && orc_uniform01(1234567, 0) < 1.0);

    /* a ragged grid: a dam block and a falling sphere */
    const orc_grid g = {13, 9, 11, 1.0 / 12};
    orc_region regs[2];
    memset(regs, 0, sizeof regs);
    regs[0].kind = ORC_REGION_BOX;
    regs[0].hi[0] = 0.5;
    regs[0].hi[1] = 0.4;
    regs[0].hi[2] = 1.0;
    regs[1].kind = ORC_REGION_SPHERE;
    regs[1].center[0] = 0.7;
    regs[1].center[1] = 0.5;
    regs[1].center[2] = 0.45;
    regs[1].radius = 0.2;
    regs[1].vel[1] = -1.0;
    const int64_t n = orc_seed(&g, regs, 2, 2, 9, NULL, NULL, NULL, NULL, NULL, NULL);
    CHECK(n > 0 && n % 8 == 0);
    double* p = dalloc(3 * n);
    double* v = dalloc(3 * n);
    CHECK(orc_seed(&g, regs, 2, 2, 9, p, p + n, p + 2 * n, v, v + n, v + 2 * n) == n);
    /* a few particles exactly on the domain's faces and corners */
    p[0] = 0.0;
    p[n + 1] = g.ny * g.dx;
    p[2 * n + 2] = g.nz * g.dx;
    for (int s = 0; s < 3; ++s) {
        one_step(&g, n, p, v, s == 1 ? ORC_PRECOND_JACOBI : ORC_PRECOND_MIC0,
                 s == 2 ? ORC_ADVECT_PARTICLE_VEL : 0u);
    }
    surface(&g, n, p, 1);
    surface(&g, n, p, 2);

    /* no particles at all */
    one_step(&g, 0, p, v, ORC_PRECOND_MIC0, 0u);
    surface(&g, 0, p, 1);

    /* a one-cell grid */
    const orc_grid g1 = {1, 1, 1, 0.5};
    double p1[3] = {0.25, 0.25, 0.25}, v1[3] = {0.0, 0.0, 0.0};
    one_step(&g1, 1, p1, v1, ORC_PRECOND_MIC0, 0u);
    surface(&g1, 1, p1, 3);

    free(p);
    free(v);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitize driver: %lld particles, all checks passed\n", (long long)n);
    return 0;
}
