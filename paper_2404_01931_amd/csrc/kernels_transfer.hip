// Particle <-> grid transfers on the staggered MAC grid.
//
// Particle-to-grid (paper Sec. 3.1.6, Eq. (4)) as an LDS splat: the particles
// of a block of cells and its one-cell ring are added into the block's face
// samples in colour phases, so every sample sums its contributions in a fixed
// order (deterministic, no atomics). The kernel also applies the force step
// (gravity, Sec. 2.1.3) and the solid-wall condition (zero normal velocity on
// the six domain faces, Sec. 3.1.7), and keeps the raw transfer for the FLIP
// change.
//
// Grid-to-particle (Sec. 3.1.8) with forward-Euler advection and the skin-width
// clamp (Sec. 3.1.3): one workgroup per tile, face samples staged in LDS.
#include <algorithm>

#include "batch.h"
#include "common.h"
#include "device_util.h"

namespace flipmi {

// Particle-to-grid as an LDS splat, one wave per 10x10x10 block of cells.
//
// The wave owns the block's faces and accumulates their weight sums W and
// weighted velocity sums M in LDS (u: 11x10x10 samples, v: 10x11x10, w:
// 10x10x11; the eleventh layer covers the domain's high side). It scatters
// every particle of the block and of the one-cell ring around it; samples
// outside the block are left to the neighbouring block. A particle of cell c
// only reaches samples within one index of c on each axis, so cells whose
// coordinates agree modulo 3 never reach a common sample: the cells are
// visited in 27 phases, one per residue class (4 x 4 x 4 cells of the 12^3
// ring box, one per lane: the block side is chosen so that every lane has a
// cell in every phase), and within a phase every lane adds to its own
// samples only. Each sample therefore sums its contributions in a fixed
// order (phase, then particle order in the cell): the result is the same on
// every run and - because each weight is rounded once and enters W and M
// unchanged (no contraction) - a uniform power-of-two velocity comes back
// exactly. Hat arguments are formed in double: in float, x / dx carries an
// absolute error of ~1e-6 cells, a large relative error for the small
// weights near the edge of a hat's support.
constexpr int P2G_T = 10;
constexpr int P2G_BOX = (P2G_T + 1) * P2G_T * P2G_T;  // 1100 samples per component

// blocks of the particle-to-grid launch, x fastest
__host__ __device__ inline int p2g_bx(const Geo& g) { return (g.nx + P2G_T - 1) / P2G_T; }
__host__ __device__ inline int p2g_by(const Geo& g) { return (g.ny + P2G_T - 1) / P2G_T; }
__host__ __device__ inline int p2g_bz(const Geo& g) { return (g.nz + P2G_T - 1) / P2G_T; }
int64_t p2g_blocks(const Geo& g) { return (int64_t)p2g_bx(g) * p2g_by(g) * p2g_bz(g); }

// Add to an LDS word without reading it back into the wave (the LDS unit's
// float add, rounded to nearest like the VALU's). Only one lane of a
// workgroup adds to a given sample between two barriers, and a lane's adds
// are applied in its program order, so each sum is still formed in a fixed
// order. Used for FP64 sums (at 256^3: 2.86 ms per step against 3.74 ms with
// read-modify-writes); FP32 sums keep the read-modify-write, which measured
// several times faster than the LDS unit's FP32 add (1.85 against 12.2 ms).
template <typename T>
struct P2GAdd {
    static constexpr bool lds_unit = sizeof(T) == 8;
};
__device__ inline void lds_add(float* a, float v) { __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ inline void lds_add(double* a, double v) { __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }

// The two sample planes of one axis that bracket coordinate x of a particle
// in cell c (the binning's exact floor of x / dx) and their hat weights
// (Eq. (4b)). Face axis (CENTRE false, samples on cell faces): planes c and
// c + 1. Centre axis (samples at cell-centre height, plane p at (p + 1/2) dx):
// planes c - 1 and c below the cell's centre, else c and c + 1. The weight
// of a plane is the distance from x to the other plane of the pair over dx,
// each distance x minus the exact product plane * dx rounded once (fma): a
// weight is zero exactly when the particle lies on the other plane, so every
// face receives a weight exactly when the exact hat is positive, whatever
// the rounding of x / dx (a hat formed as 1 - r with r rounded near 1 could
// vanish, and a face reached only by that particle would flip between 0 and
// the particle's velocity in Eq. (4)). Returns the lower plane.
template <bool CENTRE>
__device__ inline int bracket(double x, int c, double dx, double inv_dx, double& w0, double& w1)
{
    int lo = c;
    if (CENTRE && fma(-((double)c + 0.5), dx, x) < 0.0) lo = c - 1;
    const double off = CENTRE ? 0.5 : 0.0;
    const double below = fma(-((double)lo + off), dx, x);       // x - plane lo
    const double above = fma((double)lo + (1.0 + off), dx, -x);  // plane lo + 1 - x
    w0 = above > 0.0 ? above * inv_dx : 0.0;
    w1 = below > 0.0 ? below * inv_dx : 0.0;
    return lo;
}

template <typename T, int A>
__device__ inline void splat(T (*acc)[2], int x0, int y0, int z0, int cx, int cy, int cz, double x, double y,
                             double z, double dx, double inv_dx, T v)
{
    constexpr int DX = P2G_T + (A == 0), DY = P2G_T + (A == 1), DZ = P2G_T + (A == 2);
    // FP32 (read-modify-write sums): samples outside the block's box get
    // weight 0 and the index of the nearest sample inside it, which lies
    // within one index of the particle's cell and is therefore touched by no
    // other lane of the phase, so every update runs unconditionally (no
    // branch per sample: 1.84 -> 1.77 ms at 256^3) and adding an exact zero
    // leaves a sum unchanged. FP64 (LDS-unit adds) skips those samples
    // instead: there the extra adds cost more than the branches.
    constexpr bool masked = !P2GAdd<T>::lds_unit;
    double wx[2], wy[2], wz[2];
    const int i0 = bracket<A != 0>(x, cx, dx, inv_dx, wx[0], wx[1]) - x0;
    const int j0 = bracket<A != 1>(y, cy, dx, inv_dx, wy[0], wy[1]) - y0;
    const int k0 = bracket<A != 2>(z, cz, dx, inv_dx, wz[0], wz[1]) - z0;
    int li[2], lj[2], lk[2];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        const int i = i0 + d, j = j0 + d, k = k0 + d;
        wx[d] = (i >= 0 && i < DX) ? wx[d] : 0.0;
        wy[d] = (j >= 0 && j < DY) ? wy[d] : 0.0;
        wz[d] = (k >= 0 && k < DZ) ? wz[d] : 0.0;
        li[d] = min(max(i, 0), DX - 1);
        lj[d] = min(max(j, 0), DY - 1);
        lk[d] = min(max(k, 0), DZ - 1);
    }
#pragma unroll
    for (int dk = 0; dk < 2; ++dk)
#pragma unroll
        for (int dj = 0; dj < 2; ++dj)
#pragma unroll
            for (int di = 0; di < 2; ++di) {
                if (!masked && (i0 + di < 0 || i0 + di >= DX || j0 + dj < 0 || j0 + dj >= DY || k0 + dk < 0 ||
                                k0 + dk >= DZ))
                    continue;
                const T w = (T)(wx[di] * wy[dj] * wz[dk]);
                T* a = acc[li[di] + DX * (lj[dj] + DY * lk[dk])];
                if (P2GAdd<T>::lds_unit) {
                    lds_add(a, w);
                    lds_add(a + 1, v * w);
                } else {
                    a[0] = a[0] + w;
                    a[1] = fma(v, w, a[1]);
                }
            }
}

// Particles of one cell, up to P2G_BATCH of them, held in registers: the
// loads of a whole cell are issued together, one colour phase ahead of their
// use, instead of one particle at a time.
constexpr int P2G_BATCH = 8;
static_assert(P2G_BATCH <= PARTICLE_PAD, "particle reads past the last particle need slack");

template <typename T>
struct CellParticles {
    T x[P2G_BATCH], y[P2G_BATCH], z[P2G_BATCH], v[P2G_BATCH];  // position and one velocity component
};

// Eight consecutive values p[s .. s + 7] with 16-byte loads from any 4-byte
// aligned start (a lane's particles are contiguous; one wide load per four
// floats keeps the address unit from issuing one address per particle).
typedef float P2GF4 __attribute__((ext_vector_type(4), aligned(4)));
typedef double P2GD2 __attribute__((ext_vector_type(2), aligned(8)));

__device__ inline void load8(const float* __restrict__ p, uint32_t s, float (&o)[P2G_BATCH])
{
    const P2GF4 a = *(const P2GF4*)(p + s), b = *(const P2GF4*)(p + s + 4);
    o[0] = a.x;
    o[1] = a.y;
    o[2] = a.z;
    o[3] = a.w;
    o[4] = b.x;
    o[5] = b.y;
    o[6] = b.z;
    o[7] = b.w;
}

__device__ inline void load8(const double* __restrict__ p, uint32_t s, double (&o)[P2G_BATCH])
{
#pragma unroll
    for (int k = 0; k < P2G_BATCH; k += 2) {
        const P2GD2 a = *(const P2GD2*)(p + s + k);
        o[k] = a.x;
        o[k + 1] = a.y;
    }
}

// Load particles s .. s + 7 of a cell's range (values past the cell's own
// particles are not used). The state arrays are followed by PARTICLE_PAD
// elements of slack, so the reads stay inside the workspace for any s <= n.
template <typename T>
__device__ inline void load_cell(CellParticles<T>& r, const T* __restrict__ px, const T* __restrict__ py,
                                 const T* __restrict__ pz, const T* __restrict__ vc, uint32_t s)
{
    load8(px, s, r.x);
    load8(py, s, r.y);
    load8(pz, s, r.z);
    load8(vc, s, r.v);
}

// FP32: a lane sums its cell's particles in registers over the cell's
// window of samples of component A (2 along A, where the samples sit on cell
// faces; 3 across it, where they sit at cell-centre height: every particle of
// the cell reaches only these), then adds the window to LDS once per cell.
// Consecutive particles of a cell reach the same samples, and per-particle
// LDS read-modify-writes made each particle wait for the previous one's
// round trip.
template <int A>
struct Window {
    static constexpr int NX = A == 0 ? 2 : 3, NY = A == 1 ? 2 : 3, NZ = A == 2 ? 2 : 3;
    float W[NZ][NY][NX], M[NZ][NY][NX];
};

// the 1D weights of one axis over the window: 2 samples (face axis: c and
// c + 1) or 3 (centre axis: c - 1 .. c + 1, of which the bracketing pair
// gets the weights and the third sample 0). The planes come from the binned
// cell, not from floor(x / dx): with a spacing that is not a power of two,
// x * (1/dx) can land just below the face a particle was binned across.
template <int N>
__device__ inline void axis_weights(double x, int c, double dx, double inv_dx, float (&w)[N])
{
    double w0, w1;
    if (N == 2) {
        (void)bracket<false>(x, c, dx, inv_dx, w0, w1);
        w[0] = (float)w0;
        w[1] = (float)w1;
    } else {
        const bool up = bracket<true>(x, c, dx, inv_dx, w0, w1) == c;
        w[0] = up ? 0.0f : (float)w0;
        w[1] = up ? (float)w0 : (float)w1;
        w[N - 1] = up ? (float)w1 : 0.0f;
    }
}

// The same weights when dx is a power of two, from f = x / dx - c, the
// particle's offset in its binned cell in cell units: x / dx is a scaling by a
// power of two and c <= x / dx < c + 1, so f is exact in FP32, and each weight
// below is its exact value or one rounding of it - the values the FP64
// bracket gives, with FP32 operations. A weight is clamped at 0 as there (a
// non-finite coordinate gets weight 0 everywhere).
template <int N>
__device__ inline void axis_weights_dyadic(float f, float (&w)[N])
{
    if (N == 2) {
        w[0] = fmaxf(1.0f - f, 0.0f);
        w[1] = fmaxf(f, 0.0f);
    } else {
        const bool below = f < 0.5f;  // below the cell's centre: planes c - 1 and c
        w[0] = fmaxf(0.5f - f, 0.0f);
        w[1] = fmaxf(below ? 0.5f + f : 1.5f - f, 0.0f);
        w[N - 1] = fmaxf(f - 0.5f, 0.0f);
    }
}

// the particle's contribution to the window: W += wz wy wx and M += wz wy (v wx)
// for each of the window's samples, each with one fused multiply-add (the x
// weights scaled by v once per particle). With v a power of two, v wx is exact
// and every step of M is v times the same step of W, so M = v W exactly: a
// uniform power-of-two velocity comes back unchanged.
template <int A>
__device__ inline void window_accumulate(Window<A>& win, const float (&wx)[Window<A>::NX],
                                         const float (&wy)[Window<A>::NY], const float (&wz)[Window<A>::NZ],
                                         float v)
{
#pragma clang fp contract(off)
    using Wn = Window<A>;
    float vwx[Wn::NX];
#pragma unroll
    for (int i = 0; i < Wn::NX; ++i) vwx[i] = v * wx[i];
#pragma unroll
    for (int k = 0; k < Wn::NZ; ++k)
#pragma unroll
        for (int j = 0; j < Wn::NY; ++j) {
            const float wyz = wz[k] * wy[j];
#pragma unroll
            for (int i = 0; i < Wn::NX; ++i) {
                win.W[k][j][i] = fma(wyz, wx[i], win.W[k][j][i]);
                win.M[k][j][i] = fma(wyz, vwx[i], win.M[k][j][i]);
            }
        }
}

// dyadic form: fx, fy, fz are the exact in-cell offsets
template <int A>
__device__ inline void window_add_dyadic(Window<A>& win, float fx, float fy, float fz, float v)
{
    using Wn = Window<A>;
    float wx[Wn::NX], wy[Wn::NY], wz[Wn::NZ];
    axis_weights_dyadic<Wn::NX>(fx, wx);
    axis_weights_dyadic<Wn::NY>(fy, wy);
    axis_weights_dyadic<Wn::NZ>(fz, wz);
    window_accumulate<A>(win, wx, wy, wz, v);
}

template <int A>
__device__ inline void window_add(Window<A>& win, int cx, int cy, int cz, double x, double y, double z, double dx,
                                  double inv_dx, float v)
{
#pragma clang fp contract(off)
    using Wn = Window<A>;
    float wx[Wn::NX], wy[Wn::NY], wz[Wn::NZ];
    axis_weights<Wn::NX>(x, cx, dx, inv_dx, wx);
    axis_weights<Wn::NY>(y, cy, dx, inv_dx, wy);
    axis_weights<Wn::NZ>(z, cz, dx, inv_dx, wz);
    window_accumulate<A>(win, wx, wy, wz, v);
}

// add the window of cell (cx, cy, cz) to the block's samples; window samples
// outside the box go to the spare sample acc[P2G_BOX], which no output reads
// (lanes of a phase may race on it; every sample inside the box is touched by
// one lane of the phase only)
template <int A>
__device__ inline void window_flush(const Window<A>& win, float (*acc)[2], int cx, int cy, int cz, int x0, int y0,
                                    int z0)
{
#pragma clang fp contract(off)
    using Wn = Window<A>;
    constexpr int DX = P2G_T + (A == 0), DY = P2G_T + (A == 1), DZ = P2G_T + (A == 2);
    const int bi = cx - x0 - (A == 0 ? 0 : 1), bj = cy - y0 - (A == 1 ? 0 : 1), bk = cz - z0 - (A == 2 ? 0 : 1);
    const int base = bi + DX * (bj + DY * bk);
    bool in_i[Wn::NX], in_j[Wn::NY], in_k[Wn::NZ];
#pragma unroll
    for (int i = 0; i < Wn::NX; ++i) in_i[i] = (unsigned)(bi + i) < (unsigned)DX;
#pragma unroll
    for (int j = 0; j < Wn::NY; ++j) in_j[j] = (unsigned)(bj + j) < (unsigned)DY;
#pragma unroll
    for (int k = 0; k < Wn::NZ; ++k) in_k[k] = (unsigned)(bk + k) < (unsigned)DZ;
    // all reads of a plane of the window, then all writes: samples inside the
    // box are distinct, so only the spare sample can be read after a write
    // of the same flush, and its value is never used
    typedef float F2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int k = 0; k < Wn::NZ; ++k) {
        F2* a[Wn::NY][Wn::NX];
        F2 old[Wn::NY][Wn::NX];
#pragma unroll
        for (int j = 0; j < Wn::NY; ++j)
#pragma unroll
            for (int i = 0; i < Wn::NX; ++i) {
                a[j][i] = (F2*)acc[in_i[i] && in_j[j] && in_k[k] ? base + i + DX * (j + DY * k) : P2G_BOX];
                old[j][i] = *a[j][i];
            }
#pragma unroll
        for (int j = 0; j < Wn::NY; ++j)
#pragma unroll
            for (int i = 0; i < Wn::NX; ++i) {
                F2 v = old[j][i];
                v.x = v.x + win.W[k][j][i];
                v.y = v.y + win.M[k][j][i];
                *a[j][i] = v;
            }
    }
}

// the cell that lane handles in colour phase ph (ring box [r0, r1] per axis),
// or -1 when that position is outside the box
__device__ inline int64_t phase_cell(const Geo& g, int ph, int lane, int rx0, int ry0, int rz0, int rx1, int ry1,
                                     int rz1, int& cx, int& cy, int& cz)
{
    cx = rx0 + ((ph % 3) - rx0 % 3 + 3) % 3 + 3 * (lane & 3);
    cy = ry0 + (((ph / 3) % 3) - ry0 % 3 + 3) % 3 + 3 * ((lane >> 2) & 3);
    cz = rz0 + ((ph / 9) - rz0 % 3 + 3) % 3 + 3 * (lane >> 4);
    if (cx > rx1 || cy > ry1 || cz > rz1) return -1;
    return cx + (int64_t)g.nx * (cy + (int64_t)g.ny * cz);
}

// Whether any 8^3 tile of the binning's tile flags that meets the ring box
// [r0, r1] holds a particle (a box of at most 12 cells per axis meets at most
// 3 tiles per axis; lane t < 27 reads one flag). A block whose ring box holds
// no particle adds nothing to its samples.
__device__ inline bool ring_has_particles(const Geo& g, const uint32_t* __restrict__ tile_flag, int lane, int rx0,
                                          int ry0, int rz0, int rx1, int ry1, int rz1)
{
    const int tx = rx0 / TILE + lane % 3, ty = ry0 / TILE + (lane / 3) % 3, tz = rz0 / TILE + lane / 9;
    bool any = false;
    if (lane < 27 && tx <= rx1 / TILE && ty <= ry1 / TILE && tz <= rz1 / TILE)
        any = tile_flag[tx + (int64_t)g.tx * (ty + (int64_t)g.ty * tz)] != 0u;
    return __ballot(any) != 0;
}

// a particle's offset in its binned cell along one axis, in cells (exact
// when dx is a power of two; see axis_weights_dyadic)
__device__ inline float cell_offset(float x, float inv_dx, int c)
{
#pragma clang fp contract(off)
    return x * inv_dx - (float)c;
}

// A lane's eight floats in LDS, stored as two groups of four whose groups
// for the 64 lanes are contiguous (lane l at p + 4 l and p + 256 + 4 l), so a
// wave's 16-byte reads cover consecutive banks (a lane's eight floats side by
// side would put lanes l and l + 4 on the same banks)
__device__ inline void lds_load8(const float* p, float (&o)[P2G_BATCH])
{
    const float4 a = *(const float4*)p, b = *(const float4*)(p + 4 * 64);
    o[0] = a.x;
    o[1] = a.y;
    o[2] = a.z;
    o[3] = a.w;
    o[4] = b.x;
    o[5] = b.y;
    o[6] = b.z;
    o[7] = b.w;
}

__device__ inline void lds_store8(float* p, const float (&v)[P2G_BATCH])
{
    *(float4*)p = make_float4(v[0], v[1], v[2], v[3]);
    *(float4*)(p + 4 * 64) = make_float4(v[4], v[5], v[6], v[7]);
}

// Coordinates of the phase's particles shared by the workgroup's three waves:
// [buffer][axis][particle group of four][lane][4]; wave A loads axis A of its cell's particles
// (and its own velocity component) and the others read it from LDS, so each
// particle's position is read from memory once per phase instead of three times.
constexpr int P2G_CRD = 2 * 3 * 64 * P2G_BATCH;

// FP32 form of the component wave (see p2g_component): the three waves of the
// workgroup take the phases in step, with a workgroup barrier per phase for
// the shared coordinates.
template <int A, bool DYADIC>
__device__ __forceinline__ void p2g_phases_f32(const Geo& g, int lane, int x0, int y0, int z0, int rx0, int ry0,
                                               int rz0, int rx1, int ry1, int rz1, const float* __restrict__ px,
                                               const float* __restrict__ py, const float* __restrict__ pz,
                                               const float* __restrict__ vc, const uint32_t* __restrict__ start,
                                               const uint32_t* __restrict__ count, float (*acc)[2], float* crd)
{
#pragma clang fp contract(off)
    const float* const pa = A == 0 ? px : (A == 1 ? py : pz);  // the axis this wave loads
    const double inv = g.inv_dx, dx = g.dx;
    const float invf = (float)inv;
    auto row = [&](int buf, int axis) { return crd + (buf * 3 + axis) * 64 * P2G_BATCH + 4 * lane; };
    int cxa, cya, cza, cxb, cyb, czb, cxc, cyc, czc;
    int64_t c = phase_cell(g, 0, lane, rx0, ry0, rz0, rx1, ry1, rz1, cxa, cya, cza);
    uint32_t s_a = start[c >= 0 ? c : 0], n_a = c >= 0 ? count[c] : 0u;
    c = phase_cell(g, 1, lane, rx0, ry0, rz0, rx1, ry1, rz1, cxb, cyb, czb);
    uint32_t s_b = start[c >= 0 ? c : 0], n_b = c >= 0 ? count[c] : 0u;
    float Pv[P2G_BATCH], La[P2G_BATCH];
    load8(pa, s_a, La);
    load8(vc, s_a, Pv);
    lds_store8(row(0, A), La);
    lds_barrier();
#pragma unroll 1
    for (int ph = 0; ph < 27; ++ph) {
        c = phase_cell(g, min(ph + 2, 26), lane, rx0, ry0, rz0, rx1, ry1, rz1, cxc, cyc, czc);
        const uint32_t s_c = start[c >= 0 ? c : 0], n_c = c >= 0 ? count[c] : 0u;
        // the next phase's axis and velocity, in flight while this phase is splatted
        float Qa[P2G_BATCH], Qv[P2G_BATCH];
        load8(pa, s_b, Qa);
        load8(vc, s_b, Qv);
        Window<A> win;
#pragma unroll
        for (int k = 0; k < Window<A>::NZ; ++k)
#pragma unroll
            for (int j = 0; j < Window<A>::NY; ++j)
#pragma unroll
                for (int i = 0; i < Window<A>::NX; ++i) win.W[k][j][i] = win.M[k][j][i] = 0.0f;
        if (n_a > 0) {
            float X[P2G_BATCH], Y[P2G_BATCH], Z[P2G_BATCH];
            lds_load8(row(ph & 1, 0), X);
            lds_load8(row(ph & 1, 1), Y);
            lds_load8(row(ph & 1, 2), Z);
            if constexpr (DYADIC) {
#pragma unroll
                for (int k = 0; k < P2G_BATCH; ++k) {
                    if ((uint32_t)k < n_a)
                        window_add_dyadic<A>(win, cell_offset(X[k], invf, cxa), cell_offset(Y[k], invf, cya),
                                             cell_offset(Z[k], invf, cza), Pv[k]);
                }
                // cells holding more particles than a batch: the rest one by one
                for (uint32_t q = s_a + P2G_BATCH; q < s_a + n_a; ++q)
                    window_add_dyadic<A>(win, cell_offset(px[q], invf, cxa), cell_offset(py[q], invf, cya),
                                         cell_offset(pz[q], invf, cza), vc[q]);
            } else {
#pragma unroll
                for (int k = 0; k < P2G_BATCH; ++k) {
                    if ((uint32_t)k < n_a)
                        window_add<A>(win, cxa, cya, cza, (double)X[k], (double)Y[k], (double)Z[k], dx, inv, Pv[k]);
                }
                for (uint32_t q = s_a + P2G_BATCH; q < s_a + n_a; ++q)
                    window_add<A>(win, cxa, cya, cza, (double)px[q], (double)py[q], (double)pz[q], dx, inv, vc[q]);
            }
            window_flush<A>(win, acc, cxa, cya, cza, x0, y0, z0);
        }
        // the next phase's axis goes to the other buffer, which every wave
        // finished reading before the last barrier
        lds_store8(row((ph + 1) & 1, A), Qa);
        lds_barrier();
        cxa = cxb;
        cya = cyb;
        cza = czb;
        cxb = cxc;
        cyb = cyc;
        czb = czc;
#pragma unroll
        for (int k = 0; k < P2G_BATCH; ++k) Pv[k] = Qv[k];
        s_a = s_b;
        n_a = n_b;
        s_b = s_c;
        n_b = n_c;
    }
}

// One wave of the workgroup: component A of the block's faces. DYADIC: dx is
// a power of two (FP32 hat weights from exact in-cell offsets).
template <typename T, int A, bool DYADIC>
__device__ __forceinline__ void p2g_component(Geo g, int64_t n, int lane, int x0, int y0, int z0,
                                              const T* __restrict__ px, const T* __restrict__ py,
                                              const T* __restrict__ pz, const T* __restrict__ vc,
                                              const uint32_t* __restrict__ start,
                                              const uint32_t* __restrict__ count,
                                              const uint32_t* __restrict__ tile_flag, T gdt, T (*acc)[2],
                                              T* __restrict__ f_old, T* __restrict__ f_star, float* crd)
{
#pragma clang fp contract(off)
    for (int q = lane; q < P2G_BOX * 2; q += 64) (&acc[0][0])[q] = T(0);
    // ring box of cells, clipped to the domain (inclusive bounds)
    const int rx0 = max(x0 - 1, 0), rx1 = min(x0 + P2G_T, g.nx - 1);
    const int ry0 = max(y0 - 1, 0), ry1 = min(y0 + P2G_T, g.ny - 1);
    const int rz0 = max(z0 - 1, 0), rz1 = min(z0 + P2G_T, g.nz - 1);
    const double inv = g.inv_dx, dx = g.dx;
    // (the same decision in the workgroup's three waves: they share barriers)
    const bool work = n > 0 && ring_has_particles(g, tile_flag, lane, rx0, ry0, rz0, rx1, ry1, rz1);
    if constexpr (sizeof(T) == 4) {
        if (work)
            p2g_phases_f32<A, DYADIC>(g, lane, x0, y0, z0, rx0, ry0, rz0, rx1, ry1, rz1, (const float*)px,
                                      (const float*)py, (const float*)pz, (const float*)vc, start, count,
                                      (float (*)[2])acc, crd);
    } else if (work) {
        // Software pipeline over the 27 phases: the cell range of phase
        // ph + 2 and the particles of phase ph + 1 are loaded while phase ph
        // is splatted. The wave's LDS operations run in issue order, so the
        // adds of one phase are in place before the next phase reads them.
        int cxa, cya, cza, cxb, cyb, czb, cxc, cyc, czc;
        int64_t c = phase_cell(g, 0, lane, rx0, ry0, rz0, rx1, ry1, rz1, cxa, cya, cza);
        uint32_t s_a = start[c >= 0 ? c : 0], n_a = c >= 0 ? count[c] : 0u;
        c = phase_cell(g, 1, lane, rx0, ry0, rz0, rx1, ry1, rz1, cxb, cyb, czb);
        uint32_t s_b = start[c >= 0 ? c : 0], n_b = c >= 0 ? count[c] : 0u;
        CellParticles<T> P;
        load_cell(P, px, py, pz, vc, s_a);
#pragma unroll 1
        for (int ph = 0; ph < 27; ++ph) {
            c = phase_cell(g, min(ph + 2, 26), lane, rx0, ry0, rz0, rx1, ry1, rz1, cxc, cyc, czc);
            const uint32_t s_c = start[c >= 0 ? c : 0], n_c = c >= 0 ? count[c] : 0u;
            CellParticles<T> Q;
            load_cell(Q, px, py, pz, vc, s_b);
            {
#pragma unroll
                for (int k = 0; k < P2G_BATCH; ++k) {
                    if ((uint32_t)k < n_a)
                        splat<T, A>(acc, x0, y0, z0, cxa, cya, cza, (double)P.x[k], (double)P.y[k], (double)P.z[k],
                                    dx, inv, P.v[k]);
                }
                for (uint32_t q = s_a + P2G_BATCH; q < s_a + n_a; ++q)
                    splat<T, A>(acc, x0, y0, z0, cxa, cya, cza, (double)px[q], (double)py[q], (double)pz[q], dx,
                                inv, vc[q]);
            }
            __builtin_amdgcn_wave_barrier();
            cxa = cxb;
            cya = cyb;
            cza = czb;
            cxb = cxc;
            cyb = cyc;
            czb = czc;
            P = Q;
            s_a = s_b;
            n_a = n_b;
            s_b = s_c;
            n_b = n_c;
        }
    }
    // write the samples this block owns: [x0, x0+T) on every axis, plus the
    // domain's high side when the block touches it
    const int ex = min(x0 + P2G_T, g.nx), ey = min(y0 + P2G_T, g.ny), ez = min(z0 + P2G_T, g.nz);
    constexpr int DX = P2G_T + (A == 0), DY = P2G_T + (A == 1);
    const int fX = g.nx + (A == 0), fY = g.ny + (A == 1);
    const int lim = A == 0 ? g.nx : (A == 1 ? g.ny : g.nz);
    for (int q = lane; q < P2G_BOX; q += 64) {
        const int li = q % DX, lj = (q / DX) % DY, lk = q / (DX * DY);
        const int i = x0 + li, j = y0 + lj, k = z0 + lk;
        const bool own = (A == 0 ? (i < ex || i == g.nx) : i < ex) && (A == 1 ? (j < ey || j == g.ny) : j < ey) &&
                         (A == 2 ? (k < ez || k == g.nz) : k < ez) && i <= g.nx && j <= g.ny && k <= g.nz;
        if (!own) continue;
        const T W = acc[q][0], M = acc[q][1];
        const T raw = W > T(0) ? M / W : T(0);
        const int idx = A == 0 ? i : (A == 1 ? j : k);
        const int64_t f = i + (int64_t)fX * (j + (int64_t)fY * k);
        f_old[f] = raw;
        f_star[f] = (idx == 0 || idx == lim) ? T(0) : raw + gdt;
    }
}

// Three waves per block, wave a for velocity component a: each wave owns its
// component's samples (no LDS word of the sums is shared), and per wave the
// block's LDS and registers hold one component, which keeps three times as
// many waves resident as one wave doing all three. In FP32 the waves share the
// phase's particle coordinates through LDS (wave a loads axis a), with one
// workgroup barrier per phase; in FP64 each wave loads all three itself.
static_assert(P2G_NT == 3 * 64, "one wave per velocity component");

template <typename T, bool DY>
__device__ __forceinline__ void p2g_body(Blk b, Geo g, int64_t n, const T* __restrict__ px, const T* __restrict__ py,
                                         const T* __restrict__ pz, const T* __restrict__ vx,
                                         const T* __restrict__ vy, const T* __restrict__ vz,
                                         const uint32_t* __restrict__ start,
                                         const uint32_t* __restrict__ count,
                                         const uint32_t* __restrict__ tile_flag, T gdt_x, T gdt_y, T gdt_z,
                                         T* __restrict__ u_old, T* __restrict__ v_old,
                                         T* __restrict__ w_old, T* __restrict__ u_star,
                                         T* __restrict__ v_star, T* __restrict__ w_star,
                                         T (*acc)[P2G_BOX + 1][2], float* crd)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // Rows of blocks (fixed y, z) are dealt to the 8 XCDs in turn (workgroup
    // b runs on XCD b % 8), and an XCD runs its row's blocks in x order, so
    // the ring particles two x-neighbours share are read through one L2; the
    // rows interleave, so the XCDs get a similar share of the work (whole
    // slabs per XCD measured slower for the imbalance). Rows past the last
    // full group of 8 keep the plain order.
    const int nbx = p2g_bx(g), nby = p2g_by(g);
    const int nrows = nby * p2g_bz(g), full = (nrows / 8) * 8 * nbx;
    int L = b.id;
    if (b.id < full) {
        const int x = b.id & 7, k = b.id >> 3;
        L = (x + 8 * (k / nbx)) * nbx + k % nbx;
    }
    const int bx = L % nbx, by = (L / nbx) % nby, bz = L / (nbx * nby);
    const int x0 = bx * P2G_T, y0 = by * P2G_T, z0 = bz * P2G_T;
    if (wv == 0)
        p2g_component<T, 0, DY>(g, n, lane, x0, y0, z0, px, py, pz, vx, start, count, tile_flag, gdt_x, acc[0], u_old, u_star, crd);
    else if (wv == 1)
        p2g_component<T, 1, DY>(g, n, lane, x0, y0, z0, px, py, pz, vy, start, count, tile_flag, gdt_y, acc[1], v_old, v_star, crd);
    else
        p2g_component<T, 2, DY>(g, n, lane, x0, y0, z0, px, py, pz, vz, start, count, tile_flag, gdt_z, acc[2], w_old, w_star, crd);
}

// FP32 particles on a power-of-two spacing take the FP32 weights (the same values)
template <typename T, typename... Args>
__device__ __forceinline__ void p2g_dispatch(Blk b, const Geo& g, Args... args)
{
    __shared__ T acc[3][P2G_BOX + 1][2];  // one LDS block for both forms; a spare sample per component
    __shared__ float crd[sizeof(T) == 4 ? P2G_CRD : 1];  // FP32: the phase's shared coordinates
    if (sizeof(T) == 4 && g.dyadic)
        p2g_body<T, sizeof(T) == 4>(b, g, args..., acc, crd);
    else
        p2g_body<T, false>(b, g, args..., acc, crd);
}

template <typename T>
__global__ __launch_bounds__(P2G_NT) void k_p2g_tiles(Geo g, int64_t n, const T* __restrict__ px,
                                                  const T* __restrict__ py, const T* __restrict__ pz,
                                                  const T* __restrict__ vx, const T* __restrict__ vy,
                                                  const T* __restrict__ vz,
                                                  const uint32_t* __restrict__ start,
                                                  const uint32_t* __restrict__ count,
                                                  const uint32_t* __restrict__ tile_flag, T gdt_x,
                                                  T gdt_y, T gdt_z, T* __restrict__ u_old,
                                                  T* __restrict__ v_old, T* __restrict__ w_old,
                                                  T* __restrict__ u_star, T* __restrict__ v_star,
                                                  T* __restrict__ w_star)
{
    p2g_dispatch<T>(plain_blk(), g, n, px, py, pz, vx, vy, vz, start, count, tile_flag, gdt_x, gdt_y, gdt_z, u_old,
                    v_old, w_old, u_star, v_star, w_star);
}

template <typename T>
__global__ __launch_bounds__(P2G_NT) void kb_p2g_tiles(const P2GArgs<T>* __restrict__ tab,
                                                   const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const P2GArgs<T>& a) {
        p2g_dispatch<T>(b, a.g, a.n, as_global(a.px), as_global(a.py), as_global(a.pz), as_global(a.vx), as_global(a.vy), as_global(a.vz), as_global(a.start), as_global(a.count), as_global(a.tile_flag), a.gdt[0], a.gdt[1], a.gdt[2],
                    as_global(a.old[0]), as_global(a.old[1]), as_global(a.old[2]), as_global(a.star[0]), as_global(a.star[1]), as_global(a.star[2]));
    });
}

template <typename T>
void launch_p2g(const Geo& g, const T* pos, const T* vel, int64_t n, const uint32_t* start,
                const uint32_t* count, const uint32_t* tile_flag, const T gdt[3], T* const old[3],
                T* const star[3], hipStream_t st)
{
    const unsigned tiles = (unsigned)p2g_blocks(g);
    hipLaunchKernelGGL(k_p2g_tiles<T>, dim3(tiles), dim3(P2G_NT), 0, st, g, n, pos, pos + n, pos + 2 * n, vel,
                       vel + n, vel + 2 * n, start, count, tile_flag, gdt[0], gdt[1], gdt[2], old[0], old[1],
                       old[2], star[0], star[1], star[2]);
}

template <typename T>
void launch_b_p2g(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_p2g_tiles<T>, dim3(L.blocks), dim3(P2G_NT), 0, st, (const P2GArgs<T>*)L.args, L.first,
                       L.ns);
}
template void launch_b_p2g<float>(const BatchLaunch&, hipStream_t);
template void launch_b_p2g<double>(const BatchLaunch&, hipStream_t);

template void launch_p2g<float>(const Geo&, const float*, const float*, int64_t, const uint32_t*,
                                const uint32_t*, const uint32_t*, const float[3], float* const[3],
                                float* const[3], hipStream_t);
template void launch_p2g<double>(const Geo&, const double*, const double*, int64_t, const uint32_t*,
                                 const uint32_t*, const uint32_t*, const double[3], double* const[3],
                                 double* const[3], hipStream_t);

// ---------------------------------------------------------------------------
// grid-to-particle, blend, advect, clamp
// ---------------------------------------------------------------------------

// One 256-thread workgroup per 8x8x8 tile. The face samples the tile's
// particles can reach are staged in LDS first, new and old values: the
// tile's own samples plus the layer below on the two axes where samples sit
// at cell-centre height (a particle of cell c reaches samples c and c + 1
// along its component's axis and c - 1 .. c + 1 across it), i.e. a
// 9 x 10 x 10 box for u, 10 x 9 x 10 for v and 10 x 10 x 9 for w, read in
// rows. Box positions outside the domain hold the clamped edge samples, as
// a stencil clamped at the domain edge reads. Then the tile's particles -
// contiguous per x-row of the tile after binning - are processed with their
// stencils read from LDS; the arithmetic is unchanged. A stencil index that
// rounding of x / dx pushes one past the box (a particle within an ulp of a
// cell face) carries weight 0 in FP32 and about 1e-16 in FP64; it is clamped
// into the box.
constexpr int G2P_NT = 256;

template <int A>
struct G2PBox {
    static constexpr int EX = A == 0 ? 9 : 10, EY = A == 1 ? 9 : 10, EZ = A == 2 ? 9 : 10;
    static constexpr int N = EX * EY * EZ;
};
constexpr int G2P_BOX = 900;  // samples per component box
static_assert(G2PBox<0>::N == G2P_BOX && G2PBox<1>::N == G2P_BOX && G2PBox<2>::N == G2P_BOX, "box size");

template <typename T, int A>
__device__ inline void stage_box(const Geo& g, int x0, int y0, int z0, const T* __restrict__ fnew,
                                 const T* __restrict__ fold, T* sn, T* so)
{
    using B = G2PBox<A>;
    const int ox = x0 - (A != 0), oy = y0 - (A != 1), oz = z0 - (A != 2);
    const int dX = g.nx + (A == 0), dY = g.ny + (A == 1), dZ = g.nz + (A == 2);
    for (int q = threadIdx.x; q < B::N; q += G2P_NT) {
        const int lx = q % B::EX, ly = (q / B::EX) % B::EY, lz = q / (B::EX * B::EY);
        const int X = min(max(ox + lx, 0), dX - 1);
        const int Y = min(max(oy + ly, 0), dY - 1);
        const int Z = min(max(oz + lz, 0), dZ - 1);
        const int64_t fidx = X + (int64_t)dX * (Y + (int64_t)dY * Z);
        sn[q] = fnew[fidx];
        so[q] = fold[fidx];
    }
}

template <typename T>
__device__ inline T lerp(T a, T b, T t) { return a + t * (b - a); }

template <typename T>
__device__ inline T trilerp(const T v[8], T tx, T ty, T tz)
{
    const T c00 = lerp(v[0], v[1], tx), c10 = lerp(v[2], v[3], tx);
    const T c01 = lerp(v[4], v[5], tx), c11 = lerp(v[6], v[7], tx);
    return lerp(lerp(c00, c10, ty), lerp(c01, c11, ty), tz);
}

// The lower sample index along one axis and the interpolation weight t of the
// sample above it. CENTRE: samples at cell-centre height (plane p at
// (p + 1/2) dx), else on cell faces. The sample coordinate x / dx - offset is
// formed in double (see the particle-to-grid kernel). DYADIC (FP32, dx a power
// of two): X = x / dx and its fraction f are exact in FP32, and t is f, f - 1/2
// (exact) or f + 1/2 rounded once: the values the double form gives.
template <typename T, bool CENTRE, bool DYADIC>
__device__ inline int sample_coord(const Geo& g, T x, T& t)
{
    if constexpr (DYADIC) {
        const float X = (float)x * (float)g.inv_dx;
        const float c = floorf(X);
        const float f = X - c;
        if (!CENTRE) {
            t = f;
            return (int)c;
        }
        const bool above = f >= 0.5f;  // at or above the cell's centre
        t = above ? f - 0.5f : f + 0.5f;
        return (int)c - (above ? 0 : 1);
    } else {
        const double gx = (double)x * g.inv_dx - (CENTRE ? 0.5 : 0.0);
        const double fx = floor(gx);
        t = (T)(gx - fx);
        return (int)fx;
    }
}

// PIC value and FLIP change of component A at (x, y, z) from the staged box
template <typename T, int A, bool DYADIC>
__device__ inline void sample_box(const Geo& g, int x0, int y0, int z0, const T* sn, const T* so, T x, T y, T z,
                                  T& pic, T& change)
{
    using B = G2PBox<A>;
    T tx, ty, tz;
    const int ix = sample_coord<T, A != 0, DYADIC>(g, x, tx) - (x0 - (A != 0));
    const int iy = sample_coord<T, A != 1, DYADIC>(g, y, ty) - (y0 - (A != 1));
    const int iz = sample_coord<T, A != 2, DYADIC>(g, z, tz) - (z0 - (A != 2));
    const int xa = min(max(ix, 0), B::EX - 1), xb = min(max(ix + 1, 0), B::EX - 1);
    const int ya = min(max(iy, 0), B::EY - 1), yb = min(max(iy + 1, 0), B::EY - 1);
    const int za = min(max(iz, 0), B::EZ - 1), zb = min(max(iz + 1, 0), B::EZ - 1);
    const int r00 = B::EX * (ya + B::EY * za), r10 = B::EX * (yb + B::EY * za);
    const int r01 = B::EX * (ya + B::EY * zb), r11 = B::EX * (yb + B::EY * zb);
    const int idx[8] = {r00 + xa, r00 + xb, r10 + xa, r10 + xb, r01 + xa, r01 + xb, r11 + xa, r11 + xb};
    T vn[8], dv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        vn[q] = sn[idx[q]];
        dv[q] = vn[q] - so[idx[q]];
    }
    pic = trilerp(vn, tx, ty, tz);
    change = trilerp(dv, tx, ty, tz);
}

template <typename T, bool DYADIC>
__device__ __forceinline__ void g2p_body(Blk b, Geo g, const uint32_t* __restrict__ start,
                                         const uint32_t* __restrict__ count, T* __restrict__ px,
                                         T* __restrict__ py, T* __restrict__ pz, T* __restrict__ vx,
                                         T* __restrict__ vy, T* __restrict__ vz, const T* __restrict__ un,
                                         const T* __restrict__ vn, const T* __restrict__ wn,
                                         const T* __restrict__ uo, const T* __restrict__ vo,
                                         const T* __restrict__ wo, T alpha, T dt, T skin, T Lx, T Ly,
                                         T Lz, int advect_particle_vel, uint32_t* __restrict__ nonfinite,
                                         uint32_t* __restrict__ key_out, uint32_t* __restrict__ rank_out,
                                         uint32_t* __restrict__ count_next, uint32_t* __restrict__ tile_next,
                                         T (*box)[2][G2P_BOX], uint32_t* row_start, uint32_t* row_pre)
{
    const int tid = threadIdx.x;
    // the workgroups of one XCD take one contiguous run of tiles, so the face
    // samples a tile shares with its neighbours are mostly read from that
    // XCD's L2 (measured 7% faster than grid order at 256^3)
    const int tile = xcd_remap(b.id, b.n);
    const int bx = tile % g.tx, by = (tile / g.tx) % g.ty, bz = tile / (g.tx * g.ty);
    const int x0 = bx * TILE, y0 = by * TILE, z0 = bz * TILE;
    // the tile's particles: x-row r = (j, k) of the tile holds cells
    // (x0 .. x0+7, y0+j, z0+k), whose particles are contiguous after binning
    if (tid < 64) {
        const int y = y0 + (tid & 7), zc = z0 + (tid >> 3);
        uint32_t s0 = 0, cnt = 0;
        if (y < g.ny && zc < g.nz) {
            const int64_t c0 = x0 + (int64_t)g.nx * (y + (int64_t)g.ny * zc);
            const int64_t c1 = c0 + (min(x0 + TILE, g.nx) - 1 - x0);
            s0 = start[c0];
            cnt = start[c1] + count[c1] - s0;
        }
        uint32_t incl = cnt;  // inclusive scan over the 64 rows (one wave)
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const uint32_t t = __shfl_up(incl, o, WAVE);
            if (tid >= o) incl += t;
        }
        row_start[tid] = s0;
        row_pre[tid + 1] = incl;
        if (tid == 0) row_pre[0] = 0;
    }
    __syncthreads();
    const uint32_t total = row_pre[64];
    if (total == 0) return;
    stage_box<T, 0>(g, x0, y0, z0, un, uo, box[0][0], box[0][1]);
    stage_box<T, 1>(g, x0, y0, z0, vn, vo, box[1][0], box[1][1]);
    stage_box<T, 2>(g, x0, y0, z0, wn, wo, box[2][0], box[2][1]);
    __syncthreads();
    const T L[3] = {Lx, Ly, Lz};
    for (uint32_t fi = tid; fi < total; fi += G2P_NT) {
        int r = 0;  // the row holding the tile's fi-th particle
#pragma unroll
        for (int step = 32; step > 0; step >>= 1)
            if (row_pre[r + step] <= fi) r += step;
        const int64_t p = (int64_t)row_start[r] + (fi - row_pre[r]);
        const T x = px[p], y = py[p], z = pz[p];
        T pic[3], ch[3];
        sample_box<T, 0, DYADIC>(g, x0, y0, z0, box[0][0], box[0][1], x, y, z, pic[0], ch[0]);
        sample_box<T, 1, DYADIC>(g, x0, y0, z0, box[1][0], box[1][1], x, y, z, pic[1], ch[1]);
        sample_box<T, 2, DYADIC>(g, x0, y0, z0, box[2][0], box[2][1], x, y, z, pic[2], ch[2]);
        const T v[3] = {vx[p], vy[p], vz[p]};
        T vnew[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const T flip = v[a] + ch[a];
            vnew[a] = pic[a] + alpha * (flip - pic[a]);
        }
        const T pos[3] = {x, y, z};
        T out[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const T adv = advect_particle_vel ? vnew[a] : pic[a];
            T q = pos[a] + dt * adv;
            q = q < skin ? skin : q;
            q = q > L[a] - skin ? L[a] - skin : q;
            out[a] = q;
        }
        px[p] = out[0];
        py[p] = out[1];
        pz[p] = out[2];
        vx[p] = vnew[0];
        vy[p] = vnew[1];
        vz[p] = vnew[2];
        // latch non-finite particle state for the host (a NaN or an infinity
        // is never clamped back into the domain)
        bool bad = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) bad = bad || !(fabs(out[a]) <= L[a]) || !isfinite(vnew[a]);
        if (bad) atomicOr(nonfinite, 1u);
        // the next step's binning of the position just written (the live
        // lanes of this round are a prefix of the wave, as bin_rank needs)
        if (key_out) {
            int ci, cj, ck;
            bin_cell<T>(g, out[0], out[1], out[2], ci, cj, ck);
            const uint32_t cell = (uint32_t)(ci + (int64_t)g.nx * (cj + (int64_t)g.ny * ck));
            key_out[p] = cell;
            rank_out[p] = bin_rank(g, cell, ci, cj, ck, count_next, tile_next);
        }
    }
}

// FP32 particles on a power-of-two spacing take the FP32 sample coordinates
// (the same values); one set of LDS buffers for both forms
template <typename T, typename... Args>
__device__ __forceinline__ void g2p_dispatch(Blk b, const Geo& g, Args... args)
{
    __shared__ T box[3][2][G2P_BOX];
    __shared__ uint32_t row_start[64];
    __shared__ uint32_t row_pre[65];
    if (sizeof(T) == 4 && g.dyadic)
        g2p_body<T, sizeof(T) == 4>(b, g, args..., box, row_start, row_pre);
    else
        g2p_body<T, false>(b, g, args..., box, row_start, row_pre);
}

template <typename T>
__global__ __launch_bounds__(G2P_NT) void k_g2p(Geo g, const uint32_t* __restrict__ start,
                                                const uint32_t* __restrict__ count, T* __restrict__ px,
                                                T* __restrict__ py, T* __restrict__ pz, T* __restrict__ vx,
                                                T* __restrict__ vy, T* __restrict__ vz,
                                                const T* __restrict__ un, const T* __restrict__ vn,
                                                const T* __restrict__ wn, const T* __restrict__ uo,
                                                const T* __restrict__ vo, const T* __restrict__ wo, T alpha,
                                                T dt, T skin, T Lx, T Ly, T Lz, int advect_particle_vel,
                                                uint32_t* __restrict__ nonfinite, uint32_t* __restrict__ key_out,
                                                uint32_t* __restrict__ rank_out, uint32_t* __restrict__ count_next,
                                                uint32_t* __restrict__ tile_next)
{
    g2p_dispatch<T>(plain_blk(), g, start, count, px, py, pz, vx, vy, vz, un, vn, wn, uo, vo, wo, alpha, dt, skin,
                    Lx, Ly, Lz, advect_particle_vel, nonfinite, key_out, rank_out, count_next, tile_next);
}

template <typename T>
__global__ __launch_bounds__(G2P_NT) void kb_g2p(const G2PArgs<T>* __restrict__ tab,
                                                 const uint32_t* __restrict__ first, int ns)
{
    batch_for_each(tab, first, ns, [&](Blk b, const G2PArgs<T>& a) {
        g2p_dispatch<T>(b, a.g, as_global(a.start), as_global(a.count), as_global(a.px), as_global(a.py),
                    as_global(a.pz), as_global(a.vx), as_global(a.vy), as_global(a.vz), as_global(a.un),
                    as_global(a.vn), as_global(a.wn), as_global(a.uo), as_global(a.vo), as_global(a.wo), a.alpha,
                    a.dt, a.skin, a.Lx, a.Ly, a.Lz, a.advect_particle_vel, as_global(a.nonfinite),
                    (uint32_t*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr);
    });
}

template <typename T>
void launch_b_g2p(const BatchLaunch& L, hipStream_t st)
{
    if (L.blocks == 0) return;
    hipLaunchKernelGGL(kb_g2p<T>, dim3(L.blocks), dim3(G2P_NT), 0, st, (const G2PArgs<T>*)L.args, L.first, L.ns);
}
template void launch_b_g2p<float>(const BatchLaunch&, hipStream_t);
template void launch_b_g2p<double>(const BatchLaunch&, hipStream_t);

template <typename T>
void launch_g2p(const Geo& g, int64_t n, const uint32_t* start, const uint32_t* count, T* pos, T* vel,
                const T* u_new, const T* v_new, const T* w_new, const T* u_old, const T* v_old,
                const T* w_old, T alpha, T dt, int advect_particle_vel, uint32_t* nonfinite, hipStream_t st,
                uint32_t* key_out, uint32_t* rank_out, uint32_t* count_next, uint32_t* tile_next)
{
    if (n <= 0) return;
    const T skin = (T)(1e-3 * g.dx);
    const T Lx = (T)(g.nx * g.dx), Ly = (T)(g.ny * g.dx), Lz = (T)(g.nz * g.dx);
    hipLaunchKernelGGL(k_g2p<T>, dim3((unsigned)tiles_of(g)), dim3(G2P_NT), 0, st, g, start, count, pos,
                       pos + n, pos + 2 * n, vel, vel + n, vel + 2 * n, u_new, v_new, w_new, u_old, v_old,
                       w_old, alpha, dt, skin, Lx, Ly, Lz, advect_particle_vel, nonfinite, key_out, rank_out,
                       count_next, tile_next);
}

template void launch_g2p<float>(const Geo&, int64_t, const uint32_t*, const uint32_t*, float*, float*,
                                const float*, const float*, const float*, const float*, const float*,
                                const float*, float, float, int, uint32_t*, hipStream_t, uint32_t*, uint32_t*,
                                uint32_t*, uint32_t*);
template void launch_g2p<double>(const Geo&, int64_t, const uint32_t*, const uint32_t*, double*, double*,
                                 const double*, const double*, const double*, const double*, const double*,
                                 const double*, double, double, int, uint32_t*, hipStream_t, uint32_t*, uint32_t*,
                                 uint32_t*, uint32_t*);

// ---------------------------------------------------------------------------
// CFL time step (FLIP_FLAG_ADAPTIVE_DT, Sec. 3.1.4): the largest squared
// particle speed, (u^2 + v^2) + w^2 in FP64, folded into *out as the bits of
// a non-negative double (*out cleared first); the host takes the square root.
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_max_speed2(const T* __restrict__ vx, const T* __restrict__ vy,
                                                    const T* __restrict__ vz, int64_t n,
                                                    unsigned long long* __restrict__ out)
{
#pragma clang fp contract(off)
    __shared__ double red[256 / WAVE];
    double m = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const double u = vx[p], v = vy[p], w = vz[p];
        m = fmax(m, (u * u + v * v) + w * w);
    }
    m = block_max<256>(m, red);
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

template <typename T>
void launch_max_speed2(const T* vel, int64_t n, unsigned long long* out, hipStream_t st)
{
    launch_fill_u64((uint64_t*)out, 1, 0ull, st);
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_max_speed2<T>, dim3((unsigned)blocks), dim3(256), 0, st, vel, vel + n, vel + 2 * n, n, out);
}
template void launch_max_speed2<float>(const float*, int64_t, unsigned long long*, hipStream_t);
template void launch_max_speed2<double>(const double*, int64_t, unsigned long long*, hipStream_t);

}  // namespace flipmi
