// Particle <-> grid transfers on the staggered MAC grid.
//
// Particle-to-grid (paper Sec. 3.1.6, Eq. (4)), in the gather form the paper
// uses: one thread per face sample sums over the particles of the cells its
// trilinear hat can reach, in a fixed order, so the result is deterministic and
// needs no atomics. The kernel also applies the force step (gravity, Sec.
// 2.1.3) and the solid-wall condition (zero normal velocity on the six domain
// faces, Sec. 3.1.7), and keeps the raw transfer for the FLIP change.
//
// Grid-to-particle (Sec. 3.1.8) with forward-Euler advection and the skin-width
// clamp (Sec. 3.1.3): one thread per particle in binned order.
#include "common.h"
#include "device_util.h"

namespace flipmi {

template <typename T>
__device__ inline T hat(T r)
{
    T a = T(1) - fabs(r);
    return a > T(0) ? a : T(0);
}

// One thread per cell computes the three faces on the cell's low sides: u at
// (i, j+1/2, k+1/2), v at (i+1/2, j, k+1/2), w at (i+1/2, j+1/2, k) (cell
// units). Their hats can only reach particles of the 3x3x3 cells around the
// cell; neighbour cell (i+di, j+dj, k+dk) can feed u only if di <= 0, v only if
// dj <= 0 and w only if dk <= 0, which the unrolled loops resolve at compile
// time. Each weight is rounded once and the same value enters both sums (no
// contraction of products into the additions), so a uniform power-of-two
// velocity comes back exactly. The faces on the domain's high sides
// (i = nx, j = ny, k = nz) are done by k_p2g_high_faces.
template <typename T>
__global__ __launch_bounds__(256) void k_p2g_cells(Geo g, const T* __restrict__ px,
                                                   const T* __restrict__ py, const T* __restrict__ pz,
                                                   const T* __restrict__ vx, const T* __restrict__ vy,
                                                   const T* __restrict__ vz,
                                                   const uint32_t* __restrict__ start,
                                                   const uint32_t* __restrict__ count, T gdt_x,
                                                   T gdt_y, T gdt_z, T* __restrict__ u_old,
                                                   T* __restrict__ v_old, T* __restrict__ w_old,
                                                   T* __restrict__ u_star, T* __restrict__ v_star,
                                                   T* __restrict__ w_star)
{
    // block = 8 x 8 x 4 cells, one wave per z layer
    const int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
    const int t = threadIdx.x;
    const int i = bx * 8 + (t & 7), j = by * 8 + ((t >> 3) & 7), k = bz * 4 + (t >> 6);
    if (i >= g.nx || j >= g.ny || k >= g.nz) return;
    // hat arguments are formed in double: in float, x / dx carries an absolute
    // error of ~1e-6 cells, which is a large relative error in the small
    // weights of particles near the edge of a hat's support
    const double inv = g.inv_dx;

    uint32_t cs[27], cn[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        const int ii = i + (q % 3) - 1, jj = j + ((q / 3) % 3) - 1, kk = k + (q / 9) - 1;
        const bool in = ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny && kk >= 0 && kk < g.nz;
        const int64_t c = in ? ii + (int64_t)g.nx * (jj + (int64_t)g.ny * kk) : 0;
        cn[q] = in ? count[c] : 0u;
        cs[q] = in ? start[c] : 0u;
    }

    T Wu = T(0), Mu = T(0), Wv = T(0), Mv = T(0), Ww = T(0), Mw = T(0);
    {
#pragma clang fp contract(off)
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            const int di = (q % 3) - 1, dj = ((q / 3) % 3) - 1, dk = (q / 9) - 1;
            const bool fu = di <= 0, fv = dj <= 0, fw = dk <= 0;
            if (!(fu || fv || fw)) continue;
            for (uint32_t p = cs[q]; p < cs[q] + cn[q]; ++p) {
                const double gx = (double)px[p] * inv - i, gy = (double)py[p] * inv - j,
                             gz = (double)pz[p] * inv - k;
                // node-aligned and centre-aligned hats on each axis
                const double xn = hat(gx), xc = hat(gx - 0.5);
                const double yn = hat(gy), yc = hat(gy - 0.5);
                const double zn = hat(gz), zc = hat(gz - 0.5);
                if (fu) {
                    const T w = (T)(xn * yc * zc);
                    Wu = Wu + w;
                    Mu = fma(vx[p], w, Mu);
                }
                if (fv) {
                    const T w = (T)(xc * yn * zc);
                    Wv = Wv + w;
                    Mv = fma(vy[p], w, Mv);
                }
                if (fw) {
                    const T w = (T)(xc * yc * zn);
                    Ww = Ww + w;
                    Mw = fma(vz[p], w, Mw);
                }
            }
        }
    }
    const T ru = Wu > T(0) ? Mu / Wu : T(0);
    const T rv = Wv > T(0) ? Mv / Wv : T(0);
    const T rw = Ww > T(0) ? Mw / Ww : T(0);
    const int64_t fu = i + (int64_t)(g.nx + 1) * (j + (int64_t)g.ny * k);
    const int64_t fv = i + (int64_t)g.nx * (j + (int64_t)(g.ny + 1) * k);
    const int64_t fw = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
    u_old[fu] = ru;
    v_old[fv] = rv;
    w_old[fw] = rw;
    // gravity on every face, then zero normal velocity on the walls
    u_star[fu] = i == 0 ? T(0) : ru + gdt_x;
    v_star[fv] = j == 0 ? T(0) : rv + gdt_y;
    w_star[fw] = k == 0 ? T(0) : rw + gdt_z;
}

// Faces on the domain's high sides (u at i = nx, v at j = ny, w at k = nz):
// one thread per face, gathering from the cells its hat can reach.
template <typename T, int A>
__global__ __launch_bounds__(256) void k_p2g_high_faces(Geo g, const T* __restrict__ px,
                                                        const T* __restrict__ py,
                                                        const T* __restrict__ pz,
                                                        const T* __restrict__ vel,
                                                        const uint32_t* __restrict__ start,
                                                        const uint32_t* __restrict__ count,
                                                        T* __restrict__ out_old,
                                                        T* __restrict__ out_star)
{
    // the plane is indexed by the two other axes (a, b)
    const int na = A == 0 ? g.ny : g.nx, nb = A == 2 ? g.ny : g.nz;
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= (int64_t)na * nb) return;
    const int a = (int)(m % na), b = (int)(m / na);
    const int i = A == 0 ? g.nx : a;
    const int j = A == 1 ? g.ny : (A == 0 ? a : b);
    const int k = A == 2 ? g.nz : b;
    const double fx = i + (A == 0 ? 0.0 : 0.5);
    const double fy = j + (A == 1 ? 0.0 : 0.5);
    const double fz = k + (A == 2 ? 0.0 : 0.5);
    const double inv = g.inv_dx;
    const int i0 = max(i - 1, 0), i1 = min(A == 0 ? i : i + 1, g.nx - 1);
    const int j0 = max(j - 1, 0), j1 = min(A == 1 ? j : j + 1, g.ny - 1);
    const int k0 = max(k - 1, 0), k1 = min(A == 2 ? k : k + 1, g.nz - 1);
    T W = T(0), M = T(0);
    {
#pragma clang fp contract(off)
        for (int kk = k0; kk <= k1; ++kk)
            for (int jj = j0; jj <= j1; ++jj)
                for (int ii = i0; ii <= i1; ++ii) {
                    const int64_t c = ii + (int64_t)g.nx * (jj + (int64_t)g.ny * kk);
                    const uint32_t s0 = start[c], n = count[c];
                    for (uint32_t q = s0; q < s0 + n; ++q) {
                        const T w = (T)(hat((double)px[q] * inv - fx) * hat((double)py[q] * inv - fy) *
                                        hat((double)pz[q] * inv - fz));
                        W = W + w;
                        M = fma(vel[q], w, M);
                    }
                }
    }
    const int dX = g.nx + (A == 0), dY = g.ny + (A == 1);
    const int64_t f = i + (int64_t)dX * (j + (int64_t)dY * k);
    out_old[f] = W > T(0) ? M / W : T(0);
    out_star[f] = T(0);  // wall
}

template <typename T>
void launch_p2g(const Geo& g, const T* pos, const T* vel, int64_t n, const uint32_t* start,
                const uint32_t* count, const T gdt[3], T* const old[3], T* const star[3],
                hipStream_t st)
{
    const dim3 grid((unsigned)((g.nx + 7) / 8), (unsigned)((g.ny + 7) / 8), (unsigned)((g.nz + 3) / 4));
    hipLaunchKernelGGL(k_p2g_cells<T>, grid, dim3(256), 0, st, g, pos, pos + n, pos + 2 * n, vel,
                       vel + n, vel + 2 * n, start, count, gdt[0], gdt[1], gdt[2], old[0], old[1],
                       old[2], star[0], star[1], star[2]);
    const int64_t planes[3] = {(int64_t)g.ny * g.nz, (int64_t)g.nx * g.nz, (int64_t)g.nx * g.ny};
    hipLaunchKernelGGL((k_p2g_high_faces<T, 0>), dim3((unsigned)((planes[0] + 255) / 256)), dim3(256),
                       0, st, g, pos, pos + n, pos + 2 * n, vel, start, count, old[0], star[0]);
    hipLaunchKernelGGL((k_p2g_high_faces<T, 1>), dim3((unsigned)((planes[1] + 255) / 256)), dim3(256),
                       0, st, g, pos, pos + n, pos + 2 * n, vel + n, start, count, old[1], star[1]);
    hipLaunchKernelGGL((k_p2g_high_faces<T, 2>), dim3((unsigned)((planes[2] + 255) / 256)), dim3(256),
                       0, st, g, pos, pos + n, pos + 2 * n, vel + 2 * n, start, count, old[2], star[2]);
}

template void launch_p2g<float>(const Geo&, const float*, const float*, int64_t, const uint32_t*,
                                const uint32_t*, const float[3], float* const[3], float* const[3],
                                hipStream_t);
template void launch_p2g<double>(const Geo&, const double*, const double*, int64_t, const uint32_t*,
                                 const uint32_t*, const double[3], double* const[3],
                                 double* const[3], hipStream_t);

// ---------------------------------------------------------------------------
// grid-to-particle, blend, advect, clamp
// ---------------------------------------------------------------------------

template <typename T>
struct Stencil8 {
    int64_t idx[8];  // (x0,y0,z0) (x1,y0,z0) (x0,y1,z0) (x1,y1,z0) then z1
    T tx, ty, tz;
};

// eight face samples around position (x, y, z) for component A, indices
// clamped to the valid range at the domain edge
template <typename T, int A>
__device__ inline Stencil8<T> stencil(const Geo& g, T x, T y, T z)
{
    const int dX = g.nx + (A == 0), dY = g.ny + (A == 1), dZ = g.nz + (A == 2);
    // sample coordinates in double (see the particle-to-grid kernel)
    const double gx = (double)x * g.inv_dx - (A == 0 ? 0.0 : 0.5);
    const double gy = (double)y * g.inv_dx - (A == 1 ? 0.0 : 0.5);
    const double gz = (double)z * g.inv_dx - (A == 2 ? 0.0 : 0.5);
    const double fx = floor(gx), fy = floor(gy), fz = floor(gz);
    Stencil8<T> s;
    s.tx = (T)(gx - fx);
    s.ty = (T)(gy - fy);
    s.tz = (T)(gz - fz);
    const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    const int x0 = min(max(ix, 0), dX - 1), x1 = min(max(ix + 1, 0), dX - 1);
    const int y0 = min(max(iy, 0), dY - 1), y1 = min(max(iy + 1, 0), dY - 1);
    const int z0 = min(max(iz, 0), dZ - 1), z1 = min(max(iz + 1, 0), dZ - 1);
    const int64_t r00 = (int64_t)dX * (y0 + (int64_t)dY * z0), r10 = (int64_t)dX * (y1 + (int64_t)dY * z0);
    const int64_t r01 = (int64_t)dX * (y0 + (int64_t)dY * z1), r11 = (int64_t)dX * (y1 + (int64_t)dY * z1);
    s.idx[0] = r00 + x0;
    s.idx[1] = r00 + x1;
    s.idx[2] = r10 + x0;
    s.idx[3] = r10 + x1;
    s.idx[4] = r01 + x0;
    s.idx[5] = r01 + x1;
    s.idx[6] = r11 + x0;
    s.idx[7] = r11 + x1;
    return s;
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

template <typename T, int A>
__device__ inline void sample(const Geo& g, const T* __restrict__ fnew, const T* __restrict__ fold,
                              T x, T y, T z, T& pic, T& change)
{
    const Stencil8<T> s = stencil<T, A>(g, x, y, z);
    T vn[8], dv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        vn[q] = fnew[s.idx[q]];
        dv[q] = vn[q] - fold[s.idx[q]];
    }
    pic = trilerp(vn, s.tx, s.ty, s.tz);
    change = trilerp(dv, s.tx, s.ty, s.tz);
}

template <typename T>
__global__ __launch_bounds__(256) void k_g2p(Geo g, int64_t n, T* __restrict__ px,
                                             T* __restrict__ py, T* __restrict__ pz,
                                             T* __restrict__ vx, T* __restrict__ vy,
                                             T* __restrict__ vz, const T* __restrict__ un,
                                             const T* __restrict__ vn, const T* __restrict__ wn,
                                             const T* __restrict__ uo, const T* __restrict__ vo,
                                             const T* __restrict__ wo, T alpha, T dt, T skin,
                                             T Lx, T Ly, T Lz, int advect_particle_vel)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const T x = px[p], y = py[p], z = pz[p];
    T pic[3], ch[3];
    sample<T, 0>(g, un, uo, x, y, z, pic[0], ch[0]);
    sample<T, 1>(g, vn, vo, x, y, z, pic[1], ch[1]);
    sample<T, 2>(g, wn, wo, x, y, z, pic[2], ch[2]);
    const T v[3] = {vx[p], vy[p], vz[p]};
    T vnew[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T flip = v[a] + ch[a];
        vnew[a] = pic[a] + alpha * (flip - pic[a]);
    }
    const T L[3] = {Lx, Ly, Lz};
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
}

template <typename T>
void launch_g2p(const Geo& g, int64_t n, T* pos, T* vel, const T* u_new, const T* v_new,
                const T* w_new, const T* u_old, const T* v_old, const T* w_old, T alpha, T dt,
                int advect_particle_vel, hipStream_t st)
{
    if (n <= 0) return;
    const T skin = (T)(1e-3 * g.dx);
    const T Lx = (T)(g.nx * g.dx), Ly = (T)(g.ny * g.dx), Lz = (T)(g.nz * g.dx);
    hipLaunchKernelGGL(k_g2p<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, n, pos,
                       pos + n, pos + 2 * n, vel, vel + n, vel + 2 * n, u_new, v_new, w_new, u_old,
                       v_old, w_old, alpha, dt, skin, Lx, Ly, Lz, advect_particle_vel);
}

template void launch_g2p<float>(const Geo&, int64_t, float*, float*, const float*, const float*,
                                const float*, const float*, const float*, const float*, float,
                                float, int, hipStream_t);
template void launch_g2p<double>(const Geo&, int64_t, double*, double*, const double*,
                                 const double*, const double*, const double*, const double*,
                                 const double*, double, double, int, hipStream_t);

}  // namespace flipmi
