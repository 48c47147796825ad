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

// A = face component (0: u, 1: v, 2: w)
template <typename T, int A>
__global__ __launch_bounds__(256) void k_p2g(Geo g, const T* __restrict__ px,
                                             const T* __restrict__ py, const T* __restrict__ pz,
                                             const T* __restrict__ vel,
                                             const uint32_t* __restrict__ start,
                                             const uint32_t* __restrict__ count, T accel_dt,
                                             T* __restrict__ out_old, T* __restrict__ out_star)
{
    const int dX = g.nx + (A == 0), dY = g.ny + (A == 1), dZ = g.nz + (A == 2);
    const int64_t F = (int64_t)dX * dY * dZ;
    const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (f >= F) return;
    const int i = (int)(f % dX), j = (int)((f / dX) % dY), k = (int)(f / ((int64_t)dX * dY));
    // sample point in cell units
    const T fx = (T)i + (A == 0 ? T(0) : T(0.5));
    const T fy = (T)j + (A == 1 ? T(0) : T(0.5));
    const T fz = (T)k + (A == 2 ? T(0) : T(0.5));
    const T inv = (T)g.inv_dx;
    // cells whose particles can lie within one cell of the sample point
    const int i0 = max(i - 1, 0), i1 = min(A == 0 ? i : i + 1, g.nx - 1);
    const int j0 = max(j - 1, 0), j1 = min(A == 1 ? j : j + 1, g.ny - 1);
    const int k0 = max(k - 1, 0), k1 = min(A == 2 ? k : k + 1, g.nz - 1);
    T W = T(0), M = T(0);
    for (int kk = k0; kk <= k1; ++kk)
        for (int jj = j0; jj <= j1; ++jj)
            for (int ii = i0; ii <= i1; ++ii) {
                const int64_t c = ii + (int64_t)g.nx * (jj + (int64_t)g.ny * kk);
                const uint32_t s0 = start[c], n = count[c];
                for (uint32_t q = s0; q < s0 + n; ++q) {
                    const T wx = hat(px[q] * inv - fx);
                    const T wy = hat(py[q] * inv - fy);
                    const T wz = hat(pz[q] * inv - fz);
                    const T w = wx * wy * wz;
                    W += w;
                    M = fma(vel[q], w, M);
                }
            }
    const T raw = W > T(0) ? M / W : T(0);
    const int idx = A == 0 ? i : (A == 1 ? j : k);
    const int lim = A == 0 ? g.nx : (A == 1 ? g.ny : g.nz);
    out_old[f] = raw;
    out_star[f] = (idx == 0 || idx == lim) ? T(0) : raw + accel_dt;
}

template <typename T>
void launch_p2g(const Geo& g, int axis, const T* pos, int64_t n, const T* vel_axis,
                const uint32_t* start, const uint32_t* count, T accel_dt, T* out_old, T* out_star,
                hipStream_t st)
{
    const T *px = pos, *py = pos + n, *pz = pos + 2 * n;
    const int64_t F = (int64_t)(g.nx + (axis == 0)) * (g.ny + (axis == 1)) * (g.nz + (axis == 2));
    const dim3 grid((unsigned)((F + 255) / 256)), block(256);
    if (axis == 0)
        hipLaunchKernelGGL((k_p2g<T, 0>), grid, block, 0, st, g, px, py, pz, vel_axis, start, count,
                           accel_dt, out_old, out_star);
    else if (axis == 1)
        hipLaunchKernelGGL((k_p2g<T, 1>), grid, block, 0, st, g, px, py, pz, vel_axis, start, count,
                           accel_dt, out_old, out_star);
    else
        hipLaunchKernelGGL((k_p2g<T, 2>), grid, block, 0, st, g, px, py, pz, vel_axis, start, count,
                           accel_dt, out_old, out_star);
}

template void launch_p2g<float>(const Geo&, int, const float*, int64_t, const float*,
                                const uint32_t*, const uint32_t*, float, float*, float*,
                                hipStream_t);
template void launch_p2g<double>(const Geo&, int, const double*, int64_t, const double*,
                                 const uint32_t*, const uint32_t*, double, double*, double*,
                                 hipStream_t);

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
    const T inv = (T)g.inv_dx;
    const T gx = x * inv - (A == 0 ? T(0) : T(0.5));
    const T gy = y * inv - (A == 1 ? T(0) : T(0.5));
    const T gz = z * inv - (A == 2 ? T(0) : T(0.5));
    const T fx = floor(gx), fy = floor(gy), fz = floor(gz);
    Stencil8<T> s;
    s.tx = gx - fx;
    s.ty = gy - fy;
    s.tz = gz - fz;
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
