// Per-step diagnostics of the timestep, all evaluated in FP64 whatever the
// working precision (FLIP_FLAG_DIAGNOSTICS; the divergence kernel also serves
// the FLIP_FIELD_DIV readback):
//   - the discrete divergence of a face field per fluid cell (the face
//     differences of Sec. 3.1.7 over dx) and its largest magnitude, for the
//     projected and the unprojected field: their ratio is what the projection
//     (Eq. (5)) leaves of the divergence;
//   - the particles' kinetic energy 1/2 sum |v|^2 (unit particle mass; the
//     energy the paper tracks over a simulation, Sec. 4) and their largest
//     speed (the CFL number of Sec. 3.1.4 is speed * dt / dx).
// Maxima of non-negative values are folded with atomic maxima on their bit
// patterns (order-independent); the energy sum is formed in a fixed order
// (per-thread strided sums, a fixed tree per workgroup, one workgroup over
// the workgroup partials), so it is the same on every run.
#include <algorithm>

#include "common.h"
#include "device_util.h"

namespace flipmi {

constexpr int DIAG_NT = 256;
constexpr int64_t DIAG_DIV_BLOCKS = 2048;  // workgroups of the divergence kernel at most

// max of two non-negative doubles over the workgroup, thread 0's result
__device__ inline double diag_block_max(double v, double* sh)
{
    return block_max<DIAG_NT>(v, sh);
}

template <typename T>
__global__ __launch_bounds__(DIAG_NT) void k_div_max(Geo g, const uint32_t* __restrict__ count,
                                                     const T* __restrict__ un, const T* __restrict__ vn,
                                                     const T* __restrict__ wn, const T* __restrict__ us,
                                                     const T* __restrict__ vs, const T* __restrict__ ws,
                                                     double* __restrict__ div_out,
                                                     unsigned long long* __restrict__ maxbits)
{
#pragma clang fp contract(off)
    __shared__ double red[DIAG_NT / WAVE];
    const int64_t C = (int64_t)g.nx * g.ny * g.nz;
    double mn = 0.0, ms = 0.0;
    // a bounded grid, each thread striding over cells: one pair of atomic
    // maxima per workgroup (one per cell's worth of workgroups serialised on
    // the two words: 1.5 ms at 256^3)
    for (int64_t c = (int64_t)blockIdx.x * DIAG_NT + threadIdx.x; c < C; c += (int64_t)gridDim.x * DIAG_NT) {
        const int i = (int)(c % g.nx), j = (int)((c / g.nx) % g.ny), k = (int)(c / ((int64_t)g.nx * g.ny));
        // face indices of the cell's low and high faces per component
        const int64_t fu = i + (int64_t)(g.nx + 1) * (j + (int64_t)g.ny * k);
        const int64_t fv = i + (int64_t)g.nx * (j + (int64_t)(g.ny + 1) * k);
        const int64_t fw = c;
        const int64_t su = 1, sv = g.nx, sw = (int64_t)g.nx * g.ny;
        const bool fluid = count[c] > 0;
        const double dn = (((double)un[fu + su] - (double)un[fu]) + ((double)vn[fv + sv] - (double)vn[fv]) +
                           ((double)wn[fw + sw] - (double)wn[fw])) / g.dx;
        if (div_out) div_out[c] = fluid ? dn : 0.0;
        if (fluid) {
            const double ds = (((double)us[fu + su] - (double)us[fu]) + ((double)vs[fv + sv] - (double)vs[fv]) +
                               ((double)ws[fw + sw] - (double)ws[fw])) / g.dx;
            mn = fmax(mn, finite_or_inf(fabs(dn)));
            ms = fmax(ms, finite_or_inf(fabs(ds)));
        }
    }
    if (!maxbits) return;
    mn = diag_block_max(mn, red);
    ms = diag_block_max(ms, red);
    if (threadIdx.x == 0) {
        atomicMax(maxbits, (unsigned long long)__double_as_longlong(mn));
        atomicMax(maxbits + 1, (unsigned long long)__double_as_longlong(ms));
    }
}

template <typename T>
void launch_div_max(const Geo& g, const uint32_t* count, const T* const f_new[3], const T* const f_star[3],
                    double* div_out, unsigned long long* maxbits, hipStream_t st)
{
    const int64_t C = (int64_t)g.nx * g.ny * g.nz;
    if (maxbits) launch_fill_u64((uint64_t*)maxbits, 2, 0ull, st);
    const int64_t groups = std::min<int64_t>((C + DIAG_NT - 1) / DIAG_NT, DIAG_DIV_BLOCKS);
    hipLaunchKernelGGL(k_div_max<T>, dim3((unsigned)std::max<int64_t>(groups, 1)), dim3(DIAG_NT), 0, st, g, count,
                       f_new[0], f_new[1], f_new[2], f_star[0], f_star[1], f_star[2], div_out, maxbits);
}

template void launch_div_max<float>(const Geo&, const uint32_t*, const float* const[3], const float* const[3],
                                    double*, unsigned long long*, hipStream_t);
template void launch_div_max<double>(const Geo&, const uint32_t*, const double* const[3], const double* const[3],
                                     double*, unsigned long long*, hipStream_t);

// 1/2 |v|^2 summed per workgroup into part[blockIdx.x]; max |v|^2 into *speed2
template <typename T>
__global__ __launch_bounds__(DIAG_NT) void k_particle_energy(const T* __restrict__ vx, const T* __restrict__ vy,
                                                             const T* __restrict__ vz, int64_t n,
                                                             double* __restrict__ part,
                                                             unsigned long long* __restrict__ speed2)
{
#pragma clang fp contract(off)
    __shared__ double red[DIAG_NT / WAVE];
    double e = 0.0, m = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * DIAG_NT + threadIdx.x; p < n; p += (int64_t)gridDim.x * DIAG_NT) {
        const double u = vx[p], v = vy[p], w = vz[p];
        const double s2 = (u * u + v * v) + w * w;
        e += 0.5 * s2;
        m = fmax(m, finite_or_inf(s2));
    }
    e = block_sum<DIAG_NT>(e, red);
    m = diag_block_max(m, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = e;
        atomicMax(speed2, (unsigned long long)__double_as_longlong(m));
    }
}

// one workgroup: the partials summed in a fixed order
__global__ __launch_bounds__(DIAG_NT) void k_sum_partials(const double* __restrict__ part, int np,
                                                          double* __restrict__ out)
{
    __shared__ double red[DIAG_NT / WAVE];
    double e = 0.0;
    for (int q = threadIdx.x; q < np; q += DIAG_NT) e += part[q];
    e = block_sum<DIAG_NT>(e, red);
    if (threadIdx.x == 0) *out = e;
}

template <typename T>
void launch_particle_energy(const T* vel, int64_t n, double* part, double* energy, unsigned long long* speed2,
                            hipStream_t st)
{
    launch_fill_u64((uint64_t*)speed2, 1, 0ull, st);
    hipLaunchKernelGGL(k_particle_energy<T>, dim3(DIAG_ENERGY_BLOCKS), dim3(DIAG_NT), 0, st, vel, vel + n,
                       vel + 2 * n, n, part, speed2);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(DIAG_NT), 0, st, part, DIAG_ENERGY_BLOCKS, energy);
}

template void launch_particle_energy<float>(const float*, int64_t, double*, double*, unsigned long long*,
                                            hipStream_t);
template void launch_particle_energy<double>(const double*, int64_t, double*, double*, unsigned long long*,
                                             hipStream_t);

}  // namespace flipmi
