// Surface reconstruction, scalar field (paper Sec. 3.3.1): the improved-blobby
// signed distance at the corners of a sampling grid of spacing dx / refine,
//   phi(x) = |x - xbar| - r,  xbar = sum_i w_i x_i,  w_i proportional to
//   k(|x - x_i| / R), k(s) = (1 - s^2)^3 on s < 1,
// every particle having the radius r. The space hash of the binning (cell
// start and count, particles sorted by cell) limits each corner's search to
// the cells that reach within R of it. A corner with no particle closer than R
// gets phi = R (outside).
//
// One thread per corner, corners x-fastest, so the threads of a workgroup walk
// neighbouring cell ranges and share the particles through the caches. The
// sums are taken relative to the corner (xbar - x = sum k (x_i - x) / sum k),
// which keeps them small in FP32.
#include "common.h"
#include "device_util.h"

namespace flipmi {

template <typename T>
__global__ __launch_bounds__(256) void k_surface_field(Geo g, int refine, T radius, double search,
                                                       const uint32_t* __restrict__ start,
                                                       const uint32_t* __restrict__ count,
                                                       const T* __restrict__ pos, int64_t n,
                                                       T* __restrict__ phi)
{
    const int cx = g.nx * refine + 1, cy = g.ny * refine + 1, cz = g.nz * refine + 1;
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= (int64_t)cx * cy * cz) return;
    const int I = (int)(id % cx), J = (int)((id / cx) % cy), K = (int)(id / ((int64_t)cx * cy));
    const double xc[3] = {(double)I * g.dx / refine, (double)J * g.dx / refine, (double)K * g.dx / refine};
    const int nn[3] = {g.nx, g.ny, g.nz};
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = max(0, (int)floor((xc[a] - search) * g.inv_dx));
        hi[a] = min(nn[a] - 1, (int)floor((xc[a] + search) * g.inv_dx));
    }
    const T x = (T)xc[0], y = (T)xc[1], z = (T)xc[2];
    const T R2 = (T)(search * search), inv_R2 = (T)(1.0 / (search * search));
    T ks = 0, sx = 0, sy = 0, sz = 0;
    for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j) {
            const int64_t row = (int64_t)g.nx * (j + (int64_t)g.ny * k);
            // the cells lo[0] .. hi[0] of a row are one run of the sorted particles
            const uint32_t p0 = start[row + lo[0]];
            const uint32_t p1 = start[row + hi[0]] + count[row + hi[0]];
            for (uint32_t p = p0; p < p1; ++p) {
                const T dx = pos[p] - x, dy = pos[n + p] - y, dz = pos[2 * n + p] - z;
                const T d2 = dx * dx + dy * dy + dz * dz;
                if (d2 < R2) {
                    const T t = (T)1 - d2 * inv_R2;
                    const T w = t * t * t;
                    ks += w;
                    sx += w * dx;
                    sy += w * dy;
                    sz += w * dz;
                }
            }
        }
    T out = (T)search;
    if (ks > (T)0) {
        const T ex = sx / ks, ey = sy / ks, ez = sz / ks;
        out = sqrt(ex * ex + ey * ey + ez * ez) - radius;
    }
    phi[id] = out;
}

template <typename T>
void launch_surface_field(const Geo& g, int refine, double radius, double search, const uint32_t* start,
                          const uint32_t* count, const T* pos, int64_t n, T* phi, hipStream_t st)
{
    const int64_t m = (int64_t)(g.nx * refine + 1) * (g.ny * refine + 1) * (g.nz * refine + 1);
    hipLaunchKernelGGL(k_surface_field<T>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, g, refine,
                       (T)radius, search, start, count, pos, n, phi);
}

template void launch_surface_field<float>(const Geo&, int, double, double, const uint32_t*, const uint32_t*,
                                          const float*, int64_t, float*, hipStream_t);
template void launch_surface_field<double>(const Geo&, int, double, double, const uint32_t*, const uint32_t*,
                                           const double*, int64_t, double*, hipStream_t);

}  // namespace flipmi
