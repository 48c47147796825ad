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
        // particles with x - R < x_p < x + R: cells floor((x - R) / dx) up to
        // ceil((x + R) / dx) - 1 (a particle at x + R or beyond is out of reach)
        lo[a] = max(0, (int)floor((xc[a] - search) * g.inv_dx));
        hi[a] = min(nn[a] - 1, (int)ceil((xc[a] + search) * g.inv_dx) - 1);
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


// ---------------------------------------------------------------------------
// Marching cubes (paper Sec. 3.3.2). A corner is inside when phi < 0; each
// grid edge whose corners differ carries one vertex at the linear zero of phi.
// Edge id 3 * corner + axis (the edge leaving the corner in +axis), vertices
// numbered in edge order (a scan of the crossing flags); cubes x-fastest,
// their triangles counted, scanned and written from a case table.
//
// The case table follows one rule (the paper prints none): on each cube face,
// two crossing edges are joined by a segment; a face with four crossings gets
// one segment per inside corner, joining that corner's two edges; a segment is
// directed so that the inside corners it cuts off lie on its left seen from
// outside the cube; the segments close into loops, each started at its lowest
// local edge, and a loop v0 .. v(m-1) gives triangles (v0, v(k+1), v(k)),
// whose normals point out of the fluid. Local corner q = x + 2y + 4z; local
// edges 0-3 along x at (y, z) = (0,0), (1,0), (0,1), (1,1), 4-7 along y at
// (x, z), 8-11 along z at (x, y).
// ---------------------------------------------------------------------------

namespace {

struct EdgeEnds {
    int a, b;  // local corners, a at the low end
};

EdgeEnds local_edge(int e)
{
    const int axis = e >> 2, q = e & 3;
    int c[3];
    c[axis] = 0;
    c[axis == 0 ? 1 : 0] = q & 1;
    c[axis == 2 ? 1 : 2] = q >> 1;
    const int a = c[0] | (c[1] << 1) | (c[2] << 2);
    return {a, a | (1 << axis)};
}

int edge_between(int p, int q)
{
    for (int e = 0; e < 12; ++e) {
        const EdgeEnds E = local_edge(e);
        if ((E.a == p && E.b == q) || (E.a == q && E.b == p)) return e;
    }
    return -1;
}

// twice the edge midpoint, integer coordinates 0 .. 2
void mid2(int e, int m[3])
{
    const EdgeEnds E = local_edge(e);
    for (int d = 0; d < 3; ++d) m[d] = ((E.a >> d) & 1) + ((E.b >> d) & 1);
}

McTable build_mc_table()
{
    McTable t{};
    for (int inside = 0; inside < 256; ++inside) {
        int succ[12];
        for (int& s : succ) s = -1;
        for (int f = 0; f < 6; ++f) {
            const int axis = f >> 1, side = f & 1;
            const int u = (axis + 1) % 3, v = (axis + 2) % 3;
            // corners of the face, walked around its edge
            int ring[4];
            const int walk[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
            for (int r = 0; r < 4; ++r)
                ring[r] = (side << axis) | (walk[r][0] << u) | (walk[r][1] << v);
            auto in = [&](int q) { return (inside >> q) & 1; };
            int cross = 0;
            for (int r = 0; r < 4; ++r) cross += in(ring[r]) != in(ring[(r + 1) & 3]);
            struct Seg {
                int e0, e1, cut;
            } segs[2];
            int ns = 0;
            if (cross == 2) {
                Seg s{-1, -1, 0};
                for (int r = 0; r < 4; ++r) {
                    if (in(ring[r])) s.cut |= 1 << ring[r];
                    if (in(ring[r]) != in(ring[(r + 1) & 3])) {
                        const int e = edge_between(ring[r], ring[(r + 1) & 3]);
                        if (s.e0 < 0) s.e0 = e;
                        else s.e1 = e;
                    }
                }
                segs[ns++] = s;
            } else if (cross == 4) {
                for (int r = 0; r < 4; ++r)
                    if (in(ring[r]))
                        segs[ns++] = {edge_between(ring[(r + 3) & 3], ring[r]), edge_between(ring[r], ring[(r + 1) & 3]),
                                      1 << ring[r]};
            }
            for (int k = 0; k < ns; ++k) {
                // left-of test in integers: (Q - P) x (cnt * 2m - cnt... ) . n with
                // coordinates doubled and the corner mean scaled by its count
                int P[3], Q[3], sum[3] = {0, 0, 0}, cnt = 0;
                mid2(segs[k].e0, P);
                mid2(segs[k].e1, Q);
                for (int q = 0; q < 8; ++q)
                    if ((segs[k].cut >> q) & 1) {
                        for (int d = 0; d < 3; ++d) sum[d] += 2 * ((q >> d) & 1);
                        ++cnt;
                    }
                int dq[3], dm[3];
                for (int d = 0; d < 3; ++d) {
                    dq[d] = Q[d] - P[d];
                    dm[d] = sum[d] - cnt * P[d];
                }
                const int c_axis = dq[(axis + 1) % 3] * dm[(axis + 2) % 3] - dq[(axis + 2) % 3] * dm[(axis + 1) % 3];
                const int along = side ? c_axis : -c_axis;
                if (along > 0) succ[segs[k].e0] = segs[k].e1;
                else succ[segs[k].e1] = segs[k].e0;
            }
        }
        bool done[12] = {};
        int nt = 0;
        for (int e = 0; e < 12; ++e) {
            if (succ[e] < 0 || done[e]) continue;
            int loop[12], m = 0;
            for (int w = e; w >= 0 && !done[w] && m < 12; w = succ[w]) {
                done[w] = true;
                loop[m++] = w;
            }
            for (int k = 1; k + 1 < m; ++k) {
                t.edge[inside][3 * nt + 0] = (int8_t)loop[0];
                t.edge[inside][3 * nt + 1] = (int8_t)loop[k + 1];
                t.edge[inside][3 * nt + 2] = (int8_t)loop[k];
                ++nt;
            }
        }
        t.ntri[inside] = (uint8_t)nt;
    }
    return t;
}

}  // namespace

const McTable& mc_table()
{
    static const McTable t = build_mc_table();
    return t;
}

template <typename T>
__global__ __launch_bounds__(256) void k_mc_edge_flags(const T* __restrict__ phi, int cx, int cy, int cz,
                                                       uint32_t* __restrict__ flag)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= (int64_t)cx * cy * cz) return;
    const int I = (int)(c % cx), J = (int)((c / cx) % cy), K = (int)(c / ((int64_t)cx * cy));
    const bool in0 = phi[c] < (T)0;
    flag[3 * c + 0] = (I + 1 < cx) && ((phi[c + 1] < (T)0) != in0);
    flag[3 * c + 1] = (J + 1 < cy) && ((phi[c + cx] < (T)0) != in0);
    flag[3 * c + 2] = (K + 1 < cz) && ((phi[c + (int64_t)cx * cy] < (T)0) != in0);
}

template <typename T>
__device__ inline unsigned cube_case(const T* __restrict__ phi, int64_t c, int cx, int cy)
{
    const int64_t s[8] = {0, 1, cx, cx + 1, (int64_t)cx * cy, (int64_t)cx * cy + 1, (int64_t)cx * cy + cx,
                          (int64_t)cx * cy + cx + 1};
    unsigned m = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) m |= (phi[c + s[q]] < (T)0 ? 1u : 0u) << q;
    return m;
}

template <typename T>
__global__ __launch_bounds__(256) void k_mc_cube_counts(const T* __restrict__ phi, int cx, int cy, int cz,
                                                        const McTable* __restrict__ tab, uint32_t* __restrict__ cnt)
{
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int bx = cx - 1, by = cy - 1;
    if (id >= (int64_t)bx * by * (cz - 1)) return;
    const int I = (int)(id % bx), J = (int)((id / bx) % by), K = (int)(id / ((int64_t)bx * by));
    cnt[id] = tab->ntri[cube_case(phi, I + (int64_t)cx * (J + (int64_t)cy * K), cx, cy)];
}

__global__ void k_mc_totals(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ vidx, int64_t ne,
                            const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ toff, int64_t nc,
                            uint32_t* __restrict__ out)
{
    if (threadIdx.x == 0) {
        out[0] = ne > 0 ? vidx[ne - 1] + flag[ne - 1] : 0u;
        out[1] = nc > 0 ? toff[nc - 1] + cnt[nc - 1] : 0u;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_mc_vertices(const T* __restrict__ phi, int cx, int cy, int cz, double h,
                                                     const uint32_t* __restrict__ flag,
                                                     const uint32_t* __restrict__ vidx, T* __restrict__ verts,
                                                     T* __restrict__ normals)
{
#pragma clang fp contract(off)
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= (int64_t)cx * cy * cz) return;
    const int ijk[3] = {(int)(c % cx), (int)((c / cx) % cy), (int)(c / ((int64_t)cx * cy))};
    const int64_t step[3] = {1, cx, (int64_t)cx * cy};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!flag[3 * c + a]) continue;
        const T f0 = phi[c], f1 = phi[c + step[a]];
        const T t = f0 / (f0 - f1);
        const int64_t v = vidx[3 * c + a];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            verts[3 * v + d] = d == a ? (T)(((T)ijk[d] + t) * (T)h) : (T)((T)ijk[d] * (T)h);
            normals[3 * v + d] = (T)0;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_mc_triangles(const T* __restrict__ phi, int cx, int cy, int cz,
                                                      const McTable* __restrict__ tab,
                                                      const uint32_t* __restrict__ toff,
                                                      const uint32_t* __restrict__ vidx, int32_t* __restrict__ tris)
{
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int bx = cx - 1, by = cy - 1;
    if (id >= (int64_t)bx * by * (cz - 1)) return;
    const int I = (int)(id % bx), J = (int)((id / bx) % by), K = (int)(id / ((int64_t)bx * by));
    const int64_t c0 = I + (int64_t)cx * (J + (int64_t)cy * K);
    const unsigned m = cube_case(phi, c0, cx, cy);
    const int nt = tab->ntri[m];
    const int64_t base = toff[id];
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) {
            const int e = tab->edge[m][3 * t + k];
            // the edge's low corner: local edge e runs along axis e / 4 from
            // the corner with the other two offsets given by e % 4
            const int axis = e >> 2, q = e & 3;
            int off[3];
            off[axis] = 0;
            off[axis == 0 ? 1 : 0] = q & 1;
            off[axis == 2 ? 1 : 2] = q >> 1;
            const int64_t c = c0 + off[0] + (int64_t)cx * (off[1] + (int64_t)cy * off[2]);
            tris[3 * (base + t) + k] = (int32_t)vidx[3 * c + axis];
        }
}

// inverse-area weighted unit normals of the triangles, summed at their vertices
template <typename T>
__global__ __launch_bounds__(256) void k_mc_face_normals(const T* __restrict__ verts,
                                                         const int32_t* __restrict__ tris, int64_t nt,
                                                         T* __restrict__ normals)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nt) return;
    const int32_t i0 = tris[3 * t], i1 = tris[3 * t + 1], i2 = tris[3 * t + 2];
    T u[3], w[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        u[d] = verts[3 * i1 + d] - verts[3 * i0 + d];
        w[d] = verts[3 * i2 + d] - verts[3 * i0 + d];
    }
    const T cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
    const T len2 = cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2];
    if (!(len2 > (T)0)) return;
    // unit normal / area = (cr / |cr|) / (|cr| / 2) = 2 cr / |cr|^2
    const T s = (T)2 / len2;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        atomicAdd(&normals[3 * i0 + d], s * cr[d]);
        atomicAdd(&normals[3 * i1 + d], s * cr[d]);
        atomicAdd(&normals[3 * i2 + d], s * cr[d]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_mc_normalize(int64_t nv, T* __restrict__ normals)
{
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= nv) return;
    const T x = normals[3 * v], y = normals[3 * v + 1], z = normals[3 * v + 2];
    const T len = sqrt(x * x + y * y + z * z);
    if (len > (T)0) {
        normals[3 * v] = x / len;
        normals[3 * v + 1] = y / len;
        normals[3 * v + 2] = z / len;
    }
}

static unsigned grid_of(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename T>
void launch_mc_count(const T* phi, int cx, int cy, int cz, const McTable* tab, const McWork& w, hipStream_t st)
{
    const int64_t nc = (int64_t)cx * cy * cz, ncube = (int64_t)(cx - 1) * (cy - 1) * (cz - 1);
    hipLaunchKernelGGL(k_mc_edge_flags<T>, dim3(grid_of(nc)), dim3(256), 0, st, phi, cx, cy, cz, w.flag);
    launch_exclusive_scan_u32(w.flag, w.vidx, 3 * nc, w.scan_tmp, st);
    if (ncube > 0) {
        hipLaunchKernelGGL(k_mc_cube_counts<T>, dim3(grid_of(ncube)), dim3(256), 0, st, phi, cx, cy, cz, tab,
                           w.cnt);
        launch_exclusive_scan_u32(w.cnt, w.toff, ncube, w.scan_tmp, st);
    }
    hipLaunchKernelGGL(k_mc_totals, dim3(1), dim3(64), 0, st, w.flag, w.vidx, 3 * nc, w.cnt, w.toff, ncube,
                       w.totals);
}

template <typename T>
void launch_mc_emit(const T* phi, int cx, int cy, int cz, double h, const McTable* tab, const McWork& w,
                    int64_t nv, int64_t nt, T* verts, T* normals, int32_t* tris, hipStream_t st)
{
    const int64_t nc = (int64_t)cx * cy * cz, ncube = (int64_t)(cx - 1) * (cy - 1) * (cz - 1);
    hipLaunchKernelGGL(k_mc_vertices<T>, dim3(grid_of(nc)), dim3(256), 0, st, phi, cx, cy, cz, h, w.flag, w.vidx,
                       verts, normals);
    if (nt > 0) {
        hipLaunchKernelGGL(k_mc_triangles<T>, dim3(grid_of(ncube)), dim3(256), 0, st, phi, cx, cy, cz, tab, w.toff,
                           w.vidx, tris);
        hipLaunchKernelGGL(k_mc_face_normals<T>, dim3(grid_of(nt)), dim3(256), 0, st, verts, tris, nt, normals);
    }
    if (nv > 0) hipLaunchKernelGGL(k_mc_normalize<T>, dim3(grid_of(nv)), dim3(256), 0, st, nv, normals);
}

template void launch_mc_count<float>(const float*, int, int, int, const McTable*, const McWork&, hipStream_t);
template void launch_mc_count<double>(const double*, int, int, int, const McTable*, const McWork&, hipStream_t);
template void launch_mc_emit<float>(const float*, int, int, int, double, const McTable*, const McWork&, int64_t,
                                    int64_t, float*, float*, int32_t*, hipStream_t);
template void launch_mc_emit<double>(const double*, int, int, int, double, const McTable*, const McWork&, int64_t,
                                     int64_t, double*, double*, int32_t*, hipStream_t);

}  // namespace flipmi
