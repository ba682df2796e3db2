// Phase singularities in z cross-sections (the paper's `singz` device, "Input/output
// and visualization"): the points where an isoline u = u* of one state variable meets
// an isoline v = v* of another inside a grid cell, each isoline's piece in the cell
// drawn between the points where it crosses the cell's edges (linear interpolation
// along the edge).  Cell = four tissue voxels (x..x+1, y..y+1) of one z plane; a
// corner is "above" when its value is >= the level; two crossed edges give one piece,
// four (a saddle) give two, which separate the corner pair whose class differs from
// that of the four corners' mean.  Every crossing of a u piece with a v piece (both
// within their segments) is a point.
//
// Statistics are FP64 sums (count, sum x, y, z, sum x^2, y^2, z^2 in mm) in a fixed
// order: each thread walks a fixed strided set of cells, each workgroup reduces its
// threads in an LDS tree, and one workgroup sums the workgroups in index order, so
// the sums are deterministic.  Points are appended with one atomic per point (their
// order varies from run to run; the set does not).
#include "bbx_internal.h"

namespace bbx {

constexpr int kTipBlocks = 1024;
constexpr int kTipSums = 7;

template <typename T>
struct TipField {
    const T *box;          // var 0: V in box layout
    const T *list;         // var > 0: the variable over the tissue list
    const int32_t *map;    // box -> tissue index (-1 void), or null (dense box)
    __device__ double at(int64_t b) const
    {
        if (box) return (double)box[b];
        return (double)list[map ? map[b] : b];
    }
};

// Isoline pieces of one cell: corner values c (00, 10, 01, 11) relative to the level.
// Writes up to two segments (x1, y1, x2, y2) in cell coordinates; returns their count.
__device__ __forceinline__ int pieces(const double c[4], double s[2][4])
{
    const unsigned q = (c[0] >= 0.0) | (c[1] >= 0.0) << 1 | (c[2] >= 0.0) << 2 | (c[3] >= 0.0) << 3;
    // edge e: corners (i0, i1), start (sx, sy), direction along x (dirx) or y
    const int i0[4] = {0, 1, 2, 0}, i1[4] = {1, 3, 3, 2};
    double px[4], py[4];
    unsigned cut = 0;
#pragma unroll
    for (int e = 0; e < 4; e++) {
        if (((q >> i0[e]) ^ (q >> i1[e])) & 1u) {
            const double t = c[i0[e]] / (c[i0[e]] - c[i1[e]]);
            // bottom (y = 0), right (x = 1), top (y = 1), left (x = 0)
            px[e] = e == 0 || e == 2 ? t : (e == 1 ? 1.0 : 0.0);
            py[e] = e == 1 || e == 3 ? t : (e == 2 ? 1.0 : 0.0);
            cut |= 1u << e;
        }
    }
    const int n = __builtin_popcount(cut);
    if (n == 2) {
        const int e0 = __builtin_ctz(cut), e1 = 31 - __builtin_clz(cut);
        s[0][0] = px[e0]; s[0][1] = py[e0]; s[0][2] = px[e1]; s[0][3] = py[e1];
        return 1;
    }
    if (n == 4) {
        const bool mid = 0.25 * (c[0] + c[1] + c[2] + c[3]) >= 0.0;
        // mid in corner 00's class: corners 00 and 11 connect, the pieces fence off 10
        // (edges bottom, right) and 01 (top, left); else they fence off 00 and 11
        const int a0 = 0, a1 = mid == (bool)(q & 1u) ? 1 : 3;
        const int b0 = mid == (bool)(q & 1u) ? 2 : 1, b1 = mid == (bool)(q & 1u) ? 3 : 2;
        s[0][0] = px[a0]; s[0][1] = py[a0]; s[0][2] = px[a1]; s[0][3] = py[a1];
        s[1][0] = px[b0]; s[1][1] = py[b0]; s[1][2] = px[b1]; s[1][3] = py[b1];
        return 2;
    }
    return 0;
}

// Cells of planes z0 .. z1-1; plane z is reported at h (z + zoff) (a slab's global plane).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tips(int nx, int ny, int z0, int z1, int zoff, double h,
                                                 int dense, const int32_t *map, TipField<T> fu,
                                                 double ul, TipField<T> fv, double vl,
                                                 double *part, double *pts, int64_t max_pts,
                                                 unsigned long long *count)
{
    __shared__ double sh[kTipSums][kBlock];
    double acc[kTipSums] = {0, 0, 0, 0, 0, 0, 0};
    const int64_t cx = nx - 1, cy = ny - 1, ncell = cx * cy * (int64_t)(z1 - z0);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < ncell; c += stride) {
        const int64_t x = c % cx, r = c / cx, y = r % cy, z = z0 + r / cy;
        const int64_t b00 = x + nx * (y + (int64_t)ny * z);
        const int64_t bb[4] = {b00, b00 + 1, b00 + nx, b00 + nx + 1};
        if (!dense && (map[bb[0]] < 0 || map[bb[1]] < 0 || map[bb[2]] < 0 || map[bb[3]] < 0)) continue;
        double cu[4], cv[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            cu[k] = fu.at(bb[k]) - ul;
            cv[k] = fv.at(bb[k]) - vl;
        }
        double su[2][4], sv[2][4];
        const int nu = pieces(cu, su);
        if (nu == 0) continue;
        const int nv = pieces(cv, sv);
        for (int i = 0; i < nu; i++)
            for (int j = 0; j < nv; j++) {
                // P = su0 + s (su1 - su0) = sv0 + t (sv1 - sv0)
                const double rx = su[i][2] - su[i][0], ry = su[i][3] - su[i][1];
                const double qx = sv[j][2] - sv[j][0], qy = sv[j][3] - sv[j][1];
                const double det = rx * qy - ry * qx;
                if (det == 0.0) continue;
                const double wx = sv[j][0] - su[i][0], wy = sv[j][1] - su[i][1];
                const double s = (wx * qy - wy * qx) / det, t = (wx * ry - wy * rx) / det;
                if (!(s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0)) continue;
                const double X = h * ((double)x + (su[i][0] + s * rx));
                const double Y = h * ((double)y + (su[i][1] + s * ry));
                const double Z = h * (double)(z + zoff);
                acc[0] += 1.0;
                acc[1] += X; acc[2] += Y; acc[3] += Z;
                acc[4] += X * X; acc[5] += Y * Y; acc[6] += Z * Z;
                const unsigned long long k = atomicAdd(count, 1ull);
                if ((int64_t)k < max_pts) {
                    pts[3 * k] = X;
                    pts[3 * k + 1] = Y;
                    pts[3 * k + 2] = Z;
                }
            }
    }
#pragma unroll
    for (int i = 0; i < kTipSums; i++) sh[i][threadIdx.x] = acc[i];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int i = 0; i < kTipSums; i++) sh[i][threadIdx.x] += sh[i][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < kTipSums) part[(int64_t)blockIdx.x * kTipSums + threadIdx.x] = sh[threadIdx.x][0];
}

// out[i] = sum over workgroups b of part[b][i], in index order.
__global__ void k_tips_final(const double *part, int nblk, double *out)
{
    if (threadIdx.x >= kTipSums) return;
    double s = 0.0;
    for (int b = 0; b < nblk; b++) s += part[(int64_t)b * kTipSums + threadIdx.x];
    out[threadIdx.x] = s;
}

// map[b] = -1 for every box voxel, then map[idx[t]] = t for tissue voxels.
__global__ void k_map_clear(int32_t *map, int64_t nbox)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < nbox) map[i] = -1;
}

__global__ void k_map_set(int32_t *map, const int32_t *idx, int64_t nact)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < nact) map[idx[t]] = (int32_t)t;
}

hipError_t launch_box_map(int32_t *map, int64_t nbox, const int32_t *idx, int64_t nact, hipStream_t s)
{
    hipLaunchKernelGGL(k_map_clear, dim3((unsigned)((nbox + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       map, nbox);
    if (nact > 0)
        hipLaunchKernelGGL(k_map_set, dim3((unsigned)((nact + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           map, idx, nact);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tips(const TipLaunch<T> &L, hipStream_t s)
{
    TipField<T> fu{L.u_box, L.u_list, L.dense ? nullptr : L.map};
    TipField<T> fv{L.v_box, L.v_list, L.dense ? nullptr : L.map};
    hipLaunchKernelGGL((k_tips<T>), dim3(kTipBlocks), dim3(kBlock), 0, s, L.nx, L.ny, L.z0, L.z1,
                       L.zoff, L.h, L.dense, L.map, fu, L.ul, fv, L.vl, L.part, L.pts, L.max_pts,
                       L.count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tips_final, dim3(1), dim3(64), 0, s, L.part, kTipBlocks, L.out);
    return hipGetLastError();
}

template hipError_t launch_tips<float>(const TipLaunch<float> &, hipStream_t);
template hipError_t launch_tips<double>(const TipLaunch<double> &, hipStream_t);

}  // namespace bbx
