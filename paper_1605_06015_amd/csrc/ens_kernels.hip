// Batched 2D ensemble step: one launch advances every tissue of the ensemble by
// one step.  A workgroup owns one TX x TY tile of one tissue (the tile table
// lists tissues one after another, tiles row by row), so tissues of very
// different sizes share one launch with no idle workgroups beyond the ragged
// tile edges.  Workgroups are dealt so that XCD k takes the k-th contiguous
// eighth of the tile table, keeping each tissue's rows in one L2.
//
// Per voxel: the anisotropic no-flux 9-point stencil of a tissue-uniform tensor
// (the weight formulas of "Monodomain diffusion and boundary conditions" in 2D:
// face weights D_jj/h^2, edge weights +-D_xy/(2h^2), tensor-gradient term zero
// for a uniform tensor), summed in the difference form with out-of-tissue
// neighbours dropped; rectangular stimuli; the kinetics; additive coupling
// V+ = V + dt(-I_ion + I_stim + LV); the activation/APD90 recorder.
#include "ens_internal.h"
#include "step_device.h"

namespace bbx {

template <typename T>
__device__ __forceinline__ bool ens_stim_on(const EnsStim<T> &S, int64_t n)
{
    if (n < S.n0 || S.len <= 0) return false;
    const int64_t r = n - S.n0;
    if (S.per <= 0) return r < S.len;
    const int64_t c = r / S.per;
    if (S.count > 0 && c >= S.count) return false;
    return r - c * S.per < S.len;
}

template <typename T, class M, int TX, int TY, bool LDS>
__global__ __launch_bounds__(kBlock) void k_ens_step(const EnsArgs<T> a, int j)
{
    static_assert(TX * TY == kBlock, "one voxel per thread");
    constexpr int LX = TX + 2, LY = TY + 2;
    __shared__ T tile[LDS ? LX * LY : 1];
    const int lb = (int)(blockIdx.x % kXcd) * a.per_xcd + (int)(blockIdx.x / kXcd);
    if (lb >= a.ntile) return;                       // workgroup-uniform exit
    const int4 tl = a.tiles[lb];
    const EnsTissue<T> *ti = a.tis + tl.x;
    const int nx = ti->nx, ny = ti->ny;
    const int64_t n = *a.nbase + j;
    const T *Vin = (n & 1) ? a.V1 : a.V0;
    T *Vout = (n & 1) ? a.V0 : a.V1;
    const T *Vt = Vin + ti->off;
    const int tx = (int)threadIdx.x % TX, ty = (int)threadIdx.x / TX;
    const int x = tl.y + tx, y = tl.z + ty;
    const bool own = x < nx && y < ny;
    const bool px = x + 1 < nx, mx = x > 0, py = y + 1 < ny, my = y > 0;

    T Vp, E, W, N, S, NE, SW, SE, NW;
    if (LDS) {
        for (int e = (int)threadIdx.x; e < LX * LY; e += kBlock) {
            const int gx = tl.y + e % LX - 1, gy = tl.z + e / LX - 1;
            tile[e] = (gx >= 0 && gx < nx && gy >= 0 && gy < ny) ? Vt[gx + (int64_t)nx * gy] : T(0);
        }
        __syncthreads();
        if (!own) return;
        const int c = (ty + 1) * LX + tx + 1;
        Vp = tile[c];
        E = tile[c + 1];
        W = tile[c - 1];
        N = tile[c + LX];
        S = tile[c - LX];
        NE = tile[c + LX + 1];
        SW = tile[c - LX - 1];
        SE = tile[c - LX + 1];
        NW = tile[c + LX - 1];
    } else {
        if (!own) return;
        const T *q = Vt + x + (int64_t)nx * y;
        Vp = q[0];
        E = px ? q[1] : T(0);
        W = mx ? q[-1] : T(0);
        N = py ? q[nx] : T(0);
        S = my ? q[-nx] : T(0);
        NE = px && py ? q[nx + 1] : T(0);
        SW = mx && my ? q[-nx - 1] : T(0);
        SE = px && my ? q[-nx + 1] : T(0);
        NW = mx && py ? q[nx - 1] : T(0);
    }
    const T ex_ = px ? E - Vp : T(0), wx = mx ? W - Vp : T(0);
    const T ny_ = py ? N - Vp : T(0), sy_ = my ? S - Vp : T(0);
    const T exy = (px && py ? NE - Vp : T(0)) + (mx && my ? SW - Vp : T(0))
                  - (px && my ? SE - Vp : T(0)) - (mx && py ? NW - Vp : T(0));
    const T LV = ti->cxx * (ex_ + wx) + ti->cyy * (ny_ + sy_) + ti->cxy * exy;

    T Is = T(0);
    for (int k = ti->s0; k < ti->s1; k++) {
        const EnsStim<T> &St = a.stims[k];
        if (ens_stim_on(St, n) && x >= St.x0 && x < St.x1 && y >= St.y0 && y < St.y1) Is += St.amp;
    }

    const int64_t t = ti->off + x + (int64_t)nx * y;
    T g[M::NV > 1 ? M::NV - 1 : 1];
#pragma unroll
    for (int i = 0; i < M::NV - 1; i++) g[i] = a.st[i * a.pitch + t];
    const T r = M::advance(ti->prm, Vp, g, a.dt, nullptr);
    const T Vn = Vp + a.dt * (r + Is + LV);
#pragma unroll
    for (int i = 0; i < M::NV - 1; i++) a.st[i * a.pitch + t] = g[i];
    Vout[t] = Vn;
    if (a.rec) record_event(a, t, T((double)n * a.dt64), Vp, Vn);
}

__global__ void k_ens_advance(int64_t *nbase, int64_t k)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) nbase[0] += k;
}

void ens_tile_shape(int variant, int *tx, int *ty)
{
    switch (variant) {
    case 1: *tx = 32; *ty = 8; break;
    case 2: *tx = 16; *ty = 16; break;
    default: *tx = 64; *ty = 4; break;
    }
}

template <typename T, class M>
static hipError_t ens_m(int variant, const EnsArgs<T> &a, int j, hipStream_t s)
{
    const dim3 grid(a.per_xcd * kXcd), block(kBlock);
    switch (variant) {
    case 0: hipLaunchKernelGGL((k_ens_step<T, M, 64, 4, true>), grid, block, 0, s, a, j); break;
    case 1: hipLaunchKernelGGL((k_ens_step<T, M, 32, 8, true>), grid, block, 0, s, a, j); break;
    case 2: hipLaunchKernelGGL((k_ens_step<T, M, 16, 16, true>), grid, block, 0, s, a, j); break;
    case 3: hipLaunchKernelGGL((k_ens_step<T, M, 64, 4, false>), grid, block, 0, s, a, j); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ens_step(int model, int variant, const EnsArgs<T> &a, int j, hipStream_t s)
{
    switch (model) {
    case 0: return ens_m<T, kin::None<T>>(variant, a, j, s);
    case 1: return ens_m<T, kin::Barkley<T>>(variant, a, j, s);
    case 2: return ens_m<T, kin::Zfk<T>>(variant, a, j, s);
    case 3: return ens_m<T, kin::Fhn<T>>(variant, a, j, s);
    case 5: return ens_m<T, kin::Fk4<T>>(variant, a, j, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ens_advance(int64_t *nbase, int64_t k, hipStream_t s)
{
    hipLaunchKernelGGL(k_ens_advance, dim3(1), dim3(64), 0, s, nbase, k);
    return hipGetLastError();
}

template hipError_t launch_ens_step<float>(int, int, const EnsArgs<float> &, int, hipStream_t);
template hipError_t launch_ens_step<double>(int, int, const EnsArgs<double> &, int, hipStream_t);

}  // namespace bbx
