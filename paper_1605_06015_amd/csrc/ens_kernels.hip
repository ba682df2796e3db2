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
//
// Floating-point contraction is limited to single source expressions in this file
// (no cross-statement fusion chosen by the backend), so that every tile variant
// performs the same rounding and their results are bitwise identical.
#pragma clang fp contract(on)

#include "ens_internal.h"
#include "step_device.h"

namespace bbx {

template <typename T>
__device__ __forceinline__ bool ens_stim_on(const EnsStim<T> S, int64_t n)
{
    if (n < S.n0 || S.len <= 0) return false;
    const int64_t r = n - S.n0;
    if (S.per <= 0) return r < S.len;
    const int64_t c = r / S.per;
    if (S.count > 0 && c >= S.count) return false;
    return r - c * S.per < S.len;
}

// Laplacian from the nine values around a voxel (difference form, neighbours
// outside the tissue dropped).
template <typename T>
__device__ __forceinline__ T ens_laplacian(const EnsTissue<T> &ti, bool px, bool mx, bool py, bool my,
                                           T Vp, T E, T W, T N, T S, T NE, T SW, T SE, T NW)
{
    const T ex_ = px ? E - Vp : T(0), wx = mx ? W - Vp : T(0);
    const T ny_ = py ? N - Vp : T(0), sy_ = my ? S - Vp : T(0);
    const T exy = (px && py ? NE - Vp : T(0)) + (mx && my ? SW - Vp : T(0))
                  - (px && my ? SE - Vp : T(0)) - (mx && py ? NW - Vp : T(0));
    return ti.cxx * (ex_ + wx) + ti.cyy * (ny_ + sy_) + ti.cxy * exy;
}

// Stimulus current at (x, y): the tissue's stimuli [s0, s1) read whole (one wide
// scalar load each) and tested without short-circuit.
template <typename T>
__device__ __forceinline__ T ens_stim(const EnsArgs<T> &a, const EnsTissue<T> &ti, int64_t n, int x, int y)
{
    T Is = T(0);
    for (int k = ti.s0; k < ti.s1; k++) {
        const EnsStim<T> St = a.stims[k];
        const bool in = (x >= St.x0) & (x < St.x1) & (y >= St.y0) & (y < St.y1);
        if (ens_stim_on(St, n) & in) Is += St.amp;
    }
    return Is;
}

// Kinetics, V update, stores and recorder of voxel t of a tissue.
template <typename T, class M, bool NT>
__device__ __forceinline__ void ens_update(const EnsArgs<T> &a, const EnsTissue<T> &ti, int64_t n,
                                           int64_t t, T Vp, T LV, T Is, T *Vout)
{
    T g[M::NV > 1 ? M::NV - 1 : 1];
#pragma unroll
    for (int i = 0; i < M::NV - 1; i++) {
        if constexpr (NT) g[i] = __builtin_nontemporal_load(&a.st[i * a.pitch + t]);
        else g[i] = a.st[i * a.pitch + t];
    }
    const T r = M::advance(ti.prm, Vp, g, a.dt, nullptr);
    const T Vn = Vp + a.dt * (r + Is + LV);
#pragma unroll
    for (int i = 0; i < M::NV - 1; i++) a.st[i * a.pitch + t] = g[i];
    if constexpr (NT) __builtin_nontemporal_store(Vn, &Vout[t]);
    else Vout[t] = Vn;
    if (a.rec) record_event(a, t, T((double)n * a.dt64), Vp, Vn);
}

template <typename T, class M, int TX, int TY, bool LDS, bool NT>
__global__ __launch_bounds__(kBlock) void k_ens_step(const EnsArgs<T> a, int j)
{
    static_assert(TX * TY == kBlock, "one voxel per thread");
    constexpr int LX = TX + 2, LY = TY + 2;
    __shared__ T tile[LDS ? LX * LY : 1];
    const int lb = (int)(blockIdx.x % kXcd) * a.per_xcd + (int)(blockIdx.x / kXcd);
    if (lb >= a.ntile) return;                       // workgroup-uniform exit
    const int4 tl = a.tiles[lb];
    const EnsTissue<T> ti = a.tis[tl.x];
    const int nx = ti.nx, ny = ti.ny;
    const int64_t n = *a.nbase + j;
    const T *Vin = (n & 1) ? a.V1 : a.V0;
    T *Vout = (n & 1) ? a.V0 : a.V1;
    const T *Vt = Vin + ti.off;
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
        // unconditional loads at coordinates clamped into the tissue (a missing
        // neighbour reads a tissue voxel and is masked by the Laplacian)
        const int xe = px ? x + 1 : x, xw = mx ? x - 1 : x;
        const int rn = (py ? y + 1 : y) * nx, rs = (my ? y - 1 : y) * nx, rc = y * nx;
        Vp = Vt[rc + x];
        E = Vt[rc + xe];
        W = Vt[rc + xw];
        N = Vt[rn + x];
        S = Vt[rs + x];
        NE = Vt[rn + xe];
        SW = Vt[rs + xw];
        SE = Vt[rs + xe];
        NW = Vt[rn + xw];
    }
    const T LV = ens_laplacian(ti, px, mx, py, my, Vp, E, W, N, S, NE, SW, SE, NW);
    const T Is = ens_stim(a, ti, n, x, y);
    ens_update<T, M, NT>(a, ti, n, ti.off + (int64_t)(x + nx * y), Vp, LV, Is, Vout);
}

// Row-marching variant: a workgroup owns a 64-column strip of 4R rows, each wave
// R consecutive rows.  A lane keeps its column's values of rows y-1, y, y+1 in
// registers and takes the x+-1 neighbours from the adjacent lanes (cross-lane
// shuffles); lanes 0 and 63 also carry the halo columns x0-1 and x0+64.  Row y+2
// is loaded while row y is computed, so each V value is read from memory once
// and every wave keeps loads in flight through its rows.
template <typename T, class M, int R, bool NT>
__global__ __launch_bounds__(kBlock) void k_ens_march(const EnsArgs<T> a, int j)
{
    const int lb = (int)(blockIdx.x % kXcd) * a.per_xcd + (int)(blockIdx.x / kXcd);
    if (lb >= a.ntile) return;                       // workgroup-uniform exit
    const int4 tl = a.tiles[lb];
    const EnsTissue<T> ti = a.tis[tl.x];
    const int nx = ti.nx, ny = ti.ny;
    const int64_t n = *a.nbase + j;
    const T *Vt = ((n & 1) ? a.V1 : a.V0) + ti.off;
    T *Vout = (n & 1) ? a.V0 : a.V1;
    const int l = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
    const int ya = tl.z + w * R, yb = min(ny, ya + R);
    if (ya >= ny) return;                            // wave-uniform: no rows for this wave
    const int x = tl.y + l;
    const bool inx = x < nx, px = x + 1 < nx, mx = x > 0;
    const bool edge = l == 0 || l == 63;
    const int hx = l == 0 ? tl.y - 1 : tl.y + 64;    // halo column carried by lanes 0 and 63
    auto ld = [&](int xx, int yy) -> T {
        return (xx >= 0 && xx < nx && yy >= 0 && yy < ny) ? Vt[xx + (int64_t)nx * yy] : T(0);
    };
    // stimuli of this tissue: on at step n (uniform) and covering this column
    uint32_t son = 0;
    for (int k = ti.s0; k < ti.s1; k++) {
        const EnsStim<T> St = a.stims[k];
        if (ens_stim_on(St, n) & (x >= St.x0) & (x < St.x1)) son |= 1u << (k - ti.s0);
    }
    T Vm = ld(x, ya - 1), Vc = ld(x, ya), Vq = ld(x, ya + 1);
    T Hm = edge ? ld(hx, ya - 1) : T(0), Hc = edge ? ld(hx, ya) : T(0), Hq = edge ? ld(hx, ya + 1) : T(0);
    for (int y = ya; y < yb; y++) {
        const T Vn2 = ld(x, y + 2);
        const T Hn2 = edge ? ld(hx, y + 2) : T(0);
        T E = __shfl_down(Vc, 1), W = __shfl_up(Vc, 1);
        T NE = __shfl_down(Vq, 1), NW = __shfl_up(Vq, 1);
        T SE = __shfl_down(Vm, 1), SW = __shfl_up(Vm, 1);
        if (l == 63) { E = Hc; NE = Hq; SE = Hm; }
        if (l == 0) { W = Hc; NW = Hq; SW = Hm; }
        if (inx) {
            const bool py = y + 1 < ny, my = y > 0;
            const T LV = ens_laplacian(ti, px, mx, py, my, Vc, E, W, Vq, Vm, NE, SW, SE, NW);
            T Is = T(0);
            for (int k = ti.s0; k < ti.s1; k++) {
                const EnsStim<T> St = a.stims[k];
                if (((son >> (k - ti.s0)) & 1u) & (y >= St.y0) & (y < St.y1)) Is += St.amp;
            }
            ens_update<T, M, NT>(a, ti, n, ti.off + (int64_t)(x + nx * y), Vc, LV, Is, Vout);
        }
        Vm = Vc;
        Vc = Vq;
        Vq = Vn2;
        Hm = Hc;
        Hc = Hq;
        Hq = Hn2;
    }
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
    case 4: *tx = 64; *ty = 4 * 8; break;
    case 5: *tx = 64; *ty = 4 * 32; break;
    default: *tx = 64; *ty = 4; break;
    }
}

template <typename T, class M, bool NT>
static hipError_t ens_v(int variant, const EnsArgs<T> &a, int j, hipStream_t s)
{
    const dim3 grid(a.per_xcd * kXcd), block(kBlock);
    switch (variant) {
    case 0: hipLaunchKernelGGL((k_ens_step<T, M, 64, 4, true, NT>), grid, block, 0, s, a, j); break;
    case 1: hipLaunchKernelGGL((k_ens_step<T, M, 32, 8, true, NT>), grid, block, 0, s, a, j); break;
    case 2: hipLaunchKernelGGL((k_ens_step<T, M, 16, 16, true, NT>), grid, block, 0, s, a, j); break;
    case 3: hipLaunchKernelGGL((k_ens_step<T, M, 64, 4, false, NT>), grid, block, 0, s, a, j); break;
    case 4: hipLaunchKernelGGL((k_ens_march<T, M, 8, NT>), grid, block, 0, s, a, j); break;
    case 5: hipLaunchKernelGGL((k_ens_march<T, M, 32, NT>), grid, block, 0, s, a, j); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, class M>
static hipError_t ens_m(int variant, const EnsArgs<T> &a, int j, hipStream_t s)
{
    return a.nt ? ens_v<T, M, true>(variant, a, j, s) : ens_v<T, M, false>(variant, a, j, s);
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
