// Fused monodomain step: diffusion stencil + stimulus + cell kinetics +
// activation/APD90 epilogue, one thread per tissue voxel.
//
// Diffusion ("Monodomain diffusion and boundary conditions"): with the
// transversely isotropic tensor D = Dperp I + (Dpar - Dperp) f f^T (eq (sigma))
// and chi the tissue indicator (void and out-of-box neighbours count 0),
//   (L V)_p = 1/h^2 sum_j D_jj [chi(V_{+j} - V_p) + chi(V_{-j} - V_p)]
//           + 1/(2h^2) sum_{j<k} D_jk [chi(V_{+j+k} - V_p) + chi(V_{-j-k} - V_p)
//                                      - chi(V_{+j-k} - V_p) - chi(V_{-j+k} - V_p)]
//           + sum_k c_k (V_{+k} - V_{-k}),
// i.e. the paper's weights Wbar + Wtilde summed in the difference form (the
// centre weight is minus the sum of the others).  c_k, the face coefficient of
// the tensor-gradient part Wtilde, depends on the neighbours' fibres only and
// is precomputed per voxel; D^p is rebuilt in registers from the fibre, so the
// kernel streams 3+3 interleaved values per voxel instead of 18 weights.
//
// Memory: V lives in box layout (neighbour gathers; void entries stay 0 and are
// never selected), everything else is structure-of-arrays over the tissue list
// (coalesced, x-fastest order).  Workgroups are dealt to tiles in per-XCD runs
// (workgroup_tile), so that neighbour rows and planes tend to stay in one XCD's L2.
#include <type_traits>

#include "step_device.h"

namespace bbx {

// Tissue-list path: one thread per tissue voxel, 256 consecutive list entries per
// workgroup (512 when streaming), dealt to workgroups by workgroup_tile.
// Workgroup -> tile.  The tiles go out in rounds: XCD k takes the k-th run of S
// consecutive tiles of each round of 8 * S (then a last, shorter round), so that each XCD
// shares halos within its runs while the workgroups running at any moment stay within one
// region of memory.  Data that fits the Infinity Cache: runs of 256 (for up to 256
// workgroups per XCD this is one contiguous eighth of the tiles per XCD, so each XCD's L2
// keeps its part from step to step; measured: thin CRN shell 59.3 -> 56.7 us against
// eighths, CRN cup 14.2 us either way, 14.7 with runs of 16).  Streaming data (larger than
// the cache): runs of SL, measured per kernel: launch order (SL = 1) for the tissue list
// (TP06 double shell 0.977 -> 0.918 ms, 300^3 CRN box 1.010 -> 0.959 ms against eighths;
// runs of 4-64 were slower) and for the isotropic register march (200 us; 210 with runs of
// 64); runs of 64 for the LDS-ring stencil (635 -> 600 us; 623 in launch order, 615 with
// runs of 256 or 1024).
template <bool NT, int SL, typename T>
__device__ __forceinline__ int workgroup_tile(const StepArgs<T> &a)
{
    constexpr int S = NT ? SL : 256;
    const int x = (int)(blockIdx.x % kXcd), i = (int)(blockIdx.x / kXcd);
    const int full = a.per_xcd / S * S;             // per XCD: blocks in complete rounds
    if (i < full) return (i / S) * (kXcd * S) + x * S + (i % S);
    const int rem = a.per_xcd - full;                // the last, shorter round
    return full * kXcd + x * rem + (i - full);
}

template <typename T, class M, bool ANISO, bool NT, bool RK4 = false>
__global__ __launch_bounds__(NT ? kStreamBlock : kBlock) void k_step(const StepArgs<T> a)
{
    const int lb = workgroup_tile<NT, 1>(a);
    if (lb >= a.nblk) return;
    const int t = lb * (NT ? kStreamBlock : kBlock) + (int)threadIdx.x;
    if (t >= a.nact) return;
    int idx;
    uint32_t bits;
    voxel_of(a, t, idx, bits);         // dense boxes keep no index / bit arrays
    const T Vp = a.Vin[idx];
    const T LV = laplacian<T, ANISO, false>(a, a.Vin, t, idx, bits, Vp);
    update_voxel<T, M, NT, RK4>(a, step_clock(a), t, idx, Vp, LV);
}

// Dense-box path (every voxel is tissue): a workgroup owns a 64 x 4 column tile
// and marches along z through a chunk of a.zc planes.  Three planes of V, each
// with a one-voxel halo (66 x 6), live in an LDS ring; plane z+2 is fetched into
// registers while plane z is computed, so every V value is read from memory about
// once and each wave keeps loads in flight across the loop.
constexpr int kLX = kTileX + 2, kLY = kTileY + 2, kPlane = kLX * kLY;

template <typename T>
__device__ __forceinline__ T plane_val(const StepArgs<T> &a, int bx, int by, int p, int e)
{
    const int lx = e % kLX, ly = e / kLX;
    const int x = bx * kTileX + lx - 1, y = by * kTileY + ly - 1;
    if (p < 0 || p >= a.nz || x < 0 || y < 0 || x >= a.nx || y >= a.ny) return T(0);
    return a.Vin[x + a.nx * (y + a.ny * p)];
}

template <typename T, bool FULL>
__device__ __forceinline__ T lds_d(const T *P, int o, uint32_t bits, int b, T Vp)
{
    if (FULL) return P[o] - Vp;
    return ((bits >> b) & 1u) ? P[o] - Vp : T(0);
}

template <typename T, bool ANISO, bool FULL>
__device__ __forceinline__ T laplacian_lds(const StepArgs<T> &a, const T *Pm, const T *Pc,
                                           const T *Pp, int c, const T *geo, uint32_t bits, T Vp)
{
    const T ex_ = lds_d<T, FULL>(Pc, c + 1, bits, 0, Vp), wx = lds_d<T, FULL>(Pc, c - 1, bits, 1, Vp);
    const T ny_ = lds_d<T, FULL>(Pc, c + kLX, bits, 2, Vp), sy_ = lds_d<T, FULL>(Pc, c - kLX, bits, 3, Vp);
    const T up = lds_d<T, FULL>(Pp, c, bits, 4, Vp), dn = lds_d<T, FULL>(Pm, c, bits, 5, Vp);
    if (!ANISO) return a.Dperp * a.ih2 * ((ex_ + wx) + (ny_ + sy_) + (up + dn));
    const T fx = geo[0], fy = geo[1], fz = geo[2];
    const T cx = geo[3], cy = geo[4], cz = geo[5];
    const T dd = a.Dpar - a.Dperp;
    const T Dxx = a.Dperp + dd * fx * fx, Dyy = a.Dperp + dd * fy * fy;
    const T Dzz = a.Dperp + dd * fz * fz;
    const T Dxy = dd * fx * fy, Dxz = dd * fx * fz, Dyz = dd * fy * fz;
    const T exy = lds_d<T, FULL>(Pc, c + 1 + kLX, bits, 6, Vp) + lds_d<T, FULL>(Pc, c - 1 - kLX, bits, 7, Vp)
                  - lds_d<T, FULL>(Pc, c + 1 - kLX, bits, 8, Vp) - lds_d<T, FULL>(Pc, c - 1 + kLX, bits, 9, Vp);
    const T exz = lds_d<T, FULL>(Pp, c + 1, bits, 10, Vp) + lds_d<T, FULL>(Pm, c - 1, bits, 11, Vp)
                  - lds_d<T, FULL>(Pm, c + 1, bits, 12, Vp) - lds_d<T, FULL>(Pp, c - 1, bits, 13, Vp);
    const T eyz = lds_d<T, FULL>(Pp, c + kLX, bits, 14, Vp) + lds_d<T, FULL>(Pm, c - kLX, bits, 15, Vp)
                  - lds_d<T, FULL>(Pm, c + kLX, bits, 16, Vp) - lds_d<T, FULL>(Pp, c - kLX, bits, 17, Vp);
    return a.ih2 * (Dxx * (ex_ + wx) + Dyy * (ny_ + sy_) + Dzz * (up + dn)
                    + T(0.5) * (Dxy * exy + Dxz * exz + Dyz * eyz))
           + cx * (ex_ - wx) + cy * (ny_ - sy_) + cz * (up - dn);
}

template <typename T, class M, bool ANISO, bool NT>
__global__ __launch_bounds__(kBlock) void k_step_dense(const StepArgs<T> a)
{
    __shared__ T ring[3][kPlane];
    const int lb = workgroup_tile<NT, 64>(a);
    if (lb >= a.nblk) return;                       // workgroup-uniform exit
    const Clock<T> ck = step_clock(a);
    const int bx = lb % a.gx, r = lb / a.gx;
    const int by = r % a.gy, bz = r / a.gy;
    const int z0 = bz * a.zc, z1 = min(a.nz, z0 + a.zc);
    const int tx = (int)(threadIdx.x % kTileX), ty = (int)(threadIdx.x / kTileX);
    const int x = bx * kTileX + tx, y = by * kTileY + ty;
    const bool own = x < a.nx && y < a.ny;
    const int e0 = (int)threadIdx.x, e1 = e0 + kBlock;    // this thread's plane elements
    const bool has1 = e1 < kPlane;
    const int c = (ty + 1) * kLX + tx + 1;                 // own position in a plane
    const bool xy_in = bx > 0 && (bx + 1) * kTileX < a.nx && by > 0 && (by + 1) * kTileY < a.ny;
    const uint32_t px = x + 1 < a.nx, mx = x > 0, py = y + 1 < a.ny, my = y > 0;

    // planes z0-1, z0, z0+1 -> ring slots 0, 1, 2 (slot of plane p: (p - z0 + 1) % 3)
    for (int k = 0; k < 3; k++) {
        ring[k][e0] = plane_val(a, bx, by, z0 - 1 + k, e0);
        if (has1) ring[k][e1] = plane_val(a, bx, by, z0 - 1 + k, e1);
    }
    // this column's fibre and face coefficients at plane z0
    const int64_t col = (int64_t)x + (int64_t)a.nx * y, plane = (int64_t)a.nx * a.ny;
    T geo[6] = {};
    if (ANISO && own)
        for (int i = 0; i < 6; i++) geo[i] = a.geo[6 * (col + plane * z0) + i];
    __syncthreads();

    for (int z = z0; z < z1; z++) {
        const int k = z - z0;
        // prefetch plane z+2 of V (needed while z+1 < z1) and the geometry of z+1
        const bool pre = z + 1 < z1;
        T q0 = T(0), q1 = T(0);
        T gnext[6] = {};
        if (pre) {
            q0 = plane_val(a, bx, by, z + 2, e0);
            if (has1) q1 = plane_val(a, bx, by, z + 2, e1);
            if (ANISO && own)
                for (int i = 0; i < 6; i++) gnext[i] = a.geo[6 * (col + plane * (z + 1)) + i];
        }
        if (own) {
            const T *Pm = ring[k % 3], *Pc = ring[(k + 1) % 3], *Pp = ring[(k + 2) % 3];
            const int idx = x + a.nx * (y + a.ny * z);
            const uint32_t pz = z + 1 < a.nz, mz = z > 0;
            uint32_t bits = px | mx << 1 | py << 2 | my << 3 | pz << 4 | mz << 5;
            if (ANISO) {
                bits |= (px & py) << 6 | (mx & my) << 7 | (px & my) << 8 | (mx & py) << 9;
                bits |= (px & pz) << 10 | (mx & mz) << 11 | (px & mz) << 12 | (mx & pz) << 13;
                bits |= (py & pz) << 14 | (my & mz) << 15 | (py & mz) << 16 | (my & pz) << 17;
            }
            const T Vp = Pc[c];
            const bool full = xy_in && z > 0 && z + 1 < a.nz;
            const T LV = full ? laplacian_lds<T, ANISO, true>(a, Pm, Pc, Pp, c, geo, bits, Vp)
                              : laplacian_lds<T, ANISO, false>(a, Pm, Pc, Pp, c, geo, bits, Vp);
            update_voxel<T, M, NT>(a, ck, idx, idx, Vp, LV);
        }
        __syncthreads();                                   // slot of plane z-1 is free
        if (pre) {
            ring[k % 3][e0] = q0;
            if (has1) ring[k % 3][e1] = q1;
            for (int i = 0; i < 6; i++) geo[i] = gnext[i];
        }
        __syncthreads();
    }
}

// Isotropic dense boxes: each thread marches its own (x, y) column through the
// z-chunk keeping V of planes z-1, z, z+1 in registers; the four in-plane
// neighbours come from memory (cache hits) and plane z+2 is loaded one plane
// ahead.  No LDS and no barriers.
template <typename T, class M, bool NT>
__global__ __launch_bounds__(kBlock) void k_step_zreg(const StepArgs<T> a)
{
    const int lb = workgroup_tile<NT, 1>(a);
    if (lb >= a.nblk) return;
    const Clock<T> ck = step_clock(a);
    const int bx = lb % a.gx, r = lb / a.gx;
    const int by = r % a.gy, bz = r / a.gy;
    const int z0 = bz * a.zc, z1 = min(a.nz, z0 + a.zc);
    const int x = bx * kTileX + (int)(threadIdx.x % kTileX), y = by * kTileY + (int)(threadIdx.x / kTileX);
    if (x >= a.nx || y >= a.ny) return;
    const bool px = x + 1 < a.nx, mx = x > 0, py = y + 1 < a.ny, my = y > 0;
    const int plane = a.nx * a.ny;
    const int c0 = x + a.nx * y;
    const int de = px ? 1 : 0, dw = mx ? -1 : 0, dn = py ? a.nx : 0, ds = my ? -a.nx : 0;
    T Vm = z0 > 0 ? a.Vin[c0 + (z0 - 1) * plane] : T(0);
    T Vc = a.Vin[c0 + z0 * plane];
    T Vq = z0 + 1 < a.nz ? a.Vin[c0 + (z0 + 1) * plane] : T(0);
    for (int z = z0; z < z1; z++) {
        const T Vnext = (z + 2 < a.nz && z + 1 < z1) ? a.Vin[c0 + (z + 2) * plane] : T(0);
        const int idx = c0 + z * plane;
        const T E = a.Vin[idx + de], W = a.Vin[idx + dw], N = a.Vin[idx + dn], S = a.Vin[idx + ds];
        const bool pz = z + 1 < a.nz, mz = z > 0;
        const T ex_ = px ? E - Vc : T(0), wx = mx ? W - Vc : T(0);
        const T ny_ = py ? N - Vc : T(0), sy_ = my ? S - Vc : T(0);
        const T up = pz ? Vq - Vc : T(0), dnv = mz ? Vm - Vc : T(0);
        const T LV = a.Dperp * a.ih2 * ((ex_ + wx) + (ny_ + sy_) + (up + dnv));
        update_voxel<T, M, NT>(a, ck, idx, idx, Vc, LV);
        Vm = Vc;
        Vc = Vq;
        Vq = Vnext;
    }
}

template <typename T, class M, bool NT>
static void launch_kernel(int aniso, const StepArgs<T> &a, hipStream_t s)
{
    const dim3 grid(a.per_xcd * kXcd), block(kBlock);
    if (a.dense && a.zc > 0) {
        if (aniso) hipLaunchKernelGGL((k_step_dense<T, M, true, NT>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_step_zreg<T, M, NT>), grid, block, 0, s, a);
    } else {
        // 512-thread workgroups when streaming (measured: TP06 double shell 0.909 -> 0.885
        // ms, 300^3 CRN box 0.958 -> 0.942 ms); 256 for cached data (CRN cup 14.2 us
        // against 14.6 with 512)
        const dim3 bl(NT ? kStreamBlock : kBlock);
        if (aniso) hipLaunchKernelGGL((k_step<T, M, true, NT>), grid, bl, 0, s, a);
        else hipLaunchKernelGGL((k_step<T, M, false, NT>), grid, bl, 0, s, a);
    }
}

template <typename T, class M>
static hipError_t launch_m(int aniso, const StepArgs<T> &a, hipStream_t s)
{
    constexpr bool kTab = std::is_same<M, kin::CrnTab>::value;   // one-step factors only
    if (a.rk4) {
        // the RK4 integrator: tissue-list kernel, cached accesses (make_args)
        if constexpr (!kTab) {
            const dim3 grid(a.per_xcd * kXcd), block(kBlock);
            if (aniso) hipLaunchKernelGGL((k_step<T, M, true, false, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_step<T, M, false, false, true>), grid, block, 0, s, a);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (a.nt) {
        launch_kernel<T, M, true>(aniso, a, s);
    } else {
        launch_kernel<T, M, false>(aniso, a, s);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step(int model, int aniso, const StepArgs<T> &a, hipStream_t s)
{
    switch (model) {
    case 0: return launch_m<T, kin::None<T>>(aniso, a, s);
    case 1: return launch_m<T, kin::Barkley<T>>(aniso, a, s);
    case 2: return launch_m<T, kin::Zfk<T>>(aniso, a, s);
    case 3: return launch_m<T, kin::Fhn<T>>(aniso, a, s);
    case 4:
        if constexpr (std::is_same<T, float>::value)
            if (a.tab && !a.rk4) return launch_m<float, kin::CrnTab>(aniso, a, s);
        return launch_m<T, kin::Crn<T>>(aniso, a, s);
    case 5: return launch_m<T, kin::Fk4<T>>(aniso, a, s);
    case 6: return launch_m<T, kin::Tp06<T>>(aniso, a, s);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_step<float>(int, int, const StepArgs<float> &, hipStream_t);
template hipError_t launch_step<double>(int, int, const StepArgs<double> &, hipStream_t);

}  // namespace bbx
