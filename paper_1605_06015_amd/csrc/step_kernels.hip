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
// kernel streams 3+3 values per voxel instead of 18 weights.
//
// Memory: V lives in box layout (neighbour gathers; void entries stay 0 and are
// never selected), everything else is structure-of-arrays over the tissue list
// (coalesced, x-fastest order).  Workgroups are remapped so that each XCD works
// on one contiguous slab of the tissue list, keeping neighbour planes in that
// XCD's L2.
#include "bbx_internal.h"
#include "kinetics.h"

namespace bbx {

// V_{p+off} - V_p if neighbour bit b is set (tissue), else 0.  FULL: the whole
// workgroup is known to be interior (every neighbour is tissue).
template <typename T, bool FULL>
__device__ __forceinline__ T nbd(const T *__restrict__ V, int idx, int off, uint32_t bits, int b,
                                 T Vp)
{
    if (FULL) return V[idx + off] - Vp;
    return ((bits >> b) & 1u) ? V[idx + off] - Vp : T(0);
}

// (L V)_p in the difference form; see the header comment.
template <typename T, bool ANISO, bool FULL>
__device__ __forceinline__ T laplacian(const StepArgs<T> &a, const T *__restrict__ V, int t,
                                       int idx, uint32_t bits, T Vp)
{
    const int sy = a.nx, sz = a.nx * a.ny;
    const T ex_ = nbd<T, FULL>(V, idx, 1, bits, 0, Vp), wx = nbd<T, FULL>(V, idx, -1, bits, 1, Vp);
    const T ny_ = nbd<T, FULL>(V, idx, sy, bits, 2, Vp), sy_ = nbd<T, FULL>(V, idx, -sy, bits, 3, Vp);
    const T up = nbd<T, FULL>(V, idx, sz, bits, 4, Vp), dn = nbd<T, FULL>(V, idx, -sz, bits, 5, Vp);
    if (!ANISO) return a.Dperp * a.ih2 * ((ex_ + wx) + (ny_ + sy_) + (up + dn));
    const T fx = a.fib[t], fy = a.fib[a.pitch + t], fz = a.fib[2 * a.pitch + t];
    const T cx = a.gt[t], cy = a.gt[a.pitch + t], cz = a.gt[2 * a.pitch + t];
    const T dd = a.Dpar - a.Dperp;
    const T Dxx = a.Dperp + dd * fx * fx, Dyy = a.Dperp + dd * fy * fy;
    const T Dzz = a.Dperp + dd * fz * fz;
    const T Dxy = dd * fx * fy, Dxz = dd * fx * fz, Dyz = dd * fy * fz;
    const T exy = nbd<T, FULL>(V, idx, 1 + sy, bits, 6, Vp) + nbd<T, FULL>(V, idx, -1 - sy, bits, 7, Vp)
                  - nbd<T, FULL>(V, idx, 1 - sy, bits, 8, Vp) - nbd<T, FULL>(V, idx, -1 + sy, bits, 9, Vp);
    const T exz = nbd<T, FULL>(V, idx, 1 + sz, bits, 10, Vp) + nbd<T, FULL>(V, idx, -1 - sz, bits, 11, Vp)
                  - nbd<T, FULL>(V, idx, 1 - sz, bits, 12, Vp) - nbd<T, FULL>(V, idx, -1 + sz, bits, 13, Vp);
    const T eyz = nbd<T, FULL>(V, idx, sy + sz, bits, 14, Vp) + nbd<T, FULL>(V, idx, -sy - sz, bits, 15, Vp)
                  - nbd<T, FULL>(V, idx, sy - sz, bits, 16, Vp) - nbd<T, FULL>(V, idx, -sy + sz, bits, 17, Vp);
    return a.ih2 * (Dxx * (ex_ + wx) + Dyy * (ny_ + sy_) + Dzz * (up + dn)
                    + T(0.5) * (Dxy * exy + Dxz * exz + Dyz * eyz))
           + cx * (ex_ - wx) + cy * (ny_ - sy_) + cz * (up - dn);
}

// One workgroup = 256 tissue voxels of the list (sparse) or one 64 x 4 tile of a
// z plane (dense box).  Logical workgroup ids are dealt so that XCD k gets the
// k-th contiguous eighth of the domain.
template <typename T, class M, bool ANISO, bool DENSE>
__global__ __launch_bounds__(kBlock) void k_step(const StepArgs<T> a)
{
    const int lb = (int)(blockIdx.x % kXcd) * a.per_xcd + (int)(blockIdx.x / kXcd);
    if (lb >= a.nblk) return;

    int t, idx;
    uint32_t bits;
    bool full = false;
    if (DENSE) {
        // tile coordinates are workgroup-uniform (scalar unit)
        const int bx = lb % a.gx, r = lb / a.gx;
        const int by = r % a.gy, z = r / a.gy;
        const int x = bx * kTileX + (int)(threadIdx.x % kTileX);
        const int y = by * kTileY + (int)(threadIdx.x / kTileX);
        if (x >= a.nx || y >= a.ny) return;
        idx = x + a.nx * (y + a.ny * z);
        t = idx;
        full = bx > 0 && (bx + 1) * kTileX < a.nx && by > 0 && (by + 1) * kTileY < a.ny && z > 0 &&
               z + 1 < a.nz;
        const uint32_t px = x + 1 < a.nx, mx = x > 0, py = y + 1 < a.ny, my = y > 0;
        const uint32_t pz = z + 1 < a.nz, mz = z > 0;
        bits = px | mx << 1 | py << 2 | my << 3 | pz << 4 | mz << 5;
        if (ANISO) {
            bits |= (px & py) << 6 | (mx & my) << 7 | (px & my) << 8 | (mx & py) << 9;
            bits |= (px & pz) << 10 | (mx & mz) << 11 | (px & mz) << 12 | (mx & pz) << 13;
            bits |= (py & pz) << 14 | (my & mz) << 15 | (py & mz) << 16 | (my & pz) << 17;
        }
    } else {
        t = lb * kBlock + (int)threadIdx.x;
        if (t >= a.nact) return;
        idx = a.idx[t];
        bits = a.nbr[t];
    }

    const T *__restrict__ V = a.Vin;
    const T Vp = V[idx];
    const T LV = full ? laplacian<T, ANISO, true>(a, V, t, idx, bits, Vp)
                      : laplacian<T, ANISO, false>(a, V, t, idx, bits, Vp);

    // stimulus current
    T Is = T(0);
    if (a.stim_on) {
        const uint32_t sb = a.stimbits[t] & a.stim_on;
        for (int s = 0; s < a.nstim; s++)
            if ((sb >> s) & 1u) Is += a.stim_amp[s];
    }

    // kinetics
    T g[M::NV > 1 ? M::NV - 1 : 1];
#pragma unroll
    for (int i = 0; i < M::NV - 1; i++) g[i] = a.st[i * a.pitch + t];
    const T Vin = a.split ? Vp + a.dt * LV : Vp;
    const T r = M::advance(a.prm, Vin, g, a.dt);
    const T Vn = a.split ? Vin + a.dt * (r + Is) : Vp + a.dt * (r + Is + LV);
#pragma unroll
    for (int i = 0; i < M::NV - 1; i++) a.st[i * a.pitch + t] = g[i];
    a.Vout[idx] = Vn;

    // activation time / peak / APD90 (per-voxel threshold-crossing recorder)
    if (a.rec) {
        uint8_t s0 = a.status[t];
        if (s0 != 3) {
            uint8_t s = s0;
            if (s == 0 && Vp < a.theta && Vn >= a.theta) {
                a.at[t] = a.tn + a.dt * (a.theta - Vp) / (Vn - Vp);
                s = 1;
            }
            if (s == 1 && Vn < Vp) {
                a.vmax[t] = Vp;
                const T rest = a.vrep[t];
                a.vrep[t] = rest + T(0.1) * (Vp - rest);
                s = 2;
            }
            if (s == 2) {
                const T vr = a.vrep[t];
                if (Vp >= vr && Vn < vr) {
                    a.apd[t] = a.tn + a.dt * (Vp - vr) / (Vp - Vn) - a.at[t];
                    s = 3;
                }
            }
            if (s != s0) a.status[t] = s;
        }
    }
}

template <typename T, class M>
static hipError_t launch_m(int aniso, const StepArgs<T> &a, hipStream_t s)
{
    const dim3 grid(a.per_xcd * kXcd), block(kBlock);
    if (a.dense) {
        if (aniso) hipLaunchKernelGGL((k_step<T, M, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_step<T, M, false, true>), grid, block, 0, s, a);
    } else {
        if (aniso) hipLaunchKernelGGL((k_step<T, M, true, false>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_step<T, M, false, false>), grid, block, 0, s, a);
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
    case 4: return launch_m<T, kin::Crn<T>>(aniso, a, s);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_step<float>(int, int, const StepArgs<float> &, hipStream_t);
template hipError_t launch_step<double>(int, int, const StepArgs<double> &, hipStream_t);

}  // namespace bbx
