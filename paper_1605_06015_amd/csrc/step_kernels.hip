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

template <typename T>
__device__ __forceinline__ T nbdiff(const T *__restrict__ V, int64_t idx, int64_t off,
                                    uint32_t bits, int b, T Vp)
{
    return ((bits >> b) & 1u) ? V[idx + off] - Vp : T(0);
}

template <typename T, class M, bool ANISO>
__global__ __launch_bounds__(kBlock) void k_step(const StepArgs<T> a)
{
    const int lb = (int)(blockIdx.x % kXcd) * a.per_xcd + (int)(blockIdx.x / kXcd);
    if (lb >= a.nblk) return;
    const int64_t t = (int64_t)lb * kBlock + threadIdx.x;
    if (t >= a.nact) return;

    const int64_t sy = a.nx, sz = (int64_t)a.nx * a.ny;
    int64_t idx;
    uint32_t bits;
    if (a.dense) {
        idx = t;
        const int64_t r = t / a.nx;
        const int x = (int)(t - r * a.nx);
        const int z = (int)(r / a.ny);
        const int y = (int)(r - (int64_t)z * a.ny);
        const uint32_t px = x + 1 < a.nx, mx = x > 0, py = y + 1 < a.ny, my = y > 0;
        const uint32_t pz = z + 1 < a.nz, mz = z > 0;
        bits = px | mx << 1 | py << 2 | my << 3 | pz << 4 | mz << 5;
        if (ANISO) {
            bits |= (px & py) << 6 | (mx & my) << 7 | (px & my) << 8 | (mx & py) << 9;
            bits |= (px & pz) << 10 | (mx & mz) << 11 | (px & mz) << 12 | (mx & pz) << 13;
            bits |= (py & pz) << 14 | (my & mz) << 15 | (py & mz) << 16 | (my & pz) << 17;
        }
    } else {
        idx = a.idx[t];
        bits = a.nbr[t];
    }

    const T *__restrict__ V = a.Vin;
    const T Vp = V[idx];
    T LV;
    if (!ANISO) {
        T s = nbdiff(V, idx, 1, bits, 0, Vp) + nbdiff(V, idx, -1, bits, 1, Vp)
              + nbdiff(V, idx, sy, bits, 2, Vp) + nbdiff(V, idx, -sy, bits, 3, Vp)
              + nbdiff(V, idx, sz, bits, 4, Vp) + nbdiff(V, idx, -sz, bits, 5, Vp);
        LV = a.Dperp * a.ih2 * s;
    } else {
        const T fx = a.fib[t], fy = a.fib[a.pitch + t], fz = a.fib[2 * a.pitch + t];
        const T cx = a.gt[t], cy = a.gt[a.pitch + t], cz = a.gt[2 * a.pitch + t];
        const T dd = a.Dpar - a.Dperp;
        const T Dxx = a.Dperp + dd * fx * fx, Dyy = a.Dperp + dd * fy * fy;
        const T Dzz = a.Dperp + dd * fz * fz;
        const T Dxy = dd * fx * fy, Dxz = dd * fx * fz, Dyz = dd * fy * fz;
        const T ex_ = nbdiff(V, idx, 1, bits, 0, Vp), wx = nbdiff(V, idx, -1, bits, 1, Vp);
        const T ny_ = nbdiff(V, idx, sy, bits, 2, Vp), sy_ = nbdiff(V, idx, -sy, bits, 3, Vp);
        const T up = nbdiff(V, idx, sz, bits, 4, Vp), dn = nbdiff(V, idx, -sz, bits, 5, Vp);
        const T exy = nbdiff(V, idx, 1 + sy, bits, 6, Vp) + nbdiff(V, idx, -1 - sy, bits, 7, Vp)
                      - nbdiff(V, idx, 1 - sy, bits, 8, Vp) - nbdiff(V, idx, -1 + sy, bits, 9, Vp);
        const T exz = nbdiff(V, idx, 1 + sz, bits, 10, Vp) + nbdiff(V, idx, -1 - sz, bits, 11, Vp)
                      - nbdiff(V, idx, 1 - sz, bits, 12, Vp) - nbdiff(V, idx, -1 + sz, bits, 13, Vp);
        const T eyz = nbdiff(V, idx, sy + sz, bits, 14, Vp) + nbdiff(V, idx, -sy - sz, bits, 15, Vp)
                      - nbdiff(V, idx, sy - sz, bits, 16, Vp) - nbdiff(V, idx, -sy + sz, bits, 17, Vp);
        LV = a.ih2 * (Dxx * (ex_ + wx) + Dyy * (ny_ + sy_) + Dzz * (up + dn)
                      + T(0.5) * (Dxy * exy + Dxz * exz + Dyz * eyz))
             + cx * (ex_ - wx) + cy * (ny_ - sy_) + cz * (up - dn);
    }

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
    const int grid = a.per_xcd * kXcd;
    if (aniso)
        hipLaunchKernelGGL((k_step<T, M, true>), dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_step<T, M, false>), dim3(grid), dim3(kBlock), 0, s, a);
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
