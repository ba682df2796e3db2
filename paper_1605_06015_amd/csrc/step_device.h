// Per-voxel device routines of the fused step, shared by the plain step kernels,
// the surrogate step and its fallback (so a fallback voxel gets exactly the
// plain path's arithmetic).  See step_kernels.hip for the stencil formula.
#pragma once

#include "bbx_internal.h"
#include "kinetics.h"

namespace bbx {

// V_{p+off} - V_p if neighbour bit b is set (tissue), else 0.  FULL: the whole
// workgroup is known to be interior (every neighbour is tissue).  The load is
// unconditional, from the voxel itself when the neighbour is absent (always in
// bounds), so that the gathers issue back to back without branches.
template <typename T, bool FULL>
__device__ __forceinline__ T nbd(const T *__restrict__ V, int idx, int off, uint32_t bits, int b,
                                 T Vp)
{
    if (FULL) return V[idx + off] - Vp;
    const bool on = (bits >> b) & 1u;
    const T v = V[on ? idx + off : idx];
    return on ? v - Vp : T(0);
}

// (L V)_p in the difference form of the paper's weights (see step_kernels.hip).
template <typename T, bool ANISO, bool FULL>
__device__ __forceinline__ T laplacian(const StepArgs<T> &a, const T *__restrict__ V, int t,
                                       int idx, uint32_t bits, T Vp)
{
    const int sy = a.nx, sz = a.nx * a.ny;
    const T ex_ = nbd<T, FULL>(V, idx, 1, bits, 0, Vp), wx = nbd<T, FULL>(V, idx, -1, bits, 1, Vp);
    const T ny_ = nbd<T, FULL>(V, idx, sy, bits, 2, Vp), sy_ = nbd<T, FULL>(V, idx, -sy, bits, 3, Vp);
    const T up = nbd<T, FULL>(V, idx, sz, bits, 4, Vp), dn = nbd<T, FULL>(V, idx, -sz, bits, 5, Vp);
    if (!ANISO) return a.Dperp * a.ih2 * ((ex_ + wx) + (ny_ + sy_) + (up + dn));
    const T *gp = a.geo + 6 * (int64_t)t;
    const T fx = gp[0], fy = gp[1], fz = gp[2];
    const T cx = gp[3], cy = gp[4], cz = gp[5];
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

// Activation / peak / APD90 recorder (per-voxel threshold-crossing test on the
// pair V_n -> V_{n+1} at time tn = n dt).  A: any argument block with the
// recorder fields (status, theta, dt, at, vmax, vrep, apd).
template <typename T, class A, typename I>
__device__ __forceinline__ void record_event(const A &a, I t, T tn, T Vp, T Vn)
{
    uint8_t s0 = a.status[t];
    if (s0 == 3) return;
    uint8_t s = s0;
    if (s == 0 && Vp < a.theta && Vn >= a.theta) {
        a.at[t] = tn + a.dt * (a.theta - Vp) / (Vn - Vp);
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
            a.apd[t] = tn + a.dt * (Vp - vr) / (Vp - Vn) - a.at[t];
            s = 3;
        }
    }
    if (s != s0) a.status[t] = s;
}

// The step's clock: the stimuli that are on and t_n.  Host-evaluated for direct
// launches; in a replayed graph read from the device step counter (same arithmetic as
// the host: windows in whole steps, t_n = n dt rounded from FP64).
template <typename T>
struct Clock {
    uint32_t stim_on;
    T tn;
};

template <typename T>
__device__ __forceinline__ Clock<T> step_clock(const StepArgs<T> &a)
{
    if (!a.nbase) return {a.stim_on, a.tn};
    const int64_t n = *a.nbase + a.jstep;
    uint32_t on = 0;
    for (int s = 0; s < a.nstim; s++) {
        const StimWin w = a.win[s];
        if (n < w.n0 || w.len <= 0) continue;
        const int64_t r = n - w.n0;
        bool hit;
        if (w.per <= 0) {
            hit = r < w.len;
        } else {
            const int64_t c = r / w.per;
            hit = !(w.count > 0 && c >= w.count) && (r - c * w.per) < w.len;
        }
        if (hit) on |= 1u << s;
    }
    return {on, (T)((double)n * a.dt64)};
}

template <typename T>
__device__ __forceinline__ void record_voxel(const StepArgs<T> &a, int t, T Vp, T Vn, T tn)
{
    if (!a.rec) return;
    record_event(a, t, tn, Vp, Vn);
}

// Stimulus current of tissue voxel t at this step.
template <typename T>
__device__ __forceinline__ T stim_current(const StepArgs<T> &a, int t, uint32_t stim_on)
{
    T Is = T(0);
    if (stim_on) {
        const uint32_t sb = a.stimbits[t] & stim_on;
        for (int s = 0; s < a.nstim; s++)
            if ((sb >> s) & 1u) Is += a.stim_amp[s];
    }
    return Is;
}

// Box index and neighbour bits of tissue voxel t.  Dense boxes derive them from
// the coordinates (t is the box index).
template <typename T>
__device__ __forceinline__ void voxel_of(const StepArgs<T> &a, int t, int &idx, uint32_t &bits)
{
    if (!a.dense) {
        idx = a.idx[t];
        bits = a.nbr[t];
        return;
    }
    idx = t;
    const int r = t / a.nx, x = t - r * a.nx, z = r / a.ny, y = r - z * a.ny;
    const uint32_t px = x + 1 < a.nx, mx = x > 0, py = y + 1 < a.ny, my = y > 0;
    const uint32_t pz = z + 1 < a.nz, mz = z > 0;
    bits = px | mx << 1 | py << 2 | my << 3 | pz << 4 | mz << 5;
    bits |= (px & py) << 6 | (mx & my) << 7 | (px & my) << 8 | (mx & py) << 9;
    bits |= (px & pz) << 10 | (mx & mz) << 11 | (px & mz) << 12 | (mx & pz) << 13;
    bits |= (py & pz) << 14 | (my & mz) << 15 | (py & mz) << 16 | (my & pz) << 17;
}

// Classical fourth-order Runge-Kutta step of one voxel's kinetics (the `rk4` solver of
// "Kinetics solvers") for dV/dt = -I_ion(V, g) + F, dg/dt = G(V, g), with the forcing F
// (stimulus, plus the Laplacian in the additive scheme) held at its step-n value
// through the four stages, as the Euler update holds it: k_i are the right-hand sides
// at y0, y0 + dt/2 k1, y0 + dt/2 k2, y0 + dt k3, and y+ = y0 + dt/6 (k1 + 2k2 + 2k3 + k4).
// Every variable, gates included (dg/dt = (g_inf - g)/tau), takes the same stages.
// g holds g0 on entry and g+ on return; returns V+.
template <typename T, class M>
__device__ __forceinline__ T rk4_voxel(const StepArgs<T> &a, T V0, T *g, T F)
{
    constexpr int NG = M::NV > 1 ? M::NV - 1 : 1;
    const T dt = a.dt, hdt = T(0.5) * a.dt;
    T y0[NG], k[NG], acc[NG];
#pragma unroll
    for (int i = 0; i < M::NV - 1; i++) y0[i] = k[i] = g[i];
    // k1
    T kV = M::template advance<kin::Rate>(a.prm, V0, k, dt, nullptr) + F;
    T accV = kV;
#pragma unroll
    for (int i = 0; i < M::NV - 1; i++) {
        acc[i] = k[i];
        k[i] = y0[i] + hdt * k[i];
    }
    // k2
    kV = M::template advance<kin::Rate>(a.prm, V0 + hdt * kV, k, dt, nullptr) + F;
    accV += T(2) * kV;
#pragma unroll
    for (int i = 0; i < M::NV - 1; i++) {
        acc[i] += T(2) * k[i];
        k[i] = y0[i] + hdt * k[i];
    }
    // k3
    kV = M::template advance<kin::Rate>(a.prm, V0 + hdt * kV, k, dt, nullptr) + F;
    accV += T(2) * kV;
#pragma unroll
    for (int i = 0; i < M::NV - 1; i++) {
        acc[i] += T(2) * k[i];
        k[i] = y0[i] + dt * k[i];
    }
    // k4
    kV = M::template advance<kin::Rate>(a.prm, V0 + dt * kV, k, dt, nullptr) + F;
    accV += kV;
    const T w = dt * T(1.0 / 6.0);
#pragma unroll
    for (int i = 0; i < M::NV - 1; i++) g[i] = y0[i] + w * (acc[i] + k[i]);
    return V0 + w * accV;
}

// Everything after the Laplacian for one voxel: stimulus, kinetics, stores and
// the recorder.  RK4: the kinetics take the fourth-order Runge-Kutta step instead of
// forward Euler / Rush-Larsen.
template <typename T, class M, bool NT = false, bool RK4 = false>
__device__ __forceinline__ void update_voxel(const StepArgs<T> &a, const Clock<T> &ck, int t, int idx,
                                             T Vp, T LV)
{
    const T Is = stim_current(a, t, ck.stim_on);

    T g[M::NV > 1 ? M::NV - 1 : 1];
#pragma unroll
    for (int i = 0; i < M::NV - 1; i++) {
        // the state is read once per step: on large boxes it streams past the caches
        // (measured: TP06 double shell 1.010 -> 0.972 ms/step; streaming its stores too,
        // or the geometry, was slower)
        if constexpr (NT) g[i] = __builtin_nontemporal_load(&a.st[i * a.pitch + t]);
        else g[i] = a.st[i * a.pitch + t];
    }
    const T Vin = a.split ? Vp + a.dt * LV : Vp;
    T Vn;
    if constexpr (RK4) {
        Vn = rk4_voxel<T, M>(a, Vin, g, a.split ? Is : Is + LV);
    } else {
        const T r = M::advance(a.prm, Vin, g, a.dt, a.tab);
        Vn = a.split ? Vin + a.dt * (r + Is) : Vp + a.dt * (r + Is + LV);
    }
#pragma unroll
    for (int i = 0; i < M::NV - 1; i++) a.st[i * a.pitch + t] = g[i];
    if constexpr (NT)
        __builtin_nontemporal_store(Vn, &a.Vout[idx]);   // streaming write (a.nt)
    else
        a.Vout[idx] = Vn;

    record_voxel(a, t, Vp, Vn, ck.tn);
}

}  // namespace bbx
