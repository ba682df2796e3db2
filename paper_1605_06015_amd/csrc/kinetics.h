// Device-side cell kinetics for the fused step kernel.
//
// Each model provides NV (state variables including V), GATE0 (variables
// GATE0..NV-1 are gating variables) and
//   T advance(const T* prm, T V, T* g, T dt, const float* tab):  given the
// voltage the kinetics see (V_n, or V* in the split scheme) and the other state
// variables g[0..NV-2], it returns the kinetic part of dV/dt (= -I_ion, with a
// positive stimulus depolarising) and advances g in place by one step:
// forward Euler (eq (Euler)) for concentrations and recovery variables,
// Rush-Larsen for gates -- y+ = y_inf + (y - y_inf) exp(-dt/tau), the exact
// solution of y' = (y_inf - y)/tau with the voltage frozen (eqs (gate), (RL),
// (RLcoeff), with the two coefficients in the order that makes it exact).
// `tab` is the optional table of voltage-only terms (CrnTab), else unused.  With
// the policy U = Rate (below) advance() instead leaves dy/dt of every variable in g
// (same return value): the right-hand side the RK4 integrator needs.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace bbx {
namespace kin {

// FP32 uses the hardware transcendental units (v_exp_f32, v_log_f32, v_rcp_f32:
// about 1 ulp) instead of the correctly rounded library routines, which cost
// 5-15 VALU instructions each; FP64 keeps the library routines.  The FP32
// error budget is set against the FP64 oracle by the tolerance tests.
__device__ __forceinline__ float ex(float x) { return __expf(x); }
__device__ __forceinline__ double ex(double x) { return exp(x); }
__device__ __forceinline__ float lg(float x) { return __logf(x); }
__device__ __forceinline__ double lg(double x) { return log(x); }
__device__ __forceinline__ float sq(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double sq(double x) { return sqrt(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float dv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double dv(double a, double b) { return a / b; }

// z / (e^z - 1).  Near z = 0 the quotient is 0/0; there the Bernoulli series
// 1 - z/2 + z^2/12 - z^4/720 + z^6/30240 replaces it (next term z^8/1209600).
// FP64 switches at |z| < 1e-3 (series error < 1e-30) and divides by expm1;
// FP32 switches at |z| < 0.1 (series error < 1e-14), beyond which e^z - 1
// loses at most a few ulp to cancellation.
__device__ __forceinline__ double bern(double z)
{
    if (fabs(z) < 1e-3) return 1.0 - z * (0.5 - z * (1.0 / 12.0));
    return z / expm1(z);
}
__device__ __forceinline__ float bern(float z)
{
    if (fabsf(z) < 0.1f) {
        const float z2 = z * z;
        return 1.0f - 0.5f * z + z2 * (1.0f / 12.0f - z2 * (1.0f / 720.0f - z2 * (1.0f / 30240.0f)));
    }
    return dv(z, __expf(z) - 1.0f);
}

// Rush-Larsen step written with the total transition rate k = 1/tau.
template <typename T>
__device__ __forceinline__ T rl_rate(T y, T yinf, T k, T dt)
{
    return yinf + (y - yinf) * ex(-dt * k);
}

// Rush-Larsen step of a gate given opening/closing rates (eq (gate)).
template <typename T>
__device__ __forceinline__ T rl_ab(T y, T a, T b, T dt)
{
    T k = a + b;
    return rl_rate(y, a * rcp(k), k, dt);
}

// tanh: the library routine in FP64; in FP32 1 - 2/(e^{2x} + 1) on the hardware
// exp/rcp units (tends to +-1 correctly as e^{2x} overflows or underflows).
__device__ __forceinline__ double th(double x) { return tanh(x); }
__device__ __forceinline__ float th(float x) { return 1.0f - 2.0f * rcp(ex(2.0f * x) + 1.0f); }

// Logistic 1 / (1 + e^x).
template <typename T>
__device__ __forceinline__ T lgs(T x)
{
    return rcp(T(1) + ex(x));
}

// How advance() treats each variable it updates.  Step: one step of the explicit
// scheme -- forward Euler y + dt r for concentrations and recovery variables (eq
// (Euler)), Rush-Larsen y_inf + (y - y_inf) e^{-dt k} for gates (k = 1/tau).  Rate:
// the right-hand side itself, dy/dt = r or k (y_inf - y), which the classical
// fourth-order Runge-Kutta integrator evaluates at its four stages (the `rk4` solver
// of "Kinetics solvers").  The Step forms keep the operand order of each model's
// update (y + dt r, y + dt s e, e^{-dt k}, e^{-dt m k}).
struct Step {
    static constexpr bool kRate = false;
    template <typename T> __device__ static T eu(T y, T r, T dt) { return y + dt * r; }
    template <typename T> __device__ static T eus(T y, T s, T e, T dt) { return y + dt * s * e; }
    template <typename T> __device__ static T rl(T y, T yinf, T k, T dt) { return rl_rate(y, yinf, k, dt); }
    // CRN voltage terms: the one-step factor e^{-dt k} (e^{-dt m k}) and its use
    template <typename T> __device__ static T fac(T k, T dt) { return ex(-dt * k); }
    template <typename T> __device__ static T facm(T m, T k, T dt) { return ex(-dt * m * k); }
    template <typename T> __device__ static T rlf(T y, T yinf, T f) { return yinf + (y - yinf) * f; }
};
struct Rate {
    static constexpr bool kRate = true;
    template <typename T> __device__ static T eu(T, T r, T) { return r; }
    template <typename T> __device__ static T eus(T, T s, T e, T) { return s * e; }
    template <typename T> __device__ static T rl(T y, T yinf, T k, T) { return k * (yinf - y); }
    template <typename T> __device__ static T fac(T k, T) { return k; }
    template <typename T> __device__ static T facm(T m, T k, T) { return m * k; }
    template <typename T> __device__ static T rlf(T y, T yinf, T k) { return k * (yinf - y); }
};

// ---------------------------------------------------------------- pure diffusion
template <typename T>
struct None {
    static constexpr int NV = 1, GATE0 = 1;
    template <class U = Step>
    __device__ static T advance(const T *, T, T *, T, const float *) { return T(0); }
};

// ---------------------------------------------------------------- Barkley (1991)
// u' = u (1 - u)(u - (v + b)/a) / eps,  v' = u - v.   prm = {a, b, eps}
template <typename T>
struct Barkley {
    static constexpr int NV = 2, GATE0 = 2;
    template <class U = Step>
    __device__ static T advance(const T *p, T u, T *g, T dt, const float *)
    {
        T v = g[0];
        T uth = (v + p[1]) / p[0];
        g[0] = U::eu(v, (u - v), dt);
        return u * (T(1) - u) * (u - uth) / p[2];
    }
};

// ---------------------------------------------------------------- ZFK / Nagumo
// V' = V (V - alpha)(1 - V)   (eq (ZFKbidomV)).   prm = {alpha}
template <typename T>
struct Zfk {
    static constexpr int NV = 1, GATE0 = 1;
    template <class U = Step>
    __device__ static T advance(const T *p, T V, T *, T, const float *)
    {
        return V * (V - p[0]) * (T(1) - V);
    }
};

// ---------------------------------------------------------------- cubic FHN
// u' = (u - u^3/3 - v)/eps,  v' = eps (u + beta - gamma v)   (eq (FHN)).
template <typename T>
struct Fhn {
    static constexpr int NV = 2, GATE0 = 2;
    template <class U = Step>
    __device__ static T advance(const T *p, T u, T *g, T dt, const float *)
    {
        T v = g[0];
        g[0] = U::eus(v, p[0], (u + p[1] - p[2] * v), dt);
        return (u - u * u * u * T(1.0 / 3.0) - v) / p[0];
    }
};

// ---------------------------------------------------------------- four-variable minimal model
// Bueno-Orovio, Cherry & Fenton (2008), the four-variable member of the
// Fenton-Karma family cited in "Cell models"; transcribed from that
// publication, epicardial parameter set.  State u, v, w, s (u dimensionless,
// time in ms); step function H(x) = [x > 0].
//   du/dt = -(J_fi + J_so + J_si)
//   J_fi = -v H(u - th_v)(u - th_v)(u_u - u)/tau_fi
//   J_so = (u - u_o)(1 - H(u - th_w))/tau_o + H(u - th_w)/tau_so
//   J_si = -H(u - th_w) w s / tau_si
// v, w, s relax linearly towards u-dependent steady states (Rush-Larsen):
//   v -> (u < th_v- ? 1 : 0) with tau_v- below th_v, -> 0 with tau_v+ above;
//   w -> w_inf with tau_w- below th_w, -> 0 with tau_w+ above;
//   s -> (1 + tanh(k_s (u - u_s)))/2 with tau_s.
// prm = {tau_fi, tau_so1, tau_si, tau_w+} (epicardial 0.11, 30.0181, 1.8875, 200).
template <typename T>
struct Fk4 {
    static constexpr int NV = 4, GATE0 = 1;
    template <class U = Step>
    __device__ static T advance(const T *p, T u, T *g, T dt, const float *)
    {
        const T thv = T(0.3), thw = T(0.13), thvm = T(0.006), tho = T(0.006);
        const bool Hv = u > thv, Hw = u > thw, Hvm = u > thvm, Ho = u > tho;
        const T v = g[0], w = g[1], s = g[2];
        // currents
        const T tso = p[1] + (T(0.9957) - p[1]) * (T(1) + th(T(2.0458) * (u - T(0.65)))) * T(0.5);
        const T to = Ho ? T(6) : T(400);
        const T Jfi = Hv ? dv(-v * (u - thv) * (T(1.55) - u), p[0]) : T(0);
        const T Jso = Hw ? rcp(tso) : dv(u, to);
        const T Jsi = Hw ? dv(-w * s, p[2]) : T(0);
        // gates
        // each gate: one Rush-Larsen step with the branch's steady state and rate
        // selected first (one exponential per gate)
        const T vinf = u < thvm ? T(1) : T(0);
        const T kvm = Hvm ? T(1.0 / 1150.0) : T(1.0 / 60.0);
        g[0] = U::rl(v, Hv ? T(0) : vinf, Hv ? T(1.0 / 1.4506) : kvm, dt);
        const T twm = T(60) + (T(15) - T(60)) * (T(1) + th(T(65) * (u - T(0.03)))) * T(0.5);
        const T winf = Ho ? T(0.94) : T(1) - dv(u, T(0.07));
        g[1] = U::rl(w, Hw ? T(0) : winf, rcp(Hw ? p[3] : twm), dt);
        const T sinf = (T(1) + th(T(2.0994) * (u - T(0.9087)))) * T(0.5);
        g[2] = U::rl(s, sinf, Hw ? T(1.0 / 16.0) : T(1.0 / 2.7342), dt);
        return -(Jfi + Jso + Jsi);
    }
};

// ---------------------------------------------------------------- ten Tusscher-Panfilov 2006
// ten Tusscher & Panfilov (2006) human ventricular model, epicardial cell, as
// cited in "Cell models"; transcribed from its publications (the 2004 model
// paper for the unchanged currents, the 2006 paper for the L-type current and
// the subspace calcium dynamics).  g = K_i, Na_i, Ca_i, Ca_ss, Ca_SR, Rbar, Xr1,
// Xr2, Xs, m, h, j, d, f, f2, fCass, s, r (V in mV, currents pA/pF, mM, ms).
// Concentrations and Rbar: forward Euler of the published derivatives with
// rapid-buffering factors; the twelve gates: Rush-Larsen.
namespace tp {
constexpr double kRTF = 8314.472 * 310.0 / 96485.3415;  // mV
constexpr double kF = 96485.3415;
constexpr double kCm = 0.185, kVc = 0.016404, kVsr = 0.001094, kVss = 0.00005468;
constexpr double kKo = 5.4, kNao = 140.0, kCao = 2.0;
constexpr double kNaCaDen = (87.5 * 87.5 * 87.5 + 140.0 * 140.0 * 140.0) * (1.38 + 2.0);
}  // namespace tp

template <typename T>
struct Tp06 {
    static constexpr int NV = 19, GATE0 = 7;
    template <class U = Step>
    __device__ static T advance(const T *, T V, T *g, T dt, const float *)
    {
        using namespace tp;
        const T Ki = g[0], Nai = g[1], Cai = g[2], Cass = g[3], CaSR = g[4], Rb = g[5];
        const T RTF = T(kRTF), iRTF = T(1.0 / kRTF);
        const T EK = RTF * lg(dv(T(kKo), Ki)), ENa = RTF * lg(dv(T(kNao), Nai));
        const T EKs = RTF * lg(dv(T(kKo + 0.03 * kNao), Ki + T(0.03) * Nai));
        const T ECa = T(0.5) * RTF * lg(dv(T(kCao), Cai));

        const T m = g[9], h = g[10], j = g[11];
        const T INa = T(14.838) * m * m * m * h * j * (V - ENa);
        // L-type: 2F (0.25 Ca_ss e^z - Ca_o) z/(e^z - 1), z = 2 (V - 15) F/(RT)
        const T z = T(2) * (V - T(15)) * iRTF;
        const T ICaL = T(3.980e-5) * g[12] * g[13] * g[14] * g[15] * T(2.0 * kF)
                       * (T(0.25) * Cass * ex(z) - T(kCao)) * bern(z);
        const T Ito = T(0.294) * g[17] * g[16] * (V - EK);
        const T IKr = T(0.153) * T(1.0) * g[6] * g[7] * (V - EK);     // sqrt(Ko/5.4) = 1
        const T IKs = T(0.392) * g[8] * g[8] * (V - EKs);
        const T aK1 = dv(T(0.1), T(1) + ex(T(0.06) * (V - EK - T(200))));
        const T bK1 = dv(T(3) * ex(T(0.0002) * (V - EK + T(100))) + ex(T(0.1) * (V - EK - T(10))),
                         T(1) + ex(T(-0.5) * (V - EK)));
        const T IK1 = T(5.405) * T(1.0) * dv(aK1, aK1 + bK1) * (V - EK);
        const T eg = ex(T(0.35) * V * iRTF), eg1 = ex(T(-0.65) * V * iRTF);
        const T INaCa = T(1000.0) * dv(eg * Nai * Nai * Nai * T(kCao) - eg1 * T(kNao * kNao * kNao) * Cai * T(2.5),
                                       T(kNaCaDen) * (T(1) + T(0.1) * eg1));
        const T INaK = T(2.724 * kKo) * dv(Nai, T(kKo + 1.0) * (Nai + T(40))
                                                   * (T(1) + T(0.1245) * ex(T(-0.1) * V * iRTF)
                                                      + T(0.0353) * ex(-V * iRTF)));
        const T IpCa = T(0.1238) * dv(Cai, T(0.0005) + Cai);
        const T IpK = T(0.0146) * dv(V - EK, T(1) + ex((T(25) - V) * T(1.0 / 5.98)));
        const T IbNa = T(0.00029) * (V - ENa);
        const T IbCa = T(0.000592) * (V - ECa);

        // calcium handling
        const T ec = dv(T(1.5), CaSR);
        const T kcasr = T(2.5) - dv(T(1.5), T(1) + ec * ec);
        const T k1 = dv(T(0.15), kcasr), k2 = T(0.045) * kcasr;
        const T c2 = Cass * Cass;
        const T O = dv(k1 * c2 * Rb, T(0.060) + k1 * c2);
        const T Irel = T(0.102) * O * (CaSR - Cass);
        const T Iup = dv(T(0.006375), T(1) + dv(T(0.00025 * 0.00025), Cai * Cai));
        const T Ileak = T(0.00036) * (CaSR - Cai);
        const T Ixfer = T(0.0038) * (Cass - Cai);
        const T bc = rcp(T(1) + dv(T(0.2 * 0.001), (Cai + T(0.001)) * (Cai + T(0.001))));
        const T bsr = rcp(T(1) + dv(T(10.0 * 0.3), (CaSR + T(0.3)) * (CaSR + T(0.3))));
        const T bss = rcp(T(1) + dv(T(0.4 * 0.00025), (Cass + T(0.00025)) * (Cass + T(0.00025))));
        const T c2f = T(kCm / (kVc * kF));
        g[0] = U::eu(Ki, (-(IK1 + Ito + IKr + IKs - T(2) * INaK + IpK) * c2f), dt);
        g[1] = U::eu(Nai, (-(INa + IbNa + T(3) * INaK + T(3) * INaCa) * c2f), dt);
        g[2] = U::eu(Cai, (bc * ((Ileak - Iup) * T(kVsr / kVc) + Ixfer
                                 - (IbCa + IpCa - T(2) * INaCa) * T(kCm / (2.0 * kVc * kF)))), dt);
        g[3] = U::eu(Cass, (bss * (-ICaL * T(kCm / (2.0 * kVss * kF)) + Irel * T(kVsr / kVss)
                                   - Ixfer * T(kVc / kVss))), dt);
        g[4] = U::eu(CaSR, (bsr * (Iup - Irel - Ileak)), dt);
        g[5] = U::eu(Rb, (-k2 * Cass * Rb + T(0.005) * (T(1) - Rb)), dt);

        // gates
        g[6] = U::rl(g[6], lgs((T(-26) - V) * T(1.0 / 7.0)),
                       rcp(dv(T(450), T(1) + ex((T(-45) - V) * T(0.1))) * dv(T(6), T(1) + ex((V + T(30)) * T(1.0 / 11.5)))), dt);
        g[7] = U::rl(g[7], lgs((V + T(88)) * T(1.0 / 24.0)),
                       rcp(dv(T(3), T(1) + ex((T(-60) - V) * T(0.05))) * dv(T(1.12), T(1) + ex((V - T(60)) * T(0.05)))), dt);
        g[8] = U::rl(g[8], lgs((T(-5) - V) * T(1.0 / 14.0)),
                       rcp(dv(T(1400), sq(T(1) + ex((T(5) - V) * T(1.0 / 6.0)))) * rcp(T(1) + ex((V - T(35)) * T(1.0 / 15.0))) + T(80)), dt);
        const T mi = lgs((T(-56.86) - V) * T(1.0 / 9.03));
        g[9] = U::rl(m, mi * mi,
                       rcp(rcp(T(1) + ex((T(-60) - V) * T(0.2)))
                           * (dv(T(0.1), T(1) + ex((V + T(35)) * T(0.2))) + dv(T(0.10), T(1) + ex((V - T(50)) * T(1.0 / 200.0))))), dt);
        const T hi = lgs((V + T(71.55)) * T(1.0 / 7.43));
        T ah, bh, aj, bj;
        if (V >= T(-40)) {
            ah = T(0);
            bh = dv(T(0.77), T(0.13) * (T(1) + ex(-(V + T(10.66)) * T(1.0 / 11.1))));
            aj = T(0);
            bj = dv(T(0.6) * ex(T(0.057) * V), T(1) + ex(T(-0.1) * (V + T(32))));
        } else {
            ah = T(0.057) * ex(-(V + T(80)) * T(1.0 / 6.8));
            bh = T(2.7) * ex(T(0.079) * V) + T(3.1e5) * ex(T(0.3485) * V);
            aj = dv((T(-2.5428e4) * ex(T(0.2444) * V) - T(6.948e-6) * ex(T(-0.04391) * V)) * (V + T(37.78)),
                    T(1) + ex(T(0.311) * (V + T(79.23))));
            bj = dv(T(0.02424) * ex(T(-0.01052) * V), T(1) + ex(T(-0.1378) * (V + T(40.14))));
        }
        g[10] = U::rl(h, hi * hi, ah + bh, dt);
        g[11] = U::rl(j, hi * hi, aj + bj, dt);
        g[12] = U::rl(g[12], lgs((T(-8) - V) * T(1.0 / 7.5)),
                        rcp((dv(T(1.4), T(1) + ex((T(-35) - V) * T(1.0 / 13.0))) + T(0.25))
                                * dv(T(1.4), T(1) + ex((V + T(5)) * T(0.2)))
                            + rcp(T(1) + ex((T(50) - V) * T(0.05)))), dt);
        const T v27 = V + T(27);
        g[13] = U::rl(g[13], lgs((V + T(20)) * T(1.0 / 7.0)),
                        rcp(T(1102.5) * ex(-v27 * v27 * T(1.0 / 225.0)) + dv(T(200), T(1) + ex((T(13) - V) * T(0.1)))
                            + dv(T(180), T(1) + ex((V + T(30)) * T(0.1))) + T(20)), dt);
        g[14] = U::rl(g[14], T(0.67) * lgs((V + T(35)) * T(1.0 / 7.0)) + T(0.33),
                        rcp(T(562) * ex(-v27 * v27 * T(1.0 / 240.0)) + dv(T(31), T(1) + ex((T(25) - V) * T(0.1)))
                            + dv(T(80), T(1) + ex((V + T(30)) * T(0.1)))), dt);
        const T cq = (Cass * T(20)) * (Cass * T(20));
        g[15] = U::rl(g[15], dv(T(0.6), T(1) + cq) + T(0.4), rcp(dv(T(80), T(1) + cq) + T(2)), dt);
        const T v45 = V + T(45), v40 = V + T(40);
        g[16] = U::rl(g[16], lgs((V + T(20)) * T(0.2)),
                        rcp(T(85) * ex(-v45 * v45 * T(1.0 / 320.0)) + dv(T(5), T(1) + ex((V - T(20)) * T(0.2))) + T(3)), dt);
        g[17] = U::rl(g[17], lgs((T(20) - V) * T(1.0 / 6.0)),
                        rcp(T(9.5) * ex(-v40 * v40 * T(1.0 / 1800.0)) + T(0.8)), dt);

        return -(INa + ICaL + Ito + IKr + IKs + IK1 + INaCa + INaK + IpCa + IpK + IbNa + IbCa);
    }
};

// ---------------------------------------------------------------- Courtemanche 1998
// Courtemanche, Ramirez & Nattel, Am J Physiol 275:H301 (1998), human atrial
// myocyte; the paper uses it for its scaling runs.  Transcribed from that
// publication.  g = Na_i, K_i, Ca_i, Ca_up, Ca_rel, m, h, j, oa, oi, ua, ui,
// xr, xs, d, f, fCa, u, v, w.  Currents per unit capacitance (pA/pF).
//
// The kinetics split into terms that depend on V alone (CRN_V entries: for the
// twelve voltage-gated gates the steady state y_inf and the one-step
// Rush-Larsen factor e^{-dt/tau}; six voltage factors of currents) and the
// rest.  The voltage-only terms are either evaluated directly (Crn) or read
// from a table over V built once per time step size (CrnTab: the start-time
// tabulation of the paper's `rushlarsen` device, "Exponential solvers").
enum {
    CV_M, CV_MA, CV_H, CV_HA, CV_J, CV_JA, CV_OA, CV_OAA, CV_OI, CV_OIA, CV_UA, CV_UAA,
    CV_UI, CV_UIA, CV_XR, CV_XRA, CV_XS, CV_XSA, CV_D, CV_DA, CV_F, CV_FA, CV_W, CV_WA,
    CV_K1, CV_KR, CV_GKUR, CV_FNAK, CV_EG, CV_EG1, CRN_V = 32  // 30 used, padded to 32
};

namespace crn {
constexpr double kRTF = 8.3143 * 310.0 / 96.4867;  // mV
constexpr double kF = 96.4867;                    // C/mmol
constexpr double kCm = 100.0;                     // pF
constexpr double kVi = 13668.0, kVup = 1109.52, kVrel = 96.48;  // um^3
constexpr double kNao = 140.0, kKo = 5.4, kCao = 1.8;           // mM
constexpr double kNaCa = 1600.0 / ((87.5 * 87.5 * 87.5 + kNao * kNao * kNao) * (1.38 + kCao));
}  // namespace crn

// Voltage-only terms at V for time step dt.
template <class U, typename T>
__device__ __forceinline__ void crn_vterms(T V, T dt, T *c)
{
    using namespace crn;
    // fast sodium current gates m, h, j from opening/closing rates
    {
        T am = T(3.2) * bern(T(-0.1) * (V + T(47.13)));
        T bm = T(0.08) * ex(-V * T(1.0 / 11.0));
        T ah, bh, aj, bj;
        if (V < T(-40)) {
            ah = T(0.135) * ex((V + T(80)) * T(-1.0 / 6.8));
            bh = T(3.56) * ex(T(0.079) * V) + T(3.1e5) * ex(T(0.35) * V);
            aj = (T(-127140) * ex(T(0.2444) * V) - T(3.474e-5) * ex(T(-0.04391) * V))
                 * (V + T(37.78)) * lgs(T(0.311) * (V + T(79.23)));
            bj = T(0.1212) * ex(T(-0.01052) * V) * lgs(T(-0.1378) * (V + T(40.14)));
        } else {
            ah = T(0);
            bh = T(1.0 / 0.13) * lgs((V + T(10.66)) * T(-1.0 / 11.1));
            aj = T(0);
            bj = T(0.3) * ex(T(-2.535e-7) * V) * lgs(T(-0.1) * (V + T(32)));
        }
        T k = am + bm;
        c[CV_M] = am * rcp(k);
        c[CV_MA] = U::fac(k, dt);
        k = ah + bh;
        c[CV_H] = ah * rcp(k);
        c[CV_HA] = U::fac(k, dt);
        k = aj + bj;
        c[CV_J] = aj * rcp(k);
        c[CV_JA] = U::fac(k, dt);
    }
    // transient outward (oa, oi) and ultrarapid (ua, ui) potassium gates; the
    // activation rates of oa and ua share one form; Q10 factor 3
    {
        T a_act = T(0.65) * rcp(ex((V + T(10)) * T(-1.0 / 8.5)) + ex((V - T(30)) * T(-1.0 / 59.0)));
        T b_act = T(0.65) * rcp(T(2.5) + ex((V + T(82)) * T(1.0 / 17.0)));
        const T ea = U::facm(T(3), (a_act + b_act), dt);
        c[CV_OA] = lgs((V + T(20.47)) * T(-1.0 / 17.54));
        c[CV_OAA] = ea;
        c[CV_UA] = lgs((V + T(30.3)) * T(-1.0 / 9.6));
        c[CV_UAA] = ea;
        T aoi = rcp(T(18.53) + ex((V + T(113.7)) * T(1.0 / 10.95)));
        T boi = rcp(T(35.56) + ex((V + T(1.26)) * T(-1.0 / 7.44)));
        c[CV_OI] = lgs((V + T(43.1)) * T(1.0 / 5.3));
        c[CV_OIA] = U::facm(T(3), (aoi + boi), dt);
        T aui = rcp(T(21) + ex((V - T(185)) * T(-1.0 / 28.0)));
        T bui = ex((V - T(158)) * T(1.0 / 16.0));
        c[CV_UI] = lgs((V - T(99.45)) * T(1.0 / 27.48));
        c[CV_UIA] = U::facm(T(3), (aui + bui), dt);
    }
    // rapid and slow delayed rectifier gates
    {
        T axr = T(0.0015) * bern(-(V + T(14.1)) * T(0.2));
        T bxr = T(7.3898e-5 * 5.1237) * bern((V - T(3.3328)) * T(1.0 / 5.1237));
        c[CV_XR] = lgs((V + T(14.1)) * T(-1.0 / 6.5));
        c[CV_XRA] = U::fac((axr + bxr), dt);
        T axs = T(4e-5 * 17.0) * bern((V - T(19.9)) * T(-1.0 / 17.0));
        T bxs = T(3.5e-5 * 9.0) * bern((V - T(19.9)) * T(1.0 / 9.0));
        c[CV_XS] = rcp(sq(T(1) + ex((V - T(19.9)) * T(-1.0 / 12.7))));
        c[CV_XSA] = U::facm(T(2), (axs + bxs), dt);
    }
    // L-type calcium gates d, f
    {
        T zd = (V + T(10)) * T(1.0 / 6.24);
        // 1/tau_d = 0.035 (V+10)(1 + e^{-zd}) / (1 - e^{-zd}) = 0.035*6.24 bern(-zd)(1 + e^{-zd})
        T kd = T(0.035 * 6.24) * bern(-zd) * (T(1) + ex(-zd));
        c[CV_D] = lgs((V + T(10)) * T(-1.0 / 8.0));
        c[CV_DA] = U::fac(kd, dt);
        T vv = V + T(10);
        T kf = (T(0.0197) * ex(T(-0.0337 * 0.0337) * vv * vv) + T(0.02)) * T(1.0 / 9.0);
        c[CV_F] = lgs((V + T(28)) * T(1.0 / 6.9));
        c[CV_FA] = U::fac(kf, dt);
    }
    // release gate w
    {
        T zw = (V - T(7.9)) * T(0.2);
        // 1/tau_w = (1 + 0.3 e^{-zw}) (V - 7.9) / (6 (1 - e^{-zw})) = 5 bern(-zw)(1 + 0.3 e^{-zw}) / 6
        T kw = T(5.0 / 6.0) * bern(-zw) * (T(1) + T(0.3) * ex(-zw));
        c[CV_W] = T(1) - lgs((V - T(40)) * T(-1.0 / 17.0));
        c[CV_WA] = U::fac(kw, dt);
    }
    // voltage factors of currents
    {
        const T vf = V * T(1.0 / kRTF);
        c[CV_K1] = lgs(T(0.07) * (V + T(80)));
        c[CV_KR] = lgs((V + T(15)) * T(1.0 / 22.4));
        c[CV_GKUR] = T(0.005) + T(0.05) * lgs((V - T(15)) * T(-1.0 / 13.0));
        const T sigma = T((8.006372134620099 - 1.0) / 7.0);  // (e^{[Na]o/67.3} - 1)/7
        c[CV_FNAK] = rcp(T(1) + T(0.1245) * ex(T(-0.1) * vf) + T(0.0365) * sigma * ex(-vf));
        const T eg = ex(T(0.35) * vf), eg1 = ex(T(-0.65) * vf);
        const T den = T(kNaCa) * rcp(T(1) + T(0.1) * eg1);
        c[CV_EG] = eg * den;
        c[CV_EG1] = eg1 * den;
    }
    c[30] = c[31] = T(0);
}

// Everything that is not univariate in V, given the voltage-only terms c.
template <class U, typename T>
__device__ __forceinline__ T crn_rest(T V, T *g, T dt, const T *c)
{
    using namespace crn;
    const T RTF = T(kRTF);
    T Nai = g[0], Ki = g[1], Cai = g[2], Caup = g[3], Carel = g[4];

    // reversal potentials
    const T ENa = RTF * lg(dv(T(kNao), Nai));
    const T EK = RTF * lg(dv(T(kKo), Ki));
    const T ECa = T(0.5) * RTF * lg(dv(T(kCao), Cai));
    const T dK = V - EK;

    // currents from the state at step n, then the Rush-Larsen gate updates
    T m = g[5], h = g[6], j = g[7];
    const T INa = T(7.8) * m * m * m * h * j * (V - ENa);
    g[5] = U::rlf(m, c[CV_M], c[CV_MA]);
    g[6] = U::rlf(h, c[CV_H], c[CV_HA]);
    g[7] = U::rlf(j, c[CV_J], c[CV_JA]);

    T oa = g[8], oi = g[9], ua = g[10], ui = g[11];
    const T Ito = T(0.1652) * oa * oa * oa * oi * dK;
    const T IKur = c[CV_GKUR] * ua * ua * ua * ui * dK;
    g[8] = U::rlf(oa, c[CV_OA], c[CV_OAA]);
    g[9] = U::rlf(oi, c[CV_OI], c[CV_OIA]);
    g[10] = U::rlf(ua, c[CV_UA], c[CV_UAA]);
    g[11] = U::rlf(ui, c[CV_UI], c[CV_UIA]);

    T xr = g[12], xs = g[13];
    const T IKr = T(0.029411765) * xr * dK * c[CV_KR];
    const T IKs = T(0.12941176) * xs * xs * dK;
    g[12] = U::rlf(xr, c[CV_XR], c[CV_XRA]);
    g[13] = U::rlf(xs, c[CV_XS], c[CV_XSA]);

    const T IK1 = T(0.09) * dK * c[CV_K1];

    T d = g[14], f = g[15], fCa = g[16];
    const T ICaL = T(0.12375) * d * f * fCa * (V - T(65));
    g[14] = U::rlf(d, c[CV_D], c[CV_DA]);
    g[15] = U::rlf(f, c[CV_F], c[CV_FA]);
    g[16] = U::rl(fCa, rcp(T(1) + Cai * T(1.0 / 0.00035)), T(0.5), dt);

    // pumps, exchanger and background currents
    const T rNa = dv(T(10), Nai);
    const T INaK = T(0.59933874 * kKo / (kKo + 1.5)) * c[CV_FNAK] * rcp(T(1) + rNa * sq(rNa));
    const T INaCa = c[CV_EG] * Nai * Nai * Nai * T(kCao) - c[CV_EG1] * T(kNao * kNao * kNao) * Cai;
    const T IbCa = T(0.001131) * (V - ECa);
    const T IbNa = T(0.0006744375) * (V - ENa);
    const T IpCa = T(0.275) * dv(Cai, T(0.0005) + Cai);

    // sarcoplasmic reticulum fluxes (mM/ms), release gates u, v, w
    T u = g[17], v = g[18], w = g[19];
    const T Irel = T(30) * u * u * v * w * (Carel - Cai);
    const T Itr = (Caup - Carel) * T(1.0 / 180.0);
    const T Iup = T(0.005) * dv(Cai, Cai + T(0.00092));
    const T Ileak = T(0.005 / 15.0) * Caup;
    {
        // release trigger from SR release and sarcolemmal Ca entry (currents in pA)
        T Fn = T(1e-12 * kVrel) * Irel - T(5e-13 / kF * kCm) * (T(0.5) * ICaL - T(0.2) * INaCa);
        T s1 = lgs(-(Fn - T(3.4175e-13)) * T(1.0 / 13.67e-16));
        g[17] = U::rl(u, s1, T(1.0 / 8.0), dt);
        g[18] = U::rl(v, T(1) - lgs(-(Fn - T(6.835e-14)) * T(1.0 / 13.67e-16)),
                        rcp(T(1.91) + T(2.09) * s1), dt);
        g[19] = U::rlf(w, c[CV_W], c[CV_WA]);
    }

    // concentrations (forward Euler); current-to-flux factor Cm / (F Vi)
    const T c2f = T(kCm / (kF * kVi));
    g[0] = U::eus(Nai, c2f, (T(-3) * (INaK + INaCa) - IbNa - INa), dt);
    g[1] = U::eus(Ki, c2f, (T(2) * INaK - IK1 - Ito - IKur - IKr - IKs), dt);
    {
        T ct = Cai + T(0.0005), cc = Cai + T(0.00238);
        T bt = T(0.07 * 0.0005) * rcp(ct * ct);
        T bc = T(0.05 * 0.00238) * rcp(cc * cc);
        T src = T(0.5) * c2f * (T(2) * INaCa - IpCa - ICaL - IbCa)
                + (T(kVup) * (Ileak - Iup) + T(kVrel) * Irel) * T(1.0 / kVi);
        g[2] = U::eus(Cai, src, rcp(T(1) + bt + bc), dt);
        g[3] = U::eu(Caup, (Iup - Ileak - Itr * T(kVrel / kVup)), dt);
        T cq = Carel + T(0.8);
        T bq = T(10.0 * 0.8) * rcp(cq * cq);
        g[4] = U::eus(Carel, (Itr - Irel), rcp(T(1) + bq), dt);
    }

    return -(INa + IK1 + Ito + IKur + IKr + IKs + IbNa + IbCa + INaK + IpCa + INaCa + ICaL);
}

template <typename T>
struct Crn {
    static constexpr int NV = 21, GATE0 = 6;  // variables GATE0.. are gates in [0, 1]
    template <class U = Step>
    __device__ static T advance(const T *, T V, T *g, T dt, const float *)
    {
        T c[CRN_V];
        crn_vterms<U>(V, dt, c);
        return crn_rest<U>(V, g, dt, c);
    }
};

// Table of the voltage-only terms: header {vmin, 1/dv, n} in the first CRN_V
// floats, then n nodes of CRN_V floats at V = vmin + k dv.  Linear
// interpolation; V outside the table is clamped to its range.
__device__ __forceinline__ void crn_lookup(const float *tab, float V, float *c)
{
    const float vmin = tab[0], inv = tab[1];
    const int n = (int)tab[2];
    const float x = (V - vmin) * inv;
    int i = (int)floorf(x);
    i = i < 0 ? 0 : (i > n - 2 ? n - 2 : i);
    const float f = fminf(fmaxf(x - (float)i, 0.0f), 1.0f);
    const float4 *p0 = (const float4 *)(tab + CRN_V * (1 + i));
    const float4 *p1 = p0 + CRN_V / 4;
#pragma unroll
    for (int q = 0; q < CRN_V / 4; q++) {
        const float4 a = p0[q], b = p1[q];
        c[4 * q + 0] = a.x + f * (b.x - a.x);
        c[4 * q + 1] = a.y + f * (b.y - a.y);
        c[4 * q + 2] = a.z + f * (b.z - a.z);
        c[4 * q + 3] = a.w + f * (b.w - a.w);
    }
}

// CRN with tabulated voltage-only terms (FP32 only).
struct CrnTab {
    static constexpr int NV = 21, GATE0 = 6;
    // the table holds the Step forms (e^{-dt/tau}): one scheme step only
    template <class U = Step>
    __device__ static float advance(const float *, float V, float *g, float dt, const float *tab)
    {
        static_assert(!U::kRate, "tabulated terms are one-step factors");
        float c[CRN_V];
        crn_lookup(tab, V, c);
        return crn_rest<Step>(V, g, dt, c);
    }
};

}  // namespace kin
}  // namespace bbx
