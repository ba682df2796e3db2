/*
 * Oracle for the monodomain explicit step -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64, scalar-loop reference of what the GPU library computes.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with the
 * GPU library; the two meet only through caller-supplied arrays.
 *
 * Paper: Antonioletti et al., "BeatBox -- HPC simulation environment for
 * biophysically and anatomically realistic cardiac electrophysiology"
 * (arXiv:1605.06015).  Citations name the paper's sections and equations.
 *
 * Layout: box index idx = x + nx*(y + ny*z); tissue ("active") voxels are
 * listed in increasing box order in act[]; state is [nvar][nbox] (only tissue
 * entries are read or written).  Stencil weights are kept literally, 27 per
 * tissue voxel, q = (dx,dy,dz) stored at (dz+1)*9 + (dy+1)*3 + (dx+1).
 *
 * Parity status (every function below is pinned by the CPU tests unless this
 * list says otherwise):
 *   - weights, diffusion, Euler, Rush-Larsen, RK4, Barkley/ZFK/FHN steps, the
 *     phase-singularity finder: pinned (closed forms, invariants, brute force,
 *     plane-wave speed, orders of convergence).
 *   - weights at boundary voxels with variable fibres (the paper leaves the
 *     tensor of a void neighbour undefined; here it is the centre's): pinned by
 *     the vanishing of the tissue integral's drift under refinement (the
 *     continuous no-flux problem conserves it for any tensor).
 *   - Courtemanche-Ramirez-Nattel 1998 cell model: transcribed from the
 *     original model publication (not part of the paper); parity partially
 *     pinned, by that publication's resting state and action-potential shape,
 *     and by charge conservation of its concentration equations.
 *   - four-variable Fenton-Karma-type minimal model (Bueno-Orovio, Cherry &
 *     Fenton 2008, epicardial set): transcribed from that publication; pinned
 *     by its exact resting state and the closed-form subthreshold relaxation;
 *     its suprathreshold constants are partially pinned (action-potential shape).
 *   - ten Tusscher-Panfilov 2006 ventricular model (epicardial): transcribed
 *     from its publications; parity partially pinned, by its resting state,
 *     action-potential shape and charge conservation of its concentration
 *     equations.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { M_NONE = 0, M_BARKLEY = 1, M_ZFK = 2, M_FHN = 3, M_CRN = 4, M_FK4 = 5, M_TP06 = 6 };
enum { S_ADDITIVE = 0, S_SPLIT = 1 };
enum { I_EULER_RL = 0, I_RK4 = 1 };

#define NVAR_MAX 32

/* ------------------------------------------------------------------------- */
/* Geometry: "Monodomain diffusion and boundary conditions", eqs (Lu),      */
/* (nonflux), (sigma) and the weight formulas that follow them.             */
/* ------------------------------------------------------------------------- */

/* D_jk = Dperp delta_jk + (Dpar - Dperp) f_j f_k  -- eq (sigma), f a unit vector.
 * With no fibre field the tissue is isotropic with coefficient Dperp. */
static int tensor_of(const double *fibre, int64_t idx, double Dpar, double Dperp,
                     double D[3][3])
{
    double f[3] = {0, 0, 0};
    double g = 0.0;
    if (fibre) {
        for (int j = 0; j < 3; j++) f[j] = fibre[3 * idx + j];
        double n = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        if (!(n >= 1e-12)) return -1;   /* cannot be a unit vector */
        for (int j = 0; j < 3; j++) f[j] /= n;
        g = Dpar - Dperp;
    }
    for (int j = 0; j < 3; j++)
        for (int k = 0; k < 3; k++)
            D[j][k] = (j == k ? Dperp : 0.0) + g * f[j] * f[k];
    return 0;
}

static int in_box(int nx, int ny, int nz, int x, int y, int z)
{
    return x >= 0 && y >= 0 && z >= 0 && x < nx && y < ny && z < nz;
}

/* chi_p: grid indicator of the tissue; outside the box counts as void. */
static int chi(int nx, int ny, int nz, const uint8_t *mask, int x, int y, int z)
{
    if (!in_box(nx, ny, nz, x, y, z)) return 0;
    return mask[(int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z)] != 0;
}

/* Stencil weights W^p_q = Wbar^p_q + Wtilde^p_q for every tissue voxel p and
 * q in {0,+-1}^3, with W^p_0 = -sum_{q!=0} W^p_q.
 *  Wbar:   chi_{p+q}/h^2 * { D^p_jj on faces q=+-q_j;
 *                            +D^p_jk/2 on edges q=+-(q_j+q_k);
 *                            -D^p_jk/2 on edges q=+-(q_j-q_k);  0 on corners }
 *          (each unordered pair j<k gives one edge weight, as quadratic
 *          exactness requires);
 *  Wtilde: chi_{p+q} chi_{p-q}/(4h^2) * (+-) sum_j (D^{p+q_j}_jk - D^{p-q_j}_jk)
 *          on faces q=+-q_k, 0 elsewhere.
 * D at a void or out-of-box neighbour inside Wtilde is replaced by D^p
 * (the paper leaves that case open).  Returns 0, or -1 if a tissue fibre has
 * (near) zero length. */
int orc_weights(int nx, int ny, int nz, double h, const uint8_t *mask,
                const double *fibre, double Dpar, double Dperp,
                int64_t nact, const int64_t *act, double *W)
{
    const double ih2 = 1.0 / (h * h);
    int bad = 0;
    /* voxels are independent: the loop is split over threads, results unchanged */
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t a = 0; a < nact; a++) {
        int64_t idx = act[a];
        int x = (int)(idx % nx), y = (int)((idx / nx) % ny), z = (int)(idx / ((int64_t)nx * ny));
        double Dp[3][3];
        if (tensor_of(fibre, idx, Dpar, Dperp, Dp)) { bad = 1; continue; }

        /* D at p+q_j and p-q_j for j = 0..2 (substituted by D^p when void). */
        double Dplus[3][3][3], Dminus[3][3][3];
        for (int j = 0; j < 3; j++) {
            int e[3] = {0, 0, 0};
            e[j] = 1;
            for (int s = -1; s <= 1; s += 2) {
                int xx = x + s * e[0], yy = y + s * e[1], zz = z + s * e[2];
                double (*dst)[3] = (s > 0) ? Dplus[j] : Dminus[j];
                if (chi(nx, ny, nz, mask, xx, yy, zz)) {
                    int64_t nidx = (int64_t)xx + (int64_t)nx * ((int64_t)yy + (int64_t)ny * zz);
                    if (tensor_of(fibre, nidx, Dpar, Dperp, dst)) bad = 1;
                } else {
                    memcpy(dst, Dp, sizeof(Dp));
                }
            }
        }

        double *w = W + 27 * a;
        double sum = 0.0;
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int qi = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                    int q[3] = {dx, dy, dz};
                    int nnz = (dx != 0) + (dy != 0) + (dz != 0);
                    double val = 0.0;
                    if (nnz == 0) { w[qi] = 0.0; continue; }
                    int cp = chi(nx, ny, nz, mask, x + dx, y + dy, z + dz);
                    int cm = chi(nx, ny, nz, mask, x - dx, y - dy, z - dz);
                    if (nnz == 1) {
                        int k = (dx != 0) ? 0 : (dy != 0) ? 1 : 2;
                        double sgn = (double)q[k];
                        val += cp * Dp[k][k] * ih2;                         /* Wbar, face */
                        double div = 0.0;
                        for (int j = 0; j < 3; j++) div += Dplus[j][j][k] - Dminus[j][j][k];
                        val += cp * cm * 0.25 * ih2 * sgn * div;            /* Wtilde */
                    } else if (nnz == 2) {
                        int j = -1, k = -1;
                        for (int t = 0; t < 3; t++)
                            if (q[t] != 0) { if (j < 0) j = t; else k = t; }
                        double sgn = (q[j] == q[k]) ? 0.5 : -0.5;           /* +-(q_j+q_k) vs +-(q_j-q_k) */
                        val += cp * sgn * Dp[j][k] * ih2;                   /* Wbar, edge */
                    }
                    w[qi] = val;
                    sum += val;
                }
        w[13] = -sum;
    }
    return bad ? -1 : 0;
}

/* (L u)_p = sum_q W^p_q u_{p+q}, written in the equivalent difference form
 * sum_{q!=0} W^p_q (u_{p+q} - u_p) (the difference form: equal in exact arithmetic,
 * and a constant field stays exactly constant); out-of-box q have W = 0. */
static double apply_L(int nx, int ny, int nz, const double *w, const double *u, int64_t idx)
{
    int x = (int)(idx % nx), y = (int)((idx / nx) % ny), z = (int)(idx / ((int64_t)nx * ny));
    double up = u[idx], acc = 0.0;
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                int qi = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                if (qi == 13 || w[qi] == 0.0) continue;
                if (!in_box(nx, ny, nz, x + dx, y + dy, z + dz)) continue;
                int64_t n = (int64_t)(x + dx) + (int64_t)nx * ((int64_t)(y + dy) + (int64_t)ny * (z + dz));
                acc += w[qi] * (u[n] - up);
            }
    return acc;
}

/* Apply L once to a field (used by the invariant tests). */
void orc_apply_L(int nx, int ny, int nz, int64_t nact, const int64_t *act,
                 const double *W, const double *u, double *out)
{
    for (int64_t a = 0; a < nact; a++) out[a] = apply_L(nx, ny, nz, W + 27 * a, u, act[a]);
}

/* ------------------------------------------------------------------------- */
/* Cell models.  Each fills, for state y (y[0] = V):                          */
/*   rate[i]  = dy_i/dt for variables advanced by forward Euler               */
/*              (rate[0] = -I_ion: the kinetic part of the voltage equation);  */
/*   inf[i], tau[i] for gating variables advanced by Rush-Larsen.             */
/* ------------------------------------------------------------------------- */

int orc_nvar(int model)
{
    switch (model) {
    case M_NONE: return 1;
    case M_BARKLEY: return 2;
    case M_ZFK: return 1;
    case M_FHN: return 2;
    case M_CRN: return 21;
    case M_FK4: return 4;
    case M_TP06: return 19;
    default: return -1;
    }
}

int orc_nparams(int model)
{
    switch (model) {
    case M_NONE: return 0;
    case M_BARKLEY: return 3;
    case M_ZFK: return 1;
    case M_FHN: return 3;
    case M_CRN: return 0;
    case M_FK4: return 4;
    case M_TP06: return 0;
    default: return -1;
    }
}

/* Which variables are gates (Rush-Larsen) for a model. */
static int is_gate(int model, int i)
{
    if (model == M_CRN) return i >= 6;
    if (model == M_FK4) return i >= 1;
    if (model == M_TP06) return i >= 7;
    return 0;
}

/* Barkley (1991): u' = eps^-1 u (1-u) (u - (v+b)/a),  v' = u - v.
 * The paper uses it as `fhnbkl` (Cell models; ez.bbs) without printing it. */
static void barkley_rates(const double *p, const double *y, double *rate)
{
    double a = p[0], b = p[1], eps = p[2];
    double u = y[0], v = y[1];
    rate[0] = u * (1.0 - u) * (u - (v + b) / a) / eps;
    rate[1] = u - v;
}

/* ZFK / Nagumo / Schloegl kinetics, eq (ZFKbidomV): V' = V (V - alpha)(1 - V). */
static void zfk_rates(const double *p, const double *y, double *rate)
{
    double al = p[0], V = y[0];
    rate[0] = V * (V - al) * (1.0 - V);
}

/* Cubic FitzHugh-Nagumo `fhncub`, eq (FHN): u' = (u - u^3/3 - v)/eps,
 * v' = eps (u + beta - gamma v) (the ODE's cubic term; the discrete update's
 * printed square is taken as a misprint). */
static void fhn_rates(const double *p, const double *y, double *rate)
{
    double eps = p[0], bet = p[1], gam = p[2];
    double u = y[0], v = y[1];
    rate[0] = (u - u * u * u / 3.0 - v) / eps;
    rate[1] = eps * (u + bet - gam * v);
}

/* z / (exp(z) - 1), continued by its limit 1 at z = 0. */
static double z_over_expm1(double z)
{
    return z == 0.0 ? 1.0 : z / expm1(z);
}

/* Courtemanche, Ramirez & Nattel (1998) human atrial cell model, as cited in
 * "Cell models" and used for the scaling runs.  Transcribed from the original
 * model publication (its equations are not printed in the paper).  Currents
 * are in pA/pF (membrane capacitance 100 pF), concentrations in mM, time in ms.
 * State order: V, Na_i, K_i, Ca_i, Ca_up, Ca_rel, m, h, j, oa, oi, ua, ui,
 * xr, xs, d, f, fCa, u, v, w. */
static void crn_rates(const double *y, double *rate, double *inf, double *tau)
{
    const double R = 8.3143, T = 310.0, F = 96.4867;
    const double Cm = 100.0, Vi = 13668.0, Vup = 1109.52, Vrel = 96.48;
    const double Ko = 5.4, Nao = 140.0, Cao = 1.8;
    const double gNa = 7.8, gK1 = 0.09, gto = 0.1652, gKr = 0.029411765, gKs = 0.12941176;
    const double gCaL = 0.12375, gbCa = 0.001131, gbNa = 0.0006744375;
    const double INaKmax = 0.59933874, INaCamax = 1600.0, IpCamax = 0.275, Iupmax = 0.005;
    const double KmNai = 10.0, KmKo = 1.5, KmNa = 87.5, KmCa = 1.38, ksat = 0.1, gam = 0.35;
    const double krel = 30.0, Kup = 0.00092, Caupmax = 15.0;
    const double CMDNmax = 0.05, TRPNmax = 0.07, CSQNmax = 10.0;
    const double KmCMDN = 0.00238, KmTRPN = 0.0005, KmCSQN = 0.8;
    const double KQ10 = 3.0, tau_tr = 180.0;

    double V = y[0], Nai = y[1], Ki = y[2], Cai = y[3], Caup = y[4], Carel = y[5];
    double m = y[6], h = y[7], j = y[8], oa = y[9], oi = y[10], ua = y[11], ui = y[12];
    double xr = y[13], xs = y[14], d = y[15], f = y[16], fCa = y[17];
    double u = y[18], v = y[19], w = y[20];

    double RTF = R * T / F;
    double ENa = RTF * log(Nao / Nai);
    double EK = RTF * log(Ko / Ki);
    double ECa = 0.5 * RTF * log(Cao / Cai);

    /* membrane currents, pA/pF */
    double INa = gNa * m * m * m * h * j * (V - ENa);
    double IK1 = gK1 * (V - EK) / (1.0 + exp(0.07 * (V + 80.0)));
    double Ito = gto * oa * oa * oa * oi * (V - EK);
    double gKur = 0.005 + 0.05 / (1.0 + exp((V - 15.0) / -13.0));
    double IKur = gKur * ua * ua * ua * ui * (V - EK);
    double IKr = gKr * xr * (V - EK) / (1.0 + exp((V + 15.0) / 22.4));
    double IKs = gKs * xs * xs * (V - EK);
    double ICaL = gCaL * d * f * fCa * (V - 65.0);
    double sigma = (exp(Nao / 67.3) - 1.0) / 7.0;
    double fNaK = 1.0 / (1.0 + 0.1245 * exp(-0.1 * V / RTF) + 0.0365 * sigma * exp(-V / RTF));
    double INaK = INaKmax * fNaK / (1.0 + pow(KmNai / Nai, 1.5)) * Ko / (Ko + KmKo);
    double INaCa = INaCamax * (exp(gam * V / RTF) * Nai * Nai * Nai * Cao
                               - exp((gam - 1.0) * V / RTF) * Nao * Nao * Nao * Cai)
                   / ((KmNa * KmNa * KmNa + Nao * Nao * Nao) * (KmCa + Cao)
                      * (1.0 + ksat * exp((gam - 1.0) * V / RTF)));
    double IbCa = gbCa * (V - ECa);
    double IbNa = gbNa * (V - ENa);
    double IpCa = IpCamax * Cai / (0.0005 + Cai);

    /* calcium handling, mM/ms */
    double Irel = krel * u * u * v * w * (Carel - Cai);
    double Itr = (Caup - Carel) / tau_tr;
    double Iup = Iupmax / (1.0 + Kup / Cai);
    double Iupleak = Iupmax * Caup / Caupmax;

    double Iion = INa + IK1 + Ito + IKur + IKr + IKs + IbNa + IbCa + INaK + IpCa + INaCa + ICaL;
    rate[0] = -Iion;
    rate[1] = (-3.0 * INaK - 3.0 * INaCa - IbNa - INa) * Cm / (Vi * F);
    rate[2] = (2.0 * INaK - IK1 - Ito - IKur - IKr - IKs) * Cm / (Vi * F);
    double B1 = (2.0 * INaCa - IpCa - ICaL - IbCa) * Cm / (2.0 * Vi * F)
                + (Vup * (Iupleak - Iup) + Irel * Vrel) / Vi;
    double B2 = 1.0 + TRPNmax * KmTRPN / ((Cai + KmTRPN) * (Cai + KmTRPN))
                + CMDNmax * KmCMDN / ((Cai + KmCMDN) * (Cai + KmCMDN));
    rate[3] = B1 / B2;
    rate[4] = Iup - Iupleak - Itr * Vrel / Vup;
    rate[5] = (Itr - Irel) / (1.0 + CSQNmax * KmCSQN / ((Carel + KmCSQN) * (Carel + KmCSQN)));

    /* gates: inf and tau */
    double am = 3.2 * z_over_expm1(-0.1 * (V + 47.13));
    double bm = 0.08 * exp(-V / 11.0);
    double ah, bh, aj, bj;
    if (V < -40.0) {
        ah = 0.135 * exp((V + 80.0) / -6.8);
        bh = 3.56 * exp(0.079 * V) + 3.1e5 * exp(0.35 * V);
        aj = (-127140.0 * exp(0.2444 * V) - 3.474e-5 * exp(-0.04391 * V)) * (V + 37.78)
             / (1.0 + exp(0.311 * (V + 79.23)));
        bj = 0.1212 * exp(-0.01052 * V) / (1.0 + exp(-0.1378 * (V + 40.14)));
    } else {
        ah = 0.0;
        bh = 1.0 / (0.13 * (1.0 + exp((V + 10.66) / -11.1)));
        aj = 0.0;
        bj = 0.3 * exp(-2.535e-7 * V) / (1.0 + exp(-0.1 * (V + 32.0)));
    }
    tau[6] = 1.0 / (am + bm); inf[6] = am * tau[6];
    tau[7] = 1.0 / (ah + bh); inf[7] = ah * tau[7];
    tau[8] = 1.0 / (aj + bj); inf[8] = aj * tau[8];

    double aoa = 0.65 / (exp((V + 10.0) / -8.5) + exp((V - 30.0) / -59.0));
    double boa = 0.65 / (2.5 + exp((V + 82.0) / 17.0));
    tau[9] = 1.0 / (aoa + boa) / KQ10;
    inf[9] = 1.0 / (1.0 + exp((V + 20.47) / -17.54));
    double aoi = 1.0 / (18.53 + exp((V + 113.7) / 10.95));
    double boi = 1.0 / (35.56 + exp((V + 1.26) / -7.44));
    tau[10] = 1.0 / (aoi + boi) / KQ10;
    inf[10] = 1.0 / (1.0 + exp((V + 43.1) / 5.3));

    tau[11] = tau[9];   /* alpha_ua, beta_ua have the same form as alpha_oa, beta_oa */
    inf[11] = 1.0 / (1.0 + exp((V + 30.3) / -9.6));
    double aui = 1.0 / (21.0 + exp((V - 185.0) / -28.0));
    double bui = exp((V - 158.0) / 16.0);
    tau[12] = 1.0 / (aui + bui) / KQ10;
    inf[12] = 1.0 / (1.0 + exp((V - 99.45) / 27.48));

    double axr = 0.0003 * 5.0 * z_over_expm1(-(V + 14.1) / 5.0);
    double bxr = 7.3898e-5 * 5.1237 * z_over_expm1((V - 3.3328) / 5.1237);
    tau[13] = 1.0 / (axr + bxr);
    inf[13] = 1.0 / (1.0 + exp((V + 14.1) / -6.5));
    double axs = 4e-5 * 17.0 * z_over_expm1(-(V - 19.9) / 17.0);
    double bxs = 3.5e-5 * 9.0 * z_over_expm1((V - 19.9) / 9.0);
    tau[14] = 0.5 / (axs + bxs);
    inf[14] = 1.0 / sqrt(1.0 + exp((V - 19.9) / -12.7));

    double zd = (V + 10.0) / 6.24;
    tau[15] = 1.0 / (0.035 * 6.24 * z_over_expm1(-zd) * (1.0 + exp(-zd)));
    inf[15] = 1.0 / (1.0 + exp((V + 10.0) / -8.0));
    tau[16] = 9.0 / (0.0197 * exp(-0.0337 * 0.0337 * (V + 10.0) * (V + 10.0)) + 0.02);
    inf[16] = 1.0 / (1.0 + exp((V + 28.0) / 6.9));
    tau[17] = 2.0;
    inf[17] = 1.0 / (1.0 + Cai / 0.00035);

    /* Fn: release trigger, from SR release and sarcolemmal Ca flux (currents in pA) */
    double Fn = 1e-12 * Vrel * Irel - 5e-13 / F * (0.5 * ICaL * Cm - 0.2 * INaCa * Cm);
    tau[18] = 8.0;
    inf[18] = 1.0 / (1.0 + exp(-(Fn - 3.4175e-13) / 13.67e-16));
    tau[19] = 1.91 + 2.09 / (1.0 + exp(-(Fn - 3.4175e-13) / 13.67e-16));
    inf[19] = 1.0 - 1.0 / (1.0 + exp(-(Fn - 6.835e-14) / 13.67e-16));
    double zw = (V - 7.9) / 5.0;
    tau[20] = 6.0 / (5.0 * z_over_expm1(-zw) * (1.0 + 0.3 * exp(-zw)));
    inf[20] = 1.0 - 1.0 / (1.0 + exp(-(V - 40.0) / 17.0));
}

/* Four-variable minimal ventricular model of Bueno-Orovio, Cherry & Fenton
 * (J Theor Biol 2008), the "4-variable Fenton-Karma" family member cited with
 * the Fenton-Karma model in "Cell models"; transcribed from that publication,
 * epicardial parameter set.  State u (dimensionless), v, w, s; time in ms.
 * Step function H(x) = 1 for x > 0, else 0.  p = (tau_fi, tau_so1, tau_si,
 * tau_w+) are the per-tissue parameters (epicardial: 0.11, 30.0181, 1.8875,
 * 200); every other constant is the epicardial value.  v, w and s relax
 * linearly towards u-dependent steady states and are advanced by Rush-Larsen. */
static void fk4_rates(const double *p, const double *y, double *rate, double *inf, double *tau)
{
    const double tfi = p[0], tso1 = p[1], tsi = p[2], twp = p[3];
    const double uo = 0.0, uu = 1.55, thv = 0.3, thw = 0.13, thvm = 0.006, tho = 0.006;
    const double tv1m = 60.0, tv2m = 1150.0, tvp = 1.4506;
    const double tw1m = 60.0, tw2m = 15.0, kwm = 65.0, uwm = 0.03;
    const double to1 = 400.0, to2 = 6.0, tso2 = 0.9957, kso = 2.0458, uso = 0.65;
    const double ts1 = 2.7342, ts2 = 16.0, ks = 2.0994, us = 0.9087;
    const double twinf = 0.07, winf_star = 0.94;
    double u = y[0], v = y[1], w = y[2], s = y[3];
    int Hv = u > thv, Hw = u > thw, Hvm = u > thvm, Ho = u > tho;

    double tvm = Hvm ? tv2m : tv1m;
    double twm = tw1m + (tw2m - tw1m) * (1.0 + tanh(kwm * (u - uwm))) / 2.0;
    double tso = tso1 + (tso2 - tso1) * (1.0 + tanh(kso * (u - uso))) / 2.0;
    double ts = Hw ? ts2 : ts1;
    double to = Ho ? to2 : to1;
    double vinf = u < thvm ? 1.0 : 0.0;
    double winf = Ho ? winf_star : 1.0 - u / twinf;

    double Jfi = Hv ? -v * (u - thv) * (uu - u) / tfi : 0.0;
    double Jso = Hw ? 1.0 / tso : (u - uo) / to;
    double Jsi = Hw ? -w * s / tsi : 0.0;
    rate[0] = -(Jfi + Jso + Jsi);

    /* v: towards v_inf with tau_v- below theta_v, towards 0 with tau_v+ above */
    inf[1] = Hv ? 0.0 : vinf;
    tau[1] = Hv ? tvp : tvm;
    /* w: towards w_inf with tau_w- below theta_w, towards 0 with tau_w+ above */
    inf[2] = Hw ? 0.0 : winf;
    tau[2] = Hw ? twp : twm;
    /* s: towards (1 + tanh(k_s (u - u_s)))/2 with tau_s */
    inf[3] = (1.0 + tanh(ks * (u - us))) / 2.0;
    tau[3] = ts;
}

/* ten Tusscher & Panfilov (2006) human ventricular model, epicardial cell, as
 * cited in "Cell models"; transcribed from its publications (the 2004 model
 * paper for the unchanged currents, the 2006 paper for the L-type current and
 * the subspace calcium dynamics).  V in mV, currents in pA/pF, concentrations
 * in mM, time in ms.  State order: V, K_i, Na_i, Ca_i, Ca_ss, Ca_SR, Rbar,
 * Xr1, Xr2, Xs, m, h, j, d, f, f2, fCass, s, r.  The twelve gates (Xr1..r) use
 * Rush-Larsen; concentrations and the ryanodine-receptor variable Rbar use
 * forward Euler of their published derivatives (buffering by the rapid
 * equilibrium factors). */
static void tp06_rates(const double *y, double *rate, double *inf, double *tau)
{
    const double R = 8314.472, T = 310.0, F = 96485.3415;
    const double RTF = R * T / F;
    const double Cm = 0.185, Vc = 0.016404, Vsr = 0.001094, Vss = 0.00005468;
    const double Ko = 5.4, Nao = 140.0, Cao = 2.0;
    const double GNa = 14.838, GK1 = 5.405, Gto = 0.294, GKr = 0.153, GKs = 0.392, pKNa = 0.03;
    const double GCaL = 3.980e-5, kNaCa = 1000.0, gam = 0.35, KmCa = 1.38, KmNai = 87.5;
    const double ksat = 0.1, alf = 2.5, PNaK = 2.724, KmK = 1.0, KmNa = 40.0;
    const double GpK = 0.0146, GpCa = 0.1238, KpCa = 0.0005, GbNa = 0.00029, GbCa = 0.000592;
    const double Vmaxup = 0.006375, Kup = 0.00025, Vrel = 0.102, k1p = 0.15, k2p = 0.045;
    const double k3 = 0.060, k4 = 0.005, EC = 1.5, maxsr = 2.5, minsr = 1.0;
    const double Vleak = 0.00036, Vxfer = 0.0038, Bufc = 0.2, Kbufc = 0.001;
    const double Bufsr = 10.0, Kbufsr = 0.3, Bufss = 0.4, Kbufss = 0.00025;

    double V = y[0], Ki = y[1], Nai = y[2], Cai = y[3], Cass = y[4], CaSR = y[5], Rb = y[6];
    double xr1 = y[7], xr2 = y[8], xs = y[9], m = y[10], h = y[11], j = y[12];
    double d = y[13], f = y[14], f2 = y[15], fcass = y[16], sg = y[17], rg = y[18];

    double EK = RTF * log(Ko / Ki), ENa = RTF * log(Nao / Nai);
    double EKs = RTF * log((Ko + pKNa * Nao) / (Ki + pKNa * Nai));
    double ECa = 0.5 * RTF * log(Cao / Cai);

    double INa = GNa * m * m * m * h * j * (V - ENa);
    /* L-type: 4 (V-15) F^2/(RT) (0.25 Ca_ss e^z - Ca_o)/(e^z - 1), z = 2 (V-15) F/(RT)
     *       = 2 F (0.25 Ca_ss e^z - Ca_o) z/(e^z - 1) */
    double z = 2.0 * (V - 15.0) / RTF;
    double ICaL = GCaL * d * f * f2 * fcass * 2.0 * F * (0.25 * Cass * exp(z) - Cao) * z_over_expm1(z);
    double Ito = Gto * rg * sg * (V - EK);
    double IKr = GKr * sqrt(Ko / 5.4) * xr1 * xr2 * (V - EK);
    double IKs = GKs * xs * xs * (V - EKs);
    double aK1 = 0.1 / (1.0 + exp(0.06 * (V - EK - 200.0)));
    double bK1 = (3.0 * exp(0.0002 * (V - EK + 100.0)) + exp(0.1 * (V - EK - 10.0)))
                 / (1.0 + exp(-0.5 * (V - EK)));
    double IK1 = GK1 * sqrt(Ko / 5.4) * aK1 / (aK1 + bK1) * (V - EK);
    double eg = exp(gam * V / RTF), eg1 = exp((gam - 1.0) * V / RTF);
    double INaCa = kNaCa * (eg * Nai * Nai * Nai * Cao - eg1 * Nao * Nao * Nao * Cai * alf)
                   / ((KmNai * KmNai * KmNai + Nao * Nao * Nao) * (KmCa + Cao) * (1.0 + ksat * eg1));
    double INaK = PNaK * Ko * Nai / ((Ko + KmK) * (Nai + KmNa)
                                     * (1.0 + 0.1245 * exp(-0.1 * V / RTF) + 0.0353 * exp(-V / RTF)));
    double IpCa = GpCa * Cai / (KpCa + Cai);
    double IpK = GpK * (V - EK) / (1.0 + exp((25.0 - V) / 5.98));
    double IbNa = GbNa * (V - ENa);
    double IbCa = GbCa * (V - ECa);

    /* calcium handling */
    double kcasr = maxsr - (maxsr - minsr) / (1.0 + (EC / CaSR) * (EC / CaSR));
    double k1 = k1p / kcasr, k2 = k2p * kcasr;
    double O = k1 * Cass * Cass * Rb / (k3 + k1 * Cass * Cass);
    double Irel = Vrel * O * (CaSR - Cass);
    double Iup = Vmaxup / (1.0 + Kup * Kup / (Cai * Cai));
    double Ileak = Vleak * (CaSR - Cai);
    double Ixfer = Vxfer * (Cass - Cai);
    double bc = 1.0 / (1.0 + Bufc * Kbufc / ((Cai + Kbufc) * (Cai + Kbufc)));
    double bsr = 1.0 / (1.0 + Bufsr * Kbufsr / ((CaSR + Kbufsr) * (CaSR + Kbufsr)));
    double bss = 1.0 / (1.0 + Bufss * Kbufss / ((Cass + Kbufss) * (Cass + Kbufss)));

    rate[0] = -(INa + ICaL + Ito + IKr + IKs + IK1 + INaCa + INaK + IpCa + IpK + IbNa + IbCa);
    rate[1] = -(IK1 + Ito + IKr + IKs - 2.0 * INaK + IpK) * Cm / (Vc * F);
    rate[2] = -(INa + IbNa + 3.0 * INaK + 3.0 * INaCa) * Cm / (Vc * F);
    rate[3] = bc * ((Ileak - Iup) * Vsr / Vc + Ixfer - (IbCa + IpCa - 2.0 * INaCa) * Cm / (2.0 * Vc * F));
    rate[4] = bss * (-ICaL * Cm / (2.0 * Vss * F) + Irel * Vsr / Vss - Ixfer * Vc / Vss);
    rate[5] = bsr * (Iup - Irel - Ileak);
    rate[6] = -k2 * Cass * Rb + k4 * (1.0 - Rb);

    /* gates: steady states and time constants */
    inf[7] = 1.0 / (1.0 + exp((-26.0 - V) / 7.0));
    tau[7] = 450.0 / (1.0 + exp((-45.0 - V) / 10.0)) * 6.0 / (1.0 + exp((V + 30.0) / 11.5));
    inf[8] = 1.0 / (1.0 + exp((V + 88.0) / 24.0));
    tau[8] = 3.0 / (1.0 + exp((-60.0 - V) / 20.0)) * 1.12 / (1.0 + exp((V - 60.0) / 20.0));
    inf[9] = 1.0 / (1.0 + exp((-5.0 - V) / 14.0));
    tau[9] = 1400.0 / sqrt(1.0 + exp((5.0 - V) / 6.0)) / (1.0 + exp((V - 35.0) / 15.0)) + 80.0;
    double mi = 1.0 / (1.0 + exp((-56.86 - V) / 9.03));
    inf[10] = mi * mi;
    tau[10] = 1.0 / (1.0 + exp((-60.0 - V) / 5.0))
              * (0.1 / (1.0 + exp((V + 35.0) / 5.0)) + 0.10 / (1.0 + exp((V - 50.0) / 200.0)));
    double hi = 1.0 / (1.0 + exp((V + 71.55) / 7.43));
    double ah, bh, aj, bj;
    if (V >= -40.0) {
        ah = 0.0;
        bh = 0.77 / (0.13 * (1.0 + exp(-(V + 10.66) / 11.1)));
        aj = 0.0;
        bj = 0.6 * exp(0.057 * V) / (1.0 + exp(-0.1 * (V + 32.0)));
    } else {
        ah = 0.057 * exp(-(V + 80.0) / 6.8);
        bh = 2.7 * exp(0.079 * V) + 3.1e5 * exp(0.3485 * V);
        aj = (-2.5428e4 * exp(0.2444 * V) - 6.948e-6 * exp(-0.04391 * V)) * (V + 37.78)
             / (1.0 + exp(0.311 * (V + 79.23)));
        bj = 0.02424 * exp(-0.01052 * V) / (1.0 + exp(-0.1378 * (V + 40.14)));
    }
    inf[11] = hi * hi;
    tau[11] = 1.0 / (ah + bh);
    inf[12] = hi * hi;
    tau[12] = 1.0 / (aj + bj);
    inf[13] = 1.0 / (1.0 + exp((-8.0 - V) / 7.5));
    tau[13] = (1.4 / (1.0 + exp((-35.0 - V) / 13.0)) + 0.25) * 1.4 / (1.0 + exp((V + 5.0) / 5.0))
              + 1.0 / (1.0 + exp((50.0 - V) / 20.0));
    inf[14] = 1.0 / (1.0 + exp((V + 20.0) / 7.0));
    tau[14] = 1102.5 * exp(-(V + 27.0) * (V + 27.0) / 225.0) + 200.0 / (1.0 + exp((13.0 - V) / 10.0))
              + 180.0 / (1.0 + exp((V + 30.0) / 10.0)) + 20.0;
    inf[15] = 0.67 / (1.0 + exp((V + 35.0) / 7.0)) + 0.33;
    tau[15] = 562.0 * exp(-(V + 27.0) * (V + 27.0) / 240.0) + 31.0 / (1.0 + exp((25.0 - V) / 10.0))
              + 80.0 / (1.0 + exp((V + 30.0) / 10.0));
    double cq = (Cass / 0.05) * (Cass / 0.05);
    inf[16] = 0.6 / (1.0 + cq) + 0.4;
    tau[16] = 80.0 / (1.0 + cq) + 2.0;
    inf[17] = 1.0 / (1.0 + exp((V + 20.0) / 5.0));
    tau[17] = 85.0 * exp(-(V + 45.0) * (V + 45.0) / 320.0) + 5.0 / (1.0 + exp((V - 20.0) / 5.0)) + 3.0;
    inf[18] = 1.0 / (1.0 + exp((20.0 - V) / 6.0));
    tau[18] = 9.5 * exp(-(V + 40.0) * (V + 40.0) / 1800.0) + 0.8;
}

static void model_eval(int model, const double *p, const double *y,
                       double *rate, double *inf, double *tau)
{
    switch (model) {
    case M_NONE: rate[0] = 0.0; break;
    case M_BARKLEY: barkley_rates(p, y, rate); break;
    case M_ZFK: zfk_rates(p, y, rate); break;
    case M_FHN: fhn_rates(p, y, rate); break;
    case M_CRN: crn_rates(y, rate, inf, tau); break;
    case M_FK4: fk4_rates(p, y, rate, inf, tau); break;
    case M_TP06: tp06_rates(y, rate, inf, tau); break;
    }
}

/* Expose the kinetic right-hand side of one cell (for tests). */
int orc_model_eval(int model, const double *p, const double *y,
                   double *rate, double *inf, double *tau)
{
    int nv = orc_nvar(model);
    if (nv < 0) return -1;
    for (int i = 0; i < nv; i++) { rate[i] = 0.0; inf[i] = 0.0; tau[i] = 0.0; }
    model_eval(model, p, y, rate, inf, tau);
    return nv;
}

/* ------------------------------------------------------------------------- */
/* Stimulus: I_stim,p(n) = sum_s A_s [p in R_s] [step n inside a window of s] */
/* (external current term of eq (monodomain): a positive A depolarises;      */
/* windows are counted in whole steps).                                      */
/* ------------------------------------------------------------------------- */
/* Right-hand side of one voxel's kinetics at state y, with the forcing F (stimulus,
 * plus L V in the additive scheme) added to dV/dt: out[0] = -I_ion + F; gates
 * out[i] = (inf_i - y_i) / tau_i (eq (gate) written with y_inf and tau); the other
 * variables out[i] = their rate. */
static void kinetic_rhs(int model, const double *p, const double *y, double F, double *out)
{
    double rate[NVAR_MAX], inf[NVAR_MAX], tau[NVAR_MAX];
    int nv = orc_nvar(model);
    for (int i = 0; i < nv; i++) { rate[i] = 0.0; inf[i] = 0.0; tau[i] = 1.0; }
    model_eval(model, p, y, rate, inf, tau);
    out[0] = rate[0] + F;
    for (int i = 1; i < nv; i++)
        out[i] = is_gate(model, i) ? (inf[i] - y[i]) / tau[i] : rate[i];
}

/* One step of the classical fourth-order Runge-Kutta scheme ("Kinetics solvers",
 * the `rk4` solver) for one voxel: y is the state at the step's start (y[0] = V, or V*
 * in the split scheme) and is replaced by the state one step later; F is held
 * constant through the four stages. */
static void rk4_voxel(int model, const double *p, double *y, double F, double dt)
{
    int nv = orc_nvar(model);
    double k1[NVAR_MAX], k2[NVAR_MAX], k3[NVAR_MAX], k4[NVAR_MAX], t[NVAR_MAX];
    kinetic_rhs(model, p, y, F, k1);
    for (int i = 0; i < nv; i++) t[i] = y[i] + 0.5 * dt * k1[i];
    kinetic_rhs(model, p, t, F, k2);
    for (int i = 0; i < nv; i++) t[i] = y[i] + 0.5 * dt * k2[i];
    kinetic_rhs(model, p, t, F, k3);
    for (int i = 0; i < nv; i++) t[i] = y[i] + dt * k3[i];
    kinetic_rhs(model, p, t, F, k4);
    for (int i = 0; i < nv; i++) y[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

static int stim_on(int64_t n, int64_t n0, int64_t len, int64_t period, int64_t count)
{
    if (n < n0 || len <= 0) return 0;
    int64_t r = n - n0;
    if (period <= 0) return r < len;
    int64_t c = r / period;
    if (count > 0 && c >= count) return 0;
    return (r - c * period) < len;
}

/* ------------------------------------------------------------------------- */
/* Time stepping ("Splitting the problem into parts"; eq (Euler); eqs (RL),  */
/* (RLcoeff) in the order y_{n+1} = B + A y_n, the one exact for frozen V).  */
/* ------------------------------------------------------------------------- */
/*
 * Advances state (box layout [nvar][nbox]) by nsteps steps, the first of
 * which has index n0 (t_n = n dt).  vnext is an nbox scratch buffer.
 *  additive scheme: V+ = V + dt(-I_ion(V,g) + I_stim + LV), kinetics at (V, g);
 *  split scheme:    V* = V + dt LV, then V+ = V* + dt(-I_ion(V*,g) + I_stim),
 *                   kinetics at (V*, g).
 * Non-gates use forward Euler; gates y+ = yinf + (y - yinf) exp(-dt/tau).  With
 * integrator = I_RK4 every variable instead takes one classical RK4 step of its ODE,
 * with I_stim (additive: and LV) held constant through the stages.
 * If record != 0, activation time, peak and APD90 are detected from the pair
 * (V_n, V_{n+1}) per voxel: status 0 -> 1 on the first upward
 * crossing of theta (AT linearly interpolated), 1 -> 2 at the first decrease
 * (vmax = V_n), 2 -> 3 at the first downward crossing of
 * vrest + 0.1 (vmax - vrest) (APD90 = interpolated time - AT).
 */
int orc_run(int nx, int ny, int nz, int64_t nact, const int64_t *act, const double *W,
            int model, const double *params, double dt, int scheme, int integrator,
            int nstim, const uint8_t *stim_region, const double *stim_amp,
            const int64_t *stim_n0, const int64_t *stim_len, const int64_t *stim_period,
            const int64_t *stim_count,
            double *state, double *vnext, int64_t n0, int64_t nsteps,
            int record, double theta, uint8_t *status, double *at, double *vmax,
            double *apd, const double *vrest, int nthreads)
{
    int nv = orc_nvar(model);
    if (nv < 0) return -1;
    const int64_t nbox = (int64_t)nx * ny * nz;
    double *V = state;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    (void)nthreads;
#endif

    for (int64_t s = 0; s < nsteps; s++) {
        const int64_t n = n0 + s;
        const double tn = (double)n * dt;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
        for (int64_t a = 0; a < nact; a++) {
            int64_t p = act[a];
            double y[NVAR_MAX], rate[NVAR_MAX], inf[NVAR_MAX], tau[NVAR_MAX];
            double LV = apply_L(nx, ny, nz, W + 27 * a, V, p);
            double Is = 0.0;
            for (int k = 0; k < nstim; k++)
                if (stim_region[(int64_t)k * nbox + p] &&
                    stim_on(n, stim_n0[k], stim_len[k], stim_period[k], stim_count[k]))
                    Is += stim_amp[k];
            for (int i = 0; i < nv; i++) y[i] = state[(int64_t)i * nbox + p];
            double Vold = y[0];
            if (scheme == S_SPLIT) y[0] = Vold + dt * LV;
            double Vnew;
            if (integrator == I_RK4) {
                rk4_voxel(model, params, y, scheme == S_SPLIT ? Is : Is + LV, dt);
                Vnew = y[0];
                for (int i = 1; i < nv; i++) state[(int64_t)i * nbox + p] = y[i];
            } else {
                model_eval(model, params, y, rate, inf, tau);
                Vnew = (scheme == S_SPLIT) ? y[0] + dt * (rate[0] + Is)
                                           : Vold + dt * (rate[0] + Is + LV);
                for (int i = 1; i < nv; i++) {
                    double yi = y[i];
                    if (is_gate(model, i))
                        yi = inf[i] + (yi - inf[i]) * exp(-dt / tau[i]);
                    else
                        yi = yi + dt * rate[i];
                    state[(int64_t)i * nbox + p] = yi;
                }
            }
            vnext[p] = Vnew;

            if (record) {
                uint8_t st = status[a];
                if (st == 0 && Vold < theta && Vnew >= theta) {
                    at[a] = tn + dt * (theta - Vold) / (Vnew - Vold);
                    st = 1;
                }
                if (st == 1 && Vnew < Vold) {
                    vmax[a] = Vold;
                    st = 2;
                }
                if (st == 2) {
                    double vr = vrest[a] + 0.1 * (vmax[a] - vrest[a]);
                    if (Vold >= vr && Vnew < vr) {
                        apd[a] = tn + dt * (Vold - vr) / (Vold - Vnew) - at[a];
                        st = 3;
                    }
                }
                status[a] = st;
            }
        }
        for (int64_t a = 0; a < nact; a++) V[act[a]] = vnext[act[a]];
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Phase singularities in z cross-sections (the `singz` device of "Input/output */
/* and visualization"): points where an isoline of field u (u = u_level) and  */
/* an isoline of field v (v = v_level) intersect inside a grid cell, the      */
/* isolines' pieces in each cell obtained by linear interpolation along its   */
/* edges.  Reading of the details the paper leaves open:                      */
/*  - a cell is the square of four tissue voxels (x..x+1, y..y+1) of one plane;*/
/*  - a corner counts as "above" when its value is >= the level; an edge is   */
/*    crossed where its two corners differ, at the linearly interpolated      */
/*    point; 2 crossed edges give one segment; 4 (a saddle) give two segments,*/
/*    which separate the corner pair whose class differs from that of the     */
/*    average of the four corner values;                                     */
/*  - every intersection of a u segment with a v segment (both parameters in  */
/*    [0, 1]) is a point; statistics are the count and the mean and standard  */
/*    deviation (population) of the points' coordinates (mm, x_p = h (x,y,z)).*/
/* ------------------------------------------------------------------------- */

/* Isoline segments of the cell with corner values c[4] = (00, 10, 01, 11) (x, y)
 * relative to the level; seg[k] = {x1, y1, x2, y2} in cell coordinates [0,1]^2.
 * Returns the number of segments (0, 1 or 2). */
static int cell_segments(const double c[4], double seg[2][4])
{
    /* edges: bottom 00-10, right 10-11, top 01-11, left 00-01 */
    static const int ea[4] = {0, 1, 2, 0}, eb[4] = {1, 3, 3, 2};
    static const double ox[4] = {0, 1, 0, 0}, oy[4] = {0, 0, 1, 0};   /* edge start */
    static const double dx[4] = {1, 0, 1, 0}, dy[4] = {0, 1, 0, 1};   /* edge direction */
    double px[4], py[4];
    int cut[4], ncut = 0;
    for (int e = 0; e < 4; e++) {
        double a = c[ea[e]], b = c[eb[e]];
        cut[e] = (a >= 0.0) != (b >= 0.0);
        if (cut[e]) {
            double t = a / (a - b);
            px[e] = ox[e] + t * dx[e];
            py[e] = oy[e] + t * dy[e];
            ncut++;
        }
    }
    if (ncut == 2) {
        int k = 0, q[2];
        for (int e = 0; e < 4; e++) if (cut[e]) q[k++] = e;
        seg[0][0] = px[q[0]]; seg[0][1] = py[q[0]]; seg[0][2] = px[q[1]]; seg[0][3] = py[q[1]];
        return 1;
    }
    if (ncut == 4) {
        double centre = 0.25 * (c[0] + c[1] + c[2] + c[3]);
        int pair[2][2];
        if ((centre >= 0.0) == (c[0] >= 0.0)) {
            /* 00 and 11 joined through the centre: cut off corners 10 and 01 */
            pair[0][0] = 0; pair[0][1] = 1;    /* bottom, right: around 10 */
            pair[1][0] = 2; pair[1][1] = 3;    /* top, left: around 01 */
        } else {
            pair[0][0] = 0; pair[0][1] = 3;    /* bottom, left: around 00 */
            pair[1][0] = 1; pair[1][1] = 2;    /* right, top: around 11 */
        }
        for (int k = 0; k < 2; k++) {
            seg[k][0] = px[pair[k][0]]; seg[k][1] = py[pair[k][0]];
            seg[k][2] = px[pair[k][1]]; seg[k][3] = py[pair[k][1]];
        }
        return 2;
    }
    return 0;
}

/* Intersection of segments p and q; returns 1 and the point if they cross. */
static int seg_cross(const double p[4], const double q[4], double *x, double *y)
{
    double rx = p[2] - p[0], ry = p[3] - p[1], sx = q[2] - q[0], sy = q[3] - q[1];
    double den = rx * sy - ry * sx;
    if (den == 0.0) return 0;
    double wx = q[0] - p[0], wy = q[1] - p[1];
    double s = (wx * sy - wy * sx) / den, t = (wx * ry - wy * rx) / den;
    if (s < 0.0 || s > 1.0 || t < 0.0 || t > 1.0) return 0;
    *x = p[0] + s * rx;
    *y = p[1] + s * ry;
    return 1;
}

/* u, v: fields in box layout; mask: tissue.  sums[7] = count, sum x, y, z, sum x^2,
 * y^2, z^2 (mm).  Points (x, y, z in mm) are written to pts[3*k] for k < max_pts.
 * Returns the number of points. */
int64_t orc_tips(int nx, int ny, int nz, double h, const uint8_t *mask, const double *u,
                 double ul, const double *v, double vl, double *sums, double *pts,
                 int64_t max_pts)
{
    int64_t n = 0;
    for (int i = 0; i < 7; i++) sums[i] = 0.0;
    for (int z = 0; z < nz; z++)
        for (int y = 0; y + 1 < ny; y++)
            for (int x = 0; x + 1 < nx; x++) {
                int64_t b[4];
                b[0] = (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
                b[1] = b[0] + 1;
                b[2] = b[0] + nx;
                b[3] = b[2] + 1;
                if (!mask[b[0]] || !mask[b[1]] || !mask[b[2]] || !mask[b[3]]) continue;
                double cu[4], cv[4], su[2][4], sv[2][4];
                for (int k = 0; k < 4; k++) { cu[k] = u[b[k]] - ul; cv[k] = v[b[k]] - vl; }
                int nu = cell_segments(cu, su), nv = cell_segments(cv, sv);
                for (int i = 0; i < nu; i++)
                    for (int j = 0; j < nv; j++) {
                        double px, py;
                        if (!seg_cross(su[i], sv[j], &px, &py)) continue;
                        double X = h * (x + px), Y = h * (y + py), Z = h * z;
                        sums[0] += 1.0;
                        sums[1] += X; sums[2] += Y; sums[3] += Z;
                        sums[4] += X * X; sums[5] += Y * Y; sums[6] += Z * Z;
                        if (n < max_pts && pts) { pts[3 * n] = X; pts[3 * n + 1] = Y; pts[3 * n + 2] = Z; }
                        n++;
                    }
            }
    return n;
}
