// Internal declarations shared by the host side of libbbx and its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bbx {

constexpr int kBlock = 256;      // threads per workgroup (4 wave64)
constexpr int kStreamBlock = 512; // tissue-list step on data beyond the Infinity Cache
constexpr int kMaxStim = 32;     // stimuli per grid (bit per stimulus in a uint32)
constexpr int kMaxParams = 8;    // model parameters
constexpr int kXcd = 8;          // MI355X: 8 XCDs, workgroups dealt round-robin
constexpr double kInfinityCacheBytes = 256.0 * 1024 * 1024;   // MI355X Infinity Cache size

// The 18 non-corner neighbours of the 19-point stencil, in bit order: the six
// faces, then the edges of the xy, xz and yz planes as (+,+), (-,-), (+,-), (-,+).
// Corner neighbours carry zero weight in the paper's scheme and are not stored.
struct NbOff { int dx, dy, dz; };
__host__ __device__ constexpr NbOff nb_off(int b)
{
    constexpr NbOff t[18] = {
        {+1, 0, 0}, {-1, 0, 0}, {0, +1, 0}, {0, -1, 0}, {0, 0, +1}, {0, 0, -1},
        {+1, +1, 0}, {-1, -1, 0}, {+1, -1, 0}, {-1, +1, 0},
        {+1, 0, +1}, {-1, 0, -1}, {+1, 0, -1}, {-1, 0, +1},
        {0, +1, +1}, {0, -1, -1}, {0, +1, -1}, {0, -1, +1},
    };
    return t[b];
}

// Stimulus window in whole steps (as the host evaluates it): on for n0 + c*per <= n <
// n0 + c*per + len, c = 0 .. count-1 (per <= 0: once; count <= 0 with per > 0: forever).
struct StimWin {
    int64_t n0, len, per, count;
};

// Arguments of one fused step launch (passed by value in the kernarg segment).
template <typename T>
struct StepArgs {
    // geometry
    int nx, ny, nz;
    int dense;                 // 1: every box voxel is tissue, t == box index
    int64_t nact, pitch;       // tissue voxels; element pitch of the SoA arrays
    const int32_t *idx;        // [nact] box index of tissue voxel t (sparse only)
    const uint32_t *nbr;       // [nact] neighbour-is-tissue bits (sparse only)
    const T *geo;              // [nact][6] per voxel: unit fibre (3), face coefficients
                               // of the tensor-gradient term (3); anisotropic only
    T Dpar, Dperp, ih2;
    // state
    const T *Vin;              // [nbox] V at step n (box layout, void entries 0)
    T *Vout;                   // [nbox] V at step n+1
    T *st;                     // [nvar-1][pitch] other state variables, updated in place
    // model / scheme
    T prm[kMaxParams];
    T dt;
    int split;
    int rk4;                   // 1: kinetics by the classical RK4 integrator
    const float *tab;          // tabulated voltage-only kinetic terms (FP32 CRN) or null
    // stimulus
    int nstim;
    uint32_t stim_on;          // bit s: stimulus s active at this step (host-evaluated)
    const uint32_t *stimbits;  // [nact] bit s: voxel inside stimulus s region
    const T *stim_amp;         // [kMaxStim]
    // activation / APD90 recording
    int rec;
    T theta, tn;
    // device clock (graph replay): with nbase set, the step is n = *nbase + jstep, and
    // the kernel evaluates stim_on from win[] and tn = n * dt64 itself, as the host does
    const int64_t *nbase;
    int jstep;
    double dt64;
    const StimWin *win;
    uint8_t *status;
    T *at, *vmax, *apd;
    T *vrep;                   // rest level until the peak is known, then the 90% level
    // 1: the state is read and V_{n+1} written with non-temporal accesses (box or
    // state arrays larger than the Infinity Cache, where caching these streams only
    // evicts the V_n lines the neighbour gathers reuse)
    int nt;
    // XCD-aware block mapping; dense boxes use 64 x 4 (x, y) tiles, gx * gy per plane
    int nblk, per_xcd;
    int gx, gy, zc;            // dense: tiles along x, y; planes per z-chunk
};

// Dense-box tile of one workgroup: kTileX x kTileY voxels of one z plane.
constexpr int kTileX = 64;
constexpr int kTileY = kBlock / kTileX;

// The calling thread's last-error message, shared by all entry points.
int api_error(int code, const char *msg);
void api_clear_error();
void api_log(const char *msg);   // one line on stderr when BBX_LOG is set

// Launchers (step_kernels.hip).  Return hipSuccess or the launch error.
template <typename T>
hipError_t launch_step(int model, int aniso, const StepArgs<T> &a, hipStream_t s);

// Phase-singularity finder (tips_kernels.hip).  u_box / v_box: a field in box layout
// (V), else u_list / v_list over the tissue list (indexed through map unless dense).
template <typename T>
struct TipLaunch {
    int nx, ny, nz, dense;
    int z0, z1;                  // planes searched (a slab's own planes)
    int zoff;                    // global index of plane 0 (slabs), for the coordinates
    double h, ul, vl;
    const int32_t *map;
    const T *u_box, *u_list, *v_box, *v_list;
    double *part;                // [1024][7] workgroup sums
    double *out;                 // [7] count, sum x, y, z, sum x^2, y^2, z^2 (mm)
    double *pts;                 // [max_pts][3] or null
    int64_t max_pts;
    unsigned long long *count;   // points found (zeroed by the caller)
};
constexpr int kTipPartBytes = 1024 * 7 * 8;
template <typename T>
hipError_t launch_tips(const TipLaunch<T> &L, hipStream_t s);
hipError_t launch_box_map(int32_t *map, int64_t nbox, const int32_t *idx, int64_t nact, hipStream_t s);

// Pseudo-ECG electrodes (ecg_kernels.hip): positions in mm, grid step h.
constexpr int kMaxElectrodes = 16;
constexpr int kEcgPartials = 1024;   // blocks of the ECG reduction
struct EcgElectrodes {
    double x[kMaxElectrodes], y[kMaxElectrodes], z[kMaxElectrodes];
    double h;
    int n;
};
// out[e] = pseudo-ECG of a.Vin at electrode e (FP64); partials: kEcgPartials * kMaxElectrodes.
template <typename T>
hipError_t launch_ecg(const StepArgs<T> &a, int aniso, const EcgElectrodes &el, double *partials,
                      double *out, hipStream_t s);

// Auxiliary kernels (aux_kernels.hip).
template <typename T>
hipError_t launch_to_box(const T *src, int src_is_box, const int32_t *idx, int dense,
                         int64_t nact, int64_t nbox, double *out, hipStream_t s);
template <typename T>
hipError_t launch_from_box(const double *src, T *dst, int dst_is_box, const int32_t *idx,
                           int dense, int64_t nact, hipStream_t s);
template <typename T>
hipError_t launch_reduce(const T *src, int src_is_box, const int32_t *idx, int dense,
                         int64_t nact, const uint8_t *region, int op, double *partials,
                         int nparts, double *out, hipStream_t s);
template <typename T>
hipError_t launch_nonfinite(const T *V, const int32_t *idx, int dense, const T *st,
                            int nst, int64_t nact, int64_t pitch, int *flag, hipStream_t s);
template <typename T>
hipError_t launch_weights(const StepArgs<T> &a, int aniso, double *W, hipStream_t s);
template <typename T>
hipError_t launch_fill(T *p, T v, int64_t n, hipStream_t s);
// *p = v (set) or *p += v (advance), one thread: a graph's device step counter.
hipError_t launch_counter(int64_t *p, int64_t v, int add, hipStream_t s);
template <typename T>
hipError_t launch_fill_tissue(T *box, const int32_t *idx, int64_t nact, T v, hipStream_t s);
hipError_t launch_crn_table(double vmin, double dv, int n, double dt, float *tab, hipStream_t s);
constexpr double kTabVmin = -120.0, kTabVmax = 80.0;   // tabulated voltage range (mV)
constexpr int kTabWidth = 32;                           // floats per table node
template <typename T>
hipError_t launch_gather(const T *box, const int32_t *idx, int dense, int64_t nact, T *dst,
                         hipStream_t s);
// box[idx[i]] = src[i] for i < n (a slab's halo unpack).
template <typename T>
hipError_t launch_scatter(const T *src, const int32_t *idx, int64_t n, T *box, hipStream_t s);

}  // namespace bbx
