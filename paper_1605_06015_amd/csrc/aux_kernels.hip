// Auxiliary kernels: layout conversion (tissue list <-> box), FP64 reductions
// with a fixed summation order, the finite-value check, and the effective
// stencil weights (for inspection against the paper's weight formulas).
#include "bbx_internal.h"
#include "kinetics.h"

namespace bbx {

static inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

template <typename T>
__global__ void k_fill(T *p, T v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename T>
hipError_t launch_fill(T *p, T v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, v, n);
    return hipGetLastError();
}

// box[idx[t]] = v for every tissue voxel t (sparse grids; void entries untouched).
template <typename T>
__global__ void k_fill_tissue(T *box, const int32_t *idx, int64_t nact, T v)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < nact) box[idx[t]] = v;
}

template <typename T>
hipError_t launch_fill_tissue(T *box, const int32_t *idx, int64_t nact, T v, hipStream_t s)
{
    if (nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_tissue<T>, dim3(blocks_for(nact)), dim3(kBlock), 0, s, box, idx, nact, v);
    return hipGetLastError();
}

// out[box] = NaN for void, src value for tissue.
template <typename T>
__global__ void k_to_box(const T *src, int src_is_box, const int32_t *idx, int dense,
                         int64_t nact, int64_t nbox, double *out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (dense) {
        if (i < nbox) out[i] = (double)src[i];
        return;
    }
    if (i < nact) {
        const int64_t b = idx[i];
        out[b] = (double)src[src_is_box ? b : i];
    }
}

template <typename T>
hipError_t launch_to_box(const T *src, int src_is_box, const int32_t *idx, int dense,
                         int64_t nact, int64_t nbox, double *out, hipStream_t s)
{
    if (!dense) {
        hipError_t e = launch_fill<double>(out, __builtin_nan(""), nbox, s);
        if (e != hipSuccess) return e;
    }
    const int64_t n = dense ? nbox : nact;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_box<T>, dim3(blocks_for(n)), dim3(kBlock), 0, s, src, src_is_box,
                       idx, dense, nact, nbox, out);
    return hipGetLastError();
}

// dst (tissue list or box) <- src[box] for tissue voxels.
template <typename T>
__global__ void k_from_box(const double *src, T *dst, int dst_is_box, const int32_t *idx,
                           int dense, int64_t nact)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nact) return;
    const int64_t b = dense ? i : idx[i];
    dst[dst_is_box ? b : i] = (T)src[b];
}

template <typename T>
hipError_t launch_from_box(const double *src, T *dst, int dst_is_box, const int32_t *idx,
                           int dense, int64_t nact, hipStream_t s)
{
    if (nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_from_box<T>, dim3(blocks_for(nact)), dim3(kBlock), 0, s, src, dst,
                       dst_is_box, idx, dense, nact);
    return hipGetLastError();
}

// dst[t] = box[idx[t]] (same precision).
template <typename T>
__global__ void k_gather(const T *box, const int32_t *idx, int dense, int64_t nact, T *dst)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < nact) dst[i] = box[dense ? i : idx[i]];
}

template <typename T>
hipError_t launch_gather(const T *box, const int32_t *idx, int dense, int64_t nact, T *dst,
                         hipStream_t s)
{
    if (nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather<T>, dim3(blocks_for(nact)), dim3(kBlock), 0, s, box, idx, dense,
                       nact, dst);
    return hipGetLastError();
}

__global__ void k_counter(int64_t *p, int64_t v, int add)
{
    if (threadIdx.x == 0) *p = add ? *p + v : v;
}

hipError_t launch_counter(int64_t *p, int64_t v, int add, hipStream_t s)
{
    hipLaunchKernelGGL(k_counter, dim3(1), dim3(64), 0, s, p, v, add);
    return hipGetLastError();
}

// box[idx[i]] = src[i]: writes received halo values into a slab's halo plane.
template <typename T>
__global__ void k_scatter(const T *src, const int32_t *idx, int64_t n, T *box)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) box[idx[i]] = src[i];
}

template <typename T>
hipError_t launch_scatter(const T *src, const int32_t *idx, int64_t n, T *box, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter<T>, dim3(blocks_for(n)), dim3(kBlock), 0, s, src, idx, n, box);
    return hipGetLastError();
}

// Reduction over tissue voxels (optionally restricted to a region) in FP64.
// Pass 1: part p reduces the contiguous slice [p*chunk, (p+1)*chunk) of the
// tissue list, each thread a strided subsequence, then a fixed-shape tree in
// LDS.  Pass 2: one block reduces the parts in index order.  The result does
// not depend on timing: no atomics.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_reduce1(const T *src, int src_is_box,
                                                    const int32_t *idx, int dense, int64_t nact,
                                                    const uint8_t *region, int op,
                                                    int64_t chunk, double *parts)
{
    __shared__ double sh[kBlock];
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = min(nact, lo + chunk);
    double acc = op ? 0.0 : -__builtin_inf();
    for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
        const int64_t b = dense ? i : idx[i];
        if (region && !region[b]) continue;
        const double v = (double)src[src_is_box ? b : i];
        acc = op ? acc + v : fmax(acc, v);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            sh[threadIdx.x] = op ? sh[threadIdx.x] + sh[threadIdx.x + w]
                                 : fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kBlock) void k_reduce2(const double *parts, int nparts, int op,
                                                    double *out)
{
    __shared__ double sh[kBlock];
    double acc = op ? 0.0 : -__builtin_inf();
    for (int i = threadIdx.x; i < nparts; i += kBlock)
        acc = op ? acc + parts[i] : fmax(acc, parts[i]);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            sh[threadIdx.x] = op ? sh[threadIdx.x] + sh[threadIdx.x + w]
                                 : fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

template <typename T>
hipError_t launch_reduce(const T *src, int src_is_box, const int32_t *idx, int dense,
                         int64_t nact, const uint8_t *region, int op, double *parts,
                         int nparts, double *out, hipStream_t s)
{
    const int64_t chunk = nact > 0 ? (nact + nparts - 1) / nparts : 1;
    hipLaunchKernelGGL(k_reduce1<T>, dim3(nparts), dim3(kBlock), 0, s, src, src_is_box, idx,
                       dense, nact, region, op, chunk, parts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(kBlock), 0, s, parts, nparts, op, out);
    return hipGetLastError();
}

// flag |= 1 if any state value of a tissue voxel is not finite.
template <typename T>
__global__ void k_nonfinite(const T *V, const int32_t *idx, int dense, const T *st, int nst,
                            int64_t nact, int64_t pitch, int *flag)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool bad = false;
    if (i < nact) {
        const int64_t b = dense ? i : idx[i];
        bad = !isfinite(V[b]);
        for (int k = 0; k < nst; k++) bad |= !isfinite(st[k * pitch + i]);
    }
    if (__any(bad) && (threadIdx.x % warpSize) == 0) atomicOr(flag, 1);
}

template <typename T>
hipError_t launch_nonfinite(const T *V, const int32_t *idx, int dense, const T *st, int nst,
                            int64_t nact, int64_t pitch, int *flag, hipStream_t s)
{
    if (nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nonfinite<T>, dim3(blocks_for(nact)), dim3(kBlock), 0, s, V, idx,
                       dense, st, nst, nact, pitch, flag);
    return hipGetLastError();
}

// Effective weights W^p_q of every tissue voxel in the paper's 27-entry layout,
// reconstructed from the compact per-voxel geometry the step kernel reads.
template <typename T>
__global__ void k_weights(const StepArgs<T> a, int aniso, double *W)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= a.nact) return;
    uint32_t bits;
    if (a.dense) {
        const int64_t r = t / a.nx;
        const int x = (int)(t - r * a.nx);
        const int z = (int)(r / a.ny);
        const int y = (int)(r - (int64_t)z * a.ny);
        bits = 0;
        for (int b = 0; b < 18; b++) {
            const NbOff o = nb_off(b);
            const int xx = x + o.dx, yy = y + o.dy, zz = z + o.dz;
            if (xx >= 0 && yy >= 0 && zz >= 0 && xx < a.nx && yy < a.ny && zz < a.nz)
                bits |= 1u << b;
        }
    } else {
        bits = a.nbr[t];
    }
    double D[3][3] = {{(double)a.Dperp, 0, 0}, {0, (double)a.Dperp, 0}, {0, 0, (double)a.Dperp}};
    double c[3] = {0, 0, 0};
    if (aniso) {
        const T *gp = a.geo + 6 * t;
        const double f[3] = {(double)gp[0], (double)gp[1], (double)gp[2]};
        for (int j = 0; j < 3; j++) {
            for (int k = 0; k < 3; k++) D[j][k] += ((double)a.Dpar - (double)a.Dperp) * f[j] * f[k];
            c[j] = (double)gp[3 + j];
        }
    }
    double *w = W + 27 * t;
    for (int q = 0; q < 27; q++) w[q] = 0.0;
    const double ih2 = (double)a.ih2;
    double sum = 0.0;
    for (int b = 0; b < 18; b++) {
        if (!((bits >> b) & 1u)) continue;
        if (!aniso && b >= 6) continue;
        const NbOff o = nb_off(b);
        double val;
        if (b < 6) {
            const int ax = b / 2;
            const double sgn = (b & 1) ? -1.0 : 1.0;
            val = D[ax][ax] * ih2 + sgn * c[ax];
        } else {
            const int plane = (b - 6) / 4, kind = (b - 6) % 4;
            const int j = plane == 2 ? 1 : 0, k = plane == 0 ? 1 : 2;
            val = (kind < 2 ? 0.5 : -0.5) * D[j][k] * ih2;
        }
        w[(o.dz + 1) * 9 + (o.dy + 1) * 3 + (o.dx + 1)] = val;
        sum += val;
    }
    w[13] = -sum;
}

template <typename T>
hipError_t launch_weights(const StepArgs<T> &a, int aniso, double *W, hipStream_t s)
{
    if (a.nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_weights<T>, dim3(blocks_for(a.nact)), dim3(kBlock), 0, s, a, aniso, W);
    return hipGetLastError();
}

// Table of the CRN voltage-only terms for time step dt, evaluated in FP64 at
// V_k = vmin + k dv (k < n) and stored in FP32 after a header {vmin, 1/dv, n}.
__global__ void k_crn_table(double vmin, double dv, int n, double dt, float *tab)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) {
        tab[0] = (float)vmin;
        tab[1] = (float)(1.0 / dv);
        tab[2] = (float)n;
        for (int q = 3; q < kin::CRN_V; q++) tab[q] = 0.0f;
    }
    if (k >= n) return;
    double c[kin::CRN_V];
    kin::crn_vterms<kin::Step>(vmin + k * dv, dt, c);
    for (int q = 0; q < kin::CRN_V; q++) tab[kin::CRN_V * (1 + k) + q] = (float)c[q];
}

hipError_t launch_crn_table(double vmin, double dv, int n, double dt, float *tab, hipStream_t s)
{
    hipLaunchKernelGGL(k_crn_table, dim3((n + 255) / 256), dim3(256), 0, s, vmin, dv, n, dt, tab);
    return hipGetLastError();
}

#define BBX_INST(T)                                                                          \
    template hipError_t launch_fill<T>(T *, T, int64_t, hipStream_t);                         \
    template hipError_t launch_fill_tissue<T>(T *, const int32_t *, int64_t, T, hipStream_t); \
    template hipError_t launch_to_box<T>(const T *, int, const int32_t *, int, int64_t,       \
                                         int64_t, double *, hipStream_t);                     \
    template hipError_t launch_from_box<T>(const double *, T *, int, const int32_t *, int,    \
                                           int64_t, hipStream_t);                             \
    template hipError_t launch_reduce<T>(const T *, int, const int32_t *, int, int64_t,       \
                                         const uint8_t *, int, double *, int, double *,       \
                                         hipStream_t);                                        \
    template hipError_t launch_nonfinite<T>(const T *, const int32_t *, int, const T *, int,  \
                                            int64_t, int64_t, int *, hipStream_t);            \
    template hipError_t launch_weights<T>(const StepArgs<T> &, int, double *, hipStream_t);   \
    template hipError_t launch_gather<T>(const T *, const int32_t *, int, int64_t, T *,       \
                                         hipStream_t);                                        \
    template hipError_t launch_scatter<T>(const T *, const int32_t *, int64_t, T *, hipStream_t);
BBX_INST(float)
BBX_INST(double)
template hipError_t launch_fill<uint8_t>(uint8_t *, uint8_t, int64_t, hipStream_t);
template hipError_t launch_fill<int>(int *, int, int64_t, hipStream_t);

}  // namespace bbx
