// Pseudo-ECG: phi(x_e) = h^3 sum_{p in tissue} (L V)_p / |x_p - x_e| with x_p =
// h (x, y, z) and L the step's own discrete diffusion operator (the paper's
// weights in difference form).  With no-flux boundaries this is the volume
// integral of -D grad V . grad(1/r) of the classical pseudo-ECG, by summation
// by parts.  (L V)_p is evaluated in the grid's precision exactly as the step
// does; distances, quotients and every sum are FP64, reduced in a fixed order
// (deterministic).
#include "step_device.h"

namespace bbx {

constexpr int kEcgBlocks = kEcgPartials;

template <typename T, bool ANISO>
__global__ __launch_bounds__(kBlock) void k_ecg(const StepArgs<T> a, const EcgElectrodes el,
                                                double *partials)
{
    __shared__ double red[kBlock / 64][kMaxElectrodes];
    double acc[kMaxElectrodes];
#pragma unroll
    for (int e = 0; e < kMaxElectrodes; e++) acc[e] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < a.nact; t += stride) {
        int idx;
        uint32_t bits;
        voxel_of(a, (int)t, idx, bits);
        const T Vp = a.Vin[idx];
        const double LV = (double)laplacian<T, ANISO, false>(a, a.Vin, (int)t, idx, bits, Vp);
        const int r = idx / a.nx, x = idx - r * a.nx, z = r / a.ny, y = r - z * a.ny;
        const double px = el.h * x, py = el.h * y, pz = el.h * z;
#pragma unroll
        for (int e = 0; e < kMaxElectrodes; e++) {
            if (e < el.n) {
                const double dx = px - el.x[e], dy = py - el.y[e], dz = pz - el.z[e];
                acc[e] += LV / sqrt(dx * dx + dy * dy + dz * dz);
            }
        }
    }
    // wave reduction (fixed butterfly), then the block's waves in order
    const int lane = (int)threadIdx.x % 64, wave = (int)threadIdx.x / 64;
#pragma unroll
    for (int e = 0; e < kMaxElectrodes; e++) {
        double v = acc[e];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wave][e] = v;
    }
    __syncthreads();
    if (threadIdx.x < kMaxElectrodes) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; w++) s += red[w][threadIdx.x];
        partials[(int64_t)blockIdx.x * kMaxElectrodes + threadIdx.x] = s;
    }
}

// out[e] = h^3 * sum of the block partials in block order (one thread per electrode).
__global__ void k_ecg_final(const double *partials, int nblocks, int n, double h3, double *out)
{
    const int e = (int)threadIdx.x;
    if (e >= n) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; b++) s += partials[(int64_t)b * kMaxElectrodes + e];
    out[e] = h3 * s;
}

template <typename T>
hipError_t launch_ecg(const StepArgs<T> &a, int aniso, const EcgElectrodes &el, double *partials,
                      double *out, hipStream_t s)
{
    if (a.nact <= 0 || el.n <= 0) return hipErrorInvalidValue;
    const dim3 grid(kEcgBlocks), block(kBlock);
    if (aniso) hipLaunchKernelGGL((k_ecg<T, true>), grid, block, 0, s, a, el, partials);
    else hipLaunchKernelGGL((k_ecg<T, false>), grid, block, 0, s, a, el, partials);
    hipLaunchKernelGGL(k_ecg_final, dim3(1), dim3(64), 0, s, partials, kEcgBlocks, el.n,
                       el.h * el.h * el.h, out);
    return hipGetLastError();
}

template hipError_t launch_ecg<float>(const StepArgs<float> &, int, const EcgElectrodes &, double *,
                                      double *, hipStream_t);
template hipError_t launch_ecg<double>(const StepArgs<double> &, int, const EcgElectrodes &, double *,
                                       double *, hipStream_t);

}  // namespace bbx
