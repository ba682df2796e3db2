// Internal declarations of the surrogate network (host side and kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bbx_internal.h"

namespace bbx {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kH = 128;                   // hidden units per layer
constexpr int kP = 32;                    // inputs / outputs padded to one MFMA K block
constexpr int kS1 = kP + 8;               // LDS row stride (BF16) of 32-wide weight rows
constexpr int kS2 = kH + 8;               // LDS row stride (BF16) of 128-wide weight rows
constexpr int kPart = 2 * kH + kP + 1;    // per-tile partial sums: db1, db2, db3, loss
constexpr int64_t kMaxBatch = 65536;      // training batch limit
constexpr int kSurBlock = 768;            // threads per surrogate-step workgroup (12 waves)
constexpr int kSurRow = 28;               // staging row (floats) per voxel in the surrogate step:
                                          // 112 B, so the 16 rows a tile reads hit distinct banks
constexpr float kGateTol = 1e-3f;         // accepted excursion of a predicted gate outside [0, 1]

// Device copies of one network: BF16 weights in the MFMA layouts (see
// mlp_kernels.hip), FP32 biases [b1 H | b2 H | b3 kP] and normalisation
// [4][kP] = in_mean, in_scale, out_mean, out_sigma.
struct MlpDev {
    int nin, nout;
    __bf16 *w1, *w2, *w3, *w2t, *w3t;
    float *bias, *norm;
};

// Training scratch for one batch (Bp = batch rounded up to 32).
struct MlpScratch {
    __bf16 *xb;                      // [Bp][kP] inputs, sample-major
    float *tt;                       // [Bp][kP] targets, sample-major
    __bf16 *xf, *h1, *h2, *dz1, *dz2, *dO;  // feature-major [rows][Bp]
    float *part;                     // [Bp/16][kPart]
};

// Surrogate attached to a grid.
struct SurArgs {
    MlpDev net;
    const float *lo, *hi;            // [nvar] accepted input box
    float dv_max;                    // largest accepted |dV| per step
    // Per classifier workgroup b (kBlock voxels each, nblk of them): the tissue indices
    // of its voxels whose input the network accepts, at acc_list[b * kBlock ...], their
    // number acc_cnt[b] (rewritten every step), and its running fallback count fb[b].
    int32_t *acc_list;               // [nblk * kBlock]
    int32_t *acc_cnt;                // [nblk]
    unsigned long long *fb;          // [nblk]
    int nblk;
};

int mlp_nparams(int nin, int nout);
uint64_t mlp_mix64(uint64_t z);
hipError_t mlp_init(float *p, int nin, int nout, uint64_t seed, hipStream_t s);
hipError_t mlp_pack(const float *p, const MlpDev &d, hipStream_t s);
hipError_t mlp_forward(const MlpDev &d, const float *X, int64_t n, float *Y, hipStream_t s);
hipError_t mlp_grad(const MlpDev &d, const MlpScratch &w, int mode, const float *A, const float *Bm,
                    int64_t n, int64_t B, uint64_t seed, uint64_t iter, float *grad, double *loss,
                    hipStream_t s);
hipError_t mlp_adam(float *p, float *m, float *v, const float *grad, int n, float lr, float b1,
                    float b2, float eps, int64_t t, hipStream_t s);
hipError_t mlp_anchor(const MlpDev &d, const float *s0, const float *s1, float *p, hipStream_t s);
hipError_t mlp_stats(const float *S, const float *S1, int64_t n, int nin, double *out,
                     hipStream_t s);

hipError_t launch_surrogate_step(int model, int aniso, const StepArgs<float> &a, const SurArgs &su,
                                 hipStream_t s);
hipError_t launch_sample(const StepArgs<float> &a, int nvar, int64_t n, uint64_t seed, float *out,
                         hipStream_t s);
hipError_t launch_ionic_map(int model, const StepArgs<float> &a, int nvar, const float *in,
                            int64_t n, float *out, hipStream_t s);

}  // namespace bbx
