// Surrogate network kernels: a nin -> 128 -> 128 -> nout SiLU network on BF16
// MFMA (v_mfma_f32_16x16x32_bf16) with FP32 accumulation, used for training
// (forward, backward, weight gradients, Adam) and inside the fused step as a
// stand-in for the kinetic one-step map, with per-voxel fallback to the plain
// kinetics.
//
// Formulation.  Every layer is computed transposed, Y^T = W X^T: the weights
// are the MFMA A operand (rows = output units) and 16 samples form the B
// operand columns.  An accumulator fragment holds output units 4g+i of sample
// j (lane = 16 g + j); taking two consecutive 16-unit tiles gives, per lane,
// units {4g..4g+3} and {16+4g..16+4g+3} of a 32-unit block, which is exactly a
// B fragment of the next layer if that layer's weights store each 32-wide K
// block in the same permuted order.  So activations never leave registers
// between layers.  The reduction order over K is a permutation, which does
// not change the product.
#include "mlp_internal.h"
#include "step_device.h"

namespace bbx {

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4v mfma(bf8 a, bf8 b, f4v c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ __bf16 bf(float x) { return static_cast<__bf16>(x); }

__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float silu_d(float z)
{
    const float s = sigm(z);
    return s * (1.0f + z * (1.0f - s));
}

// Position j (0..31) of a permuted 32-wide K block holds unit kperm(j).
__host__ __device__ constexpr int kperm(int j)
{
    return (j % 8) < 4 ? 4 * (j / 8) + j % 8 : 16 + 4 * (j / 8) + (j % 8 - 4);
}

// SplitMix64 finaliser (Steele, Lea & Flood 2014) as a counter-based generator.
__host__ __device__ inline uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// --------------------------------------------------------------- parameters
// Flat FP32 layout: W1[H][nin] b1[H] W2[H][H] b2[H] W3[nout][H] b3[nout].
struct POff {
    int w1, b1, w2, b2, w3, b3, n;
};
__host__ __device__ inline POff poff(int nin, int nout)
{
    POff o;
    o.w1 = 0;
    o.b1 = kH * nin;
    o.w2 = o.b1 + kH;
    o.b2 = o.w2 + kH * kH;
    o.w3 = o.b2 + kH;
    o.b3 = o.w3 + nout * kH;
    o.n = o.b3 + nout;
    return o;
}

int mlp_nparams(int nin, int nout) { return poff(nin, nout).n; }

__global__ void k_init_params(float *p, int nin, int nout, uint64_t seed)
{
    const POff o = poff(nin, nout);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= o.n) return;
    float fan = 0.0f;
    if (e < o.b1) fan = (float)nin;
    else if (e >= o.w2 && e < o.b2) fan = (float)kH;
    else if (e >= o.w3 && e < o.b3) fan = (float)kH;
    float v = 0.0f;
    if (fan > 0.0f) {
        const double u = (double)(mix64(seed * 0x100000001B3ull + (uint64_t)e) >> 11) * (1.0 / 9007199254740992.0);
        v = (float)((2.0 * u - 1.0) / sqrt((double)fan));
    }
    p[e] = v;
}

// BF16 copies of the weights in the layouts the MFMA loops read.  The transposed
// copies (w2t, w3t) only exist for training; a grid's inference copy leaves them null.
__global__ void k_pack(const float *p, int nin, int nout, MlpDev d)
{
    const POff o = poff(nin, nout);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    // W1: [H][kS1], natural order over the (padded) inputs
    if (e < kH * kS1) {
        const int m = e / kS1, k = e % kS1;
        d.w1[e] = bf(k < nin ? p[o.w1 + m * nin + k] : 0.0f);
        // W3^T: [H (h2)][kS1], permuted order over the (padded) outputs
        const int oo = k < kP ? kperm(k) : kP;
        if (d.w3t) d.w3t[e] = bf(oo < nout ? p[o.w3 + oo * kH + m] : 0.0f);
    }
    if (e < kH * kS2) {
        const int m = e / kS2, k = e % kS2;
        const int kk = k < kH ? 32 * (k / 32) + kperm(k % 32) : kH;
        d.w2[e] = bf(kk < kH ? p[o.w2 + m * kH + kk] : 0.0f);          // W2[m][kk]
        if (d.w2t) d.w2t[e] = bf(kk < kH ? p[o.w2 + kk * kH + m] : 0.0f);   // W2^T[m][kk] = W2[kk][m]
        if (m < kP) d.w3[e] = bf(m < nout && kk < kH ? p[o.w3 + m * kH + kk] : 0.0f);
    }
    if (e < 2 * kH + kP) {
        float v = 0.0f;
        if (e < kH) v = p[o.b1 + e];
        else if (e < 2 * kH) v = p[o.b2 + e - kH];
        else if (e - 2 * kH < nout) v = p[o.b3 + e - 2 * kH];
        d.bias[e] = v;
    }
}

// ------------------------------------------------------------ tile routines
// Weights staged in LDS (same layouts as MlpDev).
struct MlpLds {
    const __bf16 *w1, *w2, *w3, *w2t, *w3t;
    const float *bias;  // b1 [H], b2 [H], b3 [kP]
};

__device__ __forceinline__ bf8 ld8(const __bf16 *p) { return *(const bf8 *)p; }

// Forward pass of one 16-sample tile.  x: B fragment (sample j, inputs 8g..8g+7).
// out[mt][i]: output unit 16 mt + 4 g + i of sample j.  z1/z2 receive the
// pre-activations, h1/h2 the BF16 activations (as next-layer B fragments).
__device__ __forceinline__ void fwd_tile(const MlpLds &W, bf8 x, f4v out[2], f4v z1[8],
                                         f4v z2[8], bf8 h1[4], bf8 h2[4])
{
    const int l = threadIdx.x & 63, j = l & 15, g = l >> 4;
#pragma unroll
    for (int mt = 0; mt < 8; mt++) {
        const f4v b = *(const f4v *)(W.bias + 16 * mt + 4 * g);   // bias as the initial sum
        z1[mt] = mfma(ld8(W.w1 + (16 * mt + j) * kS1 + 8 * g), x, b);
    }
#pragma unroll
    for (int ks = 0; ks < 4; ks++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            h1[ks][i] = bf(silu(z1[2 * ks][i]));
            h1[ks][4 + i] = bf(silu(z1[2 * ks + 1][i]));
        }
#pragma unroll
    for (int mt = 0; mt < 8; mt++) {
        f4v acc = *(const f4v *)(W.bias + kH + 16 * mt + 4 * g);
#pragma unroll
        for (int ks = 0; ks < 4; ks++)
            acc = mfma(ld8(W.w2 + (16 * mt + j) * kS2 + 32 * ks + 8 * g), h1[ks], acc);
        z2[mt] = acc;
    }
#pragma unroll
    for (int ks = 0; ks < 4; ks++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            h2[ks][i] = bf(silu(z2[2 * ks][i]));
            h2[ks][4 + i] = bf(silu(z2[2 * ks + 1][i]));
        }
#pragma unroll
    for (int mt = 0; mt < 2; mt++) {
        f4v acc = *(const f4v *)(W.bias + 2 * kH + 16 * mt + 4 * g);
#pragma unroll
        for (int ks = 0; ks < 4; ks++)
            acc = mfma(ld8(W.w3 + (16 * mt + j) * kS2 + 32 * ks + 8 * g), h2[ks], acc);
        out[mt] = acc;
    }
}

// Stage the weights of one network into LDS (all threads of the block).
__device__ __forceinline__ void stage_weights(const MlpDev &d, __bf16 *w1, __bf16 *w2,
                                              __bf16 *w3, __bf16 *w2t, __bf16 *w3t,
                                              float *bias)
{
    const int nt = blockDim.x, t = threadIdx.x;
    typedef uint4 u4;
    for (int e = t; e < kH * kS1 / 8; e += nt) ((u4 *)w1)[e] = ((const u4 *)d.w1)[e];
    for (int e = t; e < kH * kS2 / 8; e += nt) ((u4 *)w2)[e] = ((const u4 *)d.w2)[e];
    for (int e = t; e < kP * kS2 / 8; e += nt) ((u4 *)w3)[e] = ((const u4 *)d.w3)[e];
    if (w2t)
        for (int e = t; e < kH * kS2 / 8; e += nt) ((u4 *)w2t)[e] = ((const u4 *)d.w2t)[e];
    if (w3t)
        for (int e = t; e < kH * kS1 / 8; e += nt) ((u4 *)w3t)[e] = ((const u4 *)d.w3t)[e];
    for (int e = t; e < 2 * kH + kP; e += nt) bias[e] = d.bias[e];
}

// ------------------------------------------------------------- inference
// Y[n][nout] = network(X[n][nin]); one 16-sample tile per wave.
__global__ __launch_bounds__(256) void k_forward(MlpDev d, const float *X, int64_t n, float *Y)
{
    __shared__ __attribute__((aligned(16))) __bf16 w1[kH * kS1], w2[kH * kS2], w3[kP * kS2];
    __shared__ __attribute__((aligned(16))) float bias[2 * kH + kP];
    stage_weights(d, w1, w2, w3, nullptr, nullptr, bias);
    __syncthreads();
    const MlpLds W{w1, w2, w3, nullptr, nullptr, bias};
    const int l = threadIdx.x & 63, j = l & 15, g = l >> 4;
    const int64_t s = ((int64_t)blockIdx.x * 4 + threadIdx.x / 64) * 16 + j;
    bf8 x;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const int f = 8 * g + i;
        x[i] = bf(s < n && f < d.nin ? X[s * d.nin + f] : 0.0f);
    }
    f4v out[2], z1[8], z2[8];
    bf8 h1[4], h2[4];
    fwd_tile(W, x, out, z1, z2, h1, h2);
    if (s < n)
#pragma unroll
        for (int mt = 0; mt < 2; mt++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int f = 16 * mt + 4 * g + i;
                if (f < d.nout) Y[s * d.nout + f] = out[mt][i];
            }
}

// --------------------------------------------------------------- training
// Build the batch: Xb [Bp][kP] (BF16, sample-major) and Tt [Bp][kP] (FP32 targets).
// mode 0: X, T given (normalised).  mode 1: raw pairs S, S1 sampled with
// replacement; x = (s - in_mean) * in_scale, t = ((s1 - s) - out_mean) / out_sigma.
__global__ void k_prep(MlpDev d, int mode, const float *A, const float *Bm, int64_t n, int64_t B,
                       int64_t Bp, uint64_t seed, uint64_t iter, __bf16 *Xb, float *Tt)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Bp * kP) return;
    const int64_t s = e / kP;
    const int f = (int)(e % kP);
    float xv = 0.0f, tv = 0.0f;
    if (s < B) {
        if (mode == 0) {
            if (f < d.nin) xv = A[s * d.nin + f];
            if (f < d.nout) tv = Bm[s * d.nout + f];
        } else {
            const int64_t r = (int64_t)(mix64(seed ^ mix64(iter * 0x10000ull + (uint64_t)s)) % (uint64_t)n);
            if (f < d.nin) xv = (A[r * d.nin + f] - d.norm[f]) * d.norm[kP + f];
            const float sg = d.norm[3 * kP + f];
            if (f < d.nout && sg > 0.0f)
                tv = ((Bm[r * d.nout + f] - A[r * d.nin + f]) - d.norm[2 * kP + f]) / sg;
        }
    }
    Xb[s * kP + f] = bf(xv);
    Tt[s * kP + f] = tv;
}

// Forward + loss + backward through the data path for one 16-sample tile per
// wave.  Writes the feature-major BF16 operands of the weight gradients
// (Xf [kP][Bp], H1/H2/dZ1/dZ2 [H][Bp], dO [kP][Bp]) and, per tile, the sums over
// its samples of dZ1, dZ2, dO (bias gradients) and of the squared residuals.
__global__ __launch_bounds__(256) void k_fwd_bwd(MlpDev d, const __bf16 *Xb, const float *Tt,
                                                 int64_t B, int64_t Bp, float inv_count,
                                                 __bf16 *Xf, __bf16 *H1, __bf16 *H2, __bf16 *DZ1,
                                                 __bf16 *DZ2, __bf16 *DO, float *part)
{
    __shared__ __attribute__((aligned(16))) __bf16 w1[kH * kS1], w2[kH * kS2], w3[kP * kS2];
    __shared__ __attribute__((aligned(16))) __bf16 w2t[kH * kS2], w3t[kH * kS1];
    __shared__ __attribute__((aligned(16))) float bias[2 * kH + kP];
    stage_weights(d, w1, w2, w3, w2t, w3t, bias);
    __syncthreads();
    const MlpLds W{w1, w2, w3, w2t, w3t, bias};
    const int l = threadIdx.x & 63, j = l & 15, g = l >> 4;
    const int64_t tile = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (tile * 16 >= Bp) return;                       // wave-uniform
    const int64_t s = tile * 16 + j;
    const bool valid = s < B;
    const f4v zero = {0.f, 0.f, 0.f, 0.f};

    const bf8 x = *(const bf8 *)(Xb + s * kP + 8 * g);
    f4v out[2], z1[8], z2[8];
    bf8 h1[4], h2[4];
    fwd_tile(W, x, out, z1, z2, h1, h2);

    // residuals, loss, dO = 2 (O - T) / (B nout)
    float lsum = 0.0f;
    f4v dO[2];
#pragma unroll
    for (int mt = 0; mt < 2; mt++) {
        const f4v t4 = *(const f4v *)(Tt + s * kP + 16 * mt + 4 * g);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int f = 16 * mt + 4 * g + i;
            const float r = (valid && f < d.nout) ? out[mt][i] - t4[i] : 0.0f;
            lsum += r * r;
            dO[mt][i] = 2.0f * r * inv_count;
        }
    }
    bf8 dOb;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        dOb[i] = bf(dO[0][i]);
        dOb[4 + i] = bf(dO[1][i]);
    }
    // dH2^T = W3^T dO^T ; dZ2 = dH2 * silu'(Z2)
    f4v dz2[8];
#pragma unroll
    for (int mt = 0; mt < 8; mt++) {
        const f4v a = mfma(ld8(W.w3t + (16 * mt + j) * kS1 + 8 * g), dOb, zero);
#pragma unroll
        for (int i = 0; i < 4; i++) dz2[mt][i] = a[i] * silu_d(z2[mt][i]);
    }
    bf8 dz2b[4];
#pragma unroll
    for (int ks = 0; ks < 4; ks++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            dz2b[ks][i] = bf(dz2[2 * ks][i]);
            dz2b[ks][4 + i] = bf(dz2[2 * ks + 1][i]);
        }
    // dH1^T = W2^T dZ2^T ; dZ1 = dH1 * silu'(Z1)
    f4v dz1[8];
#pragma unroll
    for (int mt = 0; mt < 8; mt++) {
        f4v acc = zero;
#pragma unroll
        for (int ks = 0; ks < 4; ks++)
            acc = mfma(ld8(W.w2t + (16 * mt + j) * kS2 + 32 * ks + 8 * g), dz2b[ks], acc);
#pragma unroll
        for (int i = 0; i < 4; i++) dz1[mt][i] = acc[i] * silu_d(z1[mt][i]);
    }

    // feature-major operands of the weight gradients
#pragma unroll
    for (int i = 0; i < 8; i++) Xf[(int64_t)(8 * g + i) * Bp + s] = x[i];
#pragma unroll
    for (int mt = 0; mt < 8; mt++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int64_t f = 16 * mt + 4 * g + i;
            const int ks = mt / 2, q = (mt & 1) * 4 + i;
            H1[f * Bp + s] = h1[ks][q];
            H2[f * Bp + s] = h2[ks][q];
            DZ1[f * Bp + s] = bf(dz1[mt][i]);
            DZ2[f * Bp + s] = dz2b[ks][q];
        }
#pragma unroll
    for (int mt = 0; mt < 2; mt++)
#pragma unroll
        for (int i = 0; i < 4; i++) DO[(int64_t)(16 * mt + 4 * g + i) * Bp + s] = dOb[mt * 4 + i];

    // per-tile sums over the 16 samples (lanes with equal g), fixed xor tree
    float *pp = part + tile * kPart;
#pragma unroll
    for (int mt = 0; mt < 8; mt++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            float a = dz1[mt][i], b = dz2[mt][i];
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) {
                a += __shfl_xor(a, off, 16);
                b += __shfl_xor(b, off, 16);
            }
            if (j == 0) {
                pp[16 * mt + 4 * g + i] = a;
                pp[kH + 16 * mt + 4 * g + i] = b;
            }
        }
#pragma unroll
    for (int mt = 0; mt < 2; mt++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            float a = dO[mt][i];
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) a += __shfl_xor(a, off, 16);
            if (j == 0) pp[2 * kH + 16 * mt + 4 * g + i] = a;
        }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if (l == 0) pp[kPart - 1] = lsum;
}

// Weight gradients dW = sum_b dZ[:, b] A[:, b]^T as MFMA GEMMs over the batch.
// One workgroup per 16 x 16 output tile (tiles 0..15: dW1 (8 x 2); 16..79: dW2
// (8 x 8); 80..95: dW3 (2 x 8)); its kWgWaves waves split the batch, wave w
// taking the 32-sample blocks w, w + kWgWaves, ...; the wave partials are summed
// through LDS in wave order.  Deterministic (no atomics), and 96 x kWgWaves waves
// keep the MFMA pipes of many CUs busy where one wave per tile left them idle.
constexpr int kWgWaves = 16;
__global__ __launch_bounds__(64 * kWgWaves) void k_wgrad(MlpDev d, int64_t Bp, const __bf16 *Xf,
                                                         const __bf16 *H1, const __bf16 *H2,
                                                         const __bf16 *DZ1, const __bf16 *DZ2,
                                                         const __bf16 *DO, float *grad)
{
    __shared__ f4v part[kWgWaves][64];
    const int w = blockIdx.x;                   // output tile, 0..95 (grid = 96)
    const int wv = threadIdx.x / 64, l = threadIdx.x & 63, j = l & 15, g = l >> 4;
    const POff o = poff(d.nin, d.nout);
    const __bf16 *Am, *Bm;
    int mt, nt, rows, cols, base, ld;
    if (w < 16) { mt = w / 2; nt = w % 2; Am = DZ1; Bm = Xf; rows = kH; cols = d.nin; base = o.w1; ld = d.nin; }
    else if (w < 80) { mt = (w - 16) / 8; nt = (w - 16) % 8; Am = DZ2; Bm = H1; rows = kH; cols = kH; base = o.w2; ld = kH; }
    else { mt = (w - 80) / 8; nt = (w - 80) % 8; Am = DO; Bm = H2; rows = d.nout; cols = kH; base = o.w3; ld = kH; }
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    const __bf16 *ap = Am + (int64_t)(16 * mt + j) * Bp + 8 * g;
    const __bf16 *bp = Bm + (int64_t)(16 * nt + j) * Bp + 8 * g;
    for (int64_t k = 32 * wv; k < Bp; k += 32 * kWgWaves) acc = mfma(ld8(ap + k), ld8(bp + k), acc);
    part[wv][l] = acc;
    __syncthreads();
    if (wv != 0) return;
    f4v s = part[0][l];
    for (int i = 1; i < kWgWaves; i++) s += part[i][l];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int r = 16 * mt + 4 * g + i, c = 16 * nt + j;
        if (r < rows && c < cols) grad[base + r * ld + c] = s[i];
    }
}

// Bias gradients and the loss: one workgroup per column sums the per-tile
// partials (strided per thread, then a fixed LDS tree: deterministic).
__global__ __launch_bounds__(256) void k_reduce_part(MlpDev d, const float *part, int64_t ntile,
                                                     float *grad, double *loss, double inv_count)
{
    __shared__ double sh[256];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < ntile; t += 256) s += (double)part[t * kPart + c];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    s = sh[0];
    const POff o = poff(d.nin, d.nout);
    if (c < kH) grad[o.b1 + c] = (float)s;
    else if (c < 2 * kH) grad[o.b2 + c - kH] = (float)s;
    else if (c < 2 * kH + kP) {
        if (c - 2 * kH < d.nout) grad[o.b3 + c - 2 * kH] = (float)s;
    } else {
        loss[0] = s * inv_count;
    }
}

__global__ void k_adam(float *p, float *m, float *v, const float *grad, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gr = grad[e];
    const float mm = b1 * m[e] + (1.0f - b1) * gr;
    const float vv = b2 * v[e] + (1.0f - b2) * gr * gr;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// Normalisation statistics of training pairs, one block per feature, FP64,
// fixed reduction order.  Feature f < nin: the states; f >= kP: increments.
__global__ __launch_bounds__(256) void k_stats(const float *S, const float *S1, int64_t n,
                                               int nin, double *out)
{
    __shared__ double sh[4][256];
    const int f = blockIdx.x;          // 0..2*kP-1
    const int c = f % kP;
    const bool inc = f >= kP;
    double s1 = 0, s2 = 0, mn = __builtin_inf(), mx = -__builtin_inf();
    if (c < nin)
        for (int64_t r = threadIdx.x; r < n; r += 256) {
            const double v = inc ? (double)S1[r * nin + c] - (double)S[r * nin + c] : (double)S[r * nin + c];
            s1 += v;
            s2 += v * v;
            mn = fmin(mn, v);
            mx = fmax(mx, v);
        }
    sh[0][threadIdx.x] = s1;
    sh[1][threadIdx.x] = s2;
    sh[2][threadIdx.x] = mn;
    sh[3][threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
            sh[2][threadIdx.x] = fmin(sh[2][threadIdx.x], sh[2][threadIdx.x + w]);
            sh[3][threadIdx.x] = fmax(sh[3][threadIdx.x], sh[3][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mean = c < nin && n > 0 ? sh[0][0] / n : 0.0;
        const double var = c < nin && n > 0 ? fmax(sh[1][0] / n - mean * mean, 0.0) : 0.0;
        out[f * 4 + 0] = mean;
        out[f * 4 + 1] = sqrt(var);
        out[f * 4 + 2] = c < nin ? sh[2][0] : 0.0;
        out[f * 4 + 3] = c < nin ? sh[3][0] : 0.0;
    }
}

// ------------------------------------------------------------ host launchers
hipError_t mlp_init(float *p, int nin, int nout, uint64_t seed, hipStream_t s)
{
    const int n = mlp_nparams(nin, nout);
    hipLaunchKernelGGL(k_init_params, dim3((n + 255) / 256), dim3(256), 0, s, p, nin, nout, seed);
    return hipGetLastError();
}

hipError_t mlp_pack(const float *p, const MlpDev &d, hipStream_t s)
{
    const int n = kH * kS2;
    hipLaunchKernelGGL(k_pack, dim3((n + 255) / 256), dim3(256), 0, s, p, d.nin, d.nout, d);
    return hipGetLastError();
}

hipError_t mlp_forward(const MlpDev &d, const float *X, int64_t n, float *Y, hipStream_t s)
{
    const int64_t tiles = (n + 15) / 16;
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_forward, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, d, X, n, Y);
    return hipGetLastError();
}

hipError_t mlp_grad(const MlpDev &d, const MlpScratch &w, int mode, const float *A, const float *Bm,
                    int64_t n, int64_t B, uint64_t seed, uint64_t iter, float *grad, double *loss,
                    hipStream_t s)
{
    const int64_t Bp = (B + 31) / 32 * 32;
    const int64_t e = Bp * kP;
    hipLaunchKernelGGL(k_prep, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, d, mode, A, Bm, n, B,
                       Bp, seed, iter, w.xb, w.tt);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int64_t tiles = Bp / 16;
    const float inv = 1.0f / (float)(B * d.nout);
    hipLaunchKernelGGL(k_fwd_bwd, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, d, w.xb, w.tt, B,
                       Bp, inv, w.xf, w.h1, w.h2, w.dz1, w.dz2, w.dO, w.part);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(k_wgrad, dim3(96), dim3(64 * kWgWaves), 0, s, d, Bp, w.xf, w.h1, w.h2, w.dz1, w.dz2, w.dO,
                       grad);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(k_reduce_part, dim3(kPart), dim3(256), 0, s, d, w.part, tiles, grad, loss,
                       (double)inv);
    return hipGetLastError();
}

hipError_t mlp_adam(float *p, float *m, float *v, const float *grad, int n, float lr, float b1,
                    float b2, float eps, int64_t t, hipStream_t s)
{
    const float c1 = (float)(1.0 - pow((double)b1, (double)t));
    const float c2 = (float)(1.0 - pow((double)b2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, m, v, grad, n, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

hipError_t mlp_stats(const float *S, const float *S1, int64_t n, int nin, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_stats, dim3(2 * kP), dim3(256), 0, s, S, S1, n, nin, out);
    return hipGetLastError();
}

// Anchor: shift the output biases so that the network maps state s0 exactly to
// the normalised target increment of (s0 -> s1) (one wave, sample 0 of a tile).
__global__ __launch_bounds__(64) void k_anchor(MlpDev d, const float *s0, const float *s1, float *p)
{
    __shared__ __attribute__((aligned(16))) __bf16 w1[kH * kS1], w2[kH * kS2], w3[kP * kS2];
    __shared__ __attribute__((aligned(16))) float bias[2 * kH + kP];
    __shared__ float outv[kP];
    stage_weights(d, w1, w2, w3, nullptr, nullptr, bias);
    __syncthreads();
    const MlpLds W{w1, w2, w3, nullptr, nullptr, bias};
    const int l = threadIdx.x & 63, j = l & 15, g = l >> 4;
    bf8 x;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const int f = 8 * g + i;
        x[i] = bf(j == 0 && f < d.nin ? (s0[f] - d.norm[f]) * d.norm[kP + f] : 0.0f);
    }
    f4v out[2], z1[8], z2[8];
    bf8 h1[4], h2[4];
    fwd_tile(W, x, out, z1, z2, h1, h2);
    if (j == 0)
#pragma unroll
        for (int mt = 0; mt < 2; mt++)
#pragma unroll
            for (int i = 0; i < 4; i++) outv[16 * mt + 4 * g + i] = out[mt][i];
    __syncthreads();
    const POff o = poff(d.nin, d.nout);
    if (l < d.nout) {
        const float sg = d.norm[3 * kP + l];
        const float tgt = sg > 0.0f ? ((s1[l] - s0[l]) - d.norm[2 * kP + l]) / sg : 0.0f;
        p[o.b3 + l] += tgt - outv[l];
    }
}

hipError_t mlp_anchor(const MlpDev &d, const float *s0, const float *s1, float *p, hipStream_t s)
{
    hipLaunchKernelGGL(k_anchor, dim3(1), dim3(64), 0, s, d, s0, s1, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return mlp_pack(p, d, s);
}

uint64_t mlp_mix64(uint64_t z) { return mix64(z); }

// ------------------------------------------------------- surrogate step
// A surrogate step is two launches.  (1) k_sur_classify, one thread per tissue
// voxel: voxels whose kinetic input s = (V or V* = V + dt LV, g) lies in the
// accepted box [lo, hi] are listed in their workgroup's own segment of the network
// list (slots by a prefix count over the workgroup's waves: no global atomics, and
// the order is fixed); every other voxel gets the plain update right there (the plain
// step's own arithmetic).  (2) k_sur_net: one persistent workgroup per CU stages the
// weights in LDS once and walks the list segments in slots of 64 voxels (four per
// segment; empty slots are skipped): each thread recomputes its Laplacian and stimulus
// and writes its normalised input to the wave's LDS staging rows; the wave runs the
// network on its 64 voxels as four 16-sample tiles, and each thread applies or rejects
// its prediction (gate outside [0, 1], |dV| > dv_max, non-finite); rejected voxels get
// the plain update in place (rare).  Accepted gate predictions within kGateTol of
// [0, 1] are clamped into it.  The network's cost is thus paid only for the voxels it
// may take.
template <class M, bool ANISO>
__global__ __launch_bounds__(kBlock) void k_sur_classify(const StepArgs<float> a, const SurArgs su)
{
    __shared__ int wave_n[kBlock / 64];
    const int lb = (int)(blockIdx.x % kXcd) * a.per_xcd + (int)(blockIdx.x / kXcd);
    if (lb >= a.nblk) return;                              // workgroup-uniform exit
    const int t = lb * kBlock + (int)threadIdx.x;
    const bool valid = t < a.nact;
    int idx = 0;
    uint32_t bits = 0;
    float Vp = 0.f, LV = 0.f;
    bool ok = false;
    if (valid) {
        voxel_of(a, t, idx, bits);
        Vp = a.Vin[idx];
        LV = laplacian<float, ANISO, false>(a, a.Vin, t, idx, bits, Vp);
        const float s0 = a.split ? Vp + a.dt * LV : Vp;
        ok = (s0 >= su.lo[0]) & (s0 <= su.hi[0]);
        // every variable is read and tested (no short cut), so the loads are
        // unconditional and serve the update below
#pragma unroll
        for (int i = 1; i < M::NV; i++) {
            const float y = a.st[(i - 1) * a.pitch + t];
            ok = ok & (y >= su.lo[i]) & (y <= su.hi[i]);
        }
        // outside the box: the plain update, here, before anything is stored, so that
        // the compiler can reuse the state just loaded for the check
        if (!ok) update_voxel<float, M>(a, step_clock(a), t, idx, Vp, LV);
    }
    // slot of an accepted voxel: accepted voxels of the lower waves, then of the lower
    // lanes of its own wave
    const uint64_t acc = __ballot(ok);
    const int w = (int)threadIdx.x / 64, l = (int)threadIdx.x & 63;
    if (l == 0) wave_n[w] = __popcll(acc);
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; k++) {
        base += k < w ? wave_n[k] : 0;
        total += wave_n[k];
    }
    if (ok) {
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(acc >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)acc, 0u));
        su.acc_list[lb * kBlock + base + below] = t;
    }
    if (threadIdx.x == 0) {
        const int nvalid = min(kBlock, (int)(a.nact - (int64_t)lb * kBlock));
        su.acc_cnt[lb] = total;
        su.fb[lb] += (unsigned long long)(nvalid - total);  // input outside the box
    }
}

// Hand-over of LDS data between the lanes of one wave: the writes before it are
// visible to every lane's reads after it (a wave's LDS accesses complete in order).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// SiLU of the 32 pre-activations z[0..7] of one layer into next-layer B fragments
// h[ks] = units {4g..4g+3 of tile 2ks, 4g..4g+3 of tile 2ks+1}: each stage runs over all 32
// values before the next, so the transcendental latencies overlap.
__device__ __forceinline__ void silu_layer(const f4v z[8], bf8 h[4])
{
    float e[32];
#pragma unroll
    for (int k = 0; k < 32; k++) e[k] = __expf(-z[k >> 2][k & 3]);
#pragma unroll
    for (int k = 0; k < 32; k++) e[k] = __builtin_amdgcn_rcpf(1.0f + e[k]);
#pragma unroll
    for (int ks = 0; ks < 4; ks++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            h[ks][i] = bf(z[2 * ks][i] * e[8 * ks + i]);
            h[ks][4 + i] = bf(z[2 * ks + 1][i] * e[8 * ks + 4 + i]);
        }
}

// Inference pass of one 16-sample tile (fwd_tile without the saved pre-activations).
__device__ __forceinline__ void infer_tile(const MlpLds &W, bf8 x, f4v out[2])
{
    const int l = threadIdx.x & 63, j = l & 15, g = l >> 4;
    f4v z[8];
    bf8 h[4];
#pragma unroll
    for (int mt = 0; mt < 8; mt++)
        z[mt] = mfma(ld8(W.w1 + (16 * mt + j) * kS1 + 8 * g), x, *(const f4v *)(W.bias + 16 * mt + 4 * g));
    silu_layer(z, h);
#pragma unroll
    for (int mt = 0; mt < 8; mt++) {
        f4v acc = *(const f4v *)(W.bias + kH + 16 * mt + 4 * g);
#pragma unroll
        for (int ks = 0; ks < 4; ks++)
            acc = mfma(ld8(W.w2 + (16 * mt + j) * kS2 + 32 * ks + 8 * g), h[ks], acc);
        z[mt] = acc;
    }
    silu_layer(z, h);
#pragma unroll
    for (int mt = 0; mt < 2; mt++) {
        f4v acc = *(const f4v *)(W.bias + 2 * kH + 16 * mt + 4 * g);
#pragma unroll
        for (int ks = 0; ks < 4; ks++)
            acc = mfma(ld8(W.w3 + (16 * mt + j) * kS2 + 32 * ks + 8 * g), h[ks], acc);
        out[mt] = acc;
    }
}

template <class M, bool ANISO>
__global__ __launch_bounds__(kSurBlock) void k_sur_net(const StepArgs<float> a, const SurArgs su)
{
    constexpr int NV = M::NV;
    // outputs are written four at a time (units 4g..4g+3 of a 16-unit tile)
    static_assert((NV + 3) / 4 * 4 <= kSurRow, "a voxel's outputs must fit in its staging row");
    constexpr int kSlots = kBlock / 64;                 // 64-voxel slots per list segment
    const Clock<float> ck = step_clock(a);
    constexpr int NW = kSurBlock / 64;
    __shared__ __attribute__((aligned(16))) __bf16 w1[kH * kS1], w2[kH * kS2], w3[kP * kS2];
    __shared__ __attribute__((aligned(16))) float bias[2 * kH + kP];
    // one staging row per voxel: its normalised input (kP BF16 values) before the
    // network, its FP32 output increments after
    __shared__ __attribute__((aligned(16))) float rows[NW][64 * kSurRow];
    const int wv = threadIdx.x / 64, l = threadIdx.x & 63, j = l & 15, g = l >> 4;
    // slot c (segment c / kSlots, part c % kSlots): workgroup (c / NW) mod G, its wave
    // c mod NW, so that neighbouring slots (neighbouring voxels, often accepted together)
    // run side by side in one workgroup and a short list keeps most workgroups idle
    const int G = (int)gridDim.x, nslot = su.nblk * kSlots;
    const int rounds = (nslot + NW * G - 1) / (NW * G);
    // a workgroup none of whose slots holds a voxel leaves before staging the weights
    // (checked when each wave has at most kCheck slots: short lists)
    constexpr int kCheck = 4;
    if (rounds <= kCheck) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < kCheck; k++) {
            const int c = (k * G + (int)blockIdx.x) * NW + wv;
            if (k < rounds && c < nslot) any = any || su.acc_cnt[c / kSlots] > 64 * (c % kSlots);
        }
        if (!__syncthreads_or(any)) return;
    }
    // persistent workgroups: stage the weights once, then walk the slots; after this
    // barrier the waves run independently (each uses only its own rows), so one wave's
    // gathers overlap another's network
    stage_weights(su.net, w1, w2, w3, nullptr, nullptr, bias);
    __syncthreads();
    const MlpLds W{w1, w2, w3, nullptr, nullptr, bias};
    const float *nrm = su.net.norm;
    float *wrows = rows[wv];

    for (int k = 0; k < rounds; k++) {
        const int c = (k * G + (int)blockIdx.x) * NW + wv;
        if (c >= nslot) break;
        const int b = c / kSlots, q = c % kSlots;
        const int nin = su.acc_cnt[b] - 64 * q;              // wave-uniform
        if (nin <= 0) continue;
        const bool valid = l < nin;
        const int t = valid ? su.acc_list[b * kBlock + 64 * q + l] : 0;
        // only what the update needs after the network stays in registers; the gates
        // are read again afterwards (from cache)
        int idx = 0;
        float Vp = 0.f, LV = 0.f, Is = 0.f, s0 = 0.f;
        __bf16 xr[kP];
#pragma unroll
        for (int f = 0; f < kP; f++) xr[f] = bf(0.0f);
        if (valid) {
            uint32_t bits;
            voxel_of(a, t, idx, bits);
            Vp = a.Vin[idx];
            LV = laplacian<float, ANISO, false>(a, a.Vin, t, idx, bits, Vp);
            Is = stim_current(a, t, ck.stim_on);
            s0 = a.split ? Vp + a.dt * LV : Vp;
            xr[0] = bf((s0 - nrm[0]) * nrm[kP]);
#pragma unroll
            for (int i = 1; i < NV; i++) xr[i] = bf((a.st[(i - 1) * a.pitch + t] - nrm[i]) * nrm[kP + i]);
        }
        float *row = wrows + l * kSurRow;
        wave_sync();                                           // the previous slot's outputs read
#pragma unroll
        for (int qq = 0; qq < kP / 8; qq++) *(bf8 *)((__bf16 *)row + 8 * qq) = *(const bf8 *)(xr + 8 * qq);
        wave_sync();                                           // the wave's inputs staged

#pragma unroll 1
        for (int T = 0; T < 4; T++) {
            if (16 * T >= nin) break;                          // no voxel in this tile or later
            float *trow = wrows + (16 * T + j) * kSurRow;
            const bf8 x = ld8((const __bf16 *)trow + 8 * g);
            f4v out[2];
            infer_tile(W, x, out);
            wave_sync();                                       // the tile's inputs all read
            // output unit 16 mt + 4 g + i of sample j over the input row it came from
#pragma unroll
            for (int mt = 0; mt < 2; mt++)
                if (16 * mt + 4 * g < NV) *(f4v *)(trow + 16 * mt + 4 * g) = out[mt];
        }
        wave_sync();                                           // outputs staged
        if (!valid) continue;

        float d[NV], s[NV];
        bool ok = true;                                        // the input box was checked
        s[0] = s0;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            if (i > 0) s[i] = a.st[(i - 1) * a.pitch + t];
            d[i] = row[i] * nrm[3 * kP + i] + nrm[2 * kP + i];
            ok = ok && isfinite(d[i]);
        }
        ok = ok && fabsf(d[0]) <= su.dv_max;
        // gates: accept excursions of at most kGateTol outside [0, 1] (rounding-level
        // errors at resting values 0 or 1) and clamp; reject anything larger
#pragma unroll
        for (int i = M::GATE0; i < NV; i++)
            ok = ok && s[i] + d[i] >= -kGateTol && s[i] + d[i] <= 1.0f + kGateTol;
        // a rejected prediction falls back to the plain update of this voxel, here
        // (rare; counted with one atomic per wave on the segment's own counter)
        const uint64_t rej = __ballot(!ok);
        if (rej) {
            if (l == __ffsll((unsigned long long)rej) - 1) atomicAdd(&su.fb[b], (unsigned long long)__popcll(rej));
            if (!ok) {
                update_voxel<float, M>(a, ck, t, idx, Vp, LV);
                continue;
            }
        }
        const float Vn = a.split ? s[0] + d[0] + a.dt * Is : Vp + d[0] + a.dt * (Is + LV);
#pragma unroll
        for (int i = 1; i < NV; i++) {
            const float y = s[i] + d[i];
            a.st[(i - 1) * a.pitch + t] = i >= M::GATE0 ? fminf(fmaxf(y, 0.0f), 1.0f) : y;
        }
        a.Vout[idx] = Vn;
        record_voxel(a, t, Vp, Vn, ck.tn);
    }
}

// States of n tissue voxels drawn with replacement: out[k][0] = V, out[k][i] = g_i.
__global__ void k_sample(const StepArgs<float> a, int nvar, int64_t n, uint64_t seed, float *out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int t = (int)(mix64(seed ^ mix64((uint64_t)k)) % (uint64_t)a.nact);
    const int idx = a.dense ? t : a.idx[t];
    out[k * nvar] = a.Vin[idx];
    for (int i = 1; i < nvar; i++) out[k * nvar + i] = a.st[(i - 1) * a.pitch + t];
}

// Plain kinetic one-step map of n states (no diffusion, no stimulus).
template <class M>
__global__ void k_ionic(const StepArgs<float> a, const float *in, int64_t n, float *out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    constexpr int NV = M::NV;
    float g[NV > 1 ? NV - 1 : 1];
    const float V = in[k * NV];
#pragma unroll
    for (int i = 1; i < NV; i++) g[i - 1] = in[k * NV + i];
    const float r = M::advance(a.prm, V, g, a.dt, a.tab);
    out[k * NV] = V + a.dt * r;
#pragma unroll
    for (int i = 1; i < NV; i++) out[k * NV + i] = g[i - 1];
}

// Compute-unit count of the current device, queried once per device (the network launch
// takes one persistent workgroup per CU).
static int cu_count()
{
    constexpr int kMaxDev = 64;
    static int cache[kMaxDev];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return 256;
    if (cache[dev] == 0) {
        int n = 0;
        cache[dev] = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                             n > 0 ? n : 256;
    }
    return cache[dev];
}

template <class M>
static hipError_t sur_m(int aniso, const StepArgs<float> &a, const SurArgs &su, hipStream_t s)
{
    if (a.nact == 0) return hipSuccess;
    if (su.nblk != a.nblk) return hipErrorInvalidValue;   // list segments = classifier workgroups
    const int ncu = cu_count();
    const dim3 gc((unsigned)(a.per_xcd * kXcd)), bc(kBlock);
    if (aniso) hipLaunchKernelGGL((k_sur_classify<M, true>), gc, bc, 0, s, a, su);
    else hipLaunchKernelGGL((k_sur_classify<M, false>), gc, bc, 0, s, a, su);
    // enough workgroups for one slot per wave, at most one per CU
    const int64_t nslot = (int64_t)su.nblk * (kBlock / 64);
    const int64_t nwg = (nslot + kSurBlock / 64 - 1) / (kSurBlock / 64);
    const dim3 grid((unsigned)(nwg < ncu ? nwg : ncu)), block(kSurBlock);
    if (aniso) hipLaunchKernelGGL((k_sur_net<M, true>), grid, block, 0, s, a, su);
    else hipLaunchKernelGGL((k_sur_net<M, false>), grid, block, 0, s, a, su);
    return hipGetLastError();
}

hipError_t launch_surrogate_step(int model, int aniso, const StepArgs<float> &a, const SurArgs &su,
                                 hipStream_t s)
{
    switch (model) {
    case 1: return sur_m<kin::Barkley<float>>(aniso, a, su, s);
    case 3: return sur_m<kin::Fhn<float>>(aniso, a, su, s);
    case 4: return a.tab ? sur_m<kin::CrnTab>(aniso, a, su, s) : sur_m<kin::Crn<float>>(aniso, a, su, s);
    case 6: return sur_m<kin::Tp06<float>>(aniso, a, su, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sample(const StepArgs<float> &a, int nvar, int64_t n, uint64_t seed, float *out,
                         hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sample, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, nvar, n, seed,
                       out);
    return hipGetLastError();
}

hipError_t launch_ionic_map(int model, const StepArgs<float> &a, int nvar, const float *in,
                            int64_t n, float *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (model) {
    case 0: hipLaunchKernelGGL(k_ionic<kin::None<float>>, grid, block, 0, s, a, in, n, out); break;
    case 1: hipLaunchKernelGGL(k_ionic<kin::Barkley<float>>, grid, block, 0, s, a, in, n, out); break;
    case 2: hipLaunchKernelGGL(k_ionic<kin::Zfk<float>>, grid, block, 0, s, a, in, n, out); break;
    case 3: hipLaunchKernelGGL(k_ionic<kin::Fhn<float>>, grid, block, 0, s, a, in, n, out); break;
    case 4:
        if (a.tab) hipLaunchKernelGGL(k_ionic<kin::CrnTab>, grid, block, 0, s, a, in, n, out);
        else hipLaunchKernelGGL(k_ionic<kin::Crn<float>>, grid, block, 0, s, a, in, n, out);
        break;
    case 5: hipLaunchKernelGGL(k_ionic<kin::Fk4<float>>, grid, block, 0, s, a, in, n, out); break;
    case 6: hipLaunchKernelGGL(k_ionic<kin::Tp06<float>>, grid, block, 0, s, a, in, n, out); break;
    default: return hipErrorInvalidValue;
    }
    (void)nvar;
    return hipGetLastError();
}

}  // namespace bbx
