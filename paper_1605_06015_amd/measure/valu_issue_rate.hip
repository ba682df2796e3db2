// VALU issue-rate probe for gfx950: the sustained rate of one class of FP32/INT32
// vector instruction, measured on independent dependency chains (8 per thread, 32,768
// operations per thread) with every SIMD holding 8 waves.  The rates it prints fix the
// per-class issue costs that the ALU roofline of the step kernels is computed with:
// 2-source operations (mul, add, integer add, compare, select) pair, up to two wave64
// instructions per CU-cycle (measured 1.7-1.9), a 3-source FMA issues at one, a
// transcendental (exp, rcp) at a half.  Not part of the library; built by `python -m paper_1605_06015_amd.build --probe`
// (or the package's build step) into _build/valu_issue_rate, and run by hand.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int kChains = 8, kIter = 4096, kThreads = 256;

enum Op { FMA_LIT, EXP, RCP, EXP_MUL, FMA_REG, MUL, IADD, SELECT, CVT_ADD, NOPS };
const char *kName[NOPS] = {"fma (literal operand)", "exp", "rcp", "exp + dependent mul",
                           "fma (3 register operands)", "mul", "integer add",
                           "compare + mul + add + select", "cvt f32->i32->f32 + add"};
const int kInstsPerOp[NOPS] = {1, 1, 1, 2, 1, 1, 1, 4, 3};

template <int OP>
__global__ __launch_bounds__(kThreads) void k_rate(float *out, float seed)
{
    float x[kChains];
    int xi[kChains];
    const float y = seed * 1.0001f, z = seed * 1e-4f;
#pragma unroll
    for (int c = 0; c < kChains; c++) {
        x[c] = seed + 1e-3f * (float)(threadIdx.x + c);
        xi[c] = (int)threadIdx.x + c;
    }
    for (int i = 0; i < kIter; i++) {
#pragma unroll
        for (int c = 0; c < kChains; c++) {
            if (OP == FMA_LIT) x[c] = __builtin_fmaf(x[c], 0.999f, 1e-4f);
            else if (OP == EXP) x[c] = __builtin_amdgcn_exp2f(x[c]);
            else if (OP == RCP) x[c] = __builtin_amdgcn_rcpf(x[c]);
            else if (OP == EXP_MUL) x[c] = __builtin_amdgcn_exp2f(x[c]) * 0.5f;
            else if (OP == FMA_REG) x[c] = __builtin_fmaf(x[c], y, z);
            else if (OP == MUL) x[c] = x[c] * y;
            else if (OP == IADD) xi[c] = xi[c] + xi[(c + 1) % kChains];   // not foldable
            else if (OP == SELECT) x[c] = x[c] > y ? x[c] * 0.5f : x[c] + z;
            else x[c] = (float)(int)x[c] + y;
        }
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; c++) s += x[c] + (float)xi[c];
    out[blockIdx.x * kThreads + threadIdx.x] = s;   // grid * kThreads floats
}

// G operations per second of one class (an operation is kInstsPerOp instructions)
template <int OP>
double rate(float *d, int nblk)
{
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0;
    hipLaunchKernelGGL(k_rate<OP>, dim3(nblk), dim3(kThreads), 0, 0, d, 0.5f);   // warm-up
    constexpr int kReps = 5;
    (void)hipEventRecord(a, 0);
    for (int r = 0; r < kReps; r++) hipLaunchKernelGGL(k_rate<OP>, dim3(nblk), dim3(kThreads), 0, 0, d, 0.5f);
    (void)hipEventRecord(b, 0);
    float ms = 0.f;
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1.0;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    const double waves = (double)nblk * (kThreads / 64) * kReps;
    return waves * kIter * kChains / (ms * 1e-3) / 1e9;
}

template <int OP>
void report(float *d, int nblk)
{
    const double g = rate<OP>(d, nblk);
    printf("%-30s %8.1f G ops/s  %8.1f G wave-instructions/s\n", kName[OP], g, g * kInstsPerOp[OP]);
}

}  // namespace

int main()
{
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 1;
    const int nblk = ncu * 8 * 4;   // 8 resident waves per SIMD, four rounds
    float *d = nullptr;
    if (hipMalloc(&d, (size_t)nblk * kThreads * sizeof(float)) != hipSuccess) return 1;
    printf("%d CUs\n", ncu);
    report<FMA_LIT>(d, nblk);
    report<EXP>(d, nblk);
    report<RCP>(d, nblk);
    report<EXP_MUL>(d, nblk);
    report<FMA_REG>(d, nblk);
    report<MUL>(d, nblk);
    report<IADD>(d, nblk);
    report<SELECT>(d, nblk);
    report<CVT_ADD>(d, nblk);
    fflush(stdout);
    const bool ok = hipGetLastError() == hipSuccess;
    (void)hipFree(d);
    return ok ? 0 : 1;
}
