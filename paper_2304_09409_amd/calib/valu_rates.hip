// valu_rates.hip -- issue cost of the FP32 transcendental instructions against an FMA on the
// device's vector ALU (calibration of the vector-ALU view of the embedding kernels, whose
// activation tanh(x) = 1 - 2 / (2^(K x) + 1) is one v_exp_f32, one v_rcp_f32 and two FMA-class
// instructions). Eight independent chains per lane, 8 waves per SIMD, so that latency is hidden
// and issue rate is what is measured. Prints cycles per wave instruction step for each form.
#include <hip/hip_runtime.h>
#include <cstdio>

constexpr int NIT = 2048;

template <int MODE>
__global__ void __launch_bounds__(256) k_chain(float* out, float a, float b)
{
    float x[8], y[8];
    for (int i = 0; i < 8; ++i) x[i] = y[i] = 1e-3f * (threadIdx.x + i);
    for (int it = 0; it < NIT; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (MODE == 0) x[i] = __builtin_fmaf(x[i], a, b);
            if (MODE == 1) x[i] = __builtin_amdgcn_exp2f(x[i]) * a;
            if (MODE == 2) x[i] = __builtin_amdgcn_rcpf(x[i]) * a;
            if (MODE == 3) x[i] = 1.0f - 2.0f * __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(x[i]) + 1.0f);
            if (MODE == 4) {
                x[i] = __builtin_amdgcn_exp2f(x[i]) * a;
                y[i] = __builtin_fmaf(y[i], a, b);
                y[i] = __builtin_fmaf(y[i], a, b);
                y[i] = __builtin_fmaf(y[i], a, b);
            }
        }
    }
    float s = 0.0f;
    for (int i = 0; i < 8; ++i) s += x[i] + y[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;   // one slot per thread of the grid
}

#define CHECK(x)                                                                    \
    do {                                                                            \
        if ((x) != hipSuccess) {                                                    \
            std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(x));      \
            return 1;                                                               \
        }                                                                           \
    } while (0)

int main()
{
    int ncu = 0, clk = 0;
    CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0));
    CHECK(hipDeviceGetAttribute(&clk, hipDeviceAttributeClockRate, 0));
    const int blocks = ncu * 8;   // 8 blocks of 4 waves per CU: 8 waves per SIMD
    float* out = nullptr;
    CHECK(hipMalloc(&out, sizeof(float) * blocks * 256));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const char* names[5] = {"fma", "exp + mul", "rcp + mul", "tanh (exp, add, rcp, fma)", "exp + mul + 3 fma"};
    double cyc[5] = {0, 0, 0, 0, 0};
    for (int m = 0; m < 5; ++m) {
        for (int rep = 0; rep < 2; ++rep) {   // the first launch warms up
            CHECK(hipEventRecord(e0));
            switch (m) {
            case 0: hipLaunchKernelGGL(k_chain<0>, dim3(blocks), dim3(256), 0, 0, out, 0.999f, 1e-4f); break;
            case 1: hipLaunchKernelGGL(k_chain<1>, dim3(blocks), dim3(256), 0, 0, out, 0.5f, 0.0f); break;
            case 2: hipLaunchKernelGGL(k_chain<2>, dim3(blocks), dim3(256), 0, 0, out, 1.0f, 0.0f); break;
            case 3: hipLaunchKernelGGL(k_chain<3>, dim3(blocks), dim3(256), 0, 0, out, 1.0f, 0.0f); break;
            default: hipLaunchKernelGGL(k_chain<4>, dim3(blocks), dim3(256), 0, 0, out, 0.5f, 1e-4f); break;
            }
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(e1));
            CHECK(hipEventSynchronize(e1));
            float ms = 0.0f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            const double steps_per_simd = 8.0 * NIT * 8;   // waves per SIMD x iterations x chains
            cyc[m] = ms * 1e-3 * clk * 1e3 / steps_per_simd;  // clockRate is in kHz
        }
        std::printf("%-28s %6.2f cycles per wave step\n", names[m], cyc[m]);
    }
    std::printf("in FMA issue slots: exp %.2f, rcp %.2f, tanh %.2f (nominal clock %d kHz, %d CUs)\n",
                (cyc[1] - cyc[0]) / cyc[0], (cyc[2] - cyc[0]) / cyc[0], cyc[3] / cyc[0], clk, ncu);
    CHECK(hipFree(out));
    return 0;
}
