// probe_valu_rates -- issue rate of single VALU instruction kinds on gfx950:
// 16 independent dependency chains per lane, 8192 workgroups of 256 lanes,
// best of 3 launches, reported as lane-operations per second and per clock
// per compute unit at 2.4 GHz.  These rates are the cost model of the pair
// sweep (FP32 arithmetic vs the FP64 pair geometry vs the hardware exp2).
#include <hip/hip_runtime.h>
#include <cstdio>

#define CHECK(x)                                                                       \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);      \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

constexpr int C = 16;

template <int K>
__global__ __launch_bounds__(256) void kern(float* out, int iters, float seed)
{
    float f[C];
    double d[C];
    int iv[C];
    const float a = seed * 0.9999f, bconst = seed * 1e-7f;
    const int step = (int)(seed * 3.0f);
    for (int k = 0; k < C; ++k) { f[k] = seed + 1e-3f * (threadIdx.x + k); d[k] = f[k]; iv[k] = threadIdx.x * 7 + k; }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < C; ++k) {
            if (K == 0) f[k] = fmaf(f[k], 0.9999f, 1e-7f);           // v_fma_f32
            if (K == 1) f[k] = f[k] + 1e-7f;                           // v_add_f32
            if (K == 2) d[k] = fma(d[k], 0.9999, 1e-7);               // v_fma_f64
            if (K == 3) d[k] = d[k] + 1e-7;                            // v_add_f64
            if (K == 4) d[k] = d[k] * 0.99999;                         // v_mul_f64
            if (K == 5) f[k] = __builtin_amdgcn_exp2f(-f[k]);          // v_exp_f32
            if (K == 6) f[k] = fmaf(f[k], a, bconst);                  // v_fma_f32, register operands
            if (K == 7) iv[k] = iv[k] - step;                          // v_sub_u32
            if (K == 8) { iv[k] += step; f[k] += (float)iv[k]; }       // v_add_u32 + v_cvt_f32_i32 + v_add_f32
            if (K == 9) { f[k] = f[k] * a; d[k] = d[k] + (double)f[k]; } // v_mul_f32 + v_cvt_f64_f32 + v_add_f64
            if (K == 10) { f[k] = f[k] + (float)d[k]; d[k] = d[k] * 0.99999; } // v_cvt_f32_f64 + add f32 + mul f64
            if (K == 11) f[k] = f[k] * a;                              // v_mul_f32
            // pairs of independent chains: do two kinds share issue slots or run side by side?
            if (K == 12) { f[k] = fmaf(f[k], a, bconst); d[k] = fma(d[k], 0.9999, 1e-7); }   // fma_f32 + fma_f64
            if (K == 13) { f[k] = fmaf(f[k], a, bconst); iv[k] = __float_as_int(__builtin_amdgcn_exp2f(-__int_as_float(iv[k]))); } // fma_f32 + exp
            if (K == 14) { d[k] = fma(d[k], 0.9999, 1e-7); iv[k] = __float_as_int(__builtin_amdgcn_exp2f(-__int_as_float(iv[k]))); } // fma_f64 + exp
            if (K == 15) f[k] = float(d[k] * 0.99999 + (double)f[k]) * a;  // cvt_f64_f32 + add_f64 + cvt_f32_f64 + mul_f32
        }
    }
    float s = 0;
    for (int k = 0; k < C; ++k) s += f[k] + (float)d[k] + (float)iv[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

int main()
{
    const int nb = 256 * 8 * 4, nt = 256, iters = 2048;
    float* out;
    CHECK(hipMalloc(&out, sizeof(float) * nb * nt));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const char* names[] = {"v_fma_f32 (literal)", "v_add_f32 (literal)", "v_fma_f64", "v_add_f64", "v_mul_f64", "v_exp_f32",
                           "v_fma_f32 (regs)", "v_sub_u32", "add_u32+cvt_i32+add", "mul+cvt_f64_f32+add64", "cvt_f32_f64+add+mul64", "v_mul_f32",
                           "fma_f32 | fma_f64", "fma_f32 | exp_f32", "fma_f64 | exp_f32", "cvt64+add64+cvt32+mul32"};
    const int nops[] = {1, 1, 1, 1, 1, 1, 1, 1, 3, 3, 3, 1, 2, 2, 2, 4};
    for (int k = 0; k < 16; ++k) {
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            CHECK(hipEventRecord(e0));
            switch (k) {
            case 0: hipLaunchKernelGGL(kern<0>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 1: hipLaunchKernelGGL(kern<1>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 2: hipLaunchKernelGGL(kern<2>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 3: hipLaunchKernelGGL(kern<3>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 4: hipLaunchKernelGGL(kern<4>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 5: hipLaunchKernelGGL(kern<5>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 6: hipLaunchKernelGGL(kern<6>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 7: hipLaunchKernelGGL(kern<7>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 8: hipLaunchKernelGGL(kern<8>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 9: hipLaunchKernelGGL(kern<9>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 10: hipLaunchKernelGGL(kern<10>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 11: hipLaunchKernelGGL(kern<11>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 12: hipLaunchKernelGGL(kern<12>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 13: hipLaunchKernelGGL(kern<13>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 14: hipLaunchKernelGGL(kern<14>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            case 15: hipLaunchKernelGGL(kern<15>, dim3(nb), dim3(nt), 0, 0, out, iters, 1.0f); break;
            }
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(e1));
            CHECK(hipEventSynchronize(e1));
            float ms;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) best = ms;
        }
        const double ops = (double)nb * nt * iters * C * nops[k];
        printf("%-20s %.3e lane-ops/s  (%.3f ms)  = %.2f lane-ops/clk/CU at 2.4 GHz\n", names[k], ops / (best * 1e-3), best,
               ops / (best * 1e-3) / (256 * 2.4e9));
    }
    int dev;
    hipDeviceProp_t p;
    CHECK(hipGetDevice(&dev));
    CHECK(hipGetDeviceProperties(&p, dev));
    printf("device %s CUs %d clock %d kHz\n", p.gcnArchName, p.multiProcessorCount, p.clockRate);
    CHECK(hipFree(out));
    return 0;
}
