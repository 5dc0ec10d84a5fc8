// probe_mfma_f64 -- operand/result lane layout and throughput of the FP64
// matrix instruction v_mfma_f64_16x16x4_f64 on gfx950.
//
// Layout check: one wave multiplies A (16 x 4) by B (4 x 16) with
// A[i][k] = (k == 0) ? i + 1 : (k == 1 ? 1 : 0) and
// B[k][j] = (k == 0) ? 1 : (k == 1 ? 1000 (j + 1) : 0), so C[i][j] = i + 1 + 1000 (j + 1)
// identifies the row and column of every result.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; the probe reports which of two
// result layouts holds: C[4 (l / 16) + r][l % 16] or C[4 r + l / 16][l % 16]
// for result r of lane l.
//
// Throughput: 8 independent accumulators per wave, 4096 iterations, 8192
// workgroups of 256 lanes; FLOP = 2 * 16 * 16 * 4 per instruction.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <vector>

#define CHECK(x)                                                                       \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);      \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

typedef double double4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(64) void layout_kernel(double *out)
{
    const int l = threadIdx.x;
    const int i = l % 16, k = l / 16;
    const double a = (k == 0) ? double(i + 1) : (k == 1 ? 1.0 : 0.0);
    const int j = l % 16, kb = l / 16;
    const double b = (kb == 0) ? 1.0 : (kb == 1 ? 1000.0 * (j + 1) : 0.0);
    double4_t c = {0.0, 0.0, 0.0, 0.0};
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    for (int r = 0; r < 4; ++r)
        out[4 * l + r] = c[r];
}

__global__ __launch_bounds__(256) void rate_kernel(double *out, int iters, double seed)
{
    double4_t c[8];
    for (int q = 0; q < 8; ++q)
        c[q] = double4_t{seed * q, 0.0, 0.0, 0.0};
    const double a = seed + 1e-3 * threadIdx.x, b = seed * 0.5;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            c[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[q], 0, 0, 0);
    }
    double s = 0.0;
    for (int q = 0; q < 8; ++q)
        s += c[q][0] + c[q][1] + c[q][2] + c[q][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

int main()
{
    double *d;
    CHECK(hipMalloc(&d, sizeof(double) * 256));
    hipLaunchKernelGGL(layout_kernel, dim3(1), dim3(64), 0, 0, d);
    CHECK(hipGetLastError());
    std::vector<double> h(256);
    CHECK(hipMemcpy(h.data(), d, sizeof(double) * 256, hipMemcpyDeviceToHost));
    int bad_a = 0, bad_b = 0;
    for (int l = 0; l < 64; ++l)
        for (int r = 0; r < 4; ++r) {
            const int j = l % 16;
            const int ia = 4 * (l / 16) + r, ib = 4 * r + l / 16;
            bad_a += h[4 * l + r] != ia + 1 + 1000.0 * (j + 1);
            bad_b += h[4 * l + r] != ib + 1 + 1000.0 * (j + 1);
        }
    printf("layout C[4 (l/16) + r][l %% 16]: %d mismatches of 256\n", bad_a);
    printf("layout C[4 r + l/16][l %% 16]: %d mismatches of 256\n", bad_b);
    CHECK(hipFree(d));

    const int nb = 8192, nt = 256, iters = 4096;
    double *o;
    CHECK(hipMalloc(&o, sizeof(double) * nb * nt));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
        CHECK(hipEventRecord(e0));
        hipLaunchKernelGGL(rate_kernel, dim3(nb), dim3(nt), 0, 0, o, iters, 1.0);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        float ms;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best)
            best = ms;
    }
    const double waves = double(nb) * nt / 64;
    const double flop = waves * iters * 8 * (2.0 * 16 * 16 * 4);
    printf("v_mfma_f64_16x16x4_f64: %.2f TFLOP/s (%.3f ms), %.1f FLOP/clk/CU at 2.4 GHz\n", flop / (best * 1e-3) / 1e12,
           best, flop / (best * 1e-3) / (256 * 2.4e9));
    CHECK(hipFree(o));
    return 0;
}
