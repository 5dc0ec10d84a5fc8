// probe_exp2_bias -- mean, rms and maximum relative error of the hardware
// exp2 (v_exp_f32, __builtin_amdgcn_exp2f) on gfx950 against FP64 exp2, over
// FP32 arguments spread uniformly on several ranges.  The FP32 pair sweep
// divides its sums by (1 + mean error) because every FP32 pair term carries
// exactly one hardware exp2.  It also counts nonzero results of exp2 over
// [-1000, -150]: a term whose exponent is below -150 is exactly zero.
#include <hip/hip_runtime.h>

#include <cmath>
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

// grid-stride over M arguments x = lo + (hi - lo) (i + 0.5) / M rounded to FP32;
// one (sum, sum of squares, max) triple per block
__global__ void bias_kernel(long long M, float lo, float hi, double *part)
{
    __shared__ double s1[256], s2[256], s3[256];
    double a = 0, b = 0, c = 0;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < M; i += (long long)gridDim.x * 256) {
        const float x = lo + (hi - lo) * (float)((i + 0.5) / (double)M);
        const float y = __builtin_amdgcn_exp2f(x);
        const double r = (double)y / exp2((double)x) - 1.0;
        a += r;
        b += r * r;
        c = fmax(c, fabs(r));
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    s3[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
            s3[threadIdx.x] = fmax(s3[threadIdx.x], s3[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = s1[0];
        part[3 * blockIdx.x + 1] = s2[0];
        part[3 * blockIdx.x + 2] = s3[0];
    }
}

// number of x in [lo, hi) (M evenly spaced FP32 arguments) with exp2(x) != 0
__global__ void nonzero_kernel(long long M, float lo, float hi, unsigned long long *count)
{
    unsigned long long c = 0;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < M; i += (long long)gridDim.x * 256) {
        const float x = lo + (hi - lo) * (float)((i + 0.5) / (double)M);
        c += (__builtin_amdgcn_exp2f(x) != 0.0f) ? 1 : 0;
    }
    atomicAdd(count, c);
}

int main()
{
    const long long M = 1LL << 30;
    const int blocks = 4096;
    double *dpart;
    CHECK(hipMalloc(&dpart, sizeof(double) * 3 * blocks));
    std::vector<double> h(3 * blocks);
    const float ranges[][2] = {{-30.f, 0.f}, {-12.f, 0.f}, {-1.f, 0.f}, {-100.f, -30.f}};
    for (auto &r : ranges) {
        hipLaunchKernelGGL(bias_kernel, dim3(blocks), dim3(256), 0, 0, M, r[0], r[1], dpart);
        CHECK(hipGetLastError());
        CHECK(hipMemcpy(h.data(), dpart, sizeof(double) * 3 * blocks, hipMemcpyDeviceToHost));
        double a = 0, b = 0, c = 0;
        for (int i = 0; i < blocks; ++i) {
            a += h[3 * i];
            b += h[3 * i + 1];
            c = fmax(c, h[3 * i + 2]);
        }
        printf("exp2 on [%g,%g]: mean rel err %.3e  rms %.3e  max %.3e  (M=%lld)\n", r[0], r[1], a / M, sqrt(b / M), c,
               M);
    }
    CHECK(hipFree(dpart));

    unsigned long long *dcount, hcount = 0;
    CHECK(hipMalloc(&dcount, sizeof(unsigned long long)));
    CHECK(hipMemset(dcount, 0, sizeof(unsigned long long)));
    const long long Mz = 1LL << 28;
    hipLaunchKernelGGL(nonzero_kernel, dim3(blocks), dim3(256), 0, 0, Mz, -1000.f, -150.f, dcount);
    CHECK(hipGetLastError());
    CHECK(hipMemcpy(&hcount, dcount, sizeof(hcount), hipMemcpyDeviceToHost));
    printf("exp2 on [-1000,-150]: %llu nonzero results of %lld\n", hcount, Mz);
    CHECK(hipFree(dcount));
    return 0;
}
