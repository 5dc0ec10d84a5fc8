// exp2_probe.hip -- test-only probe of the hardware FP32 exp2 (v_exp_f32) on the GPU that runs
// the tests: the mean relative error of exp2f over n FP32 arguments evenly spaced on [lo, hi],
// against the FP64 exp2 of the same (FP32-rounded) argument.  The FP32 pair sweep divides its
// sums by (1 + that mean); this probe lets a test check the constant on the device at hand.
#include <hip/hip_runtime.h>

#include <cstdint>

__global__ __launch_bounds__(256) void k_exp2_rel_err(int64_t n, double lo, double step, double *partials)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        const float x = float(lo + step * (double(i) + 0.5));
        const float y = __builtin_amdgcn_exp2f(x);
        const double ref = exp2(double(x));
        acc += double(y) / ref - 1.0;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partials[blockIdx.x] = red[0];
}

// Writes nblocks partial sums of (exp2f(x)/exp2(x) - 1) into d_partials (device, nblocks doubles).
// Returns 0, or -1 for bad arguments, -4 if the launch failed.
extern "C" int exp2_probe_rel_err(int64_t n, double lo, double hi, double *d_partials, int nblocks, void *stream)
{
    if (n < 1 || !(hi > lo) || !d_partials || nblocks < 1 || nblocks > 65536)
        return -1;
    hipLaunchKernelGGL(k_exp2_rel_err, dim3(nblocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), n, lo,
                       (hi - lo) / double(n), d_partials);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}
