// hawkes_resample.hip -- the cut-posterior X-update on gfx950.
//
// Paper Section 2.2: with the cut posterior p(theta | X, t) p(X | coarsened
// data), the latent locations are redrawn from p(X | coarsened data) in O(N)
// by sampling every event uniformly inside its county.  Counties are
// axis-aligned rectangles here.  Random numbers come from the counter-based
// Philox4x64-10 generator (Salmon, Moraes, Dror and Shaw, SC'11): event i of
// draw `iteration` uses counter (i, iteration, 0, 0) and key (seed, 0), so any
// event's draw is reproducible on its own and every GPU of a multi-GPU run can
// regenerate the same locations without communication.
//
// The kernel is HBM-bound: it reads 4 B of county id and 32 B of rectangle per
// event (rectangles hit in cache) and writes 16 B.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hawkes.h"
#include "hawkes_common.h"

namespace hawkes {
namespace {

struct U64x4 {
    uint64_t w[4];
};

__device__ inline U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1)
{
    // round multipliers and Weyl key increments of the published Philox4x64
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
        const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    return U64x4{{c0, c1, c2, c3}};
}

__global__ __launch_bounds__(256) void k_resample(int64_t n, const int32_t *__restrict__ county,
                                                  const double *__restrict__ rect, int32_t n_counties, uint64_t seed,
                                                  uint64_t iteration, double *__restrict__ x, double *__restrict__ y)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int32_t c = county[i];
    if (c < 0 || c >= n_counties) {
        const double nan = __builtin_nan("");
        x[i] = nan;
        y[i] = nan;
        return;
    }
    const U64x4 w = philox4x64_10(uint64_t(i), iteration, 0, 0, seed, 0);
    const double ux = double(w.w[0] >> 11) * 0x1.0p-53;
    const double uy = double(w.w[1] >> 11) * 0x1.0p-53;
    const double *r = rect + 4 * int64_t(c);
    x[i] = __builtin_fma(ux, r[2] - r[0], r[0]);
    y[i] = __builtin_fma(uy, r[3] - r[1], r[1]);
}

}  // namespace
}  // namespace hawkes

extern "C" int hawkes_resample_locations(int64_t n, const int32_t *d_county, const double *d_rect,
                                         int32_t n_counties, uint64_t seed, uint64_t iteration, double *d_x,
                                         double *d_y, void *stream)
{
    using namespace hawkes;
    if (n < 0 || n_counties < 1 || (n > 0 && (!d_county || !d_rect || !d_x || !d_y))) {
        set_error("resample: invalid arguments (n = %lld, n_counties = %d)", (long long)n, n_counties);
        return HAWKES_EINVAL;
    }
    if (n == 0)
        return HAWKES_OK;
    const unsigned blocks = unsigned((n + 255) / 256);
    hipLaunchKernelGGL(k_resample, dim3(blocks), dim3(256), 0, as_stream(stream), n, d_county, d_rect, n_counties,
                       seed, iteration, d_x, d_y);
    return check_launch("resample");
}
