// hawkes_mlp.hip -- the BF16 surrogate network of the log-likelihood on gfx950.
//
// Network 6 -> 256 -> 256 -> 256 -> 1 with GELU activations (x Phi(x)):
//   h1 = W1 z + b1, a1 = gelu(h1), h2 = W2 a1 + b2, a2 = gelu(h2),
//   h3 = W3 a2 + b3, a3 = gelu(h3), f = w4 . a3 + b4.
// Flat parameter layout (133,633 values): W1 (256x6, out x in), b1, W2
// (256x256), b2, W3 (256x256), b3, w4 (256), b4.
//
// The state buffer holds FP32 master weights, the two Adam moment vectors,
// and BF16 working copies: the flat vector in its own layout, W2 and W3
// transposed (in x out) for the one-sample kernels, and W2, W3, W2^T, W3^T as
// matrix-core operand fragments (below) for the batched kernels.
//
// Batched kernels (value and input gradient of many inputs, the training
// pass) run the 256 x 256 products on the matrix cores with
// v_mfma_f32_16x16x32_bf16, features as rows and 16 samples as columns, a
// workgroup of 8 waves per tile of 16 samples (2 row tiles per wave; batched
// inference takes two sample tiles per workgroup, so every weight fragment a
// wave loads feeds both).  A product's
// FP32 output sits in the lanes in the k order of the next product's column
// operand, so each wave converts its own outputs and the operands meet in
// LDS.  The weights are exact BF16; each FP32 activation enters as hi + lo
// BF16 parts (x = hi + lo + O(2^-18 |x|)), two products per operand, so the
// result matches FP32 activations times BF16 weights to ~1e-5 relative.
// One-sample kernels (a value and gradient at batch <= 8, a leapfrog
// trajectory) keep the 256-lane matrix-vector form, whose latency is lower.
//
// Inference: value and input gradient per sample (k_mlp_forward for small
// batches, k_mlp_forward_mfma), or a whole leapfrog trajectory on the
// surrogate posterior in one workgroup (k_mlp_leapfrog, the stage-1 proposal
// of delayed-acceptance HMC).
//
// Training loss (value + gradient matching):
//   L = (1/B) sum_b (f(z_b) - y_b)^2 + lambda |grad_z f(z_b) - g_b|^2.
// Its parameter gradient uses d/dtheta [r . grad_z f] = d/dtheta [D_r f] for
// r = grad_z f - g held fixed: per sample a primal pass, the reverse pass for
// grad_z f, a forward tangent pass along r, and one reverse pass through the
// primal and tangent computations; the per-sample adjoint vectors are then
// contracted over the batch (matrix cores for W2 and W3, fixed-order wave
// reductions for the rest), the same way on every call (deterministic).

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "hawkes.h"
#include "hawkes_common.h"
#include "hawkes_mlp.h"

namespace hawkes {
namespace {

constexpr int H = 256;
constexpr int DZ = 6;
constexpr int64_t P = HAWKES_MLP_PARAMS;
// offsets of the parameter blocks in the flat vector
constexpr int64_t OW1 = 0, OB1 = OW1 + H * DZ, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H * H,
                  OW4 = OB3 + H, OB4 = OW4 + H;
static_assert(OB4 + 1 == P, "parameter layout");

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct StateLayout {
    size_t master, m, v, wb, wt2, wt3, frag[4], total;
};

// Matrix-core operand copies of the 256 x 256 matrices, in this order.
enum { F_W2, F_W2T, F_W3, F_W3T };

StateLayout state_layout()
{
    StateLayout s;
    size_t off = 0;
    s.master = off;
    off = align256(off + sizeof(float) * P);
    s.m = off;
    off = align256(off + sizeof(float) * P);
    s.v = off;
    off = align256(off + sizeof(float) * P);
    s.wb = off;
    off = align256(off + sizeof(uint16_t) * P);
    s.wt2 = off;
    off = align256(off + sizeof(uint16_t) * H * H);
    s.wt3 = off;
    off = align256(off + sizeof(uint16_t) * H * H);
    for (int i = 0; i < 4; ++i) {
        s.frag[i] = off;
        off = align256(off + sizeof(uint16_t) * H * H);
    }
    s.total = off;
    return s;
}

struct Net {
    const uint16_t *w;    // flat BF16 copy
    const uint16_t *wt2;  // W2 transposed: wt2[k * H + j] = W2[j][k]
    const uint16_t *wt3;
};

Net net_of(const void *state)
{
    const StateLayout L = state_layout();
    const char *b = static_cast<const char *>(state);
    return Net{reinterpret_cast<const uint16_t *>(b + L.wb), reinterpret_cast<const uint16_t *>(b + L.wt2),
               reinterpret_cast<const uint16_t *>(b + L.wt3)};
}

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) unsigned short u16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// The batched kernels' view: the flat BF16 copy and the four operand copies.
struct MfNet {
    const uint16_t *w;
    const bf16x8 *frag[4];
};

MfNet mfnet_of(const void *state)
{
    const StateLayout L = state_layout();
    const char *b = static_cast<const char *>(state);
    MfNet n;
    n.w = reinterpret_cast<const uint16_t *>(b + L.wb);
    for (int i = 0; i < 4; ++i)
        n.frag[i] = reinterpret_cast<const bf16x8 *>(b + L.frag[i]);
    return n;
}

// Operand fragments.  A product out = M v over 256 features (M[m][k], m the
// output feature) is 16 row tiles x 8 chunks of 32 k; in a chunk, lane l
// (row m = 16 mt + l % 16, lane group q = l / 16) holds 8 consecutive BF16
// values at k = 32 kc + 4q + c (c < 4) and 32 kc + 16 + 4q + (c - 4) (c >= 4).
// That k order is the order in which the FP32 output of the previous product
// sits in the lanes (two 16-row tiles, rows 4q..4q+3 of each), so the output
// becomes the next column operand without leaving the lane; the column
// operand uses the same k order, so every k pairs with itself.  A lane's
// fragment is 16 contiguous bytes: fragment (mt, kc) of lane l at
// ((mt * 8 + kc) * 64 + l) * 8.
__host__ __device__ inline int frag_index(int m, int k)
{
    const int mt = m >> 4, lm = m & 15, kc = k >> 5, r = k & 31;
    const int upper = r >> 4, q = (r & 15) >> 2, c = upper * 4 + (r & 3);
    return ((mt * 8 + kc) * 64 + q * 16 + lm) * 8 + c;
}

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// round to nearest, ties to even; NaN stays NaN
__device__ inline uint16_t f32_to_bf16(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return uint16_t((u >> 16) | 0x40u);
    const uint32_t lsb = (u >> 16) & 1u;
    return uint16_t((u + 0x7fffu + lsb) >> 16);
}

constexpr float K_SQRT1_2 = 0.70710678118654752440f;
constexpr float K_INV_SQRT_2PI = 0.39894228040143267794f;

__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * K_SQRT1_2)); }
__device__ inline float gelu_d1(float x)
{
    return 0.5f * (1.0f + erff(x * K_SQRT1_2)) + x * K_INV_SQRT_2PI * expf(-0.5f * x * x);
}
__device__ inline float gelu_d2(float x) { return K_INV_SQRT_2PI * expf(-0.5f * x * x) * (2.0f - x * x); }

// y_j = sum_k M[k * H + j] v[k]  (M stored k-major: coalesced over j)
__device__ inline float matvec_kmajor(const uint16_t *__restrict__ M, const float *v, int j)
{
    float acc = 0.0f;
#pragma unroll 32
    for (int k = 0; k < H; ++k)
        acc = fmaf(bf16_to_f32(M[k * H + j]), v[k], acc);
    return acc;
}

// Block-wide sums of seven values per thread (256 threads) in one pairwise
// tree, results in every thread.
constexpr int NS7 = 7;
__device__ inline void block_sum7(const float v[NS7], float (*red)[H], float out[NS7])
{
    const int j = threadIdx.x;
#pragma unroll
    for (int z = 0; z < NS7; ++z)
        red[z][j] = v[z];
    __syncthreads();
    for (int w = H / 2; w > 0; w >>= 1) {
        if (j < w)
#pragma unroll
            for (int z = 0; z < NS7; ++z)
                red[z][j] += red[z][j + w];
        __syncthreads();
    }
#pragma unroll
    for (int z = 0; z < NS7; ++z)
        out[z] = red[z][0];
    __syncthreads();
}

// Value and input gradient of one input sz[DZ] (in LDS) by the workgroup's
// H threads; every thread returns f and g[DZ].  The scratch arrays are the
// caller's LDS.
struct FwdLds {
    float a1[H], a2[H], d[H], red[NS7][H];
};
__device__ inline void value_and_grad(const Net &net, const float *sz, FwdLds &L, float &f, float g[DZ])
{
    const int j = threadIdx.x;
    const uint16_t *w = net.w;
    float h1 = bf16_to_f32(w[OB1 + j]);
#pragma unroll
    for (int i = 0; i < DZ; ++i)
        h1 = fmaf(bf16_to_f32(w[OW1 + j * DZ + i]), sz[i], h1);
    L.a1[j] = gelu(h1);
    const float s1 = gelu_d1(h1);
    __syncthreads();
    const float h2 = bf16_to_f32(w[OB2 + j]) + matvec_kmajor(net.wt2, L.a1, j);
    L.a2[j] = gelu(h2);
    const float s2 = gelu_d1(h2);
    __syncthreads();
    const float h3 = bf16_to_f32(w[OB3 + j]) + matvec_kmajor(net.wt3, L.a2, j);
    const float w4 = bf16_to_f32(w[OW4 + j]);
    const float vf = w4 * gelu(h3);  // summed with the input gradient below
    L.d[j] = w4 * gelu_d1(h3);
    __syncthreads();
    const float d2 = s2 * matvec_kmajor(w + OW3, L.d, j);  // (W3^T d3)_j: W3 row-major is k-major for W3^T
    __syncthreads();
    L.d[j] = d2;
    __syncthreads();
    const float d1 = s1 * matvec_kmajor(w + OW2, L.d, j);
    float v7[NS7], s7[NS7];
    v7[0] = vf;
#pragma unroll
    for (int i = 0; i < DZ; ++i)
        v7[1 + i] = bf16_to_f32(w[OW1 + j * DZ + i]) * d1;
    block_sum7(v7, L.red, s7);
    f = s7[0] + bf16_to_f32(w[OB4]);
#pragma unroll
    for (int i = 0; i < DZ; ++i)
        g[i] = s7[1 + i];
}

// Value and input gradient, one workgroup per sample.
__global__ __launch_bounds__(H) void k_mlp_forward(Net net, const float *__restrict__ z, int64_t B,
                                                   float *__restrict__ f_out, float *__restrict__ gz_out)
{
    __shared__ float sz[DZ];
    __shared__ FwdLds L;
    const int j = threadIdx.x;
    const int64_t b = blockIdx.x;
    if (j < DZ)
        sz[j] = z[b * DZ + j];
    __syncthreads();
    float f, g[DZ];
    value_and_grad(net, sz, L, f, g);
    if (j == 0) {
        f_out[b] = f;
        if (gz_out)
            for (int i = 0; i < DZ; ++i)
                gz_out[b * DZ + i] = g[i];
    }
}

// A leapfrog trajectory on the surrogate posterior in one workgroup (the
// stage-1 proposal of delayed-acceptance HMC): n_steps steps of
// H(z, p) = -s(z) + p' M^-1 p / 2 with
//   s(z) = s_y f((z - m_z) / s_z) + m_y - z.z / (2 prior_var),
// from (z, p) with grad = ds/dz at z: half a momentum step, then per step a
// position step, s and its gradient at the new point, and a full momentum
// step (half a step after the last one).  Position and momentum updates are
// FP64 without contraction, in the operation order of a host-side leapfrog
// written the same way; a step whose s or gradient is not finite ends the
// trajectory (s = -inf, no final half step).
__global__ __launch_bounds__(H) void k_mlp_leapfrog(Net net, hawkes_mlp_leapfrog_io *io, int n)
{
#pragma clang fp contract(off)
    __shared__ float sz[DZ];
    __shared__ FwdLds L;
    __shared__ double z[DZ], p[DZ], g[DZ];
    __shared__ double sval;
    __shared__ int ok;
    const int j = threadIdx.x;
    const double eps = io->eps, m_y = io->m_y, s_y = io->s_y, pv = io->prior_var;
    double im = 0.0, mz = 0.0, szc = 1.0;
    if (j < DZ) {
        z[j] = io->z[j];
        p[j] = io->p[j] + (0.5 * eps) * io->grad[j];
        im = io->inv_mass[j];
        mz = io->m_z[j];
        szc = io->s_z[j];
    }
    if (j == 0) {
        ok = 1;
        sval = 0.0;
    }
    __syncthreads();
    for (int step = 0; step < n; ++step) {
        if (j < DZ) {
            z[j] = z[j] + (eps * im) * p[j];
            sz[j] = float((z[j] - mz) / szc);
        }
        __syncthreads();
        float f, gz[DZ];
        value_and_grad(net, sz, L, f, gz);
        if (j < DZ)
            g[j] = (double(gz[j]) * s_y) / szc - z[j] / pv;
        if (j == 0) {
            double zz = 0.0;
            for (int i = 0; i < DZ; ++i)
                zz = zz + z[i] * z[i];
            sval = (double(f) * s_y + m_y) - (0.5 * zz) / pv;
        }
        __syncthreads();
        if (j == 0) {
            bool fin = isfinite(sval);
            for (int i = 0; i < DZ; ++i)
                fin = fin && isfinite(g[i]);
            ok = fin ? 1 : 0;
        }
        __syncthreads();
        if (!ok)
            break;
        if (j < DZ && step + 1 < n)
            p[j] = p[j] + eps * g[j];
        __syncthreads();
    }
    if (j < DZ) {
        if (ok && n > 0)
            p[j] = p[j] + (0.5 * eps) * g[j];
        io->z[j] = z[j];
        io->p[j] = p[j];
        io->grad[j] = g[j];
    }
    if (j == 0) {
        io->s = ok ? sval : -HUGE_VAL;
        io->status = ok ? 1.0 : 0.0;
    }
}

// ------------------------------------------------------------------ batched kernels (matrix cores)

// A workgroup of 8 waves takes 16 samples.  In every 256-feature product the
// wave w computes row tiles 2w and 2w+1 (features 32w..32w+31) for the 16
// samples: lane l (sample l % 16, lane group q = l / 16) holds v[i], i = 4 t + r,
// of feature 32 w + 16 t + 4 q + r (t = 0, 1; r = 0..3).  A product's column
// operand (all 256 features) is published through LDS: wave w converts its 8
// values to the hi + lo BF16 operands of chunk w, every wave then reads all 8
// chunks.
constexpr int NWAVE = 8;
constexpr int RT = 16 / NWAVE;  // row tiles per wave
constexpr int VPL = 4 * RT;     // values per lane

__device__ inline int feat(int w, int q, int i) { return 16 * (RT * w + (i >> 2)) + 4 * q + (i & 3); }

__device__ inline void split8(const float x[8], bf16x8 &hi, bf16x8 &lo)
{
    u16x8 h, l;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const uint16_t xh = f32_to_bf16(x[c]);
        h[c] = xh;
        l[c] = f32_to_bf16(x[c] - bf16_to_f32(xh));
    }
    hi = __builtin_bit_cast(bf16x8, h);
    lo = __builtin_bit_cast(bf16x8, l);
}

// Column operands in LDS: two slots (consecutive products alternate), 8 chunks, hi and lo, 64 lanes.
typedef bf16x8 Operands[2][8][2][64];

// The wave's 16 weight fragments of a product (its RT row tiles x 8 chunks),
// requested ahead of the product: the callers issue them before the elementwise
// work that forms the product's input, which then hides the memory latency.
typedef bf16x8 Frags[8][RT];

__device__ inline void load_frags(const bf16x8 *__restrict__ M, Frags &a)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int kc = 0; kc < 8; ++kc)
#pragma unroll
        for (int t = 0; t < RT; ++t)
            a[kc][t] = M[((RT * w + t) * 8 + kc) * 64 + l];
    // keep the loads here: the scheduler would otherwise sink each next to its use
    __builtin_amdgcn_sched_barrier(0);
}

// y = M x for the workgroup's 16 samples (M's fragments in a), x given by each
// wave's values.  Element c of chunk kc is the value of row tile 2 kc + c / 4,
// row 4 q + c % 4: for the publishing wave (kc = w) that is x[c].
__device__ inline void mf_product(const Frags &a, const float x[VPL], float y[VPL], Operands &op, int slot)
{
    static_assert(RT == 2, "one published chunk per wave");
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    {
        bf16x8 hi, lo;
        split8(x, hi, lo);
        op[slot][w][0][l] = hi;
        op[slot][w][1][l] = lo;
    }
    __syncthreads();
    f32x4 acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
        acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kc = 0; kc < 8; ++kc) {
        const bf16x8 bh = op[slot][kc][0][l], bl = op[slot][kc][1][l];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kc][t], bl, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kc][t], bh, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            y[4 * t + r] = acc[t][r];
}

// sum over the four lane groups that hold one sample (every lane gets the same bits)
__device__ inline float group_sum(float x)
{
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    return x;
}

// sum over the wave by a fixed butterfly
__device__ inline float wave_sum(float x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        x += __shfl_xor(x, o);
    return x;
}

// Per-sample sums of NRED values over all 256 features: each lane's partial, the
// lane groups of a wave, then the waves in order through LDS; every lane of the
// sample gets the same total.
constexpr int NRED = 7;
__device__ inline void sample_sums(float v[NRED], float (*red)[16][NRED])
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NRED; ++k)
        v[k] = group_sum(v[k]);
    if (l < 16)
#pragma unroll
        for (int k = 0; k < NRED; ++k)
            red[w][l][k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NRED; ++k) {
        float t = red[0][l & 15][k];
#pragma unroll
        for (int ww = 1; ww < NWAVE; ++ww)
            t += red[ww][l & 15][k];
        v[k] = t;
    }
}

// Layer-1 weights, biases and output weights in FP32, staged in LDS by each
// workgroup of the batched kernels.
struct SmallW {
    float w1[DZ][H];
    float b1[H], b2[H], b3[H], w4[H];
};

__device__ inline void stage_small(const uint16_t *__restrict__ w, SmallW &sw)
{
    for (int p = threadIdx.x; p < H * DZ; p += blockDim.x)
        sw.w1[p % DZ][p / DZ] = bf16_to_f32(w[OW1 + p]);
    for (int f = threadIdx.x; f < H; f += blockDim.x) {
        sw.b1[f] = bf16_to_f32(w[OB1 + f]);
        sw.b2[f] = bf16_to_f32(w[OB2 + f]);
        sw.b3[f] = bf16_to_f32(w[OB3 + f]);
        sw.w4[f] = bf16_to_f32(w[OW4 + f]);
    }
    __syncthreads();
}

// Several sample tiles per workgroup (inference): NS tiles of 16 samples share
// every weight fragment a wave loads, so each fragment feeds 2 NS MFMAs; the
// column operands of the NS tiles sit side by side in LDS.
template <int NS>
using OperandsN = bf16x8[2][NS][8][2][64];

template <int NS>
__device__ inline void mf_product_n(const Frags &a, const float (*x)[VPL], float (*y)[VPL], OperandsN<NS> &op, int slot)
{
    static_assert(RT == 2, "one published chunk per wave");
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        bf16x8 hi, lo;
        split8(x[s], hi, lo);
        op[slot][s][w][0][l] = hi;
        op[slot][s][w][1][l] = lo;
    }
    __syncthreads();
    f32x4 acc[NS][RT];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int t = 0; t < RT; ++t)
            acc[s][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kc = 0; kc < 8; ++kc) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const bf16x8 bh = op[slot][s][kc][0][l], bl = op[slot][s][kc][1][l];
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                acc[s][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kc][t], bl, acc[s][t], 0, 0, 0);
                acc[s][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kc][t], bh, acc[s][t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                y[s][4 * t + r] = acc[s][t][r];
}

// sample_sums for NS tiles: sample 16 s + l % 16 of the workgroup
template <int NS>
__device__ inline void sample_sums_n(float (*v)[NRED], float (*red)[16 * NS][NRED])
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int k = 0; k < NRED; ++k)
            v[s][k] = group_sum(v[s][k]);
    if (l < 16)
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int k = 0; k < NRED; ++k)
                red[w][16 * s + l][k] = v[s][k];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int k = 0; k < NRED; ++k) {
            float t = red[0][16 * s + (l & 15)][k];
#pragma unroll
            for (int ww = 1; ww < NWAVE; ++ww)
                t += red[ww][16 * s + (l & 15)][k];
            v[s][k] = t;
        }
}

// Value and input gradient of 16 NS samples per workgroup of 8 waves.
constexpr int FWD_TILES = 2;
template <int NS>
__global__ __launch_bounds__(64 * NWAVE) void k_mlp_forward_mfma(MfNet net, const float *__restrict__ z, int64_t B,
                                                         float *__restrict__ f_out, float *__restrict__ gz_out)
{
    __shared__ SmallW sw;
    __shared__ OperandsN<NS> op;
    __shared__ float red[NWAVE][16 * NS][NRED];
    __shared__ float4 slope[2][NS][NWAVE][VPL / 4][64];  // GELU slopes of layers 1 and 2, until the reverse pass
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, q = l >> 4;
    int64_t b[NS];
    bool valid[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        b[s] = int64_t(blockIdx.x) * (16 * NS) + 16 * s + (l & 15);
        valid[s] = b[s] < B;
    }
    stage_small(net.w, sw);
    float zi[NS][DZ];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int d = 0; d < DZ; ++d)
            zi[s][d] = valid[s] ? z[b[s] * DZ + d] : 0.0f;
    float v[NS][VPL], y[NS][VPL];
    auto put_slope = [&](int layer, int s, int i4, float x0, float x1, float x2, float x3) {
        slope[layer][s][w][i4][l] = make_float4(x0, x1, x2, x3);
    };
    Frags a;
    load_frags(net.frag[F_W2], a);
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
            const int f = feat(w, q, i);
            float h = sw.b1[f];
#pragma unroll
            for (int d = 0; d < DZ; ++d)
                h = fmaf(sw.w1[d][f], zi[s][d], h);
            v[s][i] = gelu(h);
            y[s][i] = gelu_d1(h);
        }
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int i4 = 0; i4 < VPL / 4; ++i4)
            put_slope(0, s, i4, y[s][4 * i4], y[s][4 * i4 + 1], y[s][4 * i4 + 2], y[s][4 * i4 + 3]);
    mf_product_n<NS>(a, v, y, op, 0);
    load_frags(net.frag[F_W3], a);
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
            const float h = y[s][i] + sw.b2[feat(w, q, i)];
            v[s][i] = gelu(h);
            y[s][i] = gelu_d1(h);
        }
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int i4 = 0; i4 < VPL / 4; ++i4)
            put_slope(1, s, i4, y[s][4 * i4], y[s][4 * i4 + 1], y[s][4 * i4 + 2], y[s][4 * i4 + 3]);
    mf_product_n<NS>(a, v, y, op, 1);
    load_frags(net.frag[F_W3T], a);
    float acc[NS][NRED] = {};
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
            const int f = feat(w, q, i);
            const float h = y[s][i] + sw.b3[f];
            acc[s][0] = fmaf(sw.w4[f], gelu(h), acc[s][0]);
            v[s][i] = sw.w4[f] * gelu_d1(h);
        }
    // input gradient: d2 = s2 (W3^T d3), d1 = s1 (W2^T d2), g = W1^T d1
    mf_product_n<NS>(a, v, y, op, 0);
    load_frags(net.frag[F_W2T], a);
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
            const float4 g = slope[1][s][w][i >> 2][l];
            const float sl[4] = {g.x, g.y, g.z, g.w};
            v[s][i] = y[s][i] * sl[i & 3];
        }
    mf_product_n<NS>(a, v, y, op, 1);
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
            const int f = feat(w, q, i);
            const float4 g = slope[0][s][w][i >> 2][l];
            const float sl[4] = {g.x, g.y, g.z, g.w};
            const float d1 = y[s][i] * sl[i & 3];
#pragma unroll
            for (int d = 0; d < DZ; ++d)
                acc[s][1 + d] = fmaf(sw.w1[d][f], d1, acc[s][1 + d]);
        }
    sample_sums_n<NS>(acc, red);
    if (w == 0 && q == 0)
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (valid[s]) {
                f_out[b[s]] = acc[s][0] + bf16_to_f32(net.w[OB4]);
                if (gz_out)
#pragma unroll
                    for (int d = 0; d < DZ; ++d)
                        gz_out[b[s] * DZ + d] = acc[s][1 + d];
            }
}

// Training pass.  Per-sample vectors of the parameter gradient, feature-major
// for the batch contraction: vec[(v * H + f) * bp + b], bp = batch rounded up
// to 32 (padding samples hold zeros).
struct TrainWs {
    float *vec;    // [12][H][bp]: h1b t1b | h2b t2b a1 u1 | h3b t3b a2 u2 | a3 u3
    float *zr;     // [12][bp]: z (6), r (6)
    float *cf;     // [bp]
    float *loss;   // [bp]
    int64_t bp;
};
constexpr int NV = 12;
enum { V_H1B, V_T1B, V_H2B, V_T2B, V_A1, V_U1, V_H3B, V_T3B, V_A2, V_U2, V_A3, V_U3 };

__device__ inline void put_vec(const TrainWs &ws, int vi, int64_t b, int w, int q, bool valid, const float x[VPL])
{
#pragma unroll
    for (int i = 0; i < VPL; ++i)
        ws.vec[(int64_t(vi) * H + feat(w, q, i)) * ws.bp + b] = valid ? x[i] : 0.0f;
}

// GELU of a layer's pre-activation h = y + bias: activation, slope and curvature
__device__ inline void layer_primal(const float *bias, int w, int q, const float y[VPL], float a[VPL], float s[VPL],
                                    float c[VPL])
{
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        const float h = y[i] + bias[feat(w, q, i)];
        a[i] = gelu(h);
        s[i] = gelu_d1(h);
        c[i] = gelu_d2(h);
    }
}

// Adjoints of one layer's pre-activation from those of its activation (ab) and
// of the activation's tangent (ub): h_b = ab s + ub c t and t_b = ub s, with
// the GELU slope s and curvature c and the tangent t of the layer.
__device__ inline void layer_adjoint(float ab[VPL], float ub[VPL], const float s[VPL], const float c[VPL],
                                     const float t[VPL])
{
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        const float hb = ab[i] * s[i] + ub[i] * c[i] * t[i];
        ub[i] = ub[i] * s[i];
        ab[i] = hb;
    }
}

__global__ __launch_bounds__(64 * NWAVE) void k_mlp_train_mfma(MfNet net, const float *__restrict__ z,
                                                       const float *__restrict__ y, const float *__restrict__ g,
                                                       int64_t B, float lam, TrainWs ws)
{
    __shared__ SmallW sw;
    __shared__ Operands op;
    __shared__ float red[NWAVE][16][NRED];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, q = l >> 4;
    const int64_t b = int64_t(blockIdx.x) * 16 + (l & 15);
    const bool valid = b < B;
    stage_small(net.w, sw);
    float zi[DZ], gt[DZ];
#pragma unroll
    for (int d = 0; d < DZ; ++d) {
        zi[d] = valid ? z[b * DZ + d] : 0.0f;
        gt[d] = valid ? g[b * DZ + d] : 0.0f;
    }
    const float yb = valid ? y[b] : 0.0f;
    float s1[VPL], s2[VPL], s3[VPL], c1[VPL], c2[VPL], c3[VPL], t1[VPL], t2[VPL], t3[VPL];
    float v[VPL], u[VPL], x[VPL];
    Frags a;
    load_frags(net.frag[F_W2], a);
    // primal pass
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        const int f = feat(w, q, i);
        float h = 0.0f;
#pragma unroll
        for (int d = 0; d < DZ; ++d)
            h = fmaf(sw.w1[d][f], zi[d], h);
        x[i] = h;
    }
    layer_primal(sw.b1, w, q, x, v, s1, c1);
    put_vec(ws, V_A1, b, w, q, valid, v);
    mf_product(a, v, x, op, 0);
    load_frags(net.frag[F_W3], a);
    layer_primal(sw.b2, w, q, x, v, s2, c2);
    put_vec(ws, V_A2, b, w, q, valid, v);
    mf_product(a, v, x, op, 1);
    load_frags(net.frag[F_W3T], a);
    layer_primal(sw.b3, w, q, x, v, s3, c3);
    put_vec(ws, V_A3, b, w, q, valid, v);
    float acc[NRED] = {};
#pragma unroll
    for (int i = 0; i < VPL; ++i)
        acc[0] = fmaf(sw.w4[feat(w, q, i)], v[i], acc[0]);
    // input gradient
#pragma unroll
    for (int i = 0; i < VPL; ++i)
        v[i] = sw.w4[feat(w, q, i)] * s3[i];
    mf_product(a, v, x, op, 0);
    load_frags(net.frag[F_W2T], a);
#pragma unroll
    for (int i = 0; i < VPL; ++i)
        v[i] = x[i] * s2[i];
    mf_product(a, v, x, op, 1);
    load_frags(net.frag[F_W2], a);
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        const int f = feat(w, q, i);
        const float d1 = s1[i] * x[i];
#pragma unroll
        for (int d = 0; d < DZ; ++d)
            acc[1 + d] = fmaf(sw.w1[d][f], d1, acc[1 + d]);
    }
    sample_sums(acc, red);
    float rr[DZ];
#pragma unroll
    for (int d = 0; d < DZ; ++d)
        rr[d] = valid ? acc[1 + d] - gt[d] : 0.0f;
    const float e = valid ? acc[0] + bf16_to_f32(net.w[OB4]) - yb : 0.0f;
    // tangent pass along r
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        const int f = feat(w, q, i);
        float t = 0.0f;
#pragma unroll
        for (int d = 0; d < DZ; ++d)
            t = fmaf(sw.w1[d][f], rr[d], t);
        t1[i] = t;
        v[i] = s1[i] * t;
    }
    put_vec(ws, V_U1, b, w, q, valid, v);
    mf_product(a, v, t2, op, 0);
    load_frags(net.frag[F_W3], a);
#pragma unroll
    for (int i = 0; i < VPL; ++i)
        v[i] = s2[i] * t2[i];
    put_vec(ws, V_U2, b, w, q, valid, v);
    mf_product(a, v, t3, op, 1);
    load_frags(net.frag[F_W3T], a);
#pragma unroll
    for (int i = 0; i < VPL; ++i)
        v[i] = s3[i] * t3[i];
    put_vec(ws, V_U3, b, w, q, valid, v);
    // reverse pass of J = cf f + ct D_r f (v: adjoint of the activation, u: of its tangent)
    const float cf = 2.0f * e / float(B);
    const float ct = 2.0f * lam / float(B);
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        const float w4 = sw.w4[feat(w, q, i)];
        v[i] = cf * w4;
        u[i] = ct * w4;
    }
    layer_adjoint(v, u, s3, c3, t3);
    put_vec(ws, V_H3B, b, w, q, valid, v);
    put_vec(ws, V_T3B, b, w, q, valid, u);
    mf_product(a, v, x, op, 0);
    mf_product(a, u, v, op, 1);
    load_frags(net.frag[F_W2T], a);
    layer_adjoint(x, v, s2, c2, t2);
    put_vec(ws, V_H2B, b, w, q, valid, x);
    put_vec(ws, V_T2B, b, w, q, valid, v);
    mf_product(a, x, u, op, 0);
    mf_product(a, v, x, op, 1);
    layer_adjoint(u, x, s1, c1, t1);
    put_vec(ws, V_H1B, b, w, q, valid, u);
    put_vec(ws, V_T1B, b, w, q, valid, x);
    if (w == 0 && q == 0) {
        float rn = 0.0f;
#pragma unroll
        for (int d = 0; d < DZ; ++d) {
            ws.zr[d * ws.bp + b] = zi[d];
            ws.zr[(DZ + d) * ws.bp + b] = rr[d];
            rn = fmaf(rr[d], rr[d], rn);
        }
        ws.cf[b] = cf;
        ws.loss[b] = valid ? e * e + lam * rn : 0.0f;
    }
}

// Parameter gradient, contracted over the padded batch, by workgroups of 4 waves:
//   workgroups 0..511: a 16 x 16 tile of dW2 (0..255) or dW3 (256..511) on the
//     matrix cores, sum_b h_b[j] a_b[k] + t_b[j] u_b[k], each FP32 factor split
//     into hi + lo BF16 parts and three products taken (hi hi, hi lo, lo hi;
//     lo lo is below 2^-16 of the product).  The (term, 32-sample chunk) items
//     are dealt to the 4 waves in turn, each wave's partial tile is added in
//     item order, and the 4 partials in wave order;
//   workgroups 512..: 4 rows each (one per wave) of W1 (6 values), b1, b2, b3,
//     w4, then b4 with the loss: lanes take samples lane + 64 i in order, then a
//     fixed butterfly over the wave.
constexpr int WG_TILES = 512;
constexpr int WG_ROWS = 5 * H + 1;
constexpr int WGRAD_WAVES = 4;

// lane group q's 8 values of a 32-sample chunk in the fragment k order
__device__ inline void load8(const float *p, int q, float4 &x0, float4 &x1)
{
    x0 = *reinterpret_cast<const float4 *>(p + 4 * q);
    x1 = *reinterpret_cast<const float4 *>(p + 16 + 4 * q);
}

__device__ inline void split_pair(const float4 &x0, const float4 &x1, bf16x8 &hi, bf16x8 &lo)
{
    const float x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
    split8(x, hi, lo);
}

__global__ __launch_bounds__(64 * WGRAD_WAVES) void k_mlp_wgrad_mfma(TrainWs ws, int64_t B, float ct,
                                                                    float *__restrict__ grad,
                                                                    float *__restrict__ loss_out)
{
    __shared__ f32x4 part[WGRAD_WAVES][64];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, q = l >> 4, lm = l & 15;
    const int64_t bp = ws.bp;
    const int wg = blockIdx.x;
    if (wg < WG_TILES) {
        const int mat = wg >> 8, jt = (wg >> 4) & 15, kt = wg & 15;
        const int vh = mat ? V_H3B : V_H2B, vt = mat ? V_T3B : V_T2B, va = mat ? V_A2 : V_A1, vu = mat ? V_U2 : V_U1;
        const int j = 16 * jt + lm, k = 16 * kt + lm;
        const int nchunk = int(bp >> 5), nitems = 2 * nchunk;
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        // this wave's items i = w, w + 4, ...: four at a time, all their loads issued before the products
        for (int i0 = w; i0 < nitems; i0 += 4 * WGRAD_WAVES) {
            float4 xa[4][2], xb[4][2];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + WGRAD_WAVES * u;
                if (i < nitems) {
                    const int term = (i >= nchunk) ? 1 : 0;
                    const int64_t c0 = 32 * int64_t(i - term * nchunk);
                    load8(ws.vec + (int64_t(term ? vt : vh) * H + j) * bp + c0, q, xa[u][0], xa[u][1]);
                    load8(ws.vec + (int64_t(term ? vu : va) * H + k) * bp + c0, q, xb[u][0], xb[u][1]);
                } else {
                    xa[u][0] = xa[u][1] = xb[u][0] = xb[u][1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (i0 + WGRAD_WAVES * u < nitems) {
                    bf16x8 ah, al, bh, bl;
                    split_pair(xa[u][0], xa[u][1], ah, al);
                    split_pair(xb[u][0], xb[u][1], bh, bl);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
                }
            }
        }
        part[w][l] = acc;
        __syncthreads();
        if (w == 0) {
            f32x4 t = part[0][l];
#pragma unroll
            for (int ww = 1; ww < WGRAD_WAVES; ++ww)
                t += part[ww][l];
            const int64_t base = mat ? OW3 : OW2;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                grad[base + int64_t(16 * jt + 4 * q + r) * H + k] = t[r];
        }
        return;
    }
    const int row = (wg - WG_TILES) * WGRAD_WAVES + w;
    if (row >= WG_ROWS)
        return;
    if (row < H) {  // W1[j][:]: sum_b h1b[j] z_b + t1b[j] r_b
        const float *hb = ws.vec + (int64_t(V_H1B) * H + row) * bp;
        const float *tb = ws.vec + (int64_t(V_T1B) * H + row) * bp;
        float acc[DZ] = {};
#pragma unroll 4
        for (int64_t b = l; b < bp; b += 64) {
            const float h = hb[b], t = tb[b];
#pragma unroll
            for (int d = 0; d < DZ; ++d) {
                acc[d] = fmaf(h, ws.zr[d * bp + b], acc[d]);
                acc[d] = fmaf(t, ws.zr[(DZ + d) * bp + b], acc[d]);
            }
        }
#pragma unroll
        for (int d = 0; d < DZ; ++d)
            acc[d] = wave_sum(acc[d]);
        if (l == 0)
#pragma unroll
            for (int d = 0; d < DZ; ++d)
                grad[OW1 + row * DZ + d] = acc[d];
    } else if (row < 4 * H) {  // b1, b2, b3: sum_b h_b[j]
        const int layer = row / H - 1, j = row % H;
        const int vi = layer == 0 ? V_H1B : layer == 1 ? V_H2B : V_H3B;
        const int64_t off = layer == 0 ? OB1 : layer == 1 ? OB2 : OB3;
        const float *hb = ws.vec + (int64_t(vi) * H + j) * bp;
        float acc = 0.0f;
#pragma unroll 4
        for (int64_t b = l; b < bp; b += 64)
            acc += hb[b];
        acc = wave_sum(acc);
        if (l == 0)
            grad[off + j] = acc;
    } else if (row < 5 * H) {  // w4[j]: sum_b cf_b a3_b[j] + ct u3_b[j]
        const int j = row - 4 * H;
        const float *a3 = ws.vec + (int64_t(V_A3) * H + j) * bp;
        const float *u3 = ws.vec + (int64_t(V_U3) * H + j) * bp;
        float acc = 0.0f;
#pragma unroll 4
        for (int64_t b = l; b < bp; b += 64) {
            acc = fmaf(ws.cf[b], a3[b], acc);
            acc = fmaf(ct, u3[b], acc);
        }
        acc = wave_sum(acc);
        if (l == 0)
            grad[OW4 + j] = acc;
    } else {  // b4 and the loss
        float acc = 0.0f, ls = 0.0f;
#pragma unroll 4
        for (int64_t b = l; b < bp; b += 64) {
            acc += ws.cf[b];
            ls += ws.loss[b];
        }
        acc = wave_sum(acc);
        ls = wave_sum(ls);
        if (l == 0) {
            grad[OB4] = acc;
            loss_out[0] = ls / float(B);
        }
    }
}

// The BF16 working copies of a parameter: flat, transposed (W2, W3) and operand fragments.
struct Copies {
    uint16_t *wb, *wt2, *wt3, *frag[4];
};

Copies copies_of(void *state)
{
    const StateLayout L = state_layout();
    char *b = static_cast<char *>(state);
    Copies c;
    c.wb = reinterpret_cast<uint16_t *>(b + L.wb);
    c.wt2 = reinterpret_cast<uint16_t *>(b + L.wt2);
    c.wt3 = reinterpret_cast<uint16_t *>(b + L.wt3);
    for (int i = 0; i < 4; ++i)
        c.frag[i] = reinterpret_cast<uint16_t *>(b + L.frag[i]);
    return c;
}

__device__ inline void write_copies(const Copies &c, int64_t p, uint16_t h)
{
    c.wb[p] = h;
    if (p >= OW2 && p < OB2) {
        const int j = int((p - OW2) / H), k = int((p - OW2) % H);
        c.wt2[k * H + j] = h;
        c.frag[F_W2][frag_index(j, k)] = h;
        c.frag[F_W2T][frag_index(k, j)] = h;
    } else if (p >= OW3 && p < OB3) {
        const int j = int((p - OW3) / H), k = int((p - OW3) % H);
        c.wt3[k * H + j] = h;
        c.frag[F_W3][frag_index(j, k)] = h;
        c.frag[F_W3T][frag_index(k, j)] = h;
    }
}

// BF16 working copies from the FP32 master.
__global__ __launch_bounds__(256) void k_mlp_refresh(const float *__restrict__ master, Copies c)
{
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= P)
        return;
    write_copies(c, p, f32_to_bf16(master[p]));
}

__global__ __launch_bounds__(256) void k_mlp_load(const float *__restrict__ src, float *__restrict__ master,
                                                  float *__restrict__ m, float *__restrict__ v)
{
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= P)
        return;
    master[p] = src[p];
    m[p] = 0.0f;
    v[p] = 0.0f;
}

__global__ __launch_bounds__(256) void k_mlp_copy(const float *__restrict__ src, float *__restrict__ dst)
{
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < P)
        dst[p] = src[p];
}

// Adam (Kingma and Ba, 2015) with bias correction on the FP32 master weights,
// followed by the BF16 working copies of the updated value.
__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ master, float *__restrict__ m,
                                                  float *__restrict__ v, const float *__restrict__ grad, float lr,
                                                  float beta1, float beta2, float eps, float c1, float c2, Copies c)
{
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= P)
        return;
    const float gr = grad[p];
    const float mm = beta1 * m[p] + (1.0f - beta1) * gr;
    const float vv = beta2 * v[p] + (1.0f - beta2) * gr * gr;
    m[p] = mm;
    v[p] = vv;
    const float th = master[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    master[p] = th;
    write_copies(c, p, f32_to_bf16(th));
}

struct TrainLayout {
    int64_t bp;
    size_t vec, zr, cf, loss, grad, total;
};

TrainLayout train_layout(int64_t B)
{
    TrainLayout t;
    t.bp = (B + 31) / 32 * 32;
    const size_t bp = size_t(t.bp);
    size_t off = 0;
    t.vec = off;
    off = align256(off + sizeof(float) * bp * NV * H);
    t.zr = off;
    off = align256(off + sizeof(float) * bp * 12);
    t.cf = off;
    off = align256(off + sizeof(float) * bp);
    t.loss = off;
    off = align256(off + sizeof(float) * bp);
    t.grad = off;
    off = align256(off + sizeof(float) * P);
    t.total = off;
    return t;
}

// Batches up to this size take the one-sample kernel (the arithmetic of k_mlp_leapfrog).
constexpr int64_t SMALL_BATCH = 8;
constexpr int64_t MAX_BATCH = int64_t(1) << 22;

bool aligned256(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

}  // namespace
}  // namespace hawkes

using namespace hawkes;

extern "C" size_t hawkes_mlp_state_bytes(void) { return state_layout().total; }

extern "C" size_t hawkes_mlp_workspace_bytes(int64_t batch)
{
    if (batch < 1 || batch > MAX_BATCH)
        return 0;
    return train_layout(batch).total;
}

extern "C" int hawkes_mlp_load(void *d_state, const float *d_params, void *stream)
{
    if (!d_state || !d_params || !aligned256(d_state)) {
        set_error("mlp_load: null or misaligned pointer");
        return HAWKES_EINVAL;
    }
    const StateLayout L = state_layout();
    char *s = static_cast<char *>(d_state);
    const unsigned blocks = unsigned((P + 255) / 256);
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_mlp_load, dim3(blocks), dim3(256), 0, st, d_params, reinterpret_cast<float *>(s + L.master),
                       reinterpret_cast<float *>(s + L.m), reinterpret_cast<float *>(s + L.v));
    hipLaunchKernelGGL(k_mlp_refresh, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const float *>(s + L.master),
                       copies_of(d_state));
    return check_launch("mlp_load");
}

extern "C" int hawkes_mlp_store(const void *d_state, float *d_params, void *stream)
{
    if (!d_state || !d_params || !aligned256(d_state)) {
        set_error("mlp_store: null or misaligned pointer");
        return HAWKES_EINVAL;
    }
    const StateLayout L = state_layout();
    hipLaunchKernelGGL(k_mlp_copy, dim3(unsigned((P + 255) / 256)), dim3(256), 0, as_stream(stream),
                       reinterpret_cast<const float *>(static_cast<const char *>(d_state) + L.master), d_params);
    return check_launch("mlp_store");
}

extern "C" int hawkes_mlp_forward(const void *d_state, const float *d_z, int64_t batch, float *d_f, float *d_gz,
                                  void *stream)
{
    if (!d_state || !d_z || !d_f || !aligned256(d_state) || batch < 1 || batch > MAX_BATCH) {
        set_error("mlp_forward: invalid arguments (batch %lld)", (long long)batch);
        return HAWKES_EINVAL;
    }
    if (batch <= SMALL_BATCH)
        hipLaunchKernelGGL(k_mlp_forward, dim3(unsigned(batch)), dim3(H), 0, as_stream(stream), net_of(d_state), d_z,
                           batch, d_f, d_gz);
    else
        hipLaunchKernelGGL(k_mlp_forward_mfma<FWD_TILES>, dim3(unsigned((batch + 16 * FWD_TILES - 1) / (16 * FWD_TILES))),
                           dim3(64 * NWAVE), 0, as_stream(stream),
                           mfnet_of(d_state), d_z, batch, d_f, d_gz);
    return check_launch("mlp_forward");
}

extern "C" int hawkes_mlp_leapfrog(const void *d_state, hawkes_mlp_leapfrog_io *d_io, int64_t n_steps, void *stream)
{
    if (!d_state || !d_io || !aligned256(d_state) || n_steps < 1 || n_steps > 4096) {
        set_error("mlp_leapfrog: invalid arguments (n_steps %lld)", (long long)n_steps);
        return HAWKES_EINVAL;
    }
    hipLaunchKernelGGL(k_mlp_leapfrog, dim3(1), dim3(H), 0, as_stream(stream), net_of(d_state), d_io,
                       int(n_steps));
    return check_launch("mlp_leapfrog");
}

extern "C" int hawkes_mlp_loss_grad(const void *d_state, const float *d_z, const float *d_y, const float *d_g,
                                    int64_t batch, float lambda_g, void *ws, size_t ws_bytes, float *d_loss,
                                    float *d_grad, void *stream)
{
    if (!d_state || !d_z || !d_y || !d_g || !d_loss || !aligned256(d_state) || batch < 1 || batch > MAX_BATCH ||
        !(lambda_g >= 0.0f)) {
        set_error("mlp_loss_grad: invalid arguments (batch %lld)", (long long)batch);
        return HAWKES_EINVAL;
    }
    const TrainLayout T = train_layout(batch);
    if (!ws || !aligned256(ws) || ws_bytes < T.total) {
        set_error("mlp_loss_grad: workspace of %zu bytes, need %zu (256-byte aligned)", ws_bytes, T.total);
        return HAWKES_EWORKSPACE;
    }
    char *w = static_cast<char *>(ws);
    TrainWs t{reinterpret_cast<float *>(w + T.vec), reinterpret_cast<float *>(w + T.zr),
              reinterpret_cast<float *>(w + T.cf), reinterpret_cast<float *>(w + T.loss), T.bp};
    float *grad = d_grad ? d_grad : reinterpret_cast<float *>(w + T.grad);
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_mlp_train_mfma, dim3(unsigned(T.bp / 16)), dim3(64 * NWAVE), 0, st, mfnet_of(d_state), d_z, d_y, d_g,
                       batch, lambda_g, t);
    hipLaunchKernelGGL(k_mlp_wgrad_mfma, dim3(unsigned(WG_TILES + (WG_ROWS + WGRAD_WAVES - 1) / WGRAD_WAVES)),
                       dim3(64 * WGRAD_WAVES), 0, st, t, batch,
                       2.0f * lambda_g / float(batch), grad, d_loss);
    return check_launch("mlp_loss_grad");
}

extern "C" int hawkes_mlp_adam_step(void *d_state, const float *d_grad, int64_t step, float lr, float beta1,
                                    float beta2, float eps, void *stream)
{
    if (!d_state || !d_grad || !aligned256(d_state) || step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f)) {
        set_error("mlp_adam_step: invalid arguments");
        return HAWKES_EINVAL;
    }
    const StateLayout L = state_layout();
    char *s = static_cast<char *>(d_state);
    const float c1 = float(1.0 - std::pow(double(beta1), double(step)));
    const float c2 = float(1.0 - std::pow(double(beta2), double(step)));
    const unsigned blocks = unsigned((P + 255) / 256);
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_mlp_adam, dim3(blocks), dim3(256), 0, st, reinterpret_cast<float *>(s + L.master),
                       reinterpret_cast<float *>(s + L.m), reinterpret_cast<float *>(s + L.v), d_grad, lr, beta1, beta2,
                       eps, c1, c2, copies_of(d_state));
    return check_launch("mlp_adam_step");
}
