// hawkes_mlp.hip -- the BF16 surrogate network of the log-likelihood on gfx950.
//
// Network 6 -> 256 -> 256 -> 256 -> 1 with GELU activations (x Phi(x)):
//   h1 = W1 z + b1, a1 = gelu(h1), h2 = W2 a1 + b2, a2 = gelu(h2),
//   h3 = W3 a2 + b3, a3 = gelu(h3), f = w4 . a3 + b4.
// Flat parameter layout (133,633 values): W1 (256x6, out x in), b1, W2
// (256x256), b2, W3 (256x256), b3, w4 (256), b4.
//
// The state buffer holds FP32 master weights, the two Adam moment vectors,
// and BF16 working copies: the flat vector in its own layout plus W2 and W3
// transposed (in x out), so that every matrix-vector product of the forward
// and backward passes reads weights coalesced across the 256 lanes of a
// workgroup.  All products accumulate in FP32.
//
// Inference: value and input gradient per sample (k_mlp_forward), or a whole
// leapfrog trajectory on the surrogate posterior in one workgroup
// (k_mlp_leapfrog, the stage-1 proposal of delayed-acceptance HMC).
//
// Training loss (value + gradient matching):
//   L = (1/B) sum_b (f(z_b) - y_b)^2 + lambda |grad_z f(z_b) - g_b|^2.
// Its parameter gradient uses d/dtheta [r . grad_z f] = d/dtheta [D_r f] for
// r = grad_z f - g held fixed: per sample a primal pass, the reverse pass for
// grad_z f, a forward tangent pass along r, and one reverse pass through the
// primal and tangent computations; per-sample adjoint vectors are then
// contracted over the batch in a fixed order (deterministic).

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
    size_t master, m, v, wb, wt2, wt3, total;
};

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

// Per-sample vectors of the Sobolev-loss gradient (see file header), 12 x 256
// floats per sample plus z, r (6 each), cf and the sample loss.
struct TrainWs {
    float *vec;     // [B][12][H]: h1b t1b | h2b t2b a1 u1 | h3b t3b a2 u2 | a3 u3
    float *zr;      // [B][12]: z, r
    float *cf;      // [B]
    float *loss;    // [B]
};
constexpr int NV = 12;
enum { V_H1B, V_T1B, V_H2B, V_T2B, V_A1, V_U1, V_H3B, V_T3B, V_A2, V_U2, V_A3, V_U3 };

__global__ __launch_bounds__(H) void k_mlp_train_sample(Net net, const float *__restrict__ z,
                                                        const float *__restrict__ y, const float *__restrict__ g,
                                                        int64_t B, float lam, TrainWs ws)
{
    __shared__ float sz[DZ], sr[DZ], v1[H], v2[H], red[NS7][H];
    const int j = threadIdx.x;
    const int64_t b = blockIdx.x;
    const uint16_t *w = net.w;
    float *vec = ws.vec + b * NV * H;
    if (j < DZ)
        sz[j] = z[b * DZ + j];
    __syncthreads();
    // primal pass
    float h1 = bf16_to_f32(w[OB1 + j]);
#pragma unroll
    for (int i = 0; i < DZ; ++i)
        h1 = fmaf(bf16_to_f32(w[OW1 + j * DZ + i]), sz[i], h1);
    const float a1 = gelu(h1), s1 = gelu_d1(h1);
    v1[j] = a1;
    __syncthreads();
    const float h2 = bf16_to_f32(w[OB2 + j]) + matvec_kmajor(net.wt2, v1, j);
    const float a2 = gelu(h2), s2 = gelu_d1(h2);
    v2[j] = a2;
    __syncthreads();
    const float h3 = bf16_to_f32(w[OB3 + j]) + matvec_kmajor(net.wt3, v2, j);
    const float a3 = gelu(h3), s3 = gelu_d1(h3);
    const float w4 = bf16_to_f32(w[OW4 + j]);
    const float vf = w4 * a3;  // summed with the input gradient below
    // input gradient
    v1[j] = w4 * s3;
    __syncthreads();
    const float d2 = s2 * matvec_kmajor(w + OW3, v1, j);
    v2[j] = d2;
    __syncthreads();
    const float d1 = s1 * matvec_kmajor(w + OW2, v2, j);
    float v7[NS7], s7[NS7], rr[DZ];
    v7[0] = vf;
#pragma unroll
    for (int i = 0; i < DZ; ++i)
        v7[1 + i] = bf16_to_f32(w[OW1 + j * DZ + i]) * d1;
    block_sum7(v7, red, s7);
    const float f = s7[0] + bf16_to_f32(w[OB4]);
#pragma unroll
    for (int i = 0; i < DZ; ++i)
        rr[i] = s7[1 + i] - g[b * DZ + i];
    const float e = f - y[b];
    if (j < DZ)
        sr[j] = rr[j];
    __syncthreads();
    // tangent pass along r
    float t1 = 0.0f;
#pragma unroll
    for (int i = 0; i < DZ; ++i)
        t1 = fmaf(bf16_to_f32(w[OW1 + j * DZ + i]), sr[i], t1);
    const float u1 = s1 * t1;
    v1[j] = u1;
    __syncthreads();
    const float t2 = matvec_kmajor(net.wt2, v1, j);
    const float u2 = s2 * t2;
    __syncthreads();
    v2[j] = u2;
    __syncthreads();
    const float t3 = matvec_kmajor(net.wt3, v2, j);
    const float u3 = s3 * t3;
    // reverse pass of J = cf f + ct D_r f
    const float cf = 2.0f * e / float(B);
    const float ct = 2.0f * lam / float(B);
    const float a3b = cf * w4, u3b = ct * w4;
    const float t3b = u3b * s3;
    const float h3b = a3b * s3 + u3b * gelu_d2(h3) * t3;
    __syncthreads();
    v1[j] = h3b;
    v2[j] = t3b;
    __syncthreads();
    const float a2b = matvec_kmajor(w + OW3, v1, j);
    const float u2b = matvec_kmajor(w + OW3, v2, j);
    const float t2b = u2b * s2;
    const float h2b = a2b * s2 + u2b * gelu_d2(h2) * t2;
    __syncthreads();
    v1[j] = h2b;
    v2[j] = t2b;
    __syncthreads();
    const float a1b = matvec_kmajor(w + OW2, v1, j);
    const float u1b = matvec_kmajor(w + OW2, v2, j);
    const float t1b = u1b * s1;
    const float h1b = a1b * s1 + u1b * gelu_d2(h1) * t1;
    vec[V_H1B * H + j] = h1b;
    vec[V_T1B * H + j] = t1b;
    vec[V_H2B * H + j] = h2b;
    vec[V_T2B * H + j] = t2b;
    vec[V_A1 * H + j] = a1;
    vec[V_U1 * H + j] = u1;
    vec[V_H3B * H + j] = h3b;
    vec[V_T3B * H + j] = t3b;
    vec[V_A2 * H + j] = a2;
    vec[V_U2 * H + j] = u2;
    vec[V_A3 * H + j] = a3;
    vec[V_U3 * H + j] = u3;
    if (j < DZ) {
        ws.zr[b * 12 + j] = sz[j];
        ws.zr[b * 12 + DZ + j] = sr[j];
    }
    if (j == 0) {
        float rn = 0.0f;
        for (int i = 0; i < DZ; ++i)
            rn = fmaf(rr[i], rr[i], rn);
        ws.cf[b] = cf;
        ws.loss[b] = e * e + lam * rn;
    }
}

// Parameter gradient: contractions of the per-sample vectors over the batch,
// one thread per parameter, samples in index order.
__global__ __launch_bounds__(256) void k_mlp_wgrad(TrainWs ws, int64_t B, float ct, float *__restrict__ grad)
{
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= P)
        return;
    float acc = 0.0f;
    if (p < OB1) {  // W1[j][i]
        const int jj = int(p / DZ), i = int(p % DZ);
        for (int64_t b = 0; b < B; ++b) {
            const float *vec = ws.vec + b * NV * H;
            acc = fmaf(vec[V_H1B * H + jj], ws.zr[b * 12 + i], acc);
            acc = fmaf(vec[V_T1B * H + jj], ws.zr[b * 12 + DZ + i], acc);
        }
    } else if (p < OW2) {
        const int jj = int(p - OB1);
        for (int64_t b = 0; b < B; ++b)
            acc += ws.vec[b * NV * H + V_H1B * H + jj];
    } else if (p < OB2) {  // W2[j][k]
        const int jj = int((p - OW2) / H), k = int((p - OW2) % H);
        for (int64_t b = 0; b < B; ++b) {
            const float *vec = ws.vec + b * NV * H;
            acc = fmaf(vec[V_H2B * H + jj], vec[V_A1 * H + k], acc);
            acc = fmaf(vec[V_T2B * H + jj], vec[V_U1 * H + k], acc);
        }
    } else if (p < OW3) {
        const int jj = int(p - OB2);
        for (int64_t b = 0; b < B; ++b)
            acc += ws.vec[b * NV * H + V_H2B * H + jj];
    } else if (p < OB3) {  // W3[j][k]
        const int jj = int((p - OW3) / H), k = int((p - OW3) % H);
        for (int64_t b = 0; b < B; ++b) {
            const float *vec = ws.vec + b * NV * H;
            acc = fmaf(vec[V_H3B * H + jj], vec[V_A2 * H + k], acc);
            acc = fmaf(vec[V_T3B * H + jj], vec[V_U2 * H + k], acc);
        }
    } else if (p < OW4) {
        const int jj = int(p - OB3);
        for (int64_t b = 0; b < B; ++b)
            acc += ws.vec[b * NV * H + V_H3B * H + jj];
    } else if (p < OB4) {  // w4[j]
        const int jj = int(p - OW4);
        for (int64_t b = 0; b < B; ++b) {
            const float *vec = ws.vec + b * NV * H;
            acc = fmaf(ws.cf[b], vec[V_A3 * H + jj], acc);
            acc = fmaf(ct, vec[V_U3 * H + jj], acc);
        }
    } else {
        for (int64_t b = 0; b < B; ++b)
            acc += ws.cf[b];
    }
    grad[p] = acc;
}

__global__ __launch_bounds__(256) void k_mlp_loss_reduce(const float *__restrict__ loss, int64_t B, float *out)
{
    __shared__ float red[256];
    const int j = threadIdx.x;
    float s = 0.0f;
    for (int64_t b = j; b < B; b += 256)
        s += loss[b];
    red[j] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (j < w)
            red[j] += red[j + w];
        __syncthreads();
    }
    if (j == 0)
        out[0] = red[0] / float(B);
}

// BF16 working copies (flat and transposed W2, W3) from the FP32 master.
__global__ __launch_bounds__(256) void k_mlp_refresh(const float *__restrict__ master, uint16_t *__restrict__ wb,
                                                     uint16_t *__restrict__ wt2, uint16_t *__restrict__ wt3)
{
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= P)
        return;
    const uint16_t h = f32_to_bf16(master[p]);
    wb[p] = h;
    if (p >= OW2 && p < OB2) {
        const int64_t q = p - OW2;
        wt2[(q % H) * H + q / H] = h;
    } else if (p >= OW3 && p < OB3) {
        const int64_t q = p - OW3;
        wt3[(q % H) * H + q / H] = h;
    }
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

// Adam (Kingma and Ba, 2015) with bias correction on the FP32 master weights.
__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ master, float *__restrict__ m,
                                                  float *__restrict__ v, const float *__restrict__ grad, float lr,
                                                  float beta1, float beta2, float eps, float c1, float c2)
{
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= P)
        return;
    const float gr = grad[p];
    const float mm = beta1 * m[p] + (1.0f - beta1) * gr;
    const float vv = beta2 * v[p] + (1.0f - beta2) * gr * gr;
    m[p] = mm;
    v[p] = vv;
    master[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

struct TrainLayout {
    size_t vec, zr, cf, loss, grad, total;
};

TrainLayout train_layout(int64_t B)
{
    TrainLayout t;
    size_t off = 0;
    t.vec = off;
    off = align256(off + sizeof(float) * size_t(B) * NV * H);
    t.zr = off;
    off = align256(off + sizeof(float) * size_t(B) * 12);
    t.cf = off;
    off = align256(off + sizeof(float) * size_t(B));
    t.loss = off;
    off = align256(off + sizeof(float) * size_t(B));
    t.grad = off;
    off = align256(off + sizeof(float) * P);
    t.total = off;
    return t;
}

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
                       reinterpret_cast<uint16_t *>(s + L.wb), reinterpret_cast<uint16_t *>(s + L.wt2),
                       reinterpret_cast<uint16_t *>(s + L.wt3));
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
    hipLaunchKernelGGL(k_mlp_forward, dim3(unsigned(batch)), dim3(H), 0, as_stream(stream), net_of(d_state), d_z,
                       batch, d_f, d_gz);
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
              reinterpret_cast<float *>(w + T.cf), reinterpret_cast<float *>(w + T.loss)};
    float *grad = d_grad ? d_grad : reinterpret_cast<float *>(w + T.grad);
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_mlp_train_sample, dim3(unsigned(batch)), dim3(H), 0, st, net_of(d_state), d_z, d_y, d_g,
                       batch, lambda_g, t);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(unsigned((P + 255) / 256)), dim3(256), 0, st, t, batch,
                       2.0f * lambda_g / float(batch), grad);
    hipLaunchKernelGGL(k_mlp_loss_reduce, dim3(1), dim3(256), 0, st, t.loss, batch, d_loss);
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
                       eps, c1, c2);
    hipLaunchKernelGGL(k_mlp_refresh, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const float *>(s + L.master),
                       reinterpret_cast<uint16_t *>(s + L.wb), reinterpret_cast<uint16_t *>(s + L.wt2),
                       reinterpret_cast<uint16_t *>(s + L.wt3));
    return check_launch("mlp_adam_step");
}
