/*
 * hawkes_mlp.h -- C ABI of the surrogate network in libhawkes.so.
 *
 * A small network replaces the exact log-likelihood inside the leapfrog
 * steps of Hamiltonian Monte Carlo; the exact GPU likelihood corrects its
 * error in a delayed-acceptance step.  The network maps standardised
 * log-parameters z (6 values) to a standardised log-likelihood:
 *
 *   6 -> 256 -> 256 -> 256 -> 1, GELU activations (GELU(x) = x Phi(x)),
 *   h1 = W1 z + b1, a1 = gelu(h1), h2 = W2 a1 + b2, a2 = gelu(h2),
 *   h3 = W3 a2 + b3, a3 = gelu(h3), f = w4 . a3 + b4.
 *
 * Parameters are one flat FP32 vector of HAWKES_MLP_PARAMS values in the order
 * W1 (256 x 6, row-major, out x in), b1 (256), W2 (256 x 256), b2, W3
 * (256 x 256), b3, w4 (256), b4 (1).  The library keeps them in a state
 * buffer (FP32 master weights, Adam moments, BF16 working copies); every
 * forward and backward product uses the BF16 weights with FP32 accumulation.
 * Batched products run on the matrix cores with each FP32 activation entering
 * as a hi + lo pair of BF16 values (relative error ~2^-17 per activation).
 *
 * Training minimises the value + gradient ("Sobolev") loss over a batch of B
 * tuples (z_b, y_b, g_b):
 *   L = (1/B) sum_b (f(z_b) - y_b)^2 + lambda_g |grad_z f(z_b) - g_b|^2.
 *
 * Conventions as in hawkes.h: device pointers, asynchronous on `stream`,
 * 256-byte aligned state and workspace buffers owned by the caller, no
 * allocation, HAWKES_OK or a negative status.  Calls that share a state or
 * workspace buffer must not overlap.
 */
#ifndef HAWKES_MLP_H
#define HAWKES_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HAWKES_MLP_PARAMS 133633

/* Bytes of the network state buffer. */
size_t hawkes_mlp_state_bytes(void);

/* Bytes of workspace hawkes_mlp_loss_grad needs for a batch of `batch`
 * tuples (0 if batch < 1 or batch > 2^22). */
size_t hawkes_mlp_workspace_bytes(int64_t batch);

/* Initialise the state from FP32 parameters d_params[HAWKES_MLP_PARAMS]
 * (device): master weights, zero Adam moments, BF16 working copies. */
int hawkes_mlp_load(void *d_state, const float *d_params, void *stream);

/* Copy the FP32 master parameters out to d_params[HAWKES_MLP_PARAMS]. */
int hawkes_mlp_store(const void *d_state, float *d_params, void *stream);

/* Value and input gradient for `batch` inputs: d_z[batch][6] ->
 * d_f[batch], d_gz[batch][6] (d_gz may be NULL).  Batches of up to 8 inputs
 * take the one-sample kernel, whose arithmetic is that of
 * hawkes_mlp_leapfrog; larger batches take the matrix cores (a workgroup of
 * 8 waves per two tiles of 16 inputs).  The two agree to ~1e-5 relative, not
 * bitwise. */
int hawkes_mlp_forward(const void *d_state, const float *d_z, int64_t batch, float *d_f, float *d_gz,
                       void *stream);

/* In/out record of hawkes_mlp_leapfrog (device memory, FP64; log-parameters z
 * of dimension 6).  The surrogate log posterior is
 *   s(z) = s_y f((z - m_z) / s_z) + m_y - z.z / (2 prior_var),
 * the network's value f rescaled to a log-likelihood plus independent
 * N(0, prior_var) priors on the z_i. */
typedef struct hawkes_mlp_leapfrog_io {
    double z[6];          /* in: start point; out: end point */
    double p[6];          /* in: momentum at the start; out: at the end */
    double grad[6];       /* in: ds/dz at the start point; out: at the end point */
    double inv_mass[6];   /* diagonal inverse mass matrix */
    double m_z[6], s_z[6]; /* input standardisation (s_z > 0) */
    double m_y, s_y;      /* output scale */
    double prior_var;     /* prior variance of each z_i */
    double eps;           /* step size */
    double s;             /* out: s at the end point; -inf if a step left the finite range */
    double status;        /* out: 1 if every step was finite, else 0 */
} hawkes_mlp_leapfrog_io;

/* A leapfrog trajectory of n_steps steps (1..4096) of H(z, p) = -s(z) +
 * p' M^-1 p / 2 on the surrogate log posterior above, run by one workgroup
 * without returning to the host: the stage-1 proposal of delayed-acceptance
 * HMC (Christen and Fox) on the network that stands in for the exact
 * likelihood.  Half a momentum step, then per step a position step, s and
 * ds/dz from the network (value and input gradient, as hawkes_mlp_forward
 * computes them), and a momentum step (half a step after the last).
 * Position and momentum updates are FP64 in the order
 *   p += (eps / 2) grad;  z += (eps inv_mass) p;  p += eps grad,
 * each product and sum rounded on its own.  A step whose s or gradient is not
 * finite ends the trajectory with s = -inf and status 0. */
int hawkes_mlp_leapfrog(const void *d_state, hawkes_mlp_leapfrog_io *d_io, int64_t n_steps, void *stream);

/* Sobolev loss of a batch (d_z[batch][6], d_y[batch], d_g[batch][6]) into
 * d_loss[1], and its gradient with respect to the flat parameter vector into
 * d_grad[HAWKES_MLP_PARAMS] (if d_grad is NULL, into the workspace).  The
 * gradient is deterministic (every call sums in the same fixed order: matrix
 * core tiles over 32-sample chunks for W2 and W3, per-lane sums then a fixed
 * wave butterfly for the other parameters). */
int hawkes_mlp_loss_grad(const void *d_state, const float *d_z, const float *d_y, const float *d_g,
                         int64_t batch, float lambda_g, void *ws, size_t ws_bytes, float *d_loss,
                         float *d_grad, void *stream);

/* One Adam update (Kingma and Ba 2015, bias-corrected; `step` counts from 1)
 * of the FP32 master weights with gradient d_grad, then a refresh of the
 * BF16 working copies (round to nearest, ties to even). */
int hawkes_mlp_adam_step(void *d_state, const float *d_grad, int64_t step, float lr, float beta1, float beta2,
                         float eps, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HAWKES_MLP_H */
