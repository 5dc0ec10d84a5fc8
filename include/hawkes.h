/*
 * hawkes.h -- C ABI of the MI355X (gfx950) spatiotemporal Hawkes likelihood
 * library (libhawkes.so).
 *
 * The model is the one of Ko, Suchard and Holbrook, "Scaling Hawkes processes
 * to one million COVID-19 cases" (arXiv 2407.11349), Section 2.1: for events
 * (x_n, t_n), n = 1..N, sorted by time,
 *
 *   lambda_n = mu * sum_{m: t_m != t_n} N2(|x_n - x_m|^2; tau_x^2) N1(t_n - t_m; tau_t^2)
 *            + xi * sum_{m: t_m <  t_n} N2(|x_n - x_m|^2; h_m^2) omega exp(-omega (t_n - t_m)),
 *              (with a domain area A > 0 in hawkes_events, N2(.; tau_x^2) becomes 1/A),
 *   h_m      = h0 * s_m      (per-source spatial sd; equation "varying" uses
 *                             s_m = D_m^(-1/2) for the county population density D_m),
 *   Lambda_n = mu [Phi((t_N - t_n)/tau_t) - Phi(-t_n/tau_t)] + xi [1 - exp(-omega (t_N - t_n))]
 *              (the compensator over the time domain (0, t_N] after the R^2 approximation),
 *   l_n      = log(max(lambda_n, 1e-40)) - Lambda_n   (the floor of Section 2.3.1),
 *
 * where N2(r^2; v) is the isotropic bivariate normal density with variance v
 * per axis and N1(d; v) the univariate normal density.  Self pairs and exact
 * time ties are excluded from both sums.  The log-likelihood of rows
 * [row_begin, row_end) is sum_{n in rows} l_n; the full range gives equation
 * "model", and any split of it adds up to the full value (the per-GPU slices
 * of Section 2.3.2).
 *
 * Conventions for every call:
 *  - All array arguments are DEVICE pointers on the current HIP device,
 *    borrowed for the duration of the call; the caller owns them.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    asynchronously on it; outputs are valid after the caller synchronises.
 *  - No call allocates device memory: scratch space comes from the
 *    caller-provided workspace `ws` of hawkes_workspace_bytes() bytes (at
 *    least hawkes_workspace_min_bytes()), 256-byte aligned.  Calls that share a workspace must not overlap; calls
 *    with distinct workspaces are independent (the library keeps no state
 *    between calls other than the calling thread's last-error message and
 *    the static device array of hawkes_loglik_grad_noalloc).
 *  - `opts` (may be NULL) carries per-call tuning and timing; see
 *    hawkes_options.
 *  - Return value: HAWKES_OK (0) or a negative status; no C++ exception
 *    crosses the ABI.  hawkes_last_error() gives a message for the calling
 *    thread's last failure.
 *  - Argument checks done on the host return an error before any work is
 *    enqueued.  Data checks (times sorted, values finite, s > 0) run on the
 *    device: on failure the outputs are set to NaN and the status word in the
 *    workspace records the reason (hawkes_workspace_status).
 */
#ifndef HAWKES_H
#define HAWKES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Model parameters in natural units: mu (-), tau_x (km), tau_t (days), xi (-),
 * h0 (km), omega (1/day).  All must be finite and > 0. */
typedef struct hawkes_theta {
    double mu, tau_x, tau_t, xi, h0, omega;
} hawkes_theta;

/* One event set: n events, all arrays device-resident, length n, FP64.
 * t must be nondecreasing (t_N = t[n-1]); s is the per-event bandwidth scale
 * (> 0): 1 for the paper's model 1, D_n^(-1/2) for its model 2.
 * area selects the background's spatial factor:
 *   0      the isotropic Gaussian N2(|x_n - x_m|^2; tau_x^2) of the formula above;
 *   > 0    the spatially uniform density 1/area (km^2) of the paper's own models
 *          (equation "fixed": mu0 / A(X) times the temporal Gaussian); tau_x then
 *          plays no part and its gradient component is 0.
 * Negative or non-finite area: HAWKES_EINVAL. */
typedef struct hawkes_events {
    int64_t n;
    const double *t;
    const double *x;
    const double *y;
    const double *s;
    double area;
} hawkes_events;

/* Arithmetic of the O(N^2) pair sweep.  FP64: every pair term in FP64.
 * FP32: pair terms in FP32 (pair differences formed in FP64 and rounded once,
 * FP32 partial sums of a few terms folded into FP64 accumulators); the
 * per-event log, the compensator and all reductions stay in FP64.  Over the
 * whole event set (row range [0, n)) the FP32 sweep uses the symmetry of the
 * background term: each term b_nm = b_mn of two events in strictly ordered
 * 512-event blocks is evaluated once and added to both events' sums.
 * FP32_SKIP: the FP32 sweep, leaving out every background term that is
 * exactly zero in FP32 because the scaled time gap alone makes its exponent
 * exceed 160 (|t_n - t_m| > sqrt(2 * 160 / log2(e)) tau_t, about 14.9 tau_t):
 * source tiles that early sweep the triggering terms only (and, for a row
 * range, tiles that late are not visited); source tiles so early that every
 * triggering term is below 2^-160 (max_m s_m^-2 exp(-omega gap) < 2^-160) are
 * not visited at all.  The result equals FP32 up to the summation order of
 * those tiles' triggering terms; the work falls when the time span is long
 * against tau_t and 1/omega.
 * Results are bitwise reproducible for a given event set, theta, precision,
 * row range and options (hawkes_options). */
enum hawkes_precision { HAWKES_FP64 = 0, HAWKES_FP32 = 1, HAWKES_FP32_SKIP = 2 };

enum hawkes_status {
    HAWKES_OK = 0,
    HAWKES_EINVAL = -1,     /* null pointer, n < 1, n too large, bad precision, theta not finite/positive */
    HAWKES_ERANGE = -2,     /* not 0 <= row_begin <= row_end <= n */
    HAWKES_EWORKSPACE = -3, /* workspace null, misaligned or too small (hawkes_workspace_min_bytes) */
    HAWKES_EHIP = -4,       /* a HIP runtime call failed; see hawkes_last_error() */
    HAWKES_EORDER = -5,     /* device check: times not nondecreasing */
    HAWKES_EDATA = -6       /* device check: a non-finite value or s <= 0 */
};

/* Per-call options (all-zero = defaults).
 *   row_workgroups    row sweep (a row range, or symmetric_groups = -1): the
 *                     workgroups (target blocks x source chunks) a call aims
 *                     for; 0 = 32768, else 1..65536.
 *   symmetric_groups  whole-set calls (row range [0, n)): the symmetric
 *                     sweep's number of row groups (and as many column
 *                     groups; one workgroup per pair of groups it needs);
 *                     0 = 384, 1..1024, or -1: whole-set calls take the row
 *                     sweep too.
 *   timing_start, timing_stop
 *                     hipEvent_t handles (both or neither): recorded on the
 *                     call's stream right before the first pair-sweep launch
 *                     and right after the last one (with the fold of its
 *                     partial sums), so that hipEventElapsedTime gives the
 *                     sweep's duration.  The caller creates and owns them.
 * Results do not depend on the options beyond the FP64 summation order of
 * partial sums (symmetric_groups = -1 also changes the order of the FP32
 * background sums), nor on the workspace size.  Values out of range:
 * HAWKES_EINVAL. */
typedef struct hawkes_options {
    int64_t row_workgroups;
    int32_t symmetric_groups;
    int32_t reserved;  /* must be 0 */
    void *timing_start;
    void *timing_stop;
} hawkes_options;

/* Bytes of workspace the likelihood calls need for n events at `precision`
 * (0 if the arguments are invalid): a part linear in n (staged source
 * records, per-row FP64 accumulators and values; about 210 bytes per event
 * at FP32) plus a slot region for the partial sums of the sweep's
 * workgroups.  The sweep runs in passes over as many workgroups as the slot
 * region holds, each pass followed by a fold of its partial sums into the
 * per-row accumulators; the returned size gives the slot region the smaller
 * of 704 MiB and what a single pass needs (at least one workgroup's slot):
 * about 0.94 * 10^9 bytes in all at n = 10^6 (FP32).  A larger workspace means fewer
 * passes and the same results. */
size_t hawkes_workspace_bytes(int64_t n, int precision);

/* The smallest workspace the calls accept for n events at `precision` with
 * default options (0 if the arguments are invalid): the part linear in n and
 * the slot of one workgroup, so that the sweep runs one workgroup per pass.
 * Between this and hawkes_workspace_bytes() the results are the same and
 * only the number of passes changes.  Options that enlarge a workgroup's
 * slot (fewer symmetric groups) may need more: such calls return
 * HAWKES_EWORKSPACE.  The minimum does not decrease with n, so a workspace
 * sized for n events (by either function) serves every smaller event set;
 * hawkes_workspace_bytes() itself is not monotone in n (its single-pass
 * size follows the group structure of the sweep). */
size_t hawkes_workspace_min_bytes(int64_t n, int precision);

/* Log-likelihood of rows [row_begin, row_end):  *d_loglik = sum_n l_n
 * (paper equation "model").  d_loglik: device pointer to 1 double.
 * Empty row ranges give 0. */
int hawkes_loglik(const hawkes_events *events, const hawkes_theta *theta, int precision,
                  int64_t row_begin, int64_t row_end, void *ws, size_t ws_bytes,
                  double *d_loglik, const hawkes_options *opts, void *stream);

/* As hawkes_loglik, plus the gradient of the same row sum with respect to
 * theta, in the order (mu, tau_x, tau_t, xi, h0, omega): d_grad is a device
 * pointer to 6 doubles.  Forward and adjoint sums come from one fused pass
 * over the pairs.  A floored event contributes no gradient from its log term. */
int hawkes_loglik_grad(const hawkes_events *events, const hawkes_theta *theta, int precision,
                       int64_t row_begin, int64_t row_end, void *ws, size_t ws_bytes,
                       double *d_loglik, double *d_grad, const hawkes_options *opts, void *stream);

/* Per-event terms of rows [row_begin, row_end): d_lambda[r] = lambda_n and
 * d_comp[r] = Lambda_n for n = row_begin + r (device arrays of
 * row_end - row_begin doubles; either may be NULL).  Uses the same pair
 * sweep as hawkes_loglik. */
int hawkes_event_terms(const hawkes_events *events, const hawkes_theta *theta, int precision,
                       int64_t row_begin, int64_t row_end, void *ws, size_t ws_bytes,
                       double *d_lambda, double *d_comp, const hawkes_options *opts, void *stream);

/* Log-likelihoods of rows [row_begin, row_end) for num_theta parameter vectors
 * on the same events: d_loglik[k] = the hawkes_loglik value at thetas[k]
 * (thetas: HOST array of num_theta structs; d_loglik: device array of
 * num_theta doubles).  The parameter kernels of the paper's sampler
 * (Section 2.3.2) and of delayed acceptance compare the likelihood at two
 * parameter vectors under the same latent locations.  FP32 and FP32_SKIP
 * evaluate vectors two at a time in one pair sweep that forms each pair's
 * differences once for both (a vector left over takes the single sweep).
 * Each value equals the hawkes_loglik value at the same vector up to a
 * last-bit FP32 rounding in a few pairs per billion (10^-15 relative at
 * n = 10^6; the first vector of each fused pair bitwise in FP32), so it does
 * not depend on the vector it is paired with (FP32_SKIP: beyond the summation
 * order of the far triggering tiles).  FP64 evaluates one vector per sweep.  Every
 * vector is checked as in hawkes_loglik before any work is enqueued;
 * num_theta < 1 or a NULL thetas: HAWKES_EINVAL.  The workspace is the one of
 * hawkes_workspace_bytes(n, precision). */
int hawkes_loglik_batch(const hawkes_events *events, const hawkes_theta *thetas, int64_t num_theta,
                        int precision, int64_t row_begin, int64_t row_end, void *ws, size_t ws_bytes,
                        double *d_loglik, const hawkes_options *opts, void *stream);

/* The X-update of the cut posterior (paper Section 2.2: latent locations drawn
 * from p(X | coarsened data) in O(N), uniformly within each event's county),
 * with counties as axis-aligned rectangles.
 *   d_county  device int32[n], county id of each event in [0, n_counties)
 *   d_rect    device double[n_counties * 4], rows (x0, y0, x1, y1), x0 < x1, y0 < y1
 *   seed, iteration  Philox4x64-10 key (seed, 0) and counter (n, iteration, 0, 0)
 *   d_x, d_y  device double[n] outputs (may alias the event arrays)
 * Event i gets u = (w >> 11) * 2^-53 from output words 0 and 1 and
 * x = fma(u, x1 - x0, x0) (likewise y), so results are bit-reproducible.
 * An out-of-range county id leaves that event's location as NaN. */
int hawkes_resample_locations(int64_t n, const int32_t *d_county, const double *d_rect,
                              int32_t n_counties, uint64_t seed, uint64_t iteration,
                              double *d_x, double *d_y, void *stream);

/* Synchronises `stream` and reads the device status word of workspace `ws`
 * written by the last likelihood call that used it: *status = HAWKES_OK,
 * HAWKES_EORDER or HAWKES_EDATA. */
int hawkes_workspace_status(const void *ws, int *status, void *stream);

/* hawkes_loglik_grad without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the workspace is a 64 MiB array in the
 * library's own device memory, one copy per GPU the library runs on, held
 * until the process ends.  Arguments and results as in hawkes_loglik_grad
 * (bitwise the same values: only the number of sweep passes differs).  n is
 * limited by the array: calls whose hawkes_workspace_min_bytes(n, precision)
 * exceeds 64 MiB (about 3 * 10^5 events at FP32) return HAWKES_EWORKSPACE
 * before any work.  The call allocates nothing.  All calls on one GPU share
 * the array, so calls that overlap on one GPU (two streams, two threads)
 * race and must be serialised by the caller; the device status word of the
 * last call is not readable (data-check failures still give NaN outputs). */
int hawkes_loglik_grad_noalloc(const hawkes_events *events, const hawkes_theta *theta, int precision,
                               int64_t row_begin, int64_t row_end, double *d_loglik, double *d_grad,
                               const hawkes_options *opts, void *stream);

/* Message for a status code, and the calling thread's last error message. */
const char *hawkes_strerror(int status);
const char *hawkes_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HAWKES_H */
