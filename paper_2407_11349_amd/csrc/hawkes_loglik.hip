// hawkes_loglik.hip -- O(N^2) spatiotemporal Hawkes log-likelihood and its
// gradient on gfx950 (MI355X), behind the C ABI declared in include/hawkes.h.
//
// Model: paper Section 2.1 (equations "fixed", "varying", "model" and the
// compensator after the R^2 approximation); floor of Section 2.3.1; row
// slices of Section 2.3.2.  See include/hawkes.h for the exact definition.
//
// Pipeline of one call (all on the caller's stream, no allocation):
//   1. k_clear_status, k_stage_common   tie-group ids, tile time ranges, data checks
//   2. k_stage_f32 (FP32 only)          per-theta source records in SoA layout
//      k_sym_bounds, k_sym_plan         (symmetric sweep) block order relations
//   3. k_pair_f32 / k_pair_f64          the pair sweep: per target row, six sums
//                                       over the sources of one source range
//   4. k_finalize                       per row: lambda_n, log, gradient terms,
//                                       compensator (FP64); FP32 rows whose sums
//                                       are underflow-limited go on a rescue list
//   5. k_rescue                         those rows again, every pair in FP64
//   6. k_blocksum, k_reduce             fixed-order FP64 sums of the row values
//
// Pair sums of target n (u_m = s_m^-2):
//   S0 = sum_{t_m != t_n} b_nm,  Sd2 = sum b d^2,  Sdt2 = sum b dt^2,
//   G0 = sum_{t_m < t_n} u_m e_nm,  G1 = sum u_m e (u_m d^2),  G2 = sum u_m e dt,
//   b_nm = exp(-d^2/(2 tau_x^2) - dt^2/(2 tau_t^2)),  e_nm = exp(-u_m d^2/(2 h0^2) - omega dt).
// With c_b = 1/((2 pi)^1.5 tau_x^2 tau_t) and c_g = omega/(2 pi h0^2):
//   lambda_n = mu c_b S0 + xi c_g G0, and every d lambda_n / d theta is a
//   linear combination of the six sums.
//
// Work decomposition: TS = 256 sources per tile are staged through LDS
// (double buffered) and read by all lanes as broadcasts; a target block of
// TB = 512 rows sits in registers (2 per lane).  Each (target block, tile)
// pair is classified from the tile's and the block's time ranges: CAUSAL
// (every source strictly earlier than every target: background +
// triggering, no masks), ANTI (every source strictly later: background
// only) or MIXED (per-pair masks from tie-group ids).  Causality is never
// decided from rounded times.  The background kernel is symmetric in the
// pair, so over the whole event set each strictly ordered pair of blocks is
// swept once, from the later block, and its background terms are added to
// both blocks' rows (the FP32 symmetric sweep); a row range sweeps all its
// tiles.  Partial sums go to per-source-range slots that the finalize adds
// in a fixed order, so results are bitwise reproducible.
//
// Several parameter vectors (hawkes_loglik_batch): k_pair_f32_batch sweeps the
// forward sums of two vectors at once, forming each pair's differences and
// squared distance once; each vector then takes its own finalize and reduction.
//
// Skip mode (HAWKES_FP32_SKIP): the same FP32 sweep without the pairs whose
// background term is exactly zero in FP32 because the time gap alone puts its
// exponent past the subnormal range; same results, less work on long spans.
//
// FP32 arithmetic (precision HAWKES_FP32):
//  * positions are pre-scaled in FP64 by sqrt(log2(e)/(2 tau_x^2)) and times
//    by sqrt(log2(e)/(2 tau_t^2)); the background exponent A = d2 + dt^2 is
//    formed in FP64 from them and rounded once, so no rounded per-theta
//    constant and no rounded time difference (integer-day data have only a
//    few distinct ones) enters the background;
//  * the triggering time factor is split at the tile's last time T_k:
//    exp(-omega dt) = exp(-omega (t_n - T_k)) * exp(-omega (T_k - t_m)); the
//    source factor is folded into v_m = u_m exp(-omega (T_k - t_m)) at
//    staging and the target factor is applied in FP64 per tile;
//  * FP32 partial sums of 8 terms are folded into FP64 accumulators; the
//    column sums of the symmetric sweep are FP32 sums over a wave's 128
//    targets, folded into FP64 per tile.

#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <mutex>

#include "hawkes.h"
#include "hawkes_common.h"

namespace hawkes {

namespace {

// Compile-time shape of the FP32 sweep (defaults measured fastest on gfx950;
// the macros exist so that other shapes can be built and timed).
#ifndef HAWKES_KT
#define HAWKES_KT 2
#endif
#ifndef HAWKES_GS
#define HAWKES_GS 8
#endif
#ifndef HAWKES_UJ
#define HAWKES_UJ 2
#endif
// source-loop unrolling of the fused loglik+gradient sweep (more registers per
// step, one more independent chain in flight)
#ifndef HAWKES_UJ_GRAD
#define HAWKES_UJ_GRAD 4
#endif
#define HK_STR(x) #x
#define HK_UNROLL(n) _Pragma(HK_STR(unroll n))

constexpr int TS = 256;                   // sources per LDS tile
constexpr int WG = 256;                   // threads per workgroup (4 wave64)
constexpr int NW = WG / 64;               // waves per workgroup
constexpr int KT = HAWKES_KT;             // target rows per lane
constexpr int TB = WG * KT;               // target rows per workgroup
constexpr int GS = HAWKES_GS;             // FP32 terms summed before folding into FP64
// row sweep: workgroups (target blocks x source chunks) a call aims for
constexpr int64_t DEFAULT_ROW_WGS = 32768;
constexpr int64_t MAX_ROW_WGS = 65536;
// row / column groups of the symmetric sweep: 384 splits 10^6 events into
// 326 x 326 groups of 6 blocks, whose ~53,000 workgroups leave a shorter tail
// than 160 groups (151 x 151 of 13 blocks) did
constexpr int DEFAULT_SYM_GROUPS = 384;
constexpr int MAX_SYM_GROUPS = 1024;
// Partial sums of the sweep's workgroups ("cells") go to slots that a fold
// kernel adds into per-row FP64 accumulators after each pass over at most as
// many cells as the slot region holds; the default region is this large (or
// what one pass over every cell needs, if less): with the part linear in n,
// under 10^9 bytes of workspace at 10^6 events (the 3072 cells a pass then
// holds at that size are a whole number of rounds of resident workgroups).
constexpr size_t DEFAULT_SLOT_BYTES = size_t(704) << 20;
constexpr int MAX_FUSED_THETA = 2;        // parameter vectors one batched sweep evaluates together
constexpr int64_t MAX_N = int64_t(1) << 30;
constexpr double LOG2E = 1.4426950408889634074;
constexpr float LN2F = 0.69314718055994530942f;
constexpr double LAMBDA_FLOOR = 1e-40;
// Padding sources (the tail of the last tile) sit far away in space and in
// time, so that every one of their terms is exactly 0 in both background forms
// (the uniform background has no spatial factor to rely on).  Their squared
// distances stay finite in FP32.
constexpr double PAD_COORD = 1e15;
constexpr double PAD_TIME = -1e15;

// Mean relative error of v_exp_f32 on gfx950, measured over 2^30 FP32
// arguments spread uniformly on [-30, 0] (and, to within 2e-10, on [-12, 0]
// and [-100, -30]): every FP32 pair term carries exactly one hardware exp2,
// so the FP32 sums are divided by (1 + this) in FP64.
constexpr double EXP2_MEAN_REL_ERR = -3.41e-9;
// Rows whose FP32 rate may have lost more than this fraction of its value to
// FP32 underflow (terms below 2^-126) are recomputed in FP64.
constexpr double RESCUE_REL = 1e-12;
// Background exponents (in units of log2) at or above this give exp2 = 0 in
// FP32 (the smallest subnormal is 2^-149); the skip mode leaves out pairs
// whose scaled time gap alone reaches it.
constexpr double SKIP_EXPONENT = 160.0;
// The skip mode also leaves out source tiles so far before a target block
// that each triggering term is below 2^-160 (u_max exp(-omega gap)): terms
// that underflow to zero in FP32 arithmetic and change no FP64 sum here.
constexpr double TRIG_SKIP_EXPONENT = 160.0;
constexpr double LN2 = 0.69314718055994530942;

constexpr int STATUS_ORDER = 1;
constexpr int STATUS_DATA = 2;

enum TileClass { CAUSAL = 0, ANTI = 1, MIXED = 2 };

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
inline bool is_fp32(int precision) { return precision == HAWKES_FP32 || precision == HAWKES_FP32_SKIP; }
inline bool valid_precision(int precision) { return precision == HAWKES_FP64 || is_fp32(precision); }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------------ layout

// Groups of the symmetric sweep: about `groups` row groups of rr target
// blocks and as many column groups of ct = KT rr source tiles (the same
// number of events), so the workgroup count is about groups^2 / 2.
struct SymPlan {
    int rr = 1, ct = 1, num_gr = 0, num_gc = 0;
};

SymPlan make_sym_plan(int64_t num_tb, int64_t num_tiles, int groups)
{
    SymPlan S;
    const int64_t s = ceil_div(num_tb, groups);
    S.rr = int(s);
    S.ct = int(KT * s);
    S.num_gr = int(ceil_div(num_tb, S.rr));
    S.num_gc = int(ceil_div(num_tiles, S.ct));
    return S;
}

// Per-source FP32 record fields in 8-byte slots (pairs), so that one index
// scale addresses every field of a source in LDS.
struct DeltaGroup {
    float d;  // T_k - t_m: the source's time offset from its tile's last time
    int g;    // tie-group id
};

// Workspace: a fixed part that grows linearly with n (staged records, per-row
// accumulators and values) followed by the slot region of the passes, whose
// size is whatever the caller's workspace leaves (at least one cell).
struct Layout {
    int64_t n = 0, n_pad = 0, num_tiles = 0, max_blocks = 0, rows_cap = 0;
    size_t status = 0, g = 0, tile = 0, rowvals = 0, rescue = 0;
    size_t xs = 0, ys = 0, tsd = 0, r2 = 0, v2 = 0, u2 = 0, dg = 0;
    size_t sblk = 0, eblk = 0, gchi = 0, g0 = 0, rowstart = 0;
    size_t acc = 0, blocks = 0, slots = 0, fixed = 0;
    size_t total = 0;    // the size hawkes_workspace_bytes returns
    size_t minimum = 0;  // the fixed part and one cell of the default plans
};

// Bytes of one cell's slot: row sums (6 per row) and, in the symmetric sweep,
// column sums (3 per source) of its group's events.
inline size_t sym_cell_bytes(const SymPlan &S) { return sizeof(double) * 9 * size_t(S.rr) * TB; }
inline size_t row_cell_bytes() { return sizeof(double) * 6 * size_t(TB); }

// Work plan of the row sweep: target blocks over the row range, source chunks.
struct Plan {
    int64_t rows = 0, num_tb = 0, rows_pad = 0, chunk_tiles = 0, num_chunks = 0;
};

Plan make_plan(int64_t rows, int64_t num_tiles, int64_t target_wgs)
{
    Plan P;
    P.rows = rows;
    P.num_tb = ceil_div(rows, TB);
    P.rows_pad = P.num_tb * TB;
    int64_t want = ceil_div(target_wgs, P.num_tb);
    if (want < 1)
        want = 1;
    if (want > num_tiles)
        want = num_tiles;
    P.chunk_tiles = ceil_div(num_tiles, want);
    P.num_chunks = ceil_div(num_tiles, P.chunk_tiles);
    return P;
}

// Slot bytes a call with the default tuning needs for a single pass (the
// symmetric sweep's bound counts every row group x column group cell).
size_t single_pass_bytes(int64_t n)
{
    const int64_t num_tiles = ceil_div(n, TS), tb = ceil_div(n, TB);
    const SymPlan S = make_sym_plan(tb, num_tiles, DEFAULT_SYM_GROUPS);
    const size_t sym = size_t(S.num_gr) * size_t(S.num_gc) * sym_cell_bytes(S);
    const Plan P = make_plan(n, num_tiles, DEFAULT_ROW_WGS);
    const size_t row = size_t(P.num_tb) * size_t(P.num_chunks) * row_cell_bytes();
    return sym > row ? sym : row;
}

Layout make_layout(int64_t n, int precision)
{
    Layout L;
    L.n = n;
    L.num_tiles = ceil_div(n, TS);
    L.n_pad = L.num_tiles * TS;
    const int64_t tb_max = ceil_div(n, TB);
    L.max_blocks = ceil_div(n, WG);
    L.rows_cap = tb_max * TB;

    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.status = take(256);
    L.g = take(sizeof(int) * L.n_pad);
    L.tile = take(sizeof(double) * 3 * L.num_tiles);
    if (is_fp32(precision)) {
        L.xs = take(sizeof(double) * L.n_pad);
        L.ys = take(sizeof(double) * L.n_pad);
        L.tsd = take(sizeof(double) * L.n_pad);
        // r_m and v_m of each vector a batched sweep evaluates (the single sweep uses the first)
        L.r2 = take(sizeof(float2) * L.n_pad * MAX_FUSED_THETA);
        L.v2 = take(sizeof(float2) * L.n_pad * MAX_FUSED_THETA);
        L.u2 = take(sizeof(float2) * L.n_pad);
        L.dg = take(sizeof(DeltaGroup) * L.n_pad);
    }
    L.sblk = take(sizeof(int) * tb_max);
    L.eblk = take(sizeof(int) * tb_max);
    L.gchi = take(sizeof(int) * MAX_SYM_GROUPS);
    L.g0 = take(sizeof(int) * MAX_SYM_GROUPS);
    L.rowstart = take(sizeof(int) * (MAX_SYM_GROUPS + 1));  // + the symmetric plan's cell count
    // per-row FP64 accumulators of the folded partial sums: 6 row sums, 3 column sums
    L.acc = take(sizeof(double) * 9 * L.rows_cap);
    L.blocks = take(sizeof(double) * 7 * L.max_blocks);
    L.rowvals = take(sizeof(double) * 7 * L.rows_cap);
    L.rescue = take(sizeof(int) * L.rows_cap);
    L.slots = off;
    L.fixed = off;
    size_t slot_bytes = single_pass_bytes(n);
    if (slot_bytes > DEFAULT_SLOT_BYTES)
        slot_bytes = DEFAULT_SLOT_BYTES;
    // at least one cell of the default plans (a symmetric cell is never smaller than a row cell)
    const SymPlan S1 = make_sym_plan(tb_max, L.num_tiles, DEFAULT_SYM_GROUPS);
    const size_t one_cell = sym_cell_bytes(S1);
    if (slot_bytes < one_cell)
        slot_bytes = one_cell;
    L.total = align256(off + slot_bytes);
    L.minimum = align256(off + one_cell);
    return L;
}

// Device view of the cells of a sweep, numbered in launch order: row groups
// from the latest down, and within a row group the column groups it reaches
// from the earliest up.  Symmetric sweep: row group gr reaches column groups
// 0..gchi[gr] (from the device plan) and its first cell is rowstart[gr];
// row sweep (rowstart == nullptr): every target block takes every chunk.
struct CellMap {
    const int *rowstart = nullptr, *gchi = nullptr;
    const int *total = nullptr;  // symmetric sweep: the plan's cell count
    int num_gr = 0, num_gc = 0;
    int cell0 = 0;               // first cell of the pass being launched
    int ncells = 0;              // cells of that pass (its workgroups)
};

// Cell of workgroup w of the current pass and its slot (false: past the last cell).  A pass's
// workgroups take its cells in reverse order: within a row group the cells nearest the diagonal,
// the costliest when far pairs are skipped, start first, and the pass ends on cheaper ones.
__host__ __device__ inline bool map_cell(const CellMap &m, unsigned w, int &gr, int &gc, int &slot)
{
    slot = m.ncells - 1 - int(w);
    const int c = m.cell0 + slot;
    if (!m.rowstart) {
        if (c >= m.num_gr * m.num_gc)
            return false;
        gr = m.num_gr - 1 - c / m.num_gc;
        gc = c % m.num_gc;
        return true;
    }
    if (c >= *m.total)
        return false;
    // rowstart decreases with gr and rowstart[num_gr - 1] = 0: the smallest
    // gr whose first cell is at or before c owns c
    int lo = 0, hi = m.num_gr - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (m.rowstart[mid] <= c)
            hi = mid;
        else
            lo = mid + 1;
    }
    gr = lo;
    gc = c - m.rowstart[lo];
    return true;
}

// ------------------------------------------------------------- kernels

// status[0]: data-check flags; status[1]: number of rows on the rescue list;
// 8-byte word STATUS_UMAX: the largest u_m = s_m^-2 (FP64 bit pattern, which
// orders like the value for non-negative numbers), set by k_umax.
constexpr int STATUS_UMAX = 1;
__global__ void k_clear_status(int *status)
{
    status[0] = 0;
    status[1] = 0;
    reinterpret_cast<unsigned long long *>(status)[STATUS_UMAX] = 0ull;
}

// Largest u_m = 1 / s_m^2 over the events (one atomic per workgroup).
__global__ __launch_bounds__(256) void k_umax(const double *__restrict__ s, int64_t n, int *status)
{
    __shared__ double red[256];
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double u = 0.0;
    if (i < n) {
        const double si = s[i];
        u = 1.0 / (si * si);
        u = (isfinite(u) && u > 0.0) ? u : 0.0;  // bad values are flagged by the data checks
    }
    red[threadIdx.x] = u;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        atomicMax(reinterpret_cast<unsigned long long *>(status) + STATUS_UMAX,
                  (unsigned long long)__double_as_longlong(red[0]));
}

__global__ void k_zero_outputs(double *loglik, double *grad)
{
    const int i = threadIdx.x;
    if (i == 0 && loglik)
        loglik[0] = 0.0;
    if (i < 6 && grad)
        grad[i] = 0.0;
}

// Tie-group ids (index of the first event with the same time), tile time
// ranges, and the device-side data checks.
__global__ __launch_bounds__(256) void k_stage_common(const double *__restrict__ t, const double *__restrict__ x,
                                                      const double *__restrict__ y, const double *__restrict__ s,
                                                      int64_t n, int64_t n_pad, int *__restrict__ g,
                                                      double *__restrict__ tile, int *status)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_pad)
        return;
    if (i >= n) {
        g[i] = INT_MAX;
        return;
    }
    const double ti = t[i];
    int flags = 0;
    if (!isfinite(ti) || !isfinite(x[i]) || !isfinite(y[i]) || !isfinite(s[i]) || !(s[i] > 0.0))
        flags |= STATUS_DATA;
    if (i + 1 < n && t[i + 1] < ti)
        flags |= STATUS_ORDER;
    if (flags)
        atomicOr(status, flags);
    // lower bound of ti in the (sorted) time array
    int64_t lo = 0, hi = i;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (t[mid] < ti)
            lo = mid + 1;
        else
            hi = mid;
    }
    g[i] = int(lo);
    if (i % TS == 0) {
        const int64_t k = i / TS;
        const int64_t last = (i + TS < n ? i + TS : n) - 1;
        tile[3 * k + 0] = ti;
        tile[3 * k + 1] = t[last];
    }
}

struct StageF32 {
    double sx, st, rr, omega;
};

// Splits an FP64 value into an FP32 pair hi + lo (hi = nearest FP32).
__device__ inline void split_f32(double v, float &hi, float &lo)
{
    hi = float(v);
    lo = float(v - double(hi));
}

// Per-theta source records for the FP32 sweep (SoA of 8-byte fields, padded to
// whole tiles): positions and times pre-scaled in FP64; r_m = u_m (tau_x/h0)^2,
// v_m = u_m exp(-omega (T_k - t_m)) and u_m as FP32 hi + lo pairs, so that
// no rounding is shared by many pairs (all sources of the paper's model 1
// have one u; integer-day times give few distinct T_k - t_m); the time offset
// T_k - t_m with the tie-group id.
__global__ __launch_bounds__(256) void k_stage_f32(const double *__restrict__ t, const double *__restrict__ x,
                                                   const double *__restrict__ y, const double *__restrict__ s,
                                                   const int *__restrict__ g, int64_t n, int64_t n_pad, StageF32 c,
                                                   const double *__restrict__ tile, double *__restrict__ xs,
                                                   double *__restrict__ ys, double *__restrict__ tsd,
                                                   float2 *__restrict__ r2, float2 *__restrict__ v2,
                                                   float2 *__restrict__ u2, DeltaGroup *__restrict__ dg)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_pad)
        return;
    if (i >= n) {
        xs[i] = PAD_COORD;
        ys[i] = PAD_COORD;
        tsd[i] = PAD_TIME;
        r2[i] = v2[i] = u2[i] = make_float2(0.0f, 0.0f);
        dg[i] = DeltaGroup{0.0f, g[i]};
        return;
    }
    const int64_t k = i / TS;
    const double tlast = tile[3 * k + 1];
    const double si = s[i];
    const double u = 1.0 / (si * si);
    const double d = tlast - t[i];
    xs[i] = x[i] * c.sx;
    ys[i] = y[i] * c.sx;
    tsd[i] = t[i] * c.st;
    float hi, lo;
    split_f32(u * c.rr, hi, lo);
    r2[i] = make_float2(hi, lo);
    split_f32(u * exp(-c.omega * d), hi, lo);
    v2[i] = make_float2(hi, lo);
    split_f32(u, hi, lo);
    u2[i] = make_float2(hi, lo);
    dg[i] = DeltaGroup{float(d), g[i]};
}

// r_m and v_m (hi, lo) of a further parameter vector for the batched sweep,
// from the same formulas as k_stage_f32 (rr and omega are that vector's).
__global__ __launch_bounds__(256) void k_stage_f32_rv(const double *__restrict__ t, const double *__restrict__ s,
                                                      int64_t n, int64_t n_pad, double rr, double omega,
                                                      const double *__restrict__ tile, float2 *__restrict__ r2,
                                                      float2 *__restrict__ v2)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_pad)
        return;
    if (i >= n) {
        r2[i] = v2[i] = make_float2(0.0f, 0.0f);
        return;
    }
    const double tlast = tile[3 * (i / TS) + 1];
    const double si = s[i];
    const double u = 1.0 / (si * si);
    float hi, lo;
    split_f32(u * rr, hi, lo);
    r2[i] = make_float2(hi, lo);
    split_f32(u * exp(-omega * (tlast - t[i])), hi, lo);
    v2[i] = make_float2(hi, lo);
}

// Restarts the rescue list (status[1]) before a further vector's finalize.
__global__ void k_clear_rescue(int *status) { status[1] = 0; }

struct PairF32 {
    const double *xs, *ys, *tsd, *t;
    const float2 *r2, *v2, *u2;  // (hi, lo) of r_m, v_m, u_m
    const DeltaGroup *dg;
    const int *g;
    const double *tile;
    // Symmetric sweep (sym = 1, the whole event set): for target block b,
    // every time in blocks < sblk[b] is below every time in b, and every
    // time in blocks >= eblk[b] is above every time in b.
    const int *sblk, *eblk;
    CellMap cells;  // the cells of the sweep and the first one of this pass
    double *srow;   // [slot][6][ge]: a cell's row sums of its row group's rows
    double *scol;   // [slot][3][ge]: a cell's background column sums of its column group's sources
    int ge;         // events per group (slot stride)
    int row_begin, row_end, rows_pad, num_tiles, num_tb;  // indices below 2^31 (n <= 2^30)
    int rr, ct;     // target blocks per row group, source tiles per column group
    int sym;
    // Skip mode: every background term of a pair further apart in time than
    // skip_gap days is exactly zero in FP32.  Tiles that far before a block
    // sweep the triggering terms only, and in the row sweep (window = 1) tiles
    // that far after it are not visited.  Without skipping, skip_gap is
    // infinite and window = 0.  With trig_cull, tiles so far before a block that
    // every triggering term is below 2^-TRIG_SKIP_EXPONENT (in units of the sum
    // G0; u_m <= u_max) are not visited either.
    int window, trig_cull;
    const unsigned long long *umax;  // the status word holding u_max
    double omega, inv_st, out_s1, out_s2, out_g1, out_exp;
    double w2;  // omega * log2(e) / time scale: the triggering exponent per scaled day
    double skip_gap;
};

// Pair geometry: the scaled squared distance D and the background exponent
// A = D + dt'^2, differences and squares in FP64, D and A each rounded once
// to FP32.
__device__ inline void geom_da(double xn, double yn, double tn, double xm, double ym, double tm, float &D, float &A)
{
    const double dx = xn - xm, dy = yn - ym, dt = tn - tm;
    const double d2 = fma(dy, dy, dx * dx);
    D = float(d2);
    A = float(fma(dt, dt, d2));
}
__device__ inline float geom_d(double xn, double yn, double xm, double ym)
{
    const double dx = xn - xm, dy = yn - ym;
    return float(fma(dy, dy, dx * dx));
}
// Spatially uniform background: the exponent is the scaled time gap alone,
// A = dt'^2, so with tied times (integer days) many pairs share one value of
// A and its FP32 rounding would not average out; A is split into a hi part
// (the exp2 argument) and a lo part that corrects the term to first order.
__device__ inline void geom_da_uni(double xn, double yn, double tn, double xm, double ym, double tm, float &D,
                                   float &A, float &Alo)
{
    const double dx = xn - xm, dy = yn - ym, dt = tn - tm;
    D = float(fma(dy, dy, dx * dx));
    const double a2 = dt * dt;
    A = float(a2);
    Alo = float(a2 - double(A));
}

// Column sums of the symmetric sweep.  Within each row of 16 lanes, the
// lanes take the 16 sources of a subgroup in rotation: at step j lane i takes
// source (i + j) mod 16, and the FP32 column accumulators of a source move
// with it (row_ror:15: lane i reads lane (i + 1) mod 16 of its row).  After 8
// steps each lane's accumulator (the row's sum over 8 steps of 2 targets) is
// kept in FP64 and a new one starts; after 16 steps the first half's FP64 sum
// of a source sits 8 lanes away from the second half's (row_ror:8).  The four
// rows take the same sources at the same lane positions and are added by the
// gfx950 row swaps (permlane16: rows 0+1 and 2+3; permlane32: the halves).
constexpr int DPP_ROW_ROR8 = 0x128, DPP_ROW_ROR15 = 0x12F;
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}
__device__ __forceinline__ float row_rotate_f32(float v)
{
    return __int_as_float(dpp_mov<DPP_ROW_ROR15>(__float_as_int(v)));
}
__device__ __forceinline__ double make_f64(unsigned lo, unsigned hi)
{
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double row_shift8_f64(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = dpp_mov<DPP_ROW_ROR8>(int(unsigned(u))), hi = dpp_mov<DPP_ROW_ROR8>(int(unsigned(u >> 32)));
    return make_f64(unsigned(lo), unsigned(hi));
}
__device__ __forceinline__ double sum_rows_f64(double v)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    auto lo = __builtin_amdgcn_permlane16_swap(unsigned(u), unsigned(u), false, false);
    auto hi = __builtin_amdgcn_permlane16_swap(unsigned(u >> 32), unsigned(u >> 32), false, false);
    v = make_f64(lo[0], hi[0]) + make_f64(lo[1], hi[1]);
    u = (unsigned long long)__double_as_longlong(v);
    lo = __builtin_amdgcn_permlane32_swap(unsigned(u), unsigned(u), false, false);
    hi = __builtin_amdgcn_permlane32_swap(unsigned(u >> 32), unsigned(u >> 32), false, false);
    return make_f64(lo[0], hi[0]) + make_f64(lo[1], hi[1]);
}
static_assert(GS == 8, "the column rotation keeps one FP64 partial per 8-source group");

// Direct global-to-LDS load of one dword per lane (global_load_lds_dword):
// lane l's dword lands at LDS address `wave_base` + 4 l; `wave_base` must be
// the same for the whole wave.  stage_wait() waits for this wave's
// outstanding vector memory operations (vmcnt 0), which include these loads.
typedef __attribute__((address_space(1))) void global_void;
typedef __attribute__((address_space(3))) void lds_void;
__device__ __forceinline__ void lds_dma4(const void *src, void *wave_base)
{
    __builtin_amdgcn_global_load_lds((global_void *)src, (lds_void *)wave_base, 4, 0, 0);
}
__device__ __forceinline__ void stage_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// The FP32 fused sweep.  GRAD = false keeps only S0 and G0 (log-likelihood).
//
// Per pair (positions and times pre-scaled so that the background exponent
// is A = |x_n - x_m|^2 + (t_n - t_m)^2):
//   d2 = |x_n - x_m|^2 and A = d2 + dt^2 in FP64, each rounded once to FP32;
//   background b = exp2(-A); triggering (earlier sources) p = v_m exp2(-t1)
//   with t1 = r_m D.  Every FP32 value that many pairs would share is split
//   hi + lo, and every rounding left is of a value that varies from pair to
//   pair, so rounding errors average out instead of adding up.
//
// A workgroup owns a rectangle: the rr target blocks of row group gr (2 rows
// per lane each, one block at a time) against the ct source tiles of column
// group gc.  Row sums stay in registers for a block's sweep over the
// rectangle's tiles and go to the row partials of column group gc.
//
// Symmetric sweep (whole event set).  The background term is symmetric in
// the pair, so a block pair whose times are strictly ordered is swept once,
// from the later block: each term b_nm goes to the row sums of n and, as a
// column sum, to the row sums of m.  The later block's view is then never
// swept from the earlier block.  Block pairs whose time ranges touch are
// swept from both sides, with per-tile classes as in the row sweep.  A
// wave's column sums of a tile come from the 16-lane rotation above (FP32
// over 8 steps, then FP64, then over the 4 rows); the tile's owner lanes add
// the 4 waves' sums in FP64 and add them to this row group's column partials,
// which the workgroup alone writes (so every sum keeps a fixed order and
// results are bitwise reproducible).
//
// Row sweep (a row range): every tile is swept for every block (rr = 1,
// no columns).
//
// At least this many waves per SIMD: the register budget the compiler must
// fit (2 waves = 256 registers per lane).  KT = 2 needs ~164 and runs at 3.
#ifndef HAWKES_WAVES_PER_EU
#define HAWKES_WAVES_PER_EU 2
#endif
#if HAWKES_WAVES_PER_EU > 0
#define HK_PAIR_ATTR __attribute__((amdgpu_waves_per_eu(HAWKES_WAVES_PER_EU)))
#else
#define HK_PAIR_ATTR
#endif
template <bool GRAD, bool UNI>
__global__ __launch_bounds__(WG) HK_PAIR_ATTR void k_pair_f32(PairF32 a)
{
    // one tile of source records; the fields sit at fixed offsets from each
    // other, so a source's loads share one address and immediate offsets
    struct TileRecs {
        double x[TS], y[TS], t[TS];
        float2 r[TS], v[TS], u[TS];
        DeltaGroup dg[TS];
    };
    __shared__ TileRecs lt2[2];
    __shared__ float lcol[2][3][NW][TS];  // per-wave column sums of the tile being swept

    constexpr int UJ = GRAD ? HAWKES_UJ_GRAD : HAWKES_UJ;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15;
    int gr, gc, slot;
    if (!map_cell(a.cells, blockIdx.x, gr, gc, slot))
        return;
    const int b_first = gr * a.rr;
    const int b_stop = (b_first + a.rr < a.num_tb) ? b_first + a.rr : a.num_tb;
    const int kg0 = gc * a.ct;
    const int kg1 = (kg0 + a.ct < a.num_tiles) ? kg0 + a.ct : a.num_tiles;
    // this workgroup's slot: row sums of rows b_first * TB.., column sums of sources kg0 * TS..
    const int64_t stride = a.ge;
    const int jb = kg0 * TS, rb0 = b_first * TB;
    double *pc = a.scol + int64_t(slot) * 3 * stride;
    if (a.sym) {
        for (int k = kg0; k < kg1; ++k) {
            const int j = k * TS + tid - jb;
            pc[j] = 0.0;
            if (GRAD) {
                pc[stride + j] = 0.0;
                pc[2 * stride + j] = 0.0;
            }
        }
    }

    // Staging of tile k into LDS buffer buf by direct global-to-LDS loads: each
    // lane moves two dwords of every 8-byte-field array, landing at the wave's
    // base + 4 * lane.  The loads of the next tile run during the sweep;
    // stage_wait() (this wave's loads done) comes before the barrier that
    // publishes the tile.
    auto stage = [&](int k, int buf) {
        TileRecs &T = lt2[buf];
        // per-lane offset kept opaque, so that the compiler forms each address
        // from the array's tile base (scalar) and this offset rather than
        // holding a per-lane pointer for every array across the loop
        int o = tid;
        asm volatile("" : "+v"(o));
        const int wb = tid & ~63;
        const unsigned *xs = reinterpret_cast<const unsigned *>(a.xs + k * TS);
        const unsigned *ys = reinterpret_cast<const unsigned *>(a.ys + k * TS);
        const unsigned *ts = reinterpret_cast<const unsigned *>(a.tsd + k * TS);
        lds_dma4(xs + o, reinterpret_cast<unsigned *>(T.x) + wb);
        lds_dma4(xs + TS + o, reinterpret_cast<unsigned *>(T.x) + TS + wb);
        lds_dma4(ys + o, reinterpret_cast<unsigned *>(T.y) + wb);
        lds_dma4(ys + TS + o, reinterpret_cast<unsigned *>(T.y) + TS + wb);
        lds_dma4(ts + o, reinterpret_cast<unsigned *>(T.t) + wb);
        lds_dma4(ts + TS + o, reinterpret_cast<unsigned *>(T.t) + TS + wb);
        const unsigned *r2 = reinterpret_cast<const unsigned *>(a.r2 + k * TS);
        const unsigned *v2 = reinterpret_cast<const unsigned *>(a.v2 + k * TS);
        const unsigned *u2 = reinterpret_cast<const unsigned *>(a.u2 + k * TS);
        const unsigned *dg = reinterpret_cast<const unsigned *>(a.dg + k * TS);
        lds_dma4(r2 + o, reinterpret_cast<unsigned *>(T.r) + wb);
        lds_dma4(r2 + TS + o, reinterpret_cast<unsigned *>(T.r) + TS + wb);
        lds_dma4(v2 + o, reinterpret_cast<unsigned *>(T.v) + wb);
        lds_dma4(v2 + TS + o, reinterpret_cast<unsigned *>(T.v) + TS + wb);
        lds_dma4(u2 + o, reinterpret_cast<unsigned *>(T.u) + wb);
        lds_dma4(u2 + TS + o, reinterpret_cast<unsigned *>(T.u) + TS + wb);
        lds_dma4(dg + o, reinterpret_cast<unsigned *>(T.dg) + wb);
        lds_dma4(dg + TS + o, reinterpret_cast<unsigned *>(T.dg) + TS + wb);
    };

    // trig_cull: a triggering term of a source more than cull_gap days before its
    // target is below u_max exp(-omega gap) < 2^-TRIG_SKIP_EXPONENT; no smaller
    // than skip_gap, so that the background terms there are exactly zero too
    double cull_gap = a.skip_gap;
    if (a.trig_cull) {
        const double um = __longlong_as_double((long long)*a.umax);
        const double tg = (log(um) + TRIG_SKIP_EXPONENT * LN2) / a.omega;
        cull_gap = (tg > cull_gap) ? tg : cull_gap;
    }

    for (int b = b_first; b < b_stop; ++b) {
        const int i0 = a.row_begin + b * TB;
        const int iend = (i0 + TB < a.row_end) ? i0 + TB : a.row_end;
        const double t_lo = a.t[i0], t_hi = a.t[iend - 1];

        // lanes past the block's end take a target far away in space and time:
        // every one of its terms is exactly 0, so its column terms add nothing
        double xn[KT], yn[KT], tsn[KT], trn[KT];
        int gn[KT];
#pragma unroll
        for (int q = 0; q < KT; ++q) {
            const int i = i0 + tid + q * WG;
            const bool in = i < iend;
            xn[q] = in ? a.xs[i] : PAD_COORD;
            yn[q] = in ? a.ys[i] : PAD_COORD;
            tsn[q] = in ? a.tsd[i] : PAD_TIME;
            trn[q] = a.t[in ? i : iend - 1];
            gn[q] = in ? a.g[i] : INT_MAX;
        }
        double acc[KT][6];
#pragma unroll
        for (int q = 0; q < KT; ++q)
#pragma unroll
            for (int z = 0; z < 6; ++z)
                acc[q][z] = 0.0;

        // tiles [0, k_strict): strictly earlier blocks, swept with column sums;
        // tiles from k_end on: not visited
        int k_strict = 0, k_end = a.num_tiles, k_lo = 0;
        if (a.trig_cull) {
            // first tile whose last time is within cull_gap days of the block
            const double limit = t_lo - cull_gap;
            int lo = 0, hi = a.num_tiles;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (a.tile[3 * mid + 1] < limit)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            k_lo = lo;
        }
        if (a.sym) {
            k_strict = KT * a.sblk[b];
            const int e = KT * a.eblk[b];
            k_end = (e < a.num_tiles) ? e : a.num_tiles;
        } else if (a.window) {
            // first tile that starts more than skip_gap days after the block ends
            const double limit = t_hi + a.skip_gap;
            int lo = 0, hi = a.num_tiles;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (a.tile[3 * mid + 0] > limit)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            k_end = lo;
        }
        const int k0 = (kg0 > k_lo) ? kg0 : k_lo;
        const int k1 = (kg1 < k_end) ? kg1 : k_end;

        if (k0 < k1)
            stage(k0, 0);
        stage_wait();
        __syncthreads();

        for (int k = k0; k < k1; ++k) {
            const int buf = (k - k0) & 1;
            if (k + 1 < k1)
                stage(k + 1, buf ^ 1);  // into the buffer every wave finished reading

            const double first = a.tile[3 * k + 0], last = a.tile[3 * k + 1];
            const int cls = (last < t_lo) ? CAUSAL : ((first > t_hi) ? ANTI : MIXED);
            const bool trig_only = (cls == CAUSAL) && (t_lo - last > a.skip_gap);
            const bool cols = (k < k_strict) && !trig_only;  // strictly earlier block (so CAUSAL)

            // Terms are summed in FP32 over groups of GS = 8 sources and each
            // group sum is folded into FP64.  Long FP32 running sums would round
            // away every Gaussian-tail term below half an ulp of the sum, a
            // systematic loss of ~1e-8 relative; groups of 8 keep it near 3e-10
            // and equal across the six sums (the gradient combines them with
            // heavy cancellation, so their errors must match).  Background sums go
            // straight into the accumulators; the CAUSAL triggering sums keep FP64
            // tile partials that take the target's time factor at the tile end.
            double gt[KT][3];
#pragma unroll
            for (int q = 0; q < KT; ++q)
                gt[q][0] = gt[q][1] = gt[q][2] = 0.0;

            const TileRecs &T = lt2[buf];
            const double *sx = T.x, *sy = T.y, *st = T.t;
            const float2 *sr = T.r, *sv = T.v;
            const DeltaGroup *sdg = T.dg;

            if (cls != MIXED) {
                const bool causal = (cls == CAUSAL);
                // column sums (CAUSAL with columns): FP32 over 8 rotation steps, then FP64.
                // FP32 sums start at -0, the exact additive identity (x + -0 = x for every
                // x, +0 included), so the compiler can drop a sum's first addition and turn
                // fma(a, b, -0) into a product; a +0 start would cost an instruction
                float e0 = -0.0f, e1 = -0.0f, e2 = -0.0f;
                double h0 = 0.0, h1 = 0.0, h2 = 0.0;
                for (int m0 = 0; m0 < TS; m0 += GS) {
                    float f[KT][6];
#pragma unroll
                    for (int q = 0; q < KT; ++q)
#pragma unroll
                        for (int z = 0; z < 6; ++z)
                            f[q][z] = -0.0f;
                    // background + triggering terms of one source for the lane's targets;
                    // adds the background terms' sums over those targets (b, b D, b A) to c0..c2
                    auto causal_pair = [&](int m, float &c0, float &c1, float &c2) {
                        const double xm = sx[m], ym = sy[m], tm = st[m];
                        const float2 rm = sr[m], vm = sv[m];
                        const float rhm = rm.x, rlm = rm.y, vhm = vm.x, vlm = vm.y, dm = sdg[m].d;
#pragma unroll
                        for (int q = 0; q < KT; ++q) {
                            float D, A, Alo = 0.0f;
                            if (UNI)
                                geom_da_uni(xn[q], yn[q], tsn[q], xm, ym, tm, D, A, Alo);
                            else
                                geom_da(xn[q], yn[q], tsn[q], xm, ym, tm, D, A);
                            float b = __builtin_amdgcn_exp2f(-A);
                            if (UNI)
                                b = fmaf(-LN2F * Alo, b, b);
                            const float t1 = fmaf(rlm, D, rhm * D);
                            const float E = __builtin_amdgcn_exp2f(-t1);
                            const float p = fmaf(vlm, E, vhm * E);
                            f[q][0] += b;
                            f[q][3] += p;
                            c0 += b;
                            if (GRAD) {
                                if (!UNI) {
                                    f[q][1] = fmaf(b, D, f[q][1]);
                                    c1 = fmaf(b, D, c1);
                                }
                                f[q][2] = fmaf(b, A, f[q][2]);
                                c2 = fmaf(b, A, c2);
                                f[q][4] = fmaf(p, t1, f[q][4]);
                                f[q][5] = fmaf(p, dm, f[q][5]);
                            }
                        }
                    };
                    // triggering terms only (the background terms are exactly zero)
                    auto trig_pair = [&](int m) {
                        const double xm = sx[m], ym = sy[m];
                        const float2 rm = sr[m], vm = sv[m];
                        const float rhm = rm.x, rlm = rm.y, vhm = vm.x, vlm = vm.y, dm = sdg[m].d;
#pragma unroll
                        for (int q = 0; q < KT; ++q) {
                            const float D = geom_d(xn[q], yn[q], xm, ym);
                            const float t1 = fmaf(rlm, D, rhm * D);
                            const float E = __builtin_amdgcn_exp2f(-t1);
                            const float p = fmaf(vlm, E, vhm * E);
                            f[q][3] += p;
                            if (GRAD) {
                                f[q][4] = fmaf(p, t1, f[q][4]);
                                f[q][5] = fmaf(p, dm, f[q][5]);
                            }
                        }
                    };
                    const int sub = m0 & ~15, s0 = m0 & 15;
                    if (trig_only) {
                        HK_UNROLL(UJ)
                        for (int j = 0; j < GS; ++j)
                            trig_pair(m0 + j);
                    } else if (cols) {
                        // 16-source rotation (row sums as in the plain causal loop): lane i
                        // takes source sub + ((i + step) mod 16) at step step of the subgroup
                        HK_UNROLL(UJ)
                        for (int j = 0; j < GS; ++j) {
                            float c0 = -0.0f, c1 = -0.0f, c2 = -0.0f;
                            causal_pair(sub + ((li + s0 + j) & 15), c0, c1, c2);
                            e0 = row_rotate_f32(e0) + c0;
                            if (GRAD) {
                                if (!UNI)
                                    e1 = row_rotate_f32(e1) + c1;
                                e2 = row_rotate_f32(e2) + c2;
                            }
                        }
                        if (s0 == 0) {
                            // first 8 steps: lane i holds source sub + ((i + 7) mod 16)
                            h0 = double(e0);
                            h1 = double(e1);
                            h2 = double(e2);
                        } else {
                            // lane i holds source sub + ((i + 15) mod 16), whose first-half sum
                            // is 8 lanes back; add the halves, then the four rows
                            double w0 = sum_rows_f64(row_shift8_f64(h0) + double(e0));
                            double w1 = 0.0, w2 = 0.0;
                            if (GRAD) {
                                if (!UNI)
                                    w1 = sum_rows_f64(row_shift8_f64(h1) + double(e1));
                                w2 = sum_rows_f64(row_shift8_f64(h2) + double(e2));
                            }
                            if (lane < 16) {
                                const int mc = sub + ((li + 15) & 15);
                                lcol[buf][0][wave][mc] = float(w0);
                                if (GRAD) {
                                    lcol[buf][1][wave][mc] = float(w1);
                                    lcol[buf][2][wave][mc] = float(w2);
                                }
                            }
                        }
                        e0 = e1 = e2 = -0.0f;
                    } else if (causal) {
                        HK_UNROLL(UJ)
                        for (int j = 0; j < GS; ++j) {
                            float c0 = -0.0f, c1 = -0.0f, c2 = -0.0f;
                            causal_pair(m0 + j, c0, c1, c2);  // column sums unused
                        }
                    } else {
                        HK_UNROLL(UJ)
                        for (int j = 0; j < GS; ++j) {
                            const int m = m0 + j;
                            const double xm = sx[m], ym = sy[m], tm = st[m];
#pragma unroll
                            for (int q = 0; q < KT; ++q) {
                                float D, A, Alo = 0.0f;
                                if (UNI)
                                    geom_da_uni(xn[q], yn[q], tsn[q], xm, ym, tm, D, A, Alo);
                                else
                                    geom_da(xn[q], yn[q], tsn[q], xm, ym, tm, D, A);
                                float b = __builtin_amdgcn_exp2f(-A);
                                if (UNI)
                                    b = fmaf(-LN2F * Alo, b, b);
                                f[q][0] += b;
                                if (GRAD) {
                                    if (!UNI)
                                        f[q][1] = fmaf(b, D, f[q][1]);
                                    f[q][2] = fmaf(b, A, f[q][2]);
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int q = 0; q < KT; ++q) {
                        if (!trig_only) {
                            acc[q][0] += double(f[q][0]);
                            if (GRAD) {
                                acc[q][1] += double(f[q][1]);
                                acc[q][2] += double(f[q][2]);
                            }
                        }
                        if (causal) {
                            gt[q][0] += double(f[q][3]);
                            if (GRAD) {
                                gt[q][1] += double(f[q][4]);
                                gt[q][2] += double(f[q][5]);
                            }
                        }
                    }
                }
                if (causal) {
#pragma unroll
                    for (int q = 0; q < KT; ++q) {
                        const double dn = trn[q] - last;
                        const double fn = exp(-a.omega * dn);
                        acc[q][3] += fn * gt[q][0];
                        if (GRAD) {
                            acc[q][4] += fn * gt[q][1];
                            acc[q][5] += fn * fma(dn, gt[q][0], gt[q][2]);
                        }
                    }
                }
            } else {
                // tiles overlapping the block's time range: per-pair tie-group
                // masks and the triggering time factor formed per pair in FP64
                const float2 *su = T.u;
                for (int m0 = 0; m0 < TS; m0 += GS) {
                    float f[KT][6];
#pragma unroll
                    for (int q = 0; q < KT; ++q)
#pragma unroll
                        for (int z = 0; z < 6; ++z)
                            f[q][z] = -0.0f;
                    for (int j = 0; j < GS; ++j) {
                        const int m = m0 + j;
                        const double xm = sx[m], ym = sy[m], tm = st[m];
                        const float2 rm = sr[m], um = su[m];
                        const float rhm = rm.x, rlm = rm.y, uhm = um.x, ulm = um.y;
                        const int gm = sdg[m].g;
#pragma unroll
                        for (int q = 0; q < KT; ++q) {
                            float D, A, Alo = 0.0f;
                            if (UNI)
                                geom_da_uni(xn[q], yn[q], tsn[q], xm, ym, tm, D, A, Alo);
                            else
                                geom_da(xn[q], yn[q], tsn[q], xm, ym, tm, D, A);
                            const double dt = tsn[q] - tm;
                            float b = __builtin_amdgcn_exp2f(-A);
                            if (UNI)
                                b = fmaf(-LN2F * Alo, b, b);
                            b = (gm != gn[q]) ? b : 0.0f;
                            const float t1 = fmaf(rlm, D, rhm * D);
                            const float arg = float(fma(a.w2, dt, double(t1)));
                            const float E = __builtin_amdgcn_exp2f(-arg);
                            float p = fmaf(ulm, E, uhm * E);
                            p = (gm < gn[q]) ? p : 0.0f;
                            f[q][0] += b;
                            f[q][3] += p;
                            if (GRAD) {
                                if (!UNI)
                                    f[q][1] = fmaf(b, D, f[q][1]);
                                f[q][2] = fmaf(b, A, f[q][2]);
                                f[q][4] = fmaf(p, t1, f[q][4]);
                                f[q][5] = fmaf(p, float(dt), f[q][5]);
                            }
                        }
                    }
#pragma unroll
                    for (int q = 0; q < KT; ++q) {
                        acc[q][0] += double(f[q][0]);
                        acc[q][3] += double(f[q][3]);
                        if (GRAD) {
                            acc[q][1] += double(f[q][1]);
                            acc[q][2] += double(f[q][2]);
                            acc[q][4] += double(f[q][4]);
                            acc[q][5] += double(f[q][5]) * a.inv_st;
                        }
                    }
                }
            }

            stage_wait();
            __syncthreads();

            if (cols) {
                // owner lane of source tid: the four waves' sums in a fixed order
                const int j = k * TS + tid - jb;
                double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    s0 += double(lcol[buf][0][w][tid]);
                    if (GRAD) {
                        s1 += double(lcol[buf][1][w][tid]);
                        s2 += double(lcol[buf][2][w][tid]);
                    }
                }
                pc[j] += s0 * a.out_exp;
                if (GRAD) {
                    if (!UNI)
                        pc[stride + j] += s1 * (a.out_s1 * a.out_exp);
                    pc[2 * stride + j] += (s2 - s1) * (a.out_s2 * a.out_exp);
                }
            }
        }

        // this block's row sums against the column group, in the sums' natural units
        double *out = a.srow + int64_t(slot) * 6 * stride;
#pragma unroll
        for (int q = 0; q < KT; ++q) {
            const int i = i0 + tid + q * WG;
            if (i >= iend)
                continue;
            const int rr = i - a.row_begin - rb0;
            const double ce = a.out_exp;
            out[0 * stride + rr] = acc[q][0] * ce;
            out[3 * stride + rr] = acc[q][3] * ce;
            if (GRAD) {
                out[1 * stride + rr] = acc[q][1] * (a.out_s1 * ce);
                out[2 * stride + rr] = (acc[q][2] - acc[q][1]) * (a.out_s2 * ce);
                out[4 * stride + rr] = acc[q][4] * (a.out_g1 * ce);
                out[5 * stride + rr] = acc[q][5] * ce;
            }
        }
    }
}

// ------------------------------------------------ several theta in one sweep
//
// The forward-only FP32 sweep for NT parameter vectors at once (S0 and G0 of
// each), on the same events and the same work decomposition as k_pair_f32.
// What the vectors share is computed once per pair: the pair differences and
// the squared distance d2 in FP64 and, for vectors after the first, the
// squared time difference.  Positions and times are scaled for theta 0; for
// theta k the squared distance in its own scale is d2 cx_k and the background
// exponent A_k = d2 cx_k + dt^2 ct_k (cx_k = (sx_k / sx_0)^2,
// ct_k = (st_k / st_0)^2), each formed in FP64 and rounded once to FP32, so
// that every FP32 value of theta k is the one a single sweep at theta k forms
// (up to FP64 rounding).  Per-theta source fields: r_m and v_m (hi, lo);
// u_m, the time offsets and tie groups are shared.
// Theta k's row sums go to row-partial slots k (S0) and 3 + k (G0) and its
// column sums to column slot k, so its finalize reads the same layout as a
// single forward-only sweep, offset by k slots.

struct PairBatchF32 {
    const double *xs, *ys, *tsd, *t;  // positions and times scaled for theta 0
    const float2 *r2, *v2;            // theta k's (hi, lo) fields at r2 + k * theta_stride
    const float2 *u2;                 // (hi, lo) of u_m
    const DeltaGroup *dg;
    const int *g;
    const double *tile;
    const int *sblk, *eblk;
    CellMap cells;
    double *srow, *scol;  // slots as in PairF32
    int ge;
    int row_begin, row_end, rows_pad, num_tiles, num_tb;
    int rr, ct;
    int sym, window, trig_cull;
    int theta_stride;
    const unsigned long long *umax;
    double skip_gap;   // the largest over the vectors: tiles that early have no background term
    double omega_min;  // the smallest omega: the latest triggering cut-off
    // (sx_k / sx_0)^2 and (st_k / st_0)^2: theta k's spatial and temporal scales against theta 0's
    double cx[MAX_FUSED_THETA], ct2[MAX_FUSED_THETA], omega[MAX_FUSED_THETA], w2[MAX_FUSED_THETA];
    double out_exp;
};

template <int NT, bool UNI>
__global__ __launch_bounds__(WG) HK_PAIR_ATTR void k_pair_f32_batch(PairBatchF32 a)
{
    static_assert(NT >= 1 && NT <= MAX_FUSED_THETA, "fused theta count");
    struct TileRecs {
        double x[TS], y[TS], t[TS];
        float2 r[NT][TS], v[NT][TS], u[TS];
        DeltaGroup dg[TS];
    };
    __shared__ TileRecs lt2[2];
    __shared__ float lcol[2][NT][NW][TS];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15;
    int gr, gc, slot;
    if (!map_cell(a.cells, blockIdx.x, gr, gc, slot))
        return;
    const int b_first = gr * a.rr;
    const int b_stop = (b_first + a.rr < a.num_tb) ? b_first + a.rr : a.num_tb;
    const int kg0 = gc * a.ct;
    const int kg1 = (kg0 + a.ct < a.num_tiles) ? kg0 + a.ct : a.num_tiles;
    const int64_t stride = a.ge;
    const int jb = kg0 * TS, rb0 = b_first * TB;
    double *pc = a.scol + int64_t(slot) * 3 * stride;
    if (a.sym) {
        for (int k = kg0; k < kg1; ++k)
#pragma unroll
            for (int z = 0; z < NT; ++z)
                pc[z * stride + k * TS + tid - jb] = 0.0;
    }

    auto stage = [&](int k, int buf) {
        TileRecs &T = lt2[buf];
        int o = tid;
        asm volatile("" : "+v"(o));
        const int wb = tid & ~63;
        auto copy = [&](const void *src, void *dst) {
            const unsigned *s = reinterpret_cast<const unsigned *>(src);
            unsigned *d = reinterpret_cast<unsigned *>(dst);
            lds_dma4(s + o, d + wb);
            lds_dma4(s + TS + o, d + TS + wb);
        };
        copy(a.xs + k * TS, T.x);
        copy(a.ys + k * TS, T.y);
        copy(a.tsd + k * TS, T.t);
#pragma unroll
        for (int z = 0; z < NT; ++z) {
            copy(a.r2 + int64_t(z) * a.theta_stride + k * TS, T.r[z]);
            copy(a.v2 + int64_t(z) * a.theta_stride + k * TS, T.v[z]);
        }
        copy(a.u2 + k * TS, T.u);
        copy(a.dg + k * TS, T.dg);
    };

    double cull_gap = a.skip_gap;
    if (a.trig_cull) {
        const double um = __longlong_as_double((long long)*a.umax);
        const double tg = (log(um) + TRIG_SKIP_EXPONENT * LN2) / a.omega_min;
        cull_gap = (tg > cull_gap) ? tg : cull_gap;
    }

    for (int b = b_first; b < b_stop; ++b) {
        const int i0 = a.row_begin + b * TB;
        const int iend = (i0 + TB < a.row_end) ? i0 + TB : a.row_end;
        const double t_lo = a.t[i0], t_hi = a.t[iend - 1];

        double xn[KT], yn[KT], tsn[KT], trn[KT];
        int gn[KT];
#pragma unroll
        for (int q = 0; q < KT; ++q) {
            const int i = i0 + tid + q * WG;
            const bool in = i < iend;
            xn[q] = in ? a.xs[i] : PAD_COORD;
            yn[q] = in ? a.ys[i] : PAD_COORD;
            tsn[q] = in ? a.tsd[i] : PAD_TIME;
            trn[q] = a.t[in ? i : iend - 1];
            gn[q] = in ? a.g[i] : INT_MAX;
        }
        double acc[KT][NT][2];
#pragma unroll
        for (int q = 0; q < KT; ++q)
#pragma unroll
            for (int z = 0; z < NT; ++z)
                acc[q][z][0] = acc[q][z][1] = 0.0;

        int k_strict = 0, k_end = a.num_tiles, k_lo = 0;
        if (a.trig_cull) {
            const double limit = t_lo - cull_gap;
            int lo = 0, hi = a.num_tiles;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (a.tile[3 * mid + 1] < limit)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            k_lo = lo;
        }
        if (a.sym) {
            k_strict = KT * a.sblk[b];
            const int e = KT * a.eblk[b];
            k_end = (e < a.num_tiles) ? e : a.num_tiles;
        } else if (a.window) {
            const double limit = t_hi + a.skip_gap;
            int lo = 0, hi = a.num_tiles;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (a.tile[3 * mid + 0] > limit)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            k_end = lo;
        }
        const int k0 = (kg0 > k_lo) ? kg0 : k_lo;
        const int k1 = (kg1 < k_end) ? kg1 : k_end;

        if (k0 < k1)
            stage(k0, 0);
        stage_wait();
        __syncthreads();

        for (int k = k0; k < k1; ++k) {
            const int buf = (k - k0) & 1;
            if (k + 1 < k1)
                stage(k + 1, buf ^ 1);

            const double first = a.tile[3 * k + 0], last = a.tile[3 * k + 1];
            const int cls = (last < t_lo) ? CAUSAL : ((first > t_hi) ? ANTI : MIXED);
            const bool trig_only = (cls == CAUSAL) && (t_lo - last > a.skip_gap);
            const bool cols = (k < k_strict) && !trig_only;

            double gt[KT][NT];
#pragma unroll
            for (int q = 0; q < KT; ++q)
#pragma unroll
                for (int z = 0; z < NT; ++z)
                    gt[q][z] = 0.0;

            const TileRecs &T = lt2[buf];

            // Per pair: each vector's squared distance in its own spatial scale,
            // d2 cx_z in FP64 rounded once to FP32 (so that its triggering exponent
            // r_m D is rounded as a single sweep at that vector rounds it), and its
            // background term.
            auto pair_terms = [&](double xn_, double yn_, double tn_, double xm, double ym, double tm,
                                  float (&Dz)[NT], float (&bz)[NT]) {
                const double dx = xn_ - xm, dy = yn_ - ym, dt = tn_ - tm;
                const double d2 = fma(dy, dy, dx * dx);
                const double dt2 = dt * dt;
#pragma unroll
                for (int z = 0; z < NT; ++z) {
                    const double dz = (z == 0) ? d2 : d2 * a.cx[z];
                    Dz[z] = float(dz);
                    if (UNI) {
                        const double a2 = (z == 0) ? dt2 : dt2 * a.ct2[z];
                        const float A = float(a2), Alo = float(a2 - double(A));
                        const float e = __builtin_amdgcn_exp2f(-A);
                        bz[z] = fmaf(-LN2F * Alo, e, e);
                    } else {
                        const float A = (z == 0) ? float(fma(dt, dt, d2)) : float(fma(dt2, a.ct2[z], dz));
                        bz[z] = __builtin_amdgcn_exp2f(-A);
                    }
                }
            };
            // squared distances only (triggering terms of tiles without background terms)
            auto dist_terms = [&](double xn_, double yn_, double xm, double ym, float (&Dz)[NT]) {
                const double dx = xn_ - xm, dy = yn_ - ym;
                const double d2 = fma(dy, dy, dx * dx);
#pragma unroll
                for (int z = 0; z < NT; ++z)
                    Dz[z] = float((z == 0) ? d2 : d2 * a.cx[z]);
            };

            if (cls != MIXED) {
                const bool causal = (cls == CAUSAL);
                float e[NT];
                double h[NT];
#pragma unroll
                for (int z = 0; z < NT; ++z) {
                    e[z] = -0.0f;
                    h[z] = 0.0;
                }
                for (int m0 = 0; m0 < TS; m0 += GS) {
                    float f[KT][NT][2];
#pragma unroll
                    for (int q = 0; q < KT; ++q)
#pragma unroll
                        for (int z = 0; z < NT; ++z)
                            f[q][z][0] = f[q][z][1] = -0.0f;
                    // background + triggering terms of source m for the lane's targets;
                    // adds each vector's background terms over those targets to c[z]
                    auto causal_pair = [&](int m, float (&c)[NT]) {
                        const double xm = T.x[m], ym = T.y[m], tm = T.t[m];
#pragma unroll
                        for (int q = 0; q < KT; ++q) {
                            float Dz[NT], bz[NT];
                            pair_terms(xn[q], yn[q], tsn[q], xm, ym, tm, Dz, bz);
#pragma unroll
                            for (int z = 0; z < NT; ++z) {
                                const float2 rm = T.r[z][m], vm = T.v[z][m];
                                const float D = Dz[z];
                                const float t1 = fmaf(rm.y, D, rm.x * D);
                                const float E = __builtin_amdgcn_exp2f(-t1);
                                const float p = fmaf(vm.y, E, vm.x * E);
                                f[q][z][0] += bz[z];
                                f[q][z][1] += p;
                                c[z] += bz[z];
                            }
                        }
                    };
                    auto trig_pair = [&](int m) {
                        const double xm = T.x[m], ym = T.y[m];
#pragma unroll
                        for (int q = 0; q < KT; ++q) {
                            float Dz[NT];
                            dist_terms(xn[q], yn[q], xm, ym, Dz);
#pragma unroll
                            for (int z = 0; z < NT; ++z) {
                                const float2 rm = T.r[z][m], vm = T.v[z][m];
                                const float D = Dz[z];
                                const float t1 = fmaf(rm.y, D, rm.x * D);
                                const float E = __builtin_amdgcn_exp2f(-t1);
                                f[q][z][1] += fmaf(vm.y, E, vm.x * E);
                            }
                        }
                    };
                    const int sub = m0 & ~15, s0 = m0 & 15;
                    if (trig_only) {
                        HK_UNROLL(HAWKES_UJ)
                        for (int j = 0; j < GS; ++j)
                            trig_pair(m0 + j);
                    } else if (cols) {
                        HK_UNROLL(HAWKES_UJ)
                        for (int j = 0; j < GS; ++j) {
                            float c[NT];
#pragma unroll
                            for (int z = 0; z < NT; ++z)
                                c[z] = -0.0f;
                            causal_pair(sub + ((li + s0 + j) & 15), c);
#pragma unroll
                            for (int z = 0; z < NT; ++z)
                                e[z] = row_rotate_f32(e[z]) + c[z];
                        }
                        if (s0 == 0) {
#pragma unroll
                            for (int z = 0; z < NT; ++z)
                                h[z] = double(e[z]);
                        } else {
                            double w[NT];
#pragma unroll
                            for (int z = 0; z < NT; ++z)
                                w[z] = sum_rows_f64(row_shift8_f64(h[z]) + double(e[z]));
                            if (lane < 16) {
                                const int mc = sub + ((li + 15) & 15);
#pragma unroll
                                for (int z = 0; z < NT; ++z)
                                    lcol[buf][z][wave][mc] = float(w[z]);
                            }
                        }
#pragma unroll
                        for (int z = 0; z < NT; ++z)
                            e[z] = -0.0f;
                    } else if (causal) {
                        HK_UNROLL(HAWKES_UJ)
                        for (int j = 0; j < GS; ++j) {
                            float c[NT];
#pragma unroll
                            for (int z = 0; z < NT; ++z)
                                c[z] = -0.0f;
                            causal_pair(m0 + j, c);  // column sums unused
                        }
                    } else {
                        HK_UNROLL(HAWKES_UJ)
                        for (int j = 0; j < GS; ++j) {
                            const int m = m0 + j;
                            const double xm = T.x[m], ym = T.y[m], tm = T.t[m];
#pragma unroll
                            for (int q = 0; q < KT; ++q) {
                                float Dz[NT], bz[NT];
                                pair_terms(xn[q], yn[q], tsn[q], xm, ym, tm, Dz, bz);
#pragma unroll
                                for (int z = 0; z < NT; ++z)
                                    f[q][z][0] += bz[z];
                            }
                        }
                    }
#pragma unroll
                    for (int q = 0; q < KT; ++q)
#pragma unroll
                        for (int z = 0; z < NT; ++z) {
                            if (!trig_only)
                                acc[q][z][0] += double(f[q][z][0]);
                            if (causal)
                                gt[q][z] += double(f[q][z][1]);
                        }
                }
                if (causal) {
#pragma unroll
                    for (int q = 0; q < KT; ++q) {
                        const double dn = trn[q] - last;
#pragma unroll
                        for (int z = 0; z < NT; ++z)
                            acc[q][z][1] += exp(-a.omega[z] * dn) * gt[q][z];
                    }
                }
            } else {
                // tiles overlapping the block's time range: tie-group masks and the
                // triggering time factor per pair in FP64
                for (int m0 = 0; m0 < TS; m0 += GS) {
                    float f[KT][NT][2];
#pragma unroll
                    for (int q = 0; q < KT; ++q)
#pragma unroll
                        for (int z = 0; z < NT; ++z)
                            f[q][z][0] = f[q][z][1] = -0.0f;
                    for (int j = 0; j < GS; ++j) {
                        const int m = m0 + j;
                        const double xm = T.x[m], ym = T.y[m], tm = T.t[m];
                        const float2 um = T.u[m];
                        const int gm = T.dg[m].g;
#pragma unroll
                        for (int q = 0; q < KT; ++q) {
                            float Dz[NT], bz[NT];
                            pair_terms(xn[q], yn[q], tsn[q], xm, ym, tm, Dz, bz);
                            const double dt = tsn[q] - tm;
#pragma unroll
                            for (int z = 0; z < NT; ++z) {
                                const float2 rm = T.r[z][m];
                                const float D = Dz[z];
                                const float b = (gm != gn[q]) ? bz[z] : 0.0f;
                                const float t1 = fmaf(rm.y, D, rm.x * D);
                                const float arg = float(fma(a.w2[z], dt, double(t1)));
                                const float E = __builtin_amdgcn_exp2f(-arg);
                                const float p = fmaf(um.y, E, um.x * E);
                                f[q][z][0] += b;
                                f[q][z][1] += (gm < gn[q]) ? p : 0.0f;
                            }
                        }
                    }
#pragma unroll
                    for (int q = 0; q < KT; ++q)
#pragma unroll
                        for (int z = 0; z < NT; ++z) {
                            acc[q][z][0] += double(f[q][z][0]);
                            acc[q][z][1] += double(f[q][z][1]);
                        }
                }
            }

            stage_wait();
            __syncthreads();

            if (cols) {
                const int j = k * TS + tid - jb;
#pragma unroll
                for (int z = 0; z < NT; ++z) {
                    double s = 0.0;
#pragma unroll
                    for (int w = 0; w < NW; ++w)
                        s += double(lcol[buf][z][w][tid]);
                    pc[z * stride + j] += s * a.out_exp;
                }
            }
        }

        double *out = a.srow + int64_t(slot) * 6 * stride;
#pragma unroll
        for (int q = 0; q < KT; ++q) {
            const int i = i0 + tid + q * WG;
            if (i >= iend)
                continue;
            const int rr = i - a.row_begin - rb0;
#pragma unroll
            for (int z = 0; z < NT; ++z) {
                out[z * stride + rr] = acc[q][z][0] * a.out_exp;
                out[(3 + z) * stride + rr] = acc[q][z][1] * a.out_exp;
            }
        }
    }
}

// Block bounds of the symmetric sweep: for each target block b, sblk[b] is
// the first block whose last time is >= b's first time, eblk[b] the first
// block whose first time is > b's last time (num_tb if none).
__global__ __launch_bounds__(256) void k_sym_bounds(const double *__restrict__ t, int64_t n, int64_t num_tb,
                                                    int *__restrict__ sblk, int *__restrict__ eblk)
{
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= num_tb)
        return;
    auto first_t = [&](int64_t c) { return t[c * TB]; };
    auto last_t = [&](int64_t c) {
        const int64_t e = (c + 1) * TB;
        return t[(e < n ? e : n) - 1];
    };
    const double tl = first_t(b), th = last_t(b);
    int64_t lo = 0, hi = b;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (last_t(mid) < tl)
            lo = mid + 1;
        else
            hi = mid;
    }
    sblk[b] = int(lo);
    lo = b + 1;
    hi = num_tb;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (first_t(mid) > th)
            hi = mid;
        else
            lo = mid + 1;
    }
    eblk[b] = int(lo);
}

// Cells of the symmetric sweep (one workgroup): row group gr reaches column
// groups 0..gchi[gr] (nondecreasing in gr), its cells are numbered from
// rowstart[gr] on (latest row groups first: rowstart[num_gr - 1] = 0),
// column group gc is reached by row groups g0[gc]..num_gr-1, and *total is
// the number of cells.
__global__ __launch_bounds__(256) void k_sym_plan(const int *__restrict__ eblk, int64_t num_tb, int64_t num_tiles,
                                                  int rr, int ct, int num_gr, int num_gc, int *__restrict__ gchi,
                                                  int *__restrict__ g0, int *__restrict__ rowstart,
                                                  int *__restrict__ total)
{
    __shared__ int hi[MAX_SYM_GROUPS];
    for (int g = threadIdx.x; g < num_gr; g += blockDim.x) {
        const int64_t bl = ((int64_t(g) + 1) * rr < num_tb ? (int64_t(g) + 1) * rr : num_tb) - 1;
        const int64_t e = KT * int64_t(eblk[bl]);
        const int64_t kend = (e < num_tiles) ? e : num_tiles;
        hi[g] = int((kend + ct - 1) / ct) - 1;
        gchi[g] = hi[g];
    }
    __syncthreads();
    for (int c = threadIdx.x; c < num_gc; c += blockDim.x) {
        int g = 0;
        while (g < num_gr && hi[g] < c)
            ++g;
        g0[c] = g;
    }
    if (threadIdx.x == 0) {
        int start = 0;
        for (int g = num_gr - 1; g >= 0; --g) {
            rowstart[g] = start;
            start += hi[g] + 1;
        }
        *total = start;
    }
}

// Per-row accumulators cleared before the first pass (a kernel rather than a
// memset node, so that callers may capture the call in a graph).
__global__ __launch_bounds__(256) void k_zero(double *__restrict__ p, int64_t count)
{
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < count)
        p[i] = 0.0;
}

// Fold of one pass: adds the slots of the pass's cells into the per-row FP64
// accumulators, cell by cell in their launch order, so that the sums (and so
// the results) do not depend on where passes begin and end.  Row sums of row
// r come from the cells of its row group (column groups from the earliest
// up); in the symmetric sweep its column sums come from the cells of its
// column group (row groups from the latest down).
struct FoldArgs {
    CellMap m;
    const int *g0;            // symmetric sweep: first row group reaching each column group
    int ncells;               // cells of this pass: m.cell0 .. m.cell0 + ncells - 1
    int rr, ct, ge, sym;
    int rowmask, colmask;     // which of the 6 row and 3 column sums the sweep wrote
    int64_t rows, rows_pad;
    const double *srow, *scol;
    double *acc_row, *acc_col;  // [6][rows_pad], [3][rows_pad]
};

// Cells of pass [c0, c1) that hold row sums of row r: row group gr, cells
// [lo, hi) (empty if lo >= hi).
__host__ __device__ inline void fold_row_cells(const CellMap &m, bool sym, int rr, int64_t r, int c0, int c1,
                                               int &gr, int &lo, int &hi)
{
    gr = int((r / TB) / rr);
    int rs, nc;
    if (sym) {
        rs = m.rowstart[gr];
        nc = m.gchi[gr] + 1;
    } else {
        rs = (m.num_gr - 1 - gr) * m.num_gc;
        nc = m.num_gc;
    }
    lo = rs > c0 ? rs : c0;
    hi = (rs + nc < c1) ? rs + nc : c1;
}

// Symmetric sweep: cells of pass [c0, c1) that hold column sums of source r:
// column group gc, row groups g from gmax down to gmin (cell rowstart[g] + gc,
// which decreases with g; empty if gmin > gmax).
__host__ __device__ inline void fold_col_cells(const CellMap &m, const int *g0, int ct, int64_t r, int c0, int c1,
                                               int &gc, int &gmin, int &gmax)
{
    gc = int((r / TS) / ct);
    const int gfirst = g0[gc];
    int lo = gfirst, hi = m.num_gr;  // first g whose cell comes before c0
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (m.rowstart[mid] + gc < c0)
            hi = mid;
        else
            lo = mid + 1;
    }
    gmax = lo - 1;
    lo = gfirst;
    hi = m.num_gr;  // first g whose cell comes before c1
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (m.rowstart[mid] + gc < c1)
            hi = mid;
        else
            lo = mid + 1;
    }
    gmin = lo;
}

__global__ __launch_bounds__(256) void k_fold(FoldArgs a)
{
    const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (r >= a.rows)
        return;
    const int c0 = a.m.cell0, c1 = c0 + a.ncells;
    if (a.sym && c0 >= *a.m.total)
        return;
    {
        int gr, lo, hi;
        fold_row_cells(a.m, a.sym != 0, a.rr, r, c0, c1, gr, lo, hi);
        if (lo < hi) {
            const int64_t rel = r - int64_t(gr) * a.rr * TB;
            double v[6];
#pragma unroll
            for (int z = 0; z < 6; ++z)
                v[z] = ((a.rowmask >> z) & 1) ? a.acc_row[z * a.rows_pad + r] : 0.0;
            for (int c = lo; c < hi; ++c) {
                const double *p = a.srow + int64_t(c - c0) * 6 * a.ge + rel;
#pragma unroll
                for (int z = 0; z < 6; ++z)
                    if ((a.rowmask >> z) & 1)
                        v[z] += p[z * a.ge];
            }
#pragma unroll
            for (int z = 0; z < 6; ++z)
                if ((a.rowmask >> z) & 1)
                    a.acc_row[z * a.rows_pad + r] = v[z];
        }
    }
    if (a.sym && a.colmask) {
        int gc, gmin, gmax;
        fold_col_cells(a.m, a.g0, a.ct, r, c0, c1, gc, gmin, gmax);
        if (gmin <= gmax) {
            const int64_t rel = r - int64_t(gc) * a.ct * TS;
            double v[3];
#pragma unroll
            for (int z = 0; z < 3; ++z)
                v[z] = ((a.colmask >> z) & 1) ? a.acc_col[z * a.rows_pad + r] : 0.0;
            for (int g = gmax; g >= gmin; --g) {
                const double *p = a.scol + int64_t(a.m.rowstart[g] + gc - c0) * 3 * a.ge + rel;
#pragma unroll
                for (int z = 0; z < 3; ++z)
                    if ((a.colmask >> z) & 1)
                        v[z] += p[z * a.ge];
            }
#pragma unroll
            for (int z = 0; z < 3; ++z)
                if ((a.colmask >> z) & 1)
                    a.acc_col[z * a.rows_pad + r] = v[z];
        }
    }
}

struct PairF64 {
    const double *t, *x, *y, *s;
    const int *g;
    const double *tile;
    const int *sblk, *eblk;  // symmetric sweep: block order bounds (as in PairF32)
    CellMap cells;
    double *srow, *scol;     // slots as in PairF32
    int ge;
    int n, row_begin, row_end, rows_pad, num_tiles, num_tb;
    int rr, ct, sym;
    double ax, at, qh, omega;  // log2(e) times: 1/(2 tau_x^2), 1/(2 tau_t^2), 1/(2 h0^2), omega
};

// 2^y for y <= 0 in FP64 (the pair terms of the FP64 sweep, whose exponents are
// formed in units of log2): y = k + f with k = rint(y) and |f| <= 1/2, 2^f from
// the Taylor series of e^(f ln 2) to degree 12 (truncation below 2.4e-16
// relative for |f ln 2| <= 0.35, of one sign and about 1e-18 on average over
// f) by Horner's rule, then scaled by 2^k (the
// classical reduction of Cody and Waite, with the reduction exact here because
// the base is 2).  Exponents below -2000 give 0.
constexpr double exp2_taylor_coef(int n)
{
    double c = 1.0;
    for (int i = 1; i <= n; ++i)
        c = c * 0.69314718055994530942 / double(i);
    return c;
}
__device__ __forceinline__ double exp2_nonpos(double y)
{
    y = fmax(y, -2000.0);
    const double k = rint(y);
    const double f = y - k;
    double p = exp2_taylor_coef(12);
    p = fma(p, f, exp2_taylor_coef(11));
    p = fma(p, f, exp2_taylor_coef(10));
    p = fma(p, f, exp2_taylor_coef(9));
    p = fma(p, f, exp2_taylor_coef(8));
    p = fma(p, f, exp2_taylor_coef(7));
    p = fma(p, f, exp2_taylor_coef(6));
    p = fma(p, f, exp2_taylor_coef(5));
    p = fma(p, f, exp2_taylor_coef(4));
    p = fma(p, f, exp2_taylor_coef(3));
    p = fma(p, f, exp2_taylor_coef(2));
    p = fma(p, f, exp2_taylor_coef(1));
    p = fma(p, f, 1.0);
    return ldexp(p, int(k));
}

__device__ __forceinline__ double row_rotate_f64(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = dpp_mov<DPP_ROW_ROR15>(int(unsigned(u))), hi = dpp_mov<DPP_ROW_ROR15>(int(unsigned(u >> 32)));
    return make_f64(unsigned(lo), unsigned(hi));
}

// The FP64 sweep: every pair term in FP64 with the direct formulas, on the
// same work decomposition as the FP32 sweep (row groups x column groups; over
// the whole event set the symmetric sweep, with the background column sums of
// a strictly earlier tile carried by the 16-lane rotation in FP64, summed over
// the 4 rows and the 4 waves and added to this row group's column partials).
template <bool GRAD>
__global__ __launch_bounds__(WG) void k_pair_f64(PairF64 a)
{
    __shared__ double lx[2][TS], ly[2][TS], lt[2][TS], lu[2][TS], lq[2][TS];  // lq: u_m qh
    __shared__ int lg[2][TS];
    __shared__ double lcol[3][NW][TS];  // per-wave column sums of the tile just swept

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15;
    int gr, gc, slot;
    if (!map_cell(a.cells, blockIdx.x, gr, gc, slot))
        return;
    const int b_first = gr * a.rr;
    const int b_stop = (b_first + a.rr < a.num_tb) ? b_first + a.rr : a.num_tb;
    const int kg0 = gc * a.ct;
    const int kg1 = (kg0 + a.ct < a.num_tiles) ? kg0 + a.ct : a.num_tiles;
    const int64_t stride = a.ge;
    const int jb = kg0 * TS, rb0 = b_first * TB;
    double *pc = a.scol + int64_t(slot) * 3 * stride;
    if (a.sym) {
        for (int k = kg0; k < kg1; ++k) {
            const int j = k * TS + tid - jb;
            pc[j] = 0.0;
            if (GRAD) {
                pc[stride + j] = 0.0;
                pc[2 * stride + j] = 0.0;
            }
        }
    }

    auto fetch = [&](int j, double &fx, double &fy, double &ft, double &fu, double &fq, int &fg) {
        if (j < a.n) {
            fx = a.x[j];
            fy = a.y[j];
            ft = a.t[j];
            const double sj = a.s[j];
            fu = 1.0 / (sj * sj);
            fq = fu * a.qh;
            fg = a.g[j];
        } else {
            fx = PAD_COORD;
            fy = PAD_COORD;
            ft = PAD_TIME;
            fu = 0.0;
            fq = 0.0;
            fg = INT_MAX;
        }
    };

    for (int b = b_first; b < b_stop; ++b) {
        const int i0 = a.row_begin + b * TB;
        const int iend = (i0 + TB < a.row_end) ? i0 + TB : a.row_end;
        const double t_lo = a.t[i0], t_hi = a.t[iend - 1];
        // lanes past the block's end take a target far away: all of its terms are 0
        double xn[KT], yn[KT], tn[KT];
        int gn[KT];
#pragma unroll
        for (int q = 0; q < KT; ++q) {
            const int i = i0 + tid + q * WG;
            const bool in = i < iend;
            xn[q] = in ? a.x[i] : PAD_COORD;
            yn[q] = in ? a.y[i] : PAD_COORD;
            tn[q] = in ? a.t[i] : PAD_TIME;
            gn[q] = in ? a.g[i] : INT_MAX;
        }
        double acc[KT][6];
#pragma unroll
        for (int q = 0; q < KT; ++q)
#pragma unroll
            for (int z = 0; z < 6; ++z)
                acc[q][z] = 0.0;

        int k_strict = 0, k_end = a.num_tiles;
        if (a.sym) {
            k_strict = KT * a.sblk[b];
            const int e = KT * a.eblk[b];
            k_end = (e < a.num_tiles) ? e : a.num_tiles;
        }
        const int k0 = kg0;
        const int k1 = (kg1 < k_end) ? kg1 : k_end;

        if (k0 < k1) {
            double fx, fy, ft, fu, fq;
            int fg;
            fetch(k0 * TS + tid, fx, fy, ft, fu, fq, fg);
            lx[0][tid] = fx;
            ly[0][tid] = fy;
            lt[0][tid] = ft;
            lu[0][tid] = fu;
            lq[0][tid] = fq;
            lg[0][tid] = fg;
        }
        __syncthreads();

        for (int k = k0; k < k1; ++k) {
            const int buf = (k - k0) & 1;
            const bool more = (k + 1 < k1);
            double px = 0, py = 0, pt = 0, pu = 0, pq = 0;
            int pg = 0;
            if (more)
                fetch((k + 1) * TS + tid, px, py, pt, pu, pq, pg);

            const double first = a.tile[3 * k + 0], last = a.tile[3 * k + 1];
            const int cls = (last < t_lo) ? CAUSAL : ((first > t_hi) ? ANTI : MIXED);
            const bool cols = k < k_strict;  // strictly earlier block (so CAUSAL, whole tile)

            // background and triggering terms of source m for the lane's targets
            auto pair = [&](int m, bool use_bg_all, double &c0, double &c1, double &c2) {
                const double xm = lx[buf][m], ym = ly[buf][m], tm = lt[buf][m], um = lu[buf][m];
                const double uq = lq[buf][m];
                const int gm = lg[buf][m];
#pragma unroll
                for (int q = 0; q < KT; ++q) {
                    const double dx = xn[q] - xm, dy = yn[q] - ym;
                    const double d2 = fma(dy, dy, dx * dx);
                    const double dt = tn[q] - tm;
                    const double dt2 = dt * dt;
                    const bool use_b = use_bg_all || (gm != gn[q]);
                    const bool use_g = (cls == CAUSAL) || (cls == MIXED && gm < gn[q]);
                    if (use_b) {
                        const double bb = exp2_nonpos(-fma(a.at, dt2, a.ax * d2));
                        acc[q][0] += bb;
                        c0 += bb;
                        if (GRAD) {
                            const double bd = bb * d2, bt = bb * dt2;
                            acc[q][1] += bd;
                            acc[q][2] += bt;
                            c1 += bd;
                            c2 += bt;
                        }
                    }
                    if (use_g) {
                        const double e = um * exp2_nonpos(-fma(uq, d2, a.omega * dt));
                        acc[q][3] += e;
                        if (GRAD) {
                            acc[q][4] = fma(e, um * d2, acc[q][4]);
                            acc[q][5] = fma(e, dt, acc[q][5]);
                        }
                    }
                }
            };

            if (cols) {
                // 16-lane rotation: lane i takes source m0 + ((i + j) mod 16) at step j
                for (int m0 = 0; m0 < TS; m0 += 16) {
                    double e0 = 0.0, e1 = 0.0, e2 = 0.0;
                    for (int j = 0; j < 16; ++j) {
                        double c0 = -0.0, c1 = -0.0, c2 = -0.0;  // -0: first addition folds away
                        pair(m0 + ((li + j) & 15), true, c0, c1, c2);
                        e0 = row_rotate_f64(e0) + c0;
                        if (GRAD) {
                            e1 = row_rotate_f64(e1) + c1;
                            e2 = row_rotate_f64(e2) + c2;
                        }
                    }
                    // lane i of each row holds the row's sums of source m0 + ((i + 15) mod 16)
                    e0 = sum_rows_f64(e0);
                    if (GRAD) {
                        e1 = sum_rows_f64(e1);
                        e2 = sum_rows_f64(e2);
                    }
                    if (lane < 16) {
                        const int mc = m0 + ((li + 15) & 15);
                        lcol[0][wave][mc] = e0;
                        if (GRAD) {
                            lcol[1][wave][mc] = e1;
                            lcol[2][wave][mc] = e2;
                        }
                    }
                }
            } else {
                const int mlen = (k * TS + TS <= a.n) ? TS : a.n - k * TS;
                for (int m = 0; m < mlen; ++m) {
                    double c0 = -0.0, c1 = -0.0, c2 = -0.0;  // -0: first addition folds away
                    pair(m, cls != MIXED, c0, c1, c2);  // column sums unused
                }
            }

            if (more) {
                const int nb = buf ^ 1;
                lx[nb][tid] = px;
                ly[nb][tid] = py;
                lt[nb][tid] = pt;
                lu[nb][tid] = pu;
                lq[nb][tid] = pq;
                lg[nb][tid] = pg;
            }
            __syncthreads();
            if (cols) {
                // owner lane of source tid: the four waves' sums in a fixed order
                const int j = k * TS + tid - jb;
                double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    s0 += lcol[0][w][tid];
                    if (GRAD) {
                        s1 += lcol[1][w][tid];
                        s2 += lcol[2][w][tid];
                    }
                }
                pc[j] += s0;
                if (GRAD) {
                    pc[stride + j] += s1;
                    pc[2 * stride + j] += s2;
                }
                __syncthreads();  // lcol is written again by the next tile's columns
            }
        }

        double *out = a.srow + int64_t(slot) * 6 * stride;
#pragma unroll
        for (int q = 0; q < KT; ++q) {
            const int i = i0 + tid + q * WG;
            if (i >= iend)
                continue;
            const int rr = i - a.row_begin - rb0;
            out[0 * stride + rr] = acc[q][0];
            out[3 * stride + rr] = acc[q][3];
            if (GRAD) {
                out[1 * stride + rr] = acc[q][1];
                out[2 * stride + rr] = acc[q][2];
                out[4 * stride + rr] = acc[q][4];
                out[5 * stride + rr] = acc[q][5];
            }
        }
    }
}

struct Fin {
    const double *t, *x, *y, *s;   // raw events (the rescue sweep reads them)
    const int *g;                  // tie-group ids
    const double *acc_row;         // folded row sums [6][rows_pad]
    const double *acc_col;         // symmetric sweep: folded column sums [3][rows_pad]
    int *status;                   // [0] flags, [1] rescue count
    int *rescue;                   // rescue list of row offsets
    double *rowvals;               // [7][rows_cap] per-row l_n and gradient terms
    double *lam_out, *comp_out;
    int64_t n, row_begin, rows, rows_pad, rows_cap;
    int sym;
    double mu, tau_x, tau_t, xi, h0, omega, c_b, c_g;
    double ax, at, qh;             // 1/(2 tau_x^2), 1/(2 tau_t^2), 1/(2 h0^2)
    double rescue_lambda;          // FP32 rows with lambda below this are recomputed (0: never)
    int uniform;                   // spatially uniform background: no tau_x dependence
};

__device__ inline double std_normal_cdf(double z) { return 0.5 * erfc(-z * 0.70710678118654752440); }
__device__ inline double std_normal_pdf(double z) { return 0.39894228040143267794 * exp(-0.5 * z * z); }

// From the six pair sums of row i (natural units): l_n, its six gradient
// terms, lambda_n and Lambda_n, all FP64.
template <bool GRAD>
__device__ void row_terms(const Fin &f, const double S[6], double ti, double tN, double v[7], double &lam,
                          double &comp)
{
    const double B = f.c_b * S[0];
    const double T = f.c_g * S[3];
    lam = f.mu * B + f.xi * T;
    const bool floored = !(lam >= LAMBDA_FLOOR);
    const double av = tN - ti;
    const double bg = std_normal_cdf(av / f.tau_t) - std_normal_cdf(-ti / f.tau_t);
    const double ea = exp(-f.omega * av);
    comp = f.mu * bg + f.xi * (1.0 - ea);
    v[0] = log(floored ? LAMBDA_FLOOR : lam) - comp;
    if (GRAD) {
        const double tx = f.tau_x, tt = f.tau_t, h0 = f.h0, om = f.omega;
        double dl[6] = {0, 0, 0, 0, 0, 0};
        if (!floored) {
            const double il = 1.0 / lam;
            dl[0] = B * il;
            dl[1] = f.uniform ? 0.0 : f.mu * f.c_b * (S[1] / (tx * tx * tx) - 2.0 * S[0] / tx) * il;
            dl[2] = f.mu * f.c_b * (S[2] / (tt * tt * tt) - S[0] / tt) * il;
            dl[3] = T * il;
            dl[4] = f.xi * f.c_g * (S[4] / (h0 * h0 * h0) - 2.0 * S[3] / h0) * il;
            dl[5] = f.xi * f.c_g * (S[3] / om - S[5]) * il;
        }
        const double dcomp_taut = -(f.mu / (tt * tt)) * (av * std_normal_pdf(av / tt) + ti * std_normal_pdf(ti / tt));
        v[1] = dl[0] - bg;
        v[2] = dl[1];
        v[3] = dl[2] - dcomp_taut;
        v[4] = dl[3] - (1.0 - ea);
        v[5] = dl[4];
        v[6] = dl[5] - f.xi * av * ea;
    }
}

// Per-row FP64 finalize: the row's folded sums (row sums, plus in the
// symmetric sweep the background column sums), then lambda_n, the floored
// log, gradient terms and the compensator.
template <bool GRAD>
__global__ __launch_bounds__(256) void k_finalize(Fin f)
{
    const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (r >= f.rows)
        return;
    double S[6] = {0, 0, 0, 0, 0, 0};
    S[0] = f.acc_row[r];
    S[3] = f.acc_row[3 * f.rows_pad + r];
    if (GRAD) {
        S[1] = f.acc_row[1 * f.rows_pad + r];
        S[2] = f.acc_row[2 * f.rows_pad + r];
        S[4] = f.acc_row[4 * f.rows_pad + r];
        S[5] = f.acc_row[5 * f.rows_pad + r];
    }
    if (f.sym) {
        S[0] += f.acc_col[r];
        if (GRAD) {
            S[1] += f.acc_col[1 * f.rows_pad + r];
            S[2] += f.acc_col[2 * f.rows_pad + r];
        }
    }
    const int64_t i = f.row_begin + r;
    double v[7] = {0, 0, 0, 0, 0, 0, 0}, lam, comp;
    row_terms<GRAD>(f, S, f.t[i], f.t[f.n - 1], v, lam, comp);
    if (lam < f.rescue_lambda) {
        const int slot = atomicAdd(&f.status[1], 1);
        f.rescue[slot] = int(r);
    }
    const int nv = GRAD ? 7 : 1;
    for (int z = 0; z < nv; ++z)
        f.rowvals[z * f.rows_cap + r] = v[z];
    if (f.lam_out)
        f.lam_out[r] = lam;
    if (f.comp_out)
        f.comp_out[r] = comp;
}

// FP64 rescue: rows whose FP32 rate is underflow-limited are swept again
// with every pair in FP64 (one workgroup per row, lanes strided over
// sources), and their row values are replaced.  Workgroups stride over the
// rescue list, so the grid size is independent of its length.
template <bool GRAD>
__global__ __launch_bounds__(256) void k_rescue(Fin f)
{
    __shared__ double red[6][256];
    const int tid = threadIdx.x;
    const int count = f.status[1];
    for (int w = blockIdx.x; w < count; w += gridDim.x) {
        const int64_t r = f.rescue[w];
        const int64_t i = f.row_begin + r;
        const double xn = f.x[i], yn = f.y[i], tn = f.t[i];
        const int gn = f.g[i];
        double S[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t m = tid; m < f.n; m += 256) {
            const int gm = f.g[m];
            if (gm == gn)
                continue;
            const double dx = xn - f.x[m], dy = yn - f.y[m];
            const double d2 = dx * dx + dy * dy;
            const double dt = tn - f.t[m];
            const double b = exp(-(f.ax * d2 + f.at * dt * dt));
            S[0] += b;
            S[1] += b * d2;
            S[2] += b * dt * dt;
            if (gm < gn) {
                const double sm = f.s[m];
                const double um = 1.0 / (sm * sm);
                const double e = um * exp(-(um * f.qh * d2 + f.omega * dt));
                S[3] += e;
                S[4] += e * (um * d2);
                S[5] += e * dt;
            }
        }
        for (int z = 0; z < 6; ++z)
            red[z][tid] = S[z];
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (tid < h)
                for (int z = 0; z < 6; ++z)
                    red[z][tid] += red[z][tid + h];
            __syncthreads();
        }
        if (tid == 0) {
            double T6[6], v[7] = {0, 0, 0, 0, 0, 0, 0}, lam, comp;
            for (int z = 0; z < 6; ++z)
                T6[z] = red[z][0];
            row_terms<GRAD>(f, T6, tn, f.t[f.n - 1], v, lam, comp);
            const int nv = GRAD ? 7 : 1;
            for (int z = 0; z < nv; ++z)
                f.rowvals[z * f.rows_cap + r] = v[z];
            if (f.lam_out)
                f.lam_out[r] = lam;
        }
        __syncthreads();
    }
}

// Fixed-order block sums of the row values.
template <bool GRAD>
__global__ __launch_bounds__(256) void k_blocksum(const double *__restrict__ rowvals, int64_t rows, int64_t rows_cap,
                                                  double *__restrict__ blocks)
{
    __shared__ double red[7][256];
    const int tid = threadIdx.x;
    const int64_t r = int64_t(blockIdx.x) * 256 + tid;
    const int nv = GRAD ? 7 : 1;
    for (int z = 0; z < nv; ++z)
        red[z][tid] = (r < rows) ? rowvals[z * rows_cap + r] : 0.0;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w)
            for (int z = 0; z < nv; ++z)
                red[z][tid] += red[z][tid + w];
        __syncthreads();
    }
    if (tid == 0)
        for (int z = 0; z < nv; ++z)
            blocks[blockIdx.x * 7 + z] = red[z][0];
}

template <bool GRAD>
__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ blocks, int64_t nblk, const int *status,
                                                double *loglik, double *grad)
{
    __shared__ double red[7][256];
    const int tid = threadIdx.x;
    const int nv = GRAD ? 7 : 1;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t b = tid; b < nblk; b += 256)
        for (int z = 0; z < nv; ++z)
            v[z] += blocks[b * 7 + z];
    for (int z = 0; z < nv; ++z)
        red[z][tid] = v[z];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w)
            for (int z = 0; z < nv; ++z)
                red[z][tid] += red[z][tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        const bool bad = status[0] != 0;
        const double nan = __builtin_nan("");
        if (loglik)
            loglik[0] = bad ? nan : red[0][0];
        if (GRAD && grad)
            for (int z = 0; z < 6; ++z)
                grad[z] = bad ? nan : red[1 + z][0];
    }
}

// Per-row outputs of hawkes_event_terms become NaN when the data checks failed.
__global__ void k_poison_rows(const int *status, double *lam, double *comp, int64_t rows)
{
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= rows || status[0] == 0)
        return;
    const double nan = __builtin_nan("");
    if (lam)
        lam[r] = nan;
    if (comp)
        comp[r] = nan;
}

// ------------------------------------------------------------ host side

thread_local char g_errbuf[512];

// Per-call tuning and timing (hawkes_options; defaults when absent).
struct Tuning {
    int64_t row_wgs = DEFAULT_ROW_WGS;
    int sym_groups = DEFAULT_SYM_GROUPS;  // 0: whole-set calls take the row sweep
    hipEvent_t t_start = nullptr, t_stop = nullptr;
};

int parse_options(const hawkes_options *o, Tuning &T)
{
    if (!o)
        return HAWKES_OK;
    if (o->row_workgroups != 0) {
        if (o->row_workgroups < 1 || o->row_workgroups > MAX_ROW_WGS) {
            set_error("row_workgroups %lld outside [1, %lld]", (long long)o->row_workgroups,
                      (long long)MAX_ROW_WGS);
            return HAWKES_EINVAL;
        }
        T.row_wgs = o->row_workgroups;
    }
    if (o->symmetric_groups != 0) {
        if (o->symmetric_groups < -1 || o->symmetric_groups > MAX_SYM_GROUPS) {
            set_error("symmetric_groups %d outside [-1, %d]", int(o->symmetric_groups), MAX_SYM_GROUPS);
            return HAWKES_EINVAL;
        }
        T.sym_groups = o->symmetric_groups < 0 ? 0 : int(o->symmetric_groups);
    }
    if (o->reserved != 0) {
        set_error("hawkes_options.reserved must be 0");
        return HAWKES_EINVAL;
    }
    if ((o->timing_start == nullptr) != (o->timing_stop == nullptr)) {
        set_error("timing_start and timing_stop must both be set or both be NULL");
        return HAWKES_EINVAL;
    }
    T.t_start = reinterpret_cast<hipEvent_t>(o->timing_start);
    T.t_stop = reinterpret_cast<hipEvent_t>(o->timing_stop);
    return HAWKES_OK;
}

int validate(const hawkes_events *ev, const hawkes_theta *th, int precision, int64_t rb, int64_t re, const void *ws,
             size_t ws_bytes, Layout *L)
{
    if (!ev || !th) {
        set_error("null events or theta");
        return HAWKES_EINVAL;
    }
    if (ev->n < 1 || ev->n > MAX_N) {
        set_error("n = %lld outside [1, %lld]", (long long)ev->n, (long long)MAX_N);
        return HAWKES_EINVAL;
    }
    if (!ev->t || !ev->x || !ev->y || !ev->s) {
        set_error("null event array");
        return HAWKES_EINVAL;
    }
    if (!(ev->area >= 0.0) || !std::isfinite(ev->area)) {
        set_error("background area %g is not finite and >= 0", ev->area);
        return HAWKES_EINVAL;
    }
    if (!valid_precision(precision)) {
        set_error("precision %d is not HAWKES_FP64, HAWKES_FP32 or HAWKES_FP32_SKIP", precision);
        return HAWKES_EINVAL;
    }
    const double p[6] = {th->mu, th->tau_x, th->tau_t, th->xi, th->h0, th->omega};
    for (int k = 0; k < 6; ++k)
        if (!(p[k] > 0.0) || !std::isfinite(p[k])) {
            set_error("theta component %d = %g is not finite and positive", k, p[k]);
            return HAWKES_EINVAL;
        }
    if (rb < 0 || re > ev->n || rb > re) {
        set_error("row range [%lld, %lld) not within [0, %lld]", (long long)rb, (long long)re, (long long)ev->n);
        return HAWKES_ERANGE;
    }
    *L = make_layout(ev->n, precision);
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0 || ws_bytes < L->minimum) {
        set_error("workspace %p of %zu bytes; need at least %zu bytes (%zu recommended), 256-byte aligned", ws,
                  ws_bytes, L->minimum, L->total);
        return HAWKES_EWORKSPACE;
    }
    return HAWKES_OK;
}

int record_event(hipEvent_t ev, hipStream_t stream)
{
    const hipError_t e = hipEventRecord(ev, stream);
    return e == hipSuccess ? HAWKES_OK : hip_failure(e, "hipEventRecord");
}

template <typename T>
T *at(void *ws, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

enum Mode { MODE_LOGLIK, MODE_GRAD, MODE_TERMS };

// What every call stages before its pair sweep: tie groups, tile time ranges
// and data checks; the work plan (cells and passes); for the symmetric sweep
// its block bounds and cell numbering.
struct Setup {
    Plan P;
    SymPlan SP;
    bool sym = false, uniform = false;
    int grid_rr = 1, grid_ct = 1;
    unsigned stage_blocks = 0;
    int64_t n = 0, rb = 0, re = 0, rows = 0;
    int *status = nullptr, *g = nullptr, *sblk = nullptr, *eblk = nullptr, *g0 = nullptr;
    double *tile = nullptr, *acc_row = nullptr, *acc_col = nullptr;
    CellMap cells;
    int ge = TB;
    size_t cell_bytes = 0, slot_avail = 0;
    int64_t cells_ub = 0, cap = 0, passes = 0;
    double *srow = nullptr, *scol = nullptr;
};

int setup(const hawkes_events *ev, int64_t rb, int64_t re, void *ws, size_t ws_bytes, const Layout &L,
          const Tuning &T, hipStream_t stream, Setup &S)
{
    int rc;
    S.n = ev->n;
    S.rb = rb;
    S.re = re;
    S.rows = re - rb;
    S.uniform = ev->area > 0.0;
    S.status = at<int>(ws, L.status);
    S.g = at<int>(ws, L.g);
    S.tile = at<double>(ws, L.tile);
    S.sblk = at<int>(ws, L.sblk);
    S.eblk = at<int>(ws, L.eblk);
    S.g0 = at<int>(ws, L.g0);

    // the plan, and whether one cell's slot fits, before any work is enqueued
    S.P = make_plan(S.rows > 0 ? S.rows : 1, L.num_tiles, T.row_wgs);
    // the symmetric sweep covers the whole event set; a row range takes the row sweep
    S.sym = T.sym_groups > 0 && rb == 0 && re == S.n;
    S.SP = S.sym ? make_sym_plan(S.P.num_tb, L.num_tiles, T.sym_groups) : SymPlan{};
    S.cell_bytes = S.sym ? sym_cell_bytes(S.SP) : row_cell_bytes();
    S.slot_avail = ws_bytes - L.slots;
    if (S.slot_avail < S.cell_bytes) {
        set_error("workspace of %zu bytes leaves %zu bytes of slots; one cell of this plan needs %zu", ws_bytes,
                  S.slot_avail, S.cell_bytes);
        return HAWKES_EWORKSPACE;
    }

    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, stream, S.status);
    S.stage_blocks = unsigned(ceil_div(L.n_pad, 256));
    hipLaunchKernelGGL(k_stage_common, dim3(S.stage_blocks), dim3(256), 0, stream, ev->t, ev->x, ev->y, ev->s, S.n,
                       L.n_pad, S.g, S.tile, S.status);
    if ((rc = check_launch("stage_common")) != HAWKES_OK || S.rows == 0)
        return rc;

    int *rowstart = at<int>(ws, L.rowstart);
    if (S.sym) {
        hipLaunchKernelGGL(k_sym_bounds, dim3(unsigned(ceil_div(S.P.num_tb, 256))), dim3(256), 0, stream, ev->t,
                           S.n, S.P.num_tb, S.sblk, S.eblk);
        if ((rc = check_launch("sym_bounds")) != HAWKES_OK)
            return rc;
        hipLaunchKernelGGL(k_sym_plan, dim3(1), dim3(256), 0, stream, S.eblk, S.P.num_tb, L.num_tiles, S.SP.rr,
                           S.SP.ct, S.SP.num_gr, S.SP.num_gc, at<int>(ws, L.gchi), S.g0, rowstart,
                           rowstart + MAX_SYM_GROUPS);
        if ((rc = check_launch("sym_plan")) != HAWKES_OK)
            return rc;
    }
    // cells: row groups x column groups (the symmetric plan), or target blocks x source chunks
    S.grid_rr = S.sym ? S.SP.rr : 1;
    S.grid_ct = S.sym ? S.SP.ct : int(S.P.chunk_tiles);
    S.cells.num_gr = S.sym ? S.SP.num_gr : int(S.P.num_tb);
    S.cells.num_gc = S.sym ? S.SP.num_gc : int(S.P.num_chunks);
    if (S.sym) {
        S.cells.rowstart = rowstart;
        S.cells.gchi = at<int>(ws, L.gchi);
        S.cells.total = rowstart + MAX_SYM_GROUPS;
    }
    S.ge = S.sym ? S.SP.rr * TB : TB;
    S.cells_ub = int64_t(S.cells.num_gr) * S.cells.num_gc;
    S.acc_row = at<double>(ws, L.acc);
    S.acc_col = S.acc_row + 6 * S.P.rows_pad;
    S.srow = at<double>(ws, L.slots);
    return HAWKES_OK;
}

// Workgroups of `kernel` the device runs at once (0 if unknown).
int device_concurrency(const void *kernel)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, WG, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return cus * per_cu;
}

// Pass plan: as many cells per pass as the slot region holds, rounded down to
// whole rounds of the workgroups the device runs at once (so that a pass ends
// without a ragged round of its own).
void plan_passes(Setup &S, const void *kernel)
{
    int64_t cap = int64_t(S.slot_avail / S.cell_bytes);
    if (cap >= S.cells_ub)
        cap = S.cells_ub;
    else {
        const int64_t conc = device_concurrency(kernel);
        if (conc > 0 && cap > conc)
            cap -= cap % conc;
    }
    S.cap = cap;
    S.passes = ceil_div(S.cells_ub, cap);
    S.scol = S.srow + cap * 6 * S.ge;  // symmetric sweep: column slots after the row slots
}

// Runs the sweep pass by pass: clears the accumulators, then for each pass
// launches the pair kernel over its cells (launch(cell0, grid)) and folds the
// slots.  The caller's timing events bracket the passes.
template <typename Launch>
int sweep_passes(const Setup &S, const Tuning &T, int rowmask, int colmask, hipStream_t stream, Launch launch)
{
    int rc;
    const int64_t acc_count = 9 * S.P.rows_pad;
    hipLaunchKernelGGL(k_zero, dim3(unsigned(ceil_div(acc_count, 256))), dim3(256), 0, stream, S.acc_row,
                       acc_count);
    if ((rc = check_launch("zero")) != HAWKES_OK)
        return rc;
    if (T.t_start && (rc = record_event(T.t_start, stream)) != HAWKES_OK)
        return rc;
    FoldArgs fa;
    fa.m = S.cells;
    fa.g0 = S.g0;
    fa.rr = S.grid_rr;
    fa.ct = S.grid_ct;
    fa.ge = S.ge;
    fa.sym = S.sym ? 1 : 0;
    fa.rowmask = rowmask;
    fa.colmask = S.sym ? colmask : 0;
    fa.rows = S.rows;
    fa.rows_pad = S.P.rows_pad;
    fa.srow = S.srow;
    fa.scol = S.scol;
    fa.acc_row = S.acc_row;
    fa.acc_col = S.acc_col;
    for (int64_t p = 0; p < S.passes; ++p) {
        const int64_t cell0 = p * S.cap;
        const int64_t grid = (S.cells_ub - cell0 < S.cap) ? S.cells_ub - cell0 : S.cap;
        launch(int(cell0), unsigned(grid));
        if ((rc = check_launch("pair sweep")) != HAWKES_OK)
            return rc;
        fa.m.cell0 = int(cell0);
        fa.m.ncells = int(grid);
        fa.ncells = int(grid);
        hipLaunchKernelGGL(k_fold, dim3(unsigned(ceil_div(S.rows, 256))), dim3(256), 0, stream, fa);
        if ((rc = check_launch("fold")) != HAWKES_OK)
            return rc;
    }
    if (T.t_stop && (rc = record_event(T.t_stop, stream)) != HAWKES_OK)
        return rc;
    return HAWKES_OK;
}

// FP32 source staging scales: positions by the background's spatial scale
// (or by the triggering bandwidth h0 when the background is spatially
// uniform), times by the temporal one.
StageF32 stage_scales(const hawkes_theta *th, bool uniform)
{
    StageF32 sc;
    const double tau_sp = uniform ? th->h0 : th->tau_x;
    sc.sx = std::sqrt(LOG2E / (2.0 * tau_sp * tau_sp));
    sc.st = std::sqrt(LOG2E / (2.0 * th->tau_t * th->tau_t));
    sc.rr = (tau_sp / th->h0) * (tau_sp / th->h0);
    sc.omega = th->omega;
    return sc;
}

// The sweep's cell and slot fields shared by the pair kernels.
template <typename A>
void fill_grid(A &a, const Setup &S, const Layout &L)
{
    a.tile = S.tile;
    a.sblk = S.sblk;
    a.eblk = S.eblk;
    a.cells = S.cells;
    a.srow = S.srow;
    a.scol = S.scol;
    a.ge = S.ge;
    a.row_begin = int(S.rb);
    a.row_end = int(S.re);
    a.rows_pad = int(S.P.rows_pad);
    a.num_tiles = int(L.num_tiles);
    a.num_tb = int(S.P.num_tb);
    a.rr = S.grid_rr;
    a.ct = S.grid_ct;
    a.sym = S.sym ? 1 : 0;
}

Fin make_fin(const hawkes_events *ev, const hawkes_theta *th, int precision, const Setup &S, const Layout &L,
             void *ws, double *d_lam, double *d_comp)
{
    const double tau_x = th->tau_x, tau_t = th->tau_t, h0 = th->h0, omega = th->omega;
    Fin f;
    f.t = ev->t;
    f.x = ev->x;
    f.y = ev->y;
    f.s = ev->s;
    f.g = S.g;
    f.acc_row = S.acc_row;
    f.acc_col = S.acc_col;
    f.status = S.status;
    f.rescue = at<int>(ws, L.rescue);
    f.rowvals = at<double>(ws, L.rowvals);
    f.lam_out = d_lam;
    f.comp_out = d_comp;
    f.n = S.n;
    f.row_begin = S.rb;
    f.rows = S.rows;
    f.rows_pad = S.P.rows_pad;
    f.rows_cap = L.rows_cap;
    f.sym = S.sym ? 1 : 0;
    f.mu = th->mu;
    f.tau_x = tau_x;
    f.tau_t = tau_t;
    f.xi = th->xi;
    f.h0 = h0;
    f.omega = omega;
    f.uniform = S.uniform ? 1 : 0;
    f.c_b = S.uniform ? 1.0 / (ev->area * std::sqrt(2.0 * M_PI) * tau_t)
                      : 1.0 / (std::pow(2.0 * M_PI, 1.5) * tau_x * tau_x * tau_t);
    f.c_g = omega / (2.0 * M_PI * h0 * h0);
    f.ax = S.uniform ? 0.0 : 1.0 / (2.0 * tau_x * tau_x);
    f.at = 1.0 / (2.0 * tau_t * tau_t);
    f.qh = 1.0 / (2.0 * h0 * h0);
    // Each FP32 pair term below 2^-126 may be lost to underflow; n of them
    // bound the loss by n 2^-126 (mu c_b + xi c_g).  Rows whose rate is not
    // 1/RESCUE_REL times larger than that are recomputed in FP64.
    f.rescue_lambda = is_fp32(precision)
                          ? double(S.n) * std::ldexp(1.0, -126) * (f.mu * f.c_b + f.xi * f.c_g) / RESCUE_REL
                          : 0.0;
    return f;
}

// After the pair sweep: per-row finalize, FP64 rescue (FP32), and either the
// per-row outputs or the fixed-order reduction.
int finish(const Fin &f, const Setup &S, const Layout &L, void *ws, int precision, Mode mode, double *d_loglik,
           double *d_grad, double *d_lam, double *d_comp, hipStream_t stream)
{
    int rc;
    const bool grad = (mode == MODE_GRAD);
    const int64_t nblk = ceil_div(S.rows, 256);
    if (grad)
        hipLaunchKernelGGL(k_finalize<true>, dim3(unsigned(nblk)), dim3(256), 0, stream, f);
    else
        hipLaunchKernelGGL(k_finalize<false>, dim3(unsigned(nblk)), dim3(256), 0, stream, f);
    if ((rc = check_launch("finalize")) != HAWKES_OK)
        return rc;
    if (is_fp32(precision)) {
        const unsigned rescue_wgs = unsigned(nblk < 256 ? nblk : 256);
        if (grad)
            hipLaunchKernelGGL(k_rescue<true>, dim3(rescue_wgs), dim3(256), 0, stream, f);
        else
            hipLaunchKernelGGL(k_rescue<false>, dim3(rescue_wgs), dim3(256), 0, stream, f);
        if ((rc = check_launch("rescue")) != HAWKES_OK)
            return rc;
    }
    if (mode == MODE_TERMS) {
        hipLaunchKernelGGL(k_poison_rows, dim3(unsigned(nblk)), dim3(256), 0, stream, S.status, d_lam, d_comp,
                           S.rows);
        return check_launch("poison_rows");
    }
    double *blocks = at<double>(ws, L.blocks);
    if (grad)
        hipLaunchKernelGGL(k_blocksum<true>, dim3(unsigned(nblk)), dim3(256), 0, stream, f.rowvals, S.rows,
                           L.rows_cap, blocks);
    else
        hipLaunchKernelGGL(k_blocksum<false>, dim3(unsigned(nblk)), dim3(256), 0, stream, f.rowvals, S.rows,
                           L.rows_cap, blocks);
    if ((rc = check_launch("blocksum")) != HAWKES_OK)
        return rc;
    if (grad)
        hipLaunchKernelGGL(k_reduce<true>, dim3(1), dim3(256), 0, stream, blocks, nblk, S.status, d_loglik, d_grad);
    else
        hipLaunchKernelGGL(k_reduce<false>, dim3(1), dim3(256), 0, stream, blocks, nblk, S.status, d_loglik,
                           nullptr);
    return check_launch("reduce");
}

int run(const hawkes_events *ev, const hawkes_theta *th, int precision, int64_t rb, int64_t re, void *ws,
        size_t ws_bytes, const hawkes_options *opts, double *d_loglik, double *d_grad, double *d_lam,
        double *d_comp, Mode mode, void *stream_)
{
    Tuning T;
    int rc = parse_options(opts, T);
    if (rc != HAWKES_OK)
        return rc;
    Layout L;
    if ((rc = validate(ev, th, precision, rb, re, ws, ws_bytes, &L)) != HAWKES_OK)
        return rc;
    if (mode != MODE_TERMS && !d_loglik) {
        set_error("null loglik output");
        return HAWKES_EINVAL;
    }
    if (mode == MODE_GRAD && !d_grad) {
        set_error("null gradient output");
        return HAWKES_EINVAL;
    }
    hipStream_t stream = as_stream(stream_);
    const bool grad = (mode == MODE_GRAD);
    Setup S;
    if ((rc = setup(ev, rb, re, ws, ws_bytes, L, T, stream, S)) != HAWKES_OK)
        return rc;
    if (S.rows == 0) {
        if (mode != MODE_TERMS)
            hipLaunchKernelGGL(k_zero_outputs, dim3(1), dim3(64), 0, stream, d_loglik, grad ? d_grad : nullptr);
        return check_launch("zero_outputs");
    }
    const double h0 = th->h0, omega = th->omega;
    const bool uniform = S.uniform;
    // row sums written by the sweeps: all six with the gradient, S0 and G0 without
    const int rowmask = grad ? 0x3F : 0x09, colmask = grad ? 0x7 : 0x1;

    if (is_fp32(precision)) {
        const StageF32 sc = stage_scales(th, uniform);
        double *xs = at<double>(ws, L.xs), *ys = at<double>(ws, L.ys), *tsd = at<double>(ws, L.tsd);
        float2 *r2 = at<float2>(ws, L.r2), *v2 = at<float2>(ws, L.v2), *u2 = at<float2>(ws, L.u2);
        DeltaGroup *dg = at<DeltaGroup>(ws, L.dg);
        hipLaunchKernelGGL(k_stage_f32, dim3(S.stage_blocks), dim3(256), 0, stream, ev->t, ev->x, ev->y, ev->s,
                           S.g, S.n, L.n_pad, sc, S.tile, xs, ys, tsd, r2, v2, u2, dg);
        if ((rc = check_launch("stage_f32")) != HAWKES_OK)
            return rc;
        const void *kfn = grad ? (uniform ? reinterpret_cast<const void *>(&k_pair_f32<true, true>)
                                          : reinterpret_cast<const void *>(&k_pair_f32<true, false>))
                               : (uniform ? reinterpret_cast<const void *>(&k_pair_f32<false, true>)
                                          : reinterpret_cast<const void *>(&k_pair_f32<false, false>));
        plan_passes(S, kfn);
        PairF32 a;
        fill_grid(a, S, L);
        a.xs = xs;
        a.ys = ys;
        a.tsd = tsd;
        a.t = ev->t;
        a.r2 = r2;
        a.v2 = v2;
        a.u2 = u2;
        a.dg = dg;
        a.g = S.g;
        a.omega = omega;
        a.inv_st = 1.0 / sc.st;
        a.out_s1 = uniform ? 0.0 : 1.0 / (sc.sx * sc.sx);  // D = d^2 sx^2
        a.out_s2 = 1.0 / (sc.st * sc.st);        // dt' = dt st
        a.out_g1 = 2.0 * h0 * h0 / LOG2E;        // t1 = u d^2 log2(e) / (2 h0^2)
        a.w2 = omega * LOG2E / sc.st;
        a.out_exp = 1.0 / (1.0 + EXP2_MEAN_REL_ERR);
        a.umax = reinterpret_cast<const unsigned long long *>(S.status) + STATUS_UMAX;
        if (precision == HAWKES_FP32_SKIP) {
            // scaled time gap whose square exceeds 160: exp2(-A) <= 2^-160 is 0 in FP32
            a.skip_gap = std::sqrt(SKIP_EXPONENT) / sc.st;
            a.window = 1;
            a.trig_cull = 1;
            hipLaunchKernelGGL(k_umax, dim3(unsigned(ceil_div(S.n, 256))), dim3(256), 0, stream, ev->s, S.n,
                               S.status);
            if ((rc = check_launch("umax")) != HAWKES_OK)
                return rc;
        } else {
            a.skip_gap = HUGE_VAL;
            a.window = 0;
            a.trig_cull = 0;
        }
        rc = sweep_passes(S, T, rowmask, colmask, stream, [&](int cell0, unsigned grid) {
            a.cells.cell0 = cell0;
            a.cells.ncells = int(grid);
            if (grad && uniform)
                hipLaunchKernelGGL((k_pair_f32<true, true>), dim3(grid), dim3(WG), 0, stream, a);
            else if (grad)
                hipLaunchKernelGGL((k_pair_f32<true, false>), dim3(grid), dim3(WG), 0, stream, a);
            else if (uniform)
                hipLaunchKernelGGL((k_pair_f32<false, true>), dim3(grid), dim3(WG), 0, stream, a);
            else
                hipLaunchKernelGGL((k_pair_f32<false, false>), dim3(grid), dim3(WG), 0, stream, a);
        });
        if (rc != HAWKES_OK)
            return rc;
    } else {
        const void *kfn = grad ? reinterpret_cast<const void *>(&k_pair_f64<true>)
                               : reinterpret_cast<const void *>(&k_pair_f64<false>);
        plan_passes(S, kfn);
        PairF64 a;
        a.t = ev->t;
        a.x = ev->x;
        a.y = ev->y;
        a.s = ev->s;
        a.g = S.g;
        a.tile = S.tile;
        a.sblk = S.sblk;
        a.eblk = S.eblk;
        a.cells = S.cells;
        a.srow = S.srow;
        a.scol = S.scol;
        a.ge = S.ge;
        a.n = int(S.n);
        a.row_begin = int(rb);
        a.row_end = int(re);
        a.rows_pad = int(S.P.rows_pad);
        a.num_tiles = int(L.num_tiles);
        a.num_tb = int(S.P.num_tb);
        a.rr = S.grid_rr;
        a.ct = S.grid_ct;
        a.sym = S.sym ? 1 : 0;
        // exponents in units of log2 (the sweep's exp2); uniform background: no spatial factor
        a.ax = uniform ? 0.0 : LOG2E / (2.0 * th->tau_x * th->tau_x);
        a.at = LOG2E / (2.0 * th->tau_t * th->tau_t);
        a.qh = LOG2E / (2.0 * h0 * h0);
        a.omega = omega * LOG2E;
        rc = sweep_passes(S, T, rowmask, colmask, stream, [&](int cell0, unsigned grid) {
            a.cells.cell0 = cell0;
            a.cells.ncells = int(grid);
            if (grad)
                hipLaunchKernelGGL(k_pair_f64<true>, dim3(grid), dim3(WG), 0, stream, a);
            else
                hipLaunchKernelGGL(k_pair_f64<false>, dim3(grid), dim3(WG), 0, stream, a);
        });
        if (rc != HAWKES_OK)
            return rc;
    }

    const Fin f = make_fin(ev, th, precision, S, L, ws, d_lam, d_comp);
    return finish(f, S, L, ws, precision, mode, d_loglik, d_grad, d_lam, d_comp, stream);
}

// Several parameter vectors on the same events and rows.  FP32: pairs of
// vectors share one forward-only sweep (k_pair_f32_batch), a vector left over
// takes the single sweep; FP64: one sweep per vector.
int run_batch(const hawkes_events *ev, const hawkes_theta *th, int64_t num_theta, int precision, int64_t rb,
              int64_t re, void *ws, size_t ws_bytes, const hawkes_options *opts, double *d_loglik, void *stream_)
{
    if (!th || num_theta < 1) {
        set_error("need at least one theta (got %lld, pointer %p)", (long long)num_theta, (const void *)th);
        return HAWKES_EINVAL;
    }
    if (!d_loglik) {
        set_error("null loglik output");
        return HAWKES_EINVAL;
    }
    Tuning T;
    int rc = parse_options(opts, T);
    if (rc != HAWKES_OK)
        return rc;
    Layout L;
    for (int64_t k = 0; k < num_theta; ++k)
        if ((rc = validate(ev, th + k, precision, rb, re, ws, ws_bytes, &L)) != HAWKES_OK)
            return rc;
    if (!is_fp32(precision) || num_theta == 1 || re == rb) {
        for (int64_t k = 0; k < num_theta; ++k)
            if ((rc = run(ev, th + k, precision, rb, re, ws, ws_bytes, opts, d_loglik + k, nullptr, nullptr,
                          nullptr, MODE_LOGLIK, stream_)) != HAWKES_OK)
                return rc;
        return HAWKES_OK;
    }
    hipStream_t stream = as_stream(stream_);
    Setup S;
    if ((rc = setup(ev, rb, re, ws, ws_bytes, L, T, stream, S)) != HAWKES_OK)
        return rc;
    if (precision == HAWKES_FP32_SKIP) {
        hipLaunchKernelGGL(k_umax, dim3(unsigned(ceil_div(S.n, 256))), dim3(256), 0, stream, ev->s, S.n, S.status);
        if ((rc = check_launch("umax")) != HAWKES_OK)
            return rc;
    }
    const void *kfn = S.uniform ? reinterpret_cast<const void *>(&k_pair_f32_batch<MAX_FUSED_THETA, true>)
                                : reinterpret_cast<const void *>(&k_pair_f32_batch<MAX_FUSED_THETA, false>);
    plan_passes(S, kfn);
    double *xs = at<double>(ws, L.xs), *ys = at<double>(ws, L.ys), *tsd = at<double>(ws, L.tsd);
    float2 *r2 = at<float2>(ws, L.r2), *v2 = at<float2>(ws, L.v2), *u2 = at<float2>(ws, L.u2);
    DeltaGroup *dg = at<DeltaGroup>(ws, L.dg);
    int64_t k = 0;
    for (; k + MAX_FUSED_THETA <= num_theta; k += MAX_FUSED_THETA) {
        const hawkes_theta *t0 = th + k;
        const StageF32 sc0 = stage_scales(t0, S.uniform);
        hipLaunchKernelGGL(k_stage_f32, dim3(S.stage_blocks), dim3(256), 0, stream, ev->t, ev->x, ev->y, ev->s,
                           S.g, S.n, L.n_pad, sc0, S.tile, xs, ys, tsd, r2, v2, u2, dg);
        if ((rc = check_launch("stage_f32")) != HAWKES_OK)
            return rc;
        PairBatchF32 a;
        fill_grid(a, S, L);
        a.xs = xs;
        a.ys = ys;
        a.tsd = tsd;
        a.t = ev->t;
        a.r2 = r2;
        a.v2 = v2;
        a.u2 = u2;
        a.dg = dg;
        a.g = S.g;
        a.theta_stride = int(L.n_pad);
        a.umax = reinterpret_cast<const unsigned long long *>(S.status) + STATUS_UMAX;
        a.out_exp = 1.0 / (1.0 + EXP2_MEAN_REL_ERR);
        double max_tau_t = 0.0, min_omega = HUGE_VAL;
        const double tau_sp0 = S.uniform ? t0->h0 : t0->tau_x;
        for (int z = 0; z < MAX_FUSED_THETA; ++z) {
            const hawkes_theta *tz = t0 + z;
            const double tau_sp = S.uniform ? tz->h0 : tz->tau_x;
            if (z > 0) {
                // theta z's r_m (for its own position scale) and v_m
                const double rr = (tau_sp / tz->h0) * (tau_sp / tz->h0);
                hipLaunchKernelGGL(k_stage_f32_rv, dim3(S.stage_blocks), dim3(256), 0, stream, ev->t, ev->s, S.n,
                                   L.n_pad, rr, tz->omega, S.tile, r2 + int64_t(z) * L.n_pad,
                                   v2 + int64_t(z) * L.n_pad);
                if ((rc = check_launch("stage_f32_rv")) != HAWKES_OK)
                    return rc;
            }
            a.cx[z] = (tau_sp0 / tau_sp) * (tau_sp0 / tau_sp);
            a.ct2[z] = (t0->tau_t / tz->tau_t) * (t0->tau_t / tz->tau_t);
            a.omega[z] = tz->omega;
            a.w2[z] = tz->omega * LOG2E / sc0.st;
            max_tau_t = std::fmax(max_tau_t, tz->tau_t);
            min_omega = std::fmin(min_omega, tz->omega);
        }
        a.omega_min = min_omega;
        if (precision == HAWKES_FP32_SKIP) {
            // every vector's background term is exactly zero past the largest gap
            a.skip_gap = std::sqrt(SKIP_EXPONENT) / std::sqrt(LOG2E / (2.0 * max_tau_t * max_tau_t));
            a.window = 1;
            a.trig_cull = 1;
        } else {
            a.skip_gap = HUGE_VAL;
            a.window = 0;
            a.trig_cull = 0;
        }
        // vector z's S0 and G0 go to row sums z and 3 + z, its column sums to z
        rc = sweep_passes(S, T, 0x1B, 0x3, stream, [&](int cell0, unsigned grid) {
            a.cells.cell0 = cell0;
            a.cells.ncells = int(grid);
            if (S.uniform)
                hipLaunchKernelGGL((k_pair_f32_batch<MAX_FUSED_THETA, true>), dim3(grid), dim3(WG), 0, stream, a);
            else
                hipLaunchKernelGGL((k_pair_f32_batch<MAX_FUSED_THETA, false>), dim3(grid), dim3(WG), 0, stream,
                                   a);
        });
        if (rc != HAWKES_OK)
            return rc;
        for (int z = 0; z < MAX_FUSED_THETA; ++z) {
            // vector z's sums sit z rows further on in the accumulators
            Fin f = make_fin(ev, t0 + z, precision, S, L, ws, nullptr, nullptr);
            f.acc_row = S.acc_row + int64_t(z) * S.P.rows_pad;
            f.acc_col = S.acc_col + int64_t(z) * S.P.rows_pad;
            hipLaunchKernelGGL(k_clear_rescue, dim3(1), dim3(1), 0, stream, S.status);
            if ((rc = check_launch("clear_rescue")) != HAWKES_OK)
                return rc;
            if ((rc = finish(f, S, L, ws, precision, MODE_LOGLIK, d_loglik + k + z, nullptr, nullptr, nullptr,
                             stream)) != HAWKES_OK)
                return rc;
        }
    }
    for (; k < num_theta; ++k)
        if ((rc = run(ev, th + k, precision, rb, re, ws, ws_bytes, opts, d_loglik + k, nullptr, nullptr, nullptr,
                      MODE_LOGLIK, stream_)) != HAWKES_OK)
            return rc;
    return HAWKES_OK;
}

}  // namespace


void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_errbuf, sizeof(g_errbuf), fmt, ap);
    va_end(ap);
}

int hip_failure(hipError_t e, const char *what)
{
    set_error("%s: %s", what, hipGetErrorString(e));
    return HAWKES_EHIP;
}

int check_launch(const char *what)
{
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HAWKES_OK : hip_failure(e, what);
}

}  // namespace hawkes

// ------------------------------------------------------------------ C ABI

using namespace hawkes;

extern "C" size_t hawkes_workspace_bytes(int64_t n, int precision)
{
    if (n < 1 || n > MAX_N || !valid_precision(precision))
        return 0;
    return make_layout(n, precision).total;
}

// ------------------------------------------------ the entry point that allocates nothing
//
// hawkes_loglik_grad_noalloc takes its workspace from a file-scope device
// array: every GPU the library runs on holds one copy of it at its own
// address until the process ends.  Host code never names the array as a
// pointer (that would be a host-side stand-in, not a device address): the
// device address is looked up once per device with hipGetSymbolAddress and
// kept.  Calls on one GPU share the array, so calls that overlap on one GPU
// race; every call clears what must start at zero (status word,
// accumulators) and stages the rest afresh.

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mutex;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The current device's address of `scratch` (looked up on the first call on that device).
int scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_failure(e, "hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        set_error("device %d beyond the %d devices hawkes_loglik_grad_noalloc supports", dev, NOALLOC_MAX_DEVICES);
        return HAWKES_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_failure(e, "hipGetSymbolAddress(scratch)");
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255u) != 0) {
            set_error("scratch array of device %d at %p is not 256-byte aligned", dev, p);
            return HAWKES_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HAWKES_OK;
}

}  // namespace

extern "C" int hawkes_loglik_grad_noalloc(const hawkes_events *events, const hawkes_theta *theta, int precision,
                                          int64_t row_begin, int64_t row_end, double *d_loglik, double *d_grad,
                                          const hawkes_options *opts, void *stream)
{
    // host-side checks first (with a placeholder workspace address), so that invalid calls touch no device
    Layout L;
    int rc = validate(events, theta, precision, row_begin, row_end, reinterpret_cast<void *>(uintptr_t(256)),
                      SIZE_MAX, &L);
    if (rc != HAWKES_OK)
        return rc;
    if (L.minimum > NOALLOC_SCRATCH_BYTES) {
        set_error("n = %lld needs a workspace of at least %zu bytes at this precision; the static scratch of "
                  "hawkes_loglik_grad_noalloc holds %zu bytes",
                  (long long)events->n, L.minimum, NOALLOC_SCRATCH_BYTES);
        return HAWKES_EWORKSPACE;
    }
    void *ws = nullptr;
    if ((rc = scratch_address(&ws)) != HAWKES_OK)
        return rc;
    return run(events, theta, precision, row_begin, row_end, ws, NOALLOC_SCRATCH_BYTES, opts, d_loglik, d_grad,
               nullptr, nullptr, MODE_GRAD, stream);
}

extern "C" size_t hawkes_workspace_min_bytes(int64_t n, int precision)
{
    if (n < 1 || n > MAX_N || !valid_precision(precision))
        return 0;
    return make_layout(n, precision).minimum;
}

extern "C" int hawkes_loglik(const hawkes_events *events, const hawkes_theta *theta, int precision,
                             int64_t row_begin, int64_t row_end, void *ws, size_t ws_bytes, double *d_loglik,
                             const hawkes_options *opts, void *stream)
{
    return run(events, theta, precision, row_begin, row_end, ws, ws_bytes, opts, d_loglik, nullptr, nullptr,
               nullptr, MODE_LOGLIK, stream);
}

extern "C" int hawkes_loglik_grad(const hawkes_events *events, const hawkes_theta *theta, int precision,
                                  int64_t row_begin, int64_t row_end, void *ws, size_t ws_bytes, double *d_loglik,
                                  double *d_grad, const hawkes_options *opts, void *stream)
{
    return run(events, theta, precision, row_begin, row_end, ws, ws_bytes, opts, d_loglik, d_grad, nullptr,
               nullptr, MODE_GRAD, stream);
}

extern "C" int hawkes_event_terms(const hawkes_events *events, const hawkes_theta *theta, int precision,
                                  int64_t row_begin, int64_t row_end, void *ws, size_t ws_bytes, double *d_lambda,
                                  double *d_comp, const hawkes_options *opts, void *stream)
{
    return run(events, theta, precision, row_begin, row_end, ws, ws_bytes, opts, nullptr, nullptr, d_lambda,
               d_comp, MODE_TERMS, stream);
}

extern "C" int hawkes_loglik_batch(const hawkes_events *events, const hawkes_theta *thetas, int64_t num_theta,
                                   int precision, int64_t row_begin, int64_t row_end, void *ws, size_t ws_bytes,
                                   double *d_loglik, const hawkes_options *opts, void *stream)
{
    return run_batch(events, thetas, num_theta, precision, row_begin, row_end, ws, ws_bytes, opts, d_loglik,
                     stream);
}

extern "C" int hawkes_workspace_status(const void *ws, int *status, void *stream)
{
    if (!ws || !status) {
        set_error("null workspace or status pointer");
        return HAWKES_EINVAL;
    }
    int word = 0;
    hipError_t e = hipStreamSynchronize(as_stream(stream));
    if (e != hipSuccess)
        return hip_failure(e, "hipStreamSynchronize");
    e = hipMemcpy(&word, ws, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_failure(e, "hipMemcpy(status)");
    *status = (word & STATUS_DATA) ? HAWKES_EDATA : ((word & STATUS_ORDER) ? HAWKES_EORDER : HAWKES_OK);
    return HAWKES_OK;
}

extern "C" const char *hawkes_strerror(int status)
{
    switch (status) {
    case HAWKES_OK: return "ok";
    case HAWKES_EINVAL: return "invalid argument";
    case HAWKES_ERANGE: return "row range out of bounds";
    case HAWKES_EWORKSPACE: return "workspace missing, misaligned or too small";
    case HAWKES_EHIP: return "HIP runtime error";
    case HAWKES_EORDER: return "event times are not sorted";
    case HAWKES_EDATA: return "non-finite event data or non-positive bandwidth scale";
    default: return "unknown status";
    }
}

extern "C" const char *hawkes_last_error(void) { return g_errbuf; }
