/*
 * gl.h -- C ABI of libgl, an MI355X (gfx950) implementation of the explicit
 * Grunwald-Letnikov (GL) scheme for the fractional reaction-diffusion
 * equation d^gamma u / dt^gamma = alpha Lap u + f(u) (Sprouse, MacDonald &
 * Silva, arXiv:1004.5128, Sec. 1 eq. (1) and Sec. 2).
 *
 * The scheme (Sec. 2.2, eq. (21)), on a grid u[k] with k = t / dt:
 *
 *   u[k+1] = u[k] + dt f(u[k]) + r * sum_{(m,c) in sched(k)} c psi(gamma,m) delta[k-m]
 *
 *   r        = alpha dt^gamma / dx^2
 *   psi      = (-1)^m binom(1 - gamma, m)           (Sec. 2.1, eqs. (8), (11), (12))
 *   delta[j] = 5-point (2D), 3-point (1D) or 7-point (3D) un-normalised
 *              Laplacian of u[j] with zero values outside the grid
 *              (eq. (17), eq. (15); 3D sums the same over a third axis)
 *   sched(k) = the memory mode's (offset m, multiplicity c) pairs:
 *              full memory   m = 0..k, c = 1          (eq. (21))
 *              short memory  m = 0..min(L, k), c = 1  (eq. (22), L in steps)
 *              adaptive      base [0, a] then intervals sampled at stride 2i-1,
 *                            each sample weighted by its increment length
 *                            (Sec. 3.2, Def. 3.1, Def. 3.2, Prop. 3.1, eq. (24))
 *   f(u)     = 0, -rate u (eq. (18)), or rate u (1 - u) (Fisher-KPP).
 *   0 < gamma <= 2: subdiffusion, diffusion (gamma = 1) and superdiffusion use
 *   the same recurrence and scheme (Sec. 2.1); at gamma = 2 every weight is 1.
 *
 * The history of the stencil values delta[j] of every past step is kept in
 * device memory as FP32 rows (one row per step, as the sum of eq. (21) is
 * written); the current state u[k], delta[k] itself, the weights and every
 * per-step sum are FP64.
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers (e.g. torch CUDA tensors on the
 *    current device), never retained after the call returns.  A grid with
 *    nx * ny points is stored u[l * nx + j], x1 index j fastest; a 3D grid
 *    u[(n * ny + l) * nx + j].  An ensemble concatenates the problems' grids
 *    in order.
 *  - Work is enqueued on the stream given at gl_init (NULL = the null
 *    stream).  gl_init, gl_step_n, gl_adjoint and gl_free return after the
 *    work they enqueued has finished (they synchronise the stream).
 *  - A gl_ctx must not be used from two threads at once.
 *  - Every gl_status is GL_OK (0) or a negative code; on failure
 *    gl_last_error(ctx) (or gl_last_error(NULL) when no context exists)
 *    returns a message.  A failed call leaves the context usable unless the
 *    code is GL_EHIP.
 */
#ifndef GL_H_
#define GL_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gl_status;

#define GL_OK 0
#define GL_EINVAL (-1)       /* an argument is out of range or a pointer is NULL */
#define GL_EUNSTABLE (-2)    /* r * 4 * ndim > 2^gamma: the explicit scheme diverges */
#define GL_ENOMEM (-3)       /* the history arena does not fit in free device memory */
#define GL_ECAPACITY (-4)    /* more steps requested than max_steps allows */
#define GL_ESTATE (-5)       /* call not valid in the context's current state */
#define GL_ENONFINITE (-6)   /* a NaN or Inf in the input or in the state */
#define GL_EHIP (-7)         /* a HIP runtime call failed (message in gl_last_error) */
#define GL_EUNSUPPORTED (-8) /* valid request that the library does not implement */

/* Reaction term f(u) (Sec. 2.2, eqs. (18)-(21)). */
#define GL_RXN_NONE 0   /* f = 0 */
#define GL_RXN_LINEAR 1 /* f = -rate u (the paper's -beta u) */
#define GL_RXN_FISHER 2 /* f = rate u (1 - u) */

/* Memory mode of the history sum. */
#define GL_MEM_FULL 0     /* eq. (21) */
#define GL_MEM_SHORT 1    /* eq. (22): offsets 0..min(L, k) */
#define GL_MEM_ADAPTIVE 2 /* Sec. 3.2, eq. (24) */

/* Reading of the adaptive rule (the paper's interval joins admit two). */
#define GL_ADAPT_PARTITION 0   /* increments of 2i-1 points tile each region (a^(i-1), a^i]
                                  exactly from its first point; a leftover shorter than one
                                  increment enters point by point (default) */
#define GL_ADAPT_LITERAL 1     /* medians a^(i-1)+(2i-1)eta-i+1 up to a^i; in the interval
                                  holding k only whole increments ending by k, then a tail of
                                  single points up to k (increments may overlap or leave gaps) */
#define GL_ADAPT_UNIT_STRIDE 2 /* PARTITION with every increment of length 1: equals full memory */

/* How the history sum is evaluated. */
#define GL_SUM_GEMV_FP32 0       /* every step reads its history rows once, FP32 loads,
                                    FP64 accumulation */
#define GL_SUM_TOEPLITZ_BF16X3 1 /* full or short memory: blocks of B steps take the part of
                                    their sums over rows before the block as one Toeplitz-weight
                                    x history product on BF16 matrix cores (hi + lo split, three
                                    products, FP32 accumulation; with short memory the weights
                                    past the window are zero and only the rows within reach are
                                    read); the rest in FP64. Adaptive memory: GL_EUNSUPPORTED */

typedef struct gl_problem {
    int32_t ndim;     /* 1, 2 or 3 */
    int32_t nx;       /* interior points along x1, >= 1 */
    int32_t ny;       /* interior points along x2, >= 1 (ignored and taken as 1 in 1D) */
    int32_t nz;       /* interior points along x3, >= 1 (ignored and taken as 1 below 3D) */
    int32_t rxn;      /* GL_RXN_* */
    double dx;        /* grid spacing, > 0 */
    double dt;        /* time step, > 0 */
    double gamma;     /* anomalous exponent, 0 < gamma <= 2 */
    double alpha;     /* diffusivity, > 0 */
    double rxn_rate;  /* rate of the reaction term (finite) */
} gl_problem;

typedef struct gl_options {
    int32_t mem_mode;   /* GL_MEM_* (same for every problem of a context) */
    int32_t adapt_rule; /* GL_ADAPT_* */
    int64_t short_L;    /* short-memory window in steps, >= 0 */
    int32_t adapt_a;    /* adaptive base interval [0, a], a >= 2 */
    int32_t sum_path;   /* GL_SUM_* */
    int32_t block_B;    /* Toeplitz block length: 32, 64, 128, 256, 512, or 0: 512 when the
                           largest problem has >= 131072 points, else 256 */
    int32_t check_finite; /* nonzero: gl_step_n fails with GL_ENONFINITE on NaN/Inf state */
    int64_t max_steps;  /* history capacity in steps, >= 1 */
    int64_t ckpt_every; /* adjoint: recompute segment length C (0 = default 500) */
    void *stream;       /* hipStream_t for all work, NULL = null stream */
} gl_options;

typedef struct gl_ctx gl_ctx;

/* Creates a solver for nprob independent problems sharing the memory options
 * and copies the initial fields u0 (device, FP64, the problems' grids
 * concatenated) into it as step k = 0.  Computes the GL weights psi(gamma,m)
 * and d psi / d gamma for m = 0..max_steps in FP64 on the device (Sec. 2.1,
 * eqs. (11)-(12): the weights are computed once and reused every step) and
 * the per-step schedules, and allocates the FP32 history arena of
 * (max_steps + 1) rows per problem.
 * Errors: GL_EINVAL (bad argument), GL_EUNSTABLE, GL_ENOMEM, GL_ENONFINITE
 * (u0 not finite), GL_EHIP.  On success *out owns all device memory it uses. */
gl_status gl_init(const gl_problem *probs, int32_t nprob, const gl_options *opt,
                  const double *u0, gl_ctx **out);

/* Advances every problem n >= 0 steps of eq. (21) (or eqs. (22), (24)) and, if
 * uT is not NULL, writes the new states u[k] (FP64, concatenated) to uT.
 * Errors: GL_EINVAL (n < 0), GL_ECAPACITY (k + n > max_steps; nothing is
 * run), GL_ENONFINITE (check_finite set and the state holds NaN/Inf),
 * GL_EHIP. */
gl_status gl_step_n(gl_ctx *ctx, int64_t n, double *uT);

/* Gradient of a loss L(u[k_end]) for the run so far (steps 0..k_end from u0,
 * all problems), dt and dx held fixed.  Input dL_duT = dL/du[k_end] (FP64,
 * concatenated).  Outputs dL_du0 = dL/du0 (FP64, concatenated) and dparams,
 * nprob x 3 FP64 = {dL/dalpha, dL/dgamma, dL/drate} per problem.  Uses the
 * reverse-time sum with transposed GL weights and d psi / d gamma; for
 * adaptive memory the transpose of the schedule (offset m of reverse step k
 * weighted by its multiplicity in the schedule of forward step k + m) is
 * built on the host at each call.  The current state is not changed.
 * Errors: GL_ESTATE (no step taken yet), GL_EINVAL, GL_ENOMEM, GL_EHIP. */
gl_status gl_adjoint(gl_ctx *ctx, const double *dL_duT, double *dL_du0, double *dparams);

/* Releases every resource of ctx.  gl_free(NULL) is a no-op. */
void gl_free(gl_ctx *ctx);

/* Message of the last failure on ctx, or of the calling thread's last failure
 * that had no context (ctx == NULL).  Owned by the library; valid until the
 * next call on the same context / thread.  Never NULL. */
const char *gl_last_error(const gl_ctx *ctx);

/* Restarts every problem from new initial fields u0 (device, FP64,
 * concatenated) at k = 0, keeping the allocations, weights and schedules.
 * Errors: GL_EINVAL, GL_ENONFINITE (u0 not finite), GL_EHIP. */
gl_status gl_reset(gl_ctx *ctx, const double *u0);

/* Launch-shape autotuning of a context (no paper passage: a property of the GPU, not of
 * the method).  At step 0 (after gl_init or gl_reset), times candidate launch shapes of the
 * history sums on this context's own problems at step max_steps / 2, the mean depth of a
 * full-memory run, and keeps the fastest:
 *   GL_TUNE_GEMV     the plain path's GEMV workgroup target (its split-K fan-out;
 *                    candidates 256 .. 4096, default 1024), one GEMV + update step each;
 *   GL_TUNE_PRODUCT  the blocked path's product workgroups per CU (its chunk count;
 *                    candidates 1, 2, 4, default 2), one block product each (skipped when
 *                    GL_TOEPLITZ_KCHUNK fixes the chunk length, or max_steps / 2 < block_B).
 * what = 0 tunes both.  The candidates read the history arena as it stands and write only
 * rows, states and sums that the run overwrites before reading, so the context stays at
 * step 0 with its initial fields.  The chosen shapes change the order of floating-point
 * sums (split and chunk boundaries), not the operation; results stay within the paths'
 * tolerances.  If chosen is not NULL (host, 2 entries) it receives the GEMV target and the
 * product's workgroups per CU in effect (0: fixed chunk length).
 * Errors: GL_EINVAL (NULL ctx, unknown bits in what), GL_ESTATE (steps taken), GL_EHIP. */
#define GL_TUNE_GEMV 1
#define GL_TUNE_PRODUCT 2
gl_status gl_autotune(gl_ctx *ctx, int32_t what, int64_t *chosen);

/* ---- inspection and component entry points (tests and benchmarks) ---- */

/* Kernels timed by the profiling mode. */
#define GL_KERNEL_HIST_GEMV 0    /* plain history sum (one launch per step and problem) */
#define GL_KERNEL_UPDATE 1       /* stencil + reaction update */
#define GL_KERNEL_TOEPLITZ 2     /* Toeplitz-weight x history product (one launch per block) */
#define GL_KERNEL_TRIANGLE 3     /* steps inside a sub-block of the blocked path (its rows,
                                    stencil, update: up to eight steps per launch) */
#define GL_KERNEL_OLD_REDUCE 4   /* FP64 sum of the Toeplitz product's history chunks (only
                                    for products cut into more than one chunk) */
#define GL_KERNEL_SUBBLOCK 5     /* Toeplitz product over a block's rows before a sub-block */
#define GL_KERNEL_SUB_REDUCE 6   /* FP64 sum of the sub-block product's chunks (likewise) */
#define GL_KERNEL_COUNT 7

/* on != 0: gl_step_n brackets each launch of the timed kernels with HIP
 * events on the context's stream and accumulates their durations; resets
 * the counters either way. */
gl_status gl_set_profiling(gl_ctx *ctx, int32_t on);

/* Launch count and summed duration (milliseconds, from HIP events) of
 * kernel `kernel` (GL_KERNEL_*) since profiling was last switched. */
gl_status gl_profile(gl_ctx *ctx, int32_t kernel, int64_t *launches, double *total_ms);

/* Number of steps taken so far (the current k), or -1 for NULL. */
int64_t gl_steps_done(const gl_ctx *ctx);

/* Copies the current states u[k] (FP64, concatenated) to u. */
gl_status gl_get_state(gl_ctx *ctx, double *u);

/* Copies problem iprob's weight tables for m = 0..count-1 (count <=
 * max_steps + 1): psi(gamma, m) to psi and d psi / d gamma to dpsi (either
 * may be NULL).  Sec. 2.1, eqs. (8), (11), (12). */
gl_status gl_get_weights(gl_ctx *ctx, int32_t iprob, int64_t count, double *psi, double *dpsi);

/* Number of schedule terms (sampled offsets) summed at step k under the
 * context's memory mode, or -1 for bad arguments. */
int64_t gl_schedule_terms(const gl_ctx *ctx, int64_t k);

/* The history sum alone, with the context's weights (problem iprob), memory
 * schedule and sum path, over a caller-supplied FP32 history (any rows, e.g.
 * delta values):
 *   S[p] = sum_{(m,c) in sched(k)} c psi(gamma,m) hist[(k - m) * ld + p],
 * p = 0..P-1 (P = problem iprob's point count).  hist holds rows 0..k with
 * leading dimension ld >= P, ld % 4 == 0, 16-byte aligned.  S is FP64.
 * k must not exceed max_steps.  With GL_SUM_TOEPLITZ_BF16X3 the rows before
 * the block holding k (blocks of block_B steps) are summed on matrix cores
 * as in gl_step_n.  Errors: GL_EINVAL, GL_EHIP. */
gl_status gl_history_sum(gl_ctx *ctx, int32_t iprob, int64_t k, const float *hist, int64_t ld,
                         double *S);

#ifdef __cplusplus
}
#endif

#endif /* GL_H_ */
