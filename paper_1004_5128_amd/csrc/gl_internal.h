// Internal declarations of libgl: device data of a context, the per-step
// schedule tables and the kernel launchers.  Not part of the C ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "gl.h"

namespace gl {

// Events the profiling mode wants stamped when the next kernel launched on this thread
// starts and ends (hipExtLaunchKernelGGL records them at the kernel's own start and end,
// so the interval excludes the dispatch gap).  Null: plain launch.
struct KernelTimer {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};
extern thread_local KernelTimer g_kernel_timer;

#define GL_LAUNCH(kernel, grid, block, shmem, stream, ...)                                      \
    do {                                                                                        \
        if (::gl::g_kernel_timer.start)                                                         \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, ::gl::g_kernel_timer.start, \
                                  ::gl::g_kernel_timer.stop, 0, __VA_ARGS__);                   \
        else                                                                                    \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                \
    } while (0)

// One run of schedule terms: offsets m = m0 + i * stride (i = 0..count-1), each
// entering the history sum with weight coef * psi(gamma, m).  A step's runs are
// stored in ascending m; flattening them gives the step's term sequence.
struct Run {
    int32_t m0;
    int32_t count;
    int32_t stride;
    int32_t coef;
};

// Per-step schedule of a context: runs[run_begin[k] .. run_begin[k+1]) for
// k = 0..max_steps, and the number of terms per step.
struct Schedule {
    std::vector<Run> runs;
    std::vector<int64_t> run_begin;  // max_steps + 2 entries
    std::vector<int64_t> terms;      // max_steps + 1 entries
};

// Builds the schedule of every step 0..max_steps for the memory options
// (full, short, adaptive with its three readings).
Schedule build_schedule(const gl_options &opt, int64_t max_steps);

// The transpose of a schedule over an n-step run, for the adjoint's reverse sweep: reverse
// step rho (forward step k = n - 1 - rho) gets the terms (m, c), m = 0..rho, where c is the
// multiplicity of offset m in the schedule of forward step k + m, as runs in ascending m.
// Full and short memory are their own transposes; adaptive memory is not, since the
// sampling of a region depends on the step that reaches it.
Schedule transpose_schedule(const Schedule &fwd, int64_t n);

// Device-side state of one problem.
struct Problem {
    gl_problem p{};
    int64_t P = 0;        // grid points
    int64_t ld = 0;       // history leading dimension in floats (multiple of 64, >= P)
    double r = 0.0;       // alpha dt^gamma / dx^2
    int64_t offset = 0;   // first point of this problem in concatenated arrays
    double *psi = nullptr;   // [max_steps + 1] FP64 weights
    double *dpsi = nullptr;  // [max_steps + 1] d psi / d gamma
    double *psi_blk = nullptr;  // weights of the blocked path: psi, zero past a short-memory
                                // window (the same array as psi otherwise)
    double *carry[2] = {nullptr, nullptr};  // in-block chain carries, kMaxFuse x P each
    int64_t carry_k = -1;   // step the valid carry starts at (-1: none)
    int32_t carry_n = 0;    // steps it covers
    int32_t carry_cur = 0;  // buffer holding it
    float *H = nullptr;      // [(max_steps + 1) * ld] FP32 history, row j = delta[j] (eq. 17)
    double *u[2] = {nullptr, nullptr};  // FP64 state, double-buffered
    int cur = 0;             // u[cur] holds the current step
    // blocked Toeplitz path
    uint16_t *psi_tab = nullptr;  // BF16 hi/lo weight tables, 2 x 8 shifted copies of tab_len
    uint16_t *dpsi_tab = nullptr; // the same for d psi / d gamma (blocked adjoint, lazily)
    int64_t tab_len = 0;
    double *old = nullptr;        // [B x P] FP64 sums over the rows before the current block
    int64_t old_k0 = -1;          // block start old[] belongs to (-1: none)
    double *old2 = nullptr;       // [B2 x P] sums over the rows of the block before the sub-block
    int64_t old2_k1 = -1;         // sub-block start old2[] belongs to (-1: none)
    // adjoint: FP64 snapshots of u every C steps, snap[i] = u[i C]
    double *snap = nullptr;
    // workgroup target of this problem's history GEMV: the context's target, shared among
    // the problems of an ensemble in proportion to their sizes
    int64_t gemv_groups = 1024;
};

// ---------------------------------------------------------------- kernels

// psi(gamma, m) and d psi / d gamma for m = 0..n.
void launch_weights(double gamma, int64_t n, double *psi, double *dpsi, hipStream_t s);

// Columns per workgroup of the history GEMV.
constexpr int kGemvCols = 1024;

// Number of row splits of the history GEMV for `terms` terms over P points,
// aiming at about target_groups workgroups.
__host__ __device__ int gemv_splits(int64_t terms, int64_t P, int64_t target_groups);
constexpr int kMaxSplits = 64;

// partial[s * P + p] = sum over terms t in split s of [t_begin, t_end) of the
// step-k schedule (runs, nruns) of coef * psi[m] * H[(k - m) * ld + p], FP64,
// accumulated in term order (reverse: from the split's last term down).
void launch_hist_gemv(const float *H, int64_t ld, int64_t P, const double *psi, const Run *runs,
                      int nruns, int64_t k, int64_t t_begin, int64_t t_end, int nsplit,
                      bool reverse, double *partial, hipStream_t s);
// The same launch with a second weight table psi2 over the same rows: partial receives
// exactly what launch_hist_gemv writes, partial2 (same layout) the sums with psi2.
void launch_hist_gemv_dual(const float *H, int64_t ld, int64_t P, const double *psi,
                           const double *psi2, const Run *runs, int nruns, int64_t k,
                           int64_t t_begin, int64_t t_end, int nsplit, bool reverse,
                           double *partial, double *partial2, hipStream_t s);

// One problem of a batched (ensemble) launch; a device-resident table, one entry per
// problem, built at gl_init.
struct BatchEntry {
    float *H;
    int64_t ld, P;
    const double *psi;
    double *u[2];
    double *partial;  // this problem's GEMV partials, up to its split count x P
    double *snap;     // adjoint snapshots: u[k+1] goes to snap[(k+1)/C] when C divides k+1
    int64_t groups;   // this problem's GEMV workgroup target (Problem::gemv_groups)
    int64_t upd_begin; // first workgroup of this problem in a batched update launch
    int32_t ndim, nx, ny, nz, rxn;
    double r, dt, rate;
};

// Workgroups of one batched GEMV launch over every problem for `terms` terms.
int64_t batched_gemv_groups(const std::vector<Problem> &probs, int64_t terms);
// One launch: for every problem, partial[s * P + p] of terms [t_begin, t_end) at step k.
void launch_hist_gemv_batched(const BatchEntry *tab, int nprob, int64_t wgs, const Run *runs,
                              int nruns, int64_t k, int64_t t_begin, int64_t t_end, bool reverse,
                              hipStream_t s);
// One launch: the update of every problem from u[cur] into u[cur ^ 1], history row k;
// `terms` = the GEMV's term count (t_end - t_begin), for each problem's split count.
void launch_update_batched(const BatchEntry *tab, int nprob, int64_t wgs, int64_t k, int cur,
                           int64_t terms, int64_t C, hipStream_t s);

// Tuning (defaults; GL_GEMV_GROUPS, GL_GEMV_SERPENTINE, GL_TOEPLITZ_KCHUNK and
// GL_SUBBLOCK in the environment override them at gl_init).
struct Tuning {
    int64_t gemv_groups = 1024;  // target workgroups per GEMV launch
    bool serpentine = false;     // alternate the traversal direction every step
    int64_t kchunk = 0;          // history rows per Toeplitz product chunk (multiple of 128);
                                 // 0: per product, the fewest chunks that fill the GPU
    int64_t sub_B = 32;          // sub-block length of the blocked path (32 or 64; 0: off)
    int64_t fuse = 8;            // in-block steps per launch (1 .. kMaxFuse; kMaxFuse3 in 3D)
    int64_t chunk_wgs = 2;       // product workgroups per CU that the column tiles x chunks
                                 // should reach (half of it for 512-row blocks); 1 .. kMaxChunkWgs
};
constexpr int64_t kMaxChunkWgs = 4;

// ---- blocked Toeplitz path
constexpr int kPsiPad = 1024;  // zero entries before psi(0) in the BF16 weight tables: a
                               // product may take rows up to BM past k0 (weights psi(m < 0) = 0)
constexpr int kMaxBlock = 512;
constexpr int kMaxTK = 128;   // history rows per Toeplitz K step, at most (chunks are multiples)

// BF16 hi/lo weight tables (8 shifted copies each) from the FP64 weights psi[0..npsi).
void launch_psi_tables(const double *psi, int64_t npsi, int64_t tab_len, uint16_t *tab,
                       hipStream_t s);

// Number of history chunks a product over `rows` rows is cut into.
int toeplitz_chunks(int64_t rows, int64_t kchunk);

// out[c][b][p] (FP32) = sum over rows j in chunk c of [j_lo, j_hi) of
// T[b][j] H[j * ld + p] with T[b][j] = psi(k0 + b - j), b < BM, three BF16 products
// (j_hi <= k0 + BM).  With one chunk and direct != nullptr the FP64 result (what the chunk
// reduction below gives, plus base[b][p] when base != nullptr) goes to direct[b][p] instead.
// Returns false, launching nothing, when k0 or j_lo is not a multiple of 32, j_hi > k0 + BM,
// kchunk is not a multiple of kMaxTK or BM is not a supported block length.  Rows j >= k0 + b
// have weight psi(k0 + b - j <= 0): psi(0) = 1 at j = k0 + b, zero past it.
bool launch_toeplitz_gemm(int BM, const float *H, int64_t ld, int64_t P, const uint16_t *tab,
                          int64_t tab_len, int64_t k0, int64_t j_lo, int64_t j_hi, int64_t kchunk,
                          float *out, double *direct, const double *base, hipStream_t s);

// old[b * P + p] = (base[b * P + p] +) sum_c part[c][b][p] in FP64, chunks in order.
void launch_old_reduce(const float *part, int nchunk, int64_t BM, int64_t P, double *old,
                       const double *base, hipStream_t s);

// Arguments of the in-block step kernel: steps k .. k + s - 1 of one problem.
struct BlockStepArgs {
    const double *psi;
    float *H;
    int64_t ld, P;
    int32_t ndim, nx, ny, nz, rxn;
    double r, dt, rate;
    // Sums over the rows before the sub-block: row pre_row + i belongs to step k + i.  The
    // block's product Old ([B x P], row b) in the first sub-block of a block, Old + the
    // sub-block's product over the block's earlier rows ([B2 x P], row b2) after it.  Before
    // any row exists has_pre is 0 and pre is still a readable [B x P] array (not used).
    const double *pre;
    int32_t pre_row;
    int32_t has_pre;
    const double *u_cur;    // u[k]
    double *u_next;         // u[k + s]
    double *u_rows;         // nullable: u[k + i + 1] for i < s - 1 at u_rows + i * u_stride
    int64_t u_stride;
    double *S_out;          // nullable: row i (stride P) receives the full sum S of step k + i
    double *snap;           // nullable: checkpoint rows of u (row j / C holds u[j])
    uint32_t snap_mask;     // bit i: C divides k + i + 1, u[k + i + 1] goes to a checkpoint
    int64_t snap_row0;      // checkpoint row of the lowest set bit (the next ones follow)
    int64_t k;              // first step of the launch
    int32_t b;              // k - k0 (offset in the block: row of old)
    int32_t b2;             // k - k1 (offset in the sub-block: row of old2; rows k1 .. k - 1
                            // are summed point by point)
    int32_t s;              // steps in this launch (1 .. kMaxFuse), inside one sub-block
    int32_t write_history;  // 0: leave history rows k .. k + s - 1 untouched (recomputation)
    // Carry (sub-blocks of at most 32 steps): carry_in, nullable, holds for every point the
    // chains of this launch's steps (row i: step k + i) over all rows before k, as the
    // previous launch left them; carry_out, nullable, receives those of the next launch's
    // n_next steps over all rows before k + s, for this launch's tile points.
    const double *carry_in;
    double *carry_out;
    int32_t n_next;
    // Reverse steps (the adjoint, through launch_adjoint_steps): k is the first reverse step
    // rho and the s steps are those of forward steps kf = n - 1 - rho down to kf - s + 1.
    // u_cur is lam[kf + 1], H the mu history (row rho + i written by reverse step rho + i),
    // pre the sums over the mu rows before the sub-block (pre_row 0, has_pre 1); u_rev holds
    // u[kf - i] at u_rev - i P and lam_rows receives lam[kf - i] at lam_rows - i P (the rows
    // descend in memory).  The forward-only outputs (u_next, u_rows, S_out, snap) are unused.
    const double *u_rev;
    double *lam_rows;
};

constexpr int kMaxFuse = 8;
constexpr int kMaxFuse3 = 2;  // 3D: the halo grows in three directions (4 would spill)

// Steps k .. k + s - 1 of one sub-block as a single kernel (history sums over the
// sub-block's rows, stencil, reaction, state update, history rows).  The result of every
// step does not depend on how steps are grouped into launches.
void launch_block_step(const BlockStepArgs &args, hipStream_t s);

// S[p] = sum_s partial[s * P + p] (+ base[p] if base != nullptr), fixed order.
void launch_reduce_partials(const double *partial, int nsplit, int64_t P, const double *base,
                            double *S, hipStream_t s);

// One explicit step after the GEMV: d = stencil(u); S = d (+ base) + sum_s partial[s];
// unew = u + dt f(u) + r S; Hk (history row k, nullable) = (float) d; S_out (nullable) = S.
void launch_update(const Problem &pb, const double *u, const double *base, double *unew,
                   float *Hk, double *S_out, const double *partial, int nsplit, hipStream_t s);

// ---- adjoint
// One reverse step of the plain path: mu = r stencil(lam1); A = mu + sum_s partial[s];
// lam0 = lam1 + dt f'(uk) lam1 + A; Mrow = (float) mu; and per-workgroup partial sums
// of lam1 * Sk, lam1 * Gk, lam1 * df/drate(uk) into grad[3 * blockIdx].
void launch_adjoint_update(const Problem &pb, const double *lam1, double *lam0, float *Mrow,
                           const double *partial, int nsplit, const double *uk, const double *Sk,
                           const double *Gk, double *grad, hipStream_t s);

// Reverse steps rho .. rho + s - 1 of one sub-block on the blocked path (forward steps
// kf, kf - 1, .. kf - s + 1, kf = n - 1 - rho), in one launch of the in-block kernel with
// lam in place of u and mu = r Lap lam in place of delta: the sum of reverse step rho + i
// over the mu history runs as the forward's chain (the sums before the sub-block, then
// psi(m) times the mu rows rho - b2 .. rho + i - 1 in ascending order, then mu itself,
// psi(0) = 1), chain carries between launches included, so the result does not depend on
// how the steps are grouped.  Arguments as BlockStepArgs describes for reverse steps.
void launch_adjoint_steps(const BlockStepArgs &args, hipStream_t s);

// Per-workgroup partial sums for the steps k = k_lo .. k_lo + nk - 1 of a segment, as the
// plain path's update forms them: lam1 * S, lam1 * G, lam1 * df/drate(u) with lam1 row
// k - k_lo + 1 of lam, S, G and u rows k - k_lo; into grad + 3 (k groups + blockIdx).
void launch_adjoint_dots(const Problem &pb, const double *lam, const double *u, const double *S,
                         const double *G, int64_t k_lo, int64_t nk, double *grad, hipStream_t s);
// Workgroups of one adjoint update launch for P points.
int adjoint_groups(int64_t P);
// dparams[0..2] = {dL/dalpha, dL/dgamma, dL/drate} from the per-step partial sums
// grad[n * 3] (n entries in the fixed order they were written), through part (the
// kAdjFinalParts x 3 sums of a first stage over consecutive ranges).
constexpr int kAdjFinalParts = 256;
void launch_adjoint_final(const double *grad, int64_t n, double r, double alpha, double lndt,
                          double dt, double *part, double *dparams, hipStream_t s);

// *flag = 1 if any of x[0..n) is NaN or Inf (flag must start at 0).
void launch_check_finite(const double *x, int64_t n, int *flag, hipStream_t s);

}  // namespace gl
