// C ABI of libgl (include/gl.h): context lifetime, validation, device memory,
// and the step driver that sequences the history-sum and update kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "gl.h"
#include "gl_internal.h"

struct gl_ctx {
    std::vector<gl::Problem> probs;
    gl_options opt{};
    hipStream_t stream = nullptr;
    int64_t k = 0;             // steps taken
    int64_t total_points = 0;  // sum of problem points
    gl::Schedule sched;
    gl::Run *d_runs = nullptr;
    double *partial = nullptr;  // GEMV partial sums of one problem: its most splits x P (FP64)
    int *d_flag = nullptr;
    float *tpart = nullptr;  // Toeplitz product chunks: max chunks x B x P (FP32)
    int64_t tpart_len = 0;   // its length in floats
    int ncu = 0;             // compute units of the device
    gl::BatchEntry *d_batch = nullptr;  // one entry per problem (batched plain-path launches)

    double *bpartial = nullptr;          // per-problem GEMV partial regions of the batch
    size_t bpart_cap = 0;                // its length in doubles
    int64_t upd_wgs = 0;                 // workgroups of one batched update launch
    int64_t C = 500;         // adjoint recompute segment length (snapshot interval)
    // adjoint work buffers, allocated on the first gl_adjoint call (sized for the largest problem)
    float *adj_M = nullptr;      // reverse-time history of mu rows, max_steps x max ld
    double *adj_u = nullptr;     // recomputed states of one segment, (C + 1) x max P
    double *adj_S = nullptr;     // the forward sums S[k] of one segment, C x max P
    double *adj_G = nullptr;     // the sums with d psi / d gamma, C x max P
    double *adj_lam[2] = {nullptr, nullptr};  // plain path: lam[k + 1] and lam[k]
    double *adj_lamseg = nullptr;  // blocked path: lam[ks .. ke] of a segment, (C + 1) x max P
    double *adj_grad = nullptr;  // per step and workgroup partial dot products, 3 each
    double *adj_fpart = nullptr; // the final reduction's first-stage sums, kAdjFinalParts x 3
    double *adj_partial2 = nullptr;  // plain path: the recompute's d psi / d gamma partials
    size_t part_len = 0;         // length of partial (and adj_partial2) in doubles
    gl::Run *adj_runs = nullptr;  // adaptive memory: the transposed schedule's runs
    size_t adj_runs_cap = 0;
    // blocked adjoint (Toeplitz path): the sums over the mu rows before a block of reverse
    // steps (psi) and before a sub-block, and the sums G of a block's steps over the delta
    // history (d psi / d gamma)
    double *adj_oldA = nullptr, *adj_oldG = nullptr;  // B x max P each
    double *adj_oldA2 = nullptr;                       // B2 x max P (sub-block sums)
    int64_t adj_oldA_r0 = -1, adj_oldA2_r1 = -1;
    // chain carries between the reverse in-block launches (as the forward's, own buffers)
    double *adj_carry[2] = {nullptr, nullptr};         // kMaxFuse x max P each
    int64_t adj_carry_rho = -1;                        // reverse step the carry starts at
    int32_t adj_carry_n = 0, adj_carry_cur = 0;
    int64_t maxP = 0, maxld = 0;
    int B = 256;             // block length of the Toeplitz path
    int B2 = 0;              // sub-block length inside a block (0: one level)
    gl::Tuning tune;
    std::vector<void *> allocs;
    std::string err;
    // profiling: events bracketing timed kernel launches, resolved at sync points
    bool prof = false;
    std::vector<hipEvent_t> event_pool;
    struct Pending {
        int kernel;
        hipEvent_t start, stop;
    };
    std::vector<Pending> pending;
    int64_t prof_launches[GL_KERNEL_COUNT] = {};
    double prof_ms[GL_KERNEL_COUNT] = {};
};

namespace gl {
thread_local KernelTimer g_kernel_timer;
}

namespace {

thread_local std::string g_thread_err;

constexpr int64_t kMaxPoints = int64_t(1) << 28;  // per problem
constexpr int64_t kLargeGrid = 131072;  // points from which the default block length is 512
constexpr int64_t kMaxGemvTarget = 4096;  // largest GEMV workgroup target gl_autotune tries

// Most splits the GEMV can cut P points into for a workgroup target (gemv_splits's bound
// without the term count): enough splits to reach the target over the column blocks.
int64_t split_bound(int64_t P, int64_t target) {
    const int64_t colblocks = (P + gl::kGemvCols - 1) / gl::kGemvCols;
    return std::min<int64_t>(gl::kMaxSplits, std::max<int64_t>(1, (target + colblocks - 1) / colblocks));
}

gl_status load_initial(gl_ctx *ctx, const double *u0);

gl_status fail(gl_ctx *ctx, gl_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_thread_err = buf;
    return code;
}

#define HIP_TRY(ctx, expr)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail((ctx), GL_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

template <class T>
gl_status dev_alloc(gl_ctx *ctx, T **ptr, size_t count) {
    void *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, GL_ENOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                    hipGetErrorString(e));
    }
    ctx->allocs.push_back(p);
    *ptr = static_cast<T *>(p);
    return GL_OK;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

gl_status validate(const gl_problem *probs, int32_t nprob, const gl_options *opt,
                   const double *u0, gl_ctx **out) {
    if (!out) return fail(nullptr, GL_EINVAL, "gl_init: out is NULL");
    *out = nullptr;
    if (!probs || nprob < 1) return fail(nullptr, GL_EINVAL, "gl_init: need nprob >= 1 problems");
    if (!opt) return fail(nullptr, GL_EINVAL, "gl_init: options are NULL");
    if (!u0) return fail(nullptr, GL_EINVAL, "gl_init: u0 is NULL");
    if (opt->mem_mode < GL_MEM_FULL || opt->mem_mode > GL_MEM_ADAPTIVE)
        return fail(nullptr, GL_EINVAL, "gl_init: unknown mem_mode %d", opt->mem_mode);
    if (opt->mem_mode == GL_MEM_SHORT && opt->short_L < 0)
        return fail(nullptr, GL_EINVAL, "gl_init: short_L must be >= 0");
    if (opt->mem_mode == GL_MEM_ADAPTIVE) {
        if (opt->adapt_a < 2) return fail(nullptr, GL_EINVAL, "gl_init: adapt_a must be >= 2");
        if (opt->adapt_rule < GL_ADAPT_PARTITION || opt->adapt_rule > GL_ADAPT_UNIT_STRIDE)
            return fail(nullptr, GL_EINVAL, "gl_init: unknown adapt_rule %d", opt->adapt_rule);
    }
    if (opt->sum_path != GL_SUM_GEMV_FP32 && opt->sum_path != GL_SUM_TOEPLITZ_BF16X3)
        return fail(nullptr, GL_EINVAL, "gl_init: unknown sum_path %d", opt->sum_path);
    if (opt->max_steps < 1 || opt->max_steps > (int64_t)INT32_MAX / 2)
        return fail(nullptr, GL_EINVAL, "gl_init: max_steps must be in [1, 2^30]");
    if (opt->ckpt_every < 0) return fail(nullptr, GL_EINVAL, "gl_init: ckpt_every must be >= 0");
    if (opt->block_B != 0 && opt->block_B != 32 && opt->block_B != 64 && opt->block_B != 128 &&
        opt->block_B != 256 && opt->block_B != 512)
        return fail(nullptr, GL_EINVAL, "gl_init: block_B must be 0, 32, 64, 128, 256 or 512");
    if (opt->sum_path == GL_SUM_TOEPLITZ_BF16X3 && opt->mem_mode == GL_MEM_ADAPTIVE)
        return fail(nullptr, GL_EUNSUPPORTED,
                    "gl_init: the Toeplitz path sums full or short memory (not adaptive)");
    for (int32_t i = 0; i < nprob; ++i) {
        const gl_problem &p = probs[i];
        if (p.ndim < 1 || p.ndim > 3)
            return fail(nullptr, GL_EINVAL, "gl_init: problem %d: ndim must be 1, 2 or 3", i);
        if (p.nx < 1 || (p.ndim >= 2 && p.ny < 1) || (p.ndim == 3 && p.nz < 1))
            return fail(nullptr, GL_EINVAL, "gl_init: problem %d: grid must have >= 1 point", i);
        // kernels address a problem's points with 32-bit byte offsets
        if ((int64_t)p.nx * (p.ndim >= 2 ? p.ny : 1) * (p.ndim == 3 ? p.nz : 1) > kMaxPoints)
            return fail(nullptr, GL_EINVAL, "gl_init: problem %d: more than 2^28 grid points", i);
        if (!(p.dx > 0) || !std::isfinite(p.dx) || !(p.dt > 0) || !std::isfinite(p.dt))
            return fail(nullptr, GL_EINVAL, "gl_init: problem %d: dx and dt must be > 0", i);
        if (!(p.gamma > 0.0 && p.gamma <= 2.0))
            return fail(nullptr, GL_EINVAL, "gl_init: problem %d: gamma must be in (0, 2]", i);
        if (!(p.alpha > 0.0) || !std::isfinite(p.alpha))
            return fail(nullptr, GL_EINVAL, "gl_init: problem %d: alpha must be > 0", i);
        if (p.rxn < GL_RXN_NONE || p.rxn > GL_RXN_FISHER || !std::isfinite(p.rxn_rate))
            return fail(nullptr, GL_EINVAL, "gl_init: problem %d: bad reaction", i);
        const double r = p.alpha * std::pow(p.dt, p.gamma) / (p.dx * p.dx);
        // von Neumann bound of the explicit scheme: the highest grid mode has
        // Lap eigenvalue -> -4 ndim, and sum psi (-1)^m = 2^(1 - gamma); for 1 < gamma <= 2
        // the characteristic roots still leave the unit circle only through z = -1.
        if (r * 4.0 * p.ndim > std::pow(2.0, p.gamma) * (1.0 + 1e-12))
            return fail(nullptr, GL_EUNSTABLE,
                        "gl_init: problem %d: r = %.6g exceeds the stability bound 2^gamma/(4 "
                        "ndim) = %.6g",
                        i, r, std::pow(2.0, p.gamma) / (4.0 * p.ndim));
    }
    return GL_OK;
}

// In-block launches hand chain carries to the next launch when a sub-block (the block with
// one level) has at most 32 steps: the rows a carry sums then fit one batch.
bool carry_ok(const gl_ctx *ctx) {
    return ctx->opt.sum_path == GL_SUM_TOEPLITZ_BF16X3 && (ctx->B2 ? ctx->B2 : ctx->B) <= 32;
}

// A tuning variable's value, or nullptr when it is unset or empty.
const char *env_value(const char *name) {
    const char *v = std::getenv(name);
    return v && *v ? v : nullptr;
}

// History rows per chunk of a Toeplitz product over `rows` rows (a multiple of the K step):
// the fixed GL_TOEPLITZ_KCHUNK length if set, else the fewest chunks for which the column
// tiles x chunks reach `wgs` workgroups per CU (half as many for the 512-row block; 2 by
// default, gl_autotune may pick another).  Fewer chunks mean fewer FP32 partial products to
// write and sum; the accumulation error is set by the BF16 split, not by the FP32 sums over
// a chunk.
int64_t chunk_cap(const gl_ctx *ctx, int BM, int64_t P, int64_t rows, int64_t wgs) {
    const int64_t tiles = (P + 127) / 128;
    const int64_t target =
        (int64_t)std::max(ctx->ncu, 1) * (BM >= 512 ? std::max<int64_t>(1, wgs / 2) : wgs);
    const int64_t nchunk = std::max<int64_t>(1, (target + tiles - 1) / tiles);
    return std::max<int64_t>(1, std::min(nchunk, (rows + gl::kMaxTK - 1) / gl::kMaxTK));
}

int64_t chunk_rows(const gl_ctx *ctx, int BM, int64_t P, int64_t rows) {
    if (ctx->tune.kchunk > 0) return ctx->tune.kchunk;
    const int64_t cap = chunk_cap(ctx, BM, P, rows, ctx->tune.chunk_wgs);
    const int64_t kc = (std::max<int64_t>(rows, 1) + cap - 1) / cap;
    return (kc + gl::kMaxTK - 1) / gl::kMaxTK * gl::kMaxTK;
}

// Most chunks any product over at most `rows` rows is cut into, for any workgroup target
// gl_autotune may choose (sizes the chunk buffer): rows / chunk_rows <= chunk_cap, which
// does not decrease with rows or with the target.
int64_t max_chunks(const gl_ctx *ctx, int BM, int64_t P, int64_t rows) {
    if (ctx->tune.kchunk > 0) return gl::toeplitz_chunks(rows, ctx->tune.kchunk);
    return chunk_cap(ctx, BM, P, rows, gl::kMaxChunkWgs);
}

// The GEMV workgroup target of every problem (an ensemble shares `groups` in proportion to
// the problems' sizes), each problem's region of batched partial sums (its largest split
// count over the schedule) and the device table of the batched launches.  The stream must
// be idle: the table is rewritten in place.
gl_status apply_gemv_target(gl_ctx *ctx, int64_t groups) {
    ctx->tune.gemv_groups = groups;
    int64_t max_terms = 1;
    for (int64_t t : ctx->sched.terms) max_terms = std::max(max_terms, t);
    const int32_t nprob = (int32_t)ctx->probs.size();
    std::vector<gl::BatchEntry> tab(nprob);
    size_t off = 0;
    int64_t upd_begin = 0;
    for (int32_t i = 0; i < nprob; ++i) {
        gl::Problem &pb = ctx->probs[i];
        pb.gemv_groups = std::max<int64_t>(
            1, (groups * pb.P + ctx->total_points - 1) / ctx->total_points);
        const int splits = std::max(1, gl::gemv_splits(max_terms - 1, pb.P, pb.gemv_groups));
        gl::BatchEntry &e = tab[i];
        e.H = pb.H;
        e.ld = pb.ld;
        e.P = pb.P;
        e.psi = pb.psi;
        e.u[0] = pb.u[0];
        e.u[1] = pb.u[1];
        e.partial = ctx->bpartial + off;
        e.snap = pb.snap;
        e.groups = pb.gemv_groups;
        e.upd_begin = upd_begin;
        upd_begin += (pb.P + 255) / 256;
        off += (size_t)splits * pb.P;
        e.ndim = pb.p.ndim;
        e.nx = pb.p.nx;
        e.ny = pb.p.ny;
        e.nz = pb.p.nz;
        e.rxn = pb.p.rxn;
        e.r = pb.r;
        e.dt = pb.p.dt;
        e.rate = pb.p.rxn_rate;
    }
    if (off > ctx->bpart_cap)
        return fail(ctx, GL_EINVAL, "internal: batched partial sums exceed their buffer");
    if (upd_begin != ctx->upd_wgs)
        return fail(ctx, GL_EINVAL, "internal: batched update layout of %lld workgroups, "
                    "launch of %lld", (long long)upd_begin, (long long)ctx->upd_wgs);
    HIP_TRY(ctx, hipMemcpy(ctx->d_batch, tab.data(), tab.size() * sizeof(gl::BatchEntry),
                           hipMemcpyHostToDevice));
    return GL_OK;
}

gl_status init_impl(gl_ctx *ctx, const gl_problem *probs, int32_t nprob, const double *u0) {
    const gl_options &opt = ctx->opt;
    const int64_t rows = opt.max_steps + 1;

    const bool toep = opt.sum_path == GL_SUM_TOEPLITZ_BF16X3;
    // default block length: 512 rows for large grids, where halving the history reads per
    // product outweighs the longer sub-block products (measured: 10% faster at 512^2, 1.6%
    // at 256^2 where the default stays 256), 256 otherwise
    int64_t largest = 0;
    for (int32_t i = 0; i < nprob; ++i)
        largest = std::max<int64_t>(largest, (int64_t)probs[i].nx *
                                                 (probs[i].ndim >= 2 ? probs[i].ny : 1) *
                                                 (probs[i].ndim == 3 ? probs[i].nz : 1));
    ctx->B = opt.block_B ? opt.block_B : (largest >= kLargeGrid ? 512 : 256);
    // a second level of blocking when the sub-block length divides the block length
    ctx->B2 = (ctx->tune.sub_B > 0 && ctx->tune.sub_B < ctx->B && ctx->B % ctx->tune.sub_B == 0)
                  ? (int)ctx->tune.sub_B
                  : 0;
    // weights are kept for m up to max_steps + kMaxBlock (the last block's rows reach past k)
    const int64_t npsi = opt.max_steps + gl::kMaxBlock + 1;
    // table entries cover psi(-kPsiPad .. npsi + 63): a K step stages up to 8 words past the
    // last index it uses
    const int64_t tab_len = (npsi + gl::kPsiPad + 128 + 7) / 8 * 8;
    int dev = 0;
    HIP_TRY(ctx, hipGetDevice(&dev));
    HIP_TRY(ctx, hipDeviceGetAttribute(&ctx->ncu, hipDeviceAttributeMultiprocessorCount, dev));

    // capacity: history arena + tables + state
    size_t need = 0;
    int64_t maxP = 0;
    ctx->probs.resize(nprob);
    for (int32_t i = 0; i < nprob; ++i) {
        gl::Problem &pb = ctx->probs[i];
        pb.p = probs[i];
        if (pb.p.ndim == 1) pb.p.ny = 1;
        if (pb.p.ndim != 3) pb.p.nz = 1;
        pb.P = (int64_t)pb.p.nx * pb.p.ny * pb.p.nz;
        pb.ld = round_up(pb.P, 64);
        pb.r = pb.p.alpha * std::pow(pb.p.dt, pb.p.gamma) / (pb.p.dx * pb.p.dx);
        pb.offset = ctx->total_points;
        ctx->total_points += pb.P;
        if (pb.P > maxP) maxP = pb.P;
        need += (size_t)rows * pb.ld * sizeof(float) + 2 * (size_t)npsi * sizeof(double) +
                2 * (size_t)pb.P * sizeof(double);
        if (toep)
            need += 16 * (size_t)tab_len * sizeof(uint16_t) +
                    (size_t)(ctx->B + ctx->tune.sub_B + 2 * gl::kMaxFuse) * pb.P * sizeof(double);
    }
    ctx->C = opt.ckpt_every > 0 ? opt.ckpt_every : 500;
    const int64_t nsnap = opt.max_steps / ctx->C + 1;
    for (const gl::Problem &pb : ctx->probs) need += (size_t)nsnap * pb.P * sizeof(double);
    // GEMV partial sums: the most splits any workgroup target up to the largest candidate can
    // give each problem (a large grid fills the GPU with column blocks alone and needs one)
    const int64_t tmax = std::max<int64_t>(kMaxGemvTarget, ctx->tune.gemv_groups);
    size_t bpart_cap = 0, part_len = 0;
    for (const gl::Problem &pb : ctx->probs) {
        const int64_t share = (tmax * pb.P + ctx->total_points - 1) / ctx->total_points;
        bpart_cap += (size_t)split_bound(pb.P, share) * pb.P;
        part_len = std::max(part_len, (size_t)split_bound(pb.P, tmax) * pb.P);
    }
    need += (bpart_cap + part_len) * sizeof(double);
    // FP32 chunk products: the largest chunks x B x P over the problems
    // (a sub-block product needs at most ceil(rows / 128) <= B / 128 chunks of B2 <= 128 rows
    // of sums, so a block product's B rows of one chunk cover it)
    int64_t tpart_len = 0;
    if (toep)
        for (const gl::Problem &pb : ctx->probs)
            tpart_len = std::max(tpart_len,
                                 max_chunks(ctx, ctx->B, pb.P, opt.max_steps) * ctx->B * pb.P);
    ctx->tpart_len = tpart_len;
    need += (size_t)tpart_len * sizeof(float);
    size_t free_b = 0, total_b = 0;
    HIP_TRY(ctx, hipMemGetInfo(&free_b, &total_b));
    if (need + (size_t)(256u << 20) > free_b)
        return fail(ctx, GL_ENOMEM, "gl_init: need %.3f GB of device memory, %.3f GB free",
                    need / 1e9, free_b / 1e9);

    ctx->sched = gl::build_schedule(opt, opt.max_steps);
    gl_status st;
    // room for every problem's largest split count, whatever GEMV target gl_autotune picks
    ctx->bpart_cap = bpart_cap;
    if ((st = dev_alloc(ctx, &ctx->bpartial, ctx->bpart_cap))) return st;
    if ((st = dev_alloc(ctx, &ctx->d_batch, (size_t)nprob))) return st;
    if ((st = dev_alloc(ctx, &ctx->d_runs, ctx->sched.runs.size()))) return st;
    HIP_TRY(ctx, hipMemcpy(ctx->d_runs, ctx->sched.runs.data(),
                           ctx->sched.runs.size() * sizeof(gl::Run), hipMemcpyHostToDevice));
    if ((st = dev_alloc(ctx, &ctx->partial, part_len))) return st;
    ctx->part_len = part_len;
    if ((st = dev_alloc(ctx, &ctx->d_flag, 1))) return st;

    if (toep && (st = dev_alloc(ctx, &ctx->tpart, (size_t)std::max<int64_t>(tpart_len, 1))))
        return st;


    for (gl::Problem &pb : ctx->probs) {
        if ((st = dev_alloc(ctx, &pb.psi, npsi))) return st;
        if ((st = dev_alloc(ctx, &pb.dpsi, npsi))) return st;
        if ((st = dev_alloc(ctx, &pb.H, (size_t)rows * pb.ld))) return st;
        if ((st = dev_alloc(ctx, &pb.u[0], pb.P))) return st;
        if ((st = dev_alloc(ctx, &pb.u[1], pb.P))) return st;
        if ((st = dev_alloc(ctx, &pb.snap, (size_t)nsnap * pb.P))) return st;
        ctx->maxP = std::max(ctx->maxP, pb.P);
        ctx->maxld = std::max(ctx->maxld, pb.ld);
        gl::launch_weights(pb.p.gamma, npsi - 1, pb.psi, pb.dpsi, ctx->stream);
        HIP_TRY(ctx, hipGetLastError());
        ctx->upd_wgs += (pb.P + 255) / 256;
        if (toep) {
            pb.tab_len = tab_len;
            if ((st = dev_alloc(ctx, &pb.psi_tab, 16 * (size_t)tab_len))) return st;
            if ((st = dev_alloc(ctx, &pb.old, (size_t)ctx->B * pb.P))) return st;
            if (ctx->B2 && (st = dev_alloc(ctx, &pb.old2, (size_t)ctx->B2 * pb.P))) return st;
            if (carry_ok(ctx))
                for (int c = 0; c < 2; ++c)
                    if ((st = dev_alloc(ctx, &pb.carry[c], (size_t)gl::kMaxFuse * pb.P))) return st;
            // short memory (eq. (22)) is full memory with psi(m) = 0 for m > L
            const int64_t nkeep = opt.mem_mode == GL_MEM_SHORT ? std::min(npsi, opt.short_L + 1) : npsi;
            pb.psi_blk = pb.psi;
            if (nkeep < npsi) {
                if ((st = dev_alloc(ctx, &pb.psi_blk, npsi))) return st;
                HIP_TRY(ctx, hipMemcpyAsync(pb.psi_blk, pb.psi, nkeep * sizeof(double),
                                            hipMemcpyDeviceToDevice, ctx->stream));
                // zeros past the window: a chunk reduction over no chunks writes 0.0
                gl::launch_old_reduce(nullptr, 0, 1, npsi - nkeep, pb.psi_blk + nkeep, nullptr,
                                      ctx->stream);
            }
            gl::launch_psi_tables(pb.psi_blk, nkeep, tab_len, pb.psi_tab, ctx->stream);
            HIP_TRY(ctx, hipGetLastError());
        }
    }
    if ((st = apply_gemv_target(ctx, ctx->tune.gemv_groups)) != GL_OK) return st;
    return load_initial(ctx, u0);
}

void release(gl_ctx *ctx) {
    for (void *p : ctx->allocs) (void)hipFree(p);
    ctx->allocs.clear();
    for (auto &pd : ctx->pending) {
        ctx->event_pool.push_back(pd.start);
        ctx->event_pool.push_back(pd.stop);
    }
    ctx->pending.clear();
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    ctx->event_pool.clear();
}

gl_status take_event(gl_ctx *ctx, hipEvent_t *ev) {
    if (ctx->event_pool.empty()) {
        HIP_TRY(ctx, hipEventCreate(ev));
    } else {
        *ev = ctx->event_pool.back();
        ctx->event_pool.pop_back();
    }
    return GL_OK;
}

// Adds the durations of the pending event pairs (the stream must be synchronised).
gl_status resolve_profile(gl_ctx *ctx) {
    for (auto &pd : ctx->pending) {
        float ms = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, pd.start, pd.stop));
        ctx->prof_ms[pd.kernel] += ms;
        ctx->prof_launches[pd.kernel] += 1;
        ctx->event_pool.push_back(pd.start);
        ctx->event_pool.push_back(pd.stop);
    }
    ctx->pending.clear();
    return GL_OK;
}

// Runs launch() (exactly one kernel launch) and, in profiling mode, has the runtime stamp
// a start and a stop event at that kernel's own start and end.
template <class F>
gl_status timed(gl_ctx *ctx, int kernel, F &&launch) {
    if (!ctx->prof) {
        launch();
        return GL_OK;
    }
    gl_ctx::Pending pd{kernel, nullptr, nullptr};
    gl_status st;
    if ((st = take_event(ctx, &pd.start)) || (st = take_event(ctx, &pd.stop))) return st;
    gl::g_kernel_timer = gl::KernelTimer{pd.start, pd.stop};
    launch();
    gl::g_kernel_timer = gl::KernelTimer{};
    HIP_TRY(ctx, hipGetLastError());
    ctx->pending.push_back(pd);
    if (ctx->pending.size() >= 4096) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        return resolve_profile(ctx);
    }
    return GL_OK;
}

// Starts every problem from u0 at k = 0 and checks u0 is finite.
gl_status load_initial(gl_ctx *ctx, const double *u0) {
    for (gl::Problem &pb : ctx->probs) {
        pb.cur = 0;
        pb.old_k0 = -1;
        pb.old2_k1 = -1;
        pb.carry_k = -1;
        HIP_TRY(ctx, hipMemcpyAsync(pb.u[0], u0 + pb.offset, pb.P * sizeof(double),
                                    hipMemcpyDeviceToDevice, ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(pb.snap, u0 + pb.offset, pb.P * sizeof(double),
                                    hipMemcpyDeviceToDevice, ctx->stream));
    }
    ctx->k = 0;
    HIP_TRY(ctx, hipMemsetAsync(ctx->d_flag, 0, sizeof(int), ctx->stream));
    for (gl::Problem &pb : ctx->probs) gl::launch_check_finite(pb.u[0], pb.P, ctx->d_flag, ctx->stream);
    int flag = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (flag) return fail(ctx, GL_ENONFINITE, "u0 holds NaN or Inf");
    return GL_OK;
}

// One step k -> k + 1 of every problem on the plain GEMV path: one batched GEMV launch
// over all problems' history rows (terms m >= 1; psi(0) delta[k] is added in FP64 by
// the update) and one batched update launch.
gl_status step_gemv(gl_ctx *ctx) {
    const int64_t k = ctx->k;
    const int64_t rb = ctx->sched.run_begin[k];
    const int nruns = (int)(ctx->sched.run_begin[k + 1] - rb);
    const int64_t T = ctx->sched.terms[k];
    const int nprob = (int)ctx->probs.size();
    const int cur = ctx->probs[0].cur;
    const bool reverse = ctx->tune.serpentine && (k & 1);
    const int64_t wgs = gl::batched_gemv_groups(ctx->probs, T - 1);
    gl_status st;
    if (wgs > 0) {
        st = timed(ctx, GL_KERNEL_HIST_GEMV, [&] {
            gl::launch_hist_gemv_batched(ctx->d_batch, nprob, wgs, ctx->d_runs + rb, nruns, k, 1, T,
                                         reverse, ctx->stream);
        });
        if (st != GL_OK) return st;
    }
    st = timed(ctx, GL_KERNEL_UPDATE, [&] {
        gl::launch_update_batched(ctx->d_batch, nprob, ctx->upd_wgs, k, cur, T - 1, ctx->C,
                                  ctx->stream);
    });
    if (st != GL_OK) return st;
    for (gl::Problem &pb : ctx->probs) pb.cur ^= 1;
    HIP_TRY(ctx, hipGetLastError());
    ctx->k = k + 1;
    return GL_OK;
}

// out[b] = sum_{j_lo <= j < j_hi} psi(k_out + b - j) hist[j] for b < BM, on the matrix
// cores (FP32 chunk products summed in FP64).
// (base[b] +) out[b] = sum_{j_lo <= j < j_hi} psi(k_out + b - j) hist[j] for b < BM, on the
// matrix cores (FP32 chunk products summed in FP64; one chunk is written by the product
// kernel itself).
gl_status block_sums(gl_ctx *ctx, gl::Problem &pb, const uint16_t *tab, const float *hist,
                     int64_t ld, int BM, int64_t k_out, int64_t j_lo, int64_t j_hi, double *out,
                     const double *base, int gemm_id, int reduce_id) {
    if (j_hi <= j_lo)  // no rows in the window: the sums are the base (or zero)
        return timed(ctx, reduce_id, [&] {
            gl::launch_old_reduce(ctx->tpart, 0, BM, pb.P, out, base, ctx->stream);
        });
    const int64_t kchunk = chunk_rows(ctx, BM, pb.P, j_hi - j_lo);
    const int nchunk = gl::toeplitz_chunks(j_hi - j_lo, kchunk);
    if (nchunk > 1 && (int64_t)nchunk * BM * pb.P > ctx->tpart_len)
        return fail(ctx, GL_EINVAL, "internal: %d chunk products of %d x %lld exceed the buffer",
                    nchunk, BM, (long long)pb.P);
    bool launched = false;
    gl_status st = timed(ctx, gemm_id, [&] {
        launched = gl::launch_toeplitz_gemm(BM, hist, ld, pb.P, tab, pb.tab_len, k_out, j_lo,
                                            j_hi, kchunk, ctx->tpart, out, base, ctx->stream);
    });
    if (st == GL_OK && !launched)
        return fail(ctx, GL_EINVAL, "internal: Toeplitz product over rows [%lld, %lld) for step "
                    "%lld, %d rows out, refused", (long long)j_lo, (long long)j_hi,
                    (long long)k_out, BM);
    if (st != GL_OK || nchunk <= 1) return st;
    return timed(ctx, reduce_id, [&] {
        gl::launch_old_reduce(ctx->tpart, nchunk, BM, pb.P, out, base, ctx->stream);
    });
}

// First history row that can reach step k_out or later: with short memory of L steps the
// weights of rows before k_out - L are zero (rounded down to the product kernel's 32-row
// alignment), otherwise row 0.
int64_t window_lo(const gl_ctx *ctx, int64_t k_out) {
    if (ctx->opt.mem_mode != GL_MEM_SHORT) return 0;
    return std::max<int64_t>(0, (k_out - ctx->opt.short_L) / 32 * 32);
}

// old[b] = sum_{j < k0} psi(k0 + b - j) hist[j] for b < B.
gl_status block_old(gl_ctx *ctx, gl::Problem &pb, const float *hist, int64_t ld, int64_t k0,
                    double *old) {
    return block_sums(ctx, pb, pb.psi_tab, hist, ld, ctx->B, k0, window_lo(ctx, k0), k0, old,
                      nullptr,
                      GL_KERNEL_TOEPLITZ, GL_KERNEL_OLD_REDUCE);
}

// Steps of the blocked path that one launch can take from step k: at most the fusion
// length, the steps left (limit) and those left in k's sub-block (its block with one level).
int64_t block_run(const gl_ctx *ctx, int64_t k, int64_t limit) {
    const int64_t b = k % ctx->B;
    const int64_t left = ctx->B2 ? ctx->B2 - b % ctx->B2 : ctx->B - b;
    return std::max<int64_t>(1, std::min({ctx->tune.fuse, limit, left}));
}

// Steps k .. k + s - 1 of one problem on the blocked path (s from block_run), from u_cur
// into u_next; u_rows (nullable, stride u_stride) receives the states in between, S_out
// (nullable, stride P) the steps' sums; write_history 0 leaves the history rows alone.
gl_status toeplitz_steps(gl_ctx *ctx, gl::Problem &pb, int64_t k, int64_t s,
                         const double *u_cur, double *u_next, double *u_rows, int64_t u_stride,
                         double *S_out, int write_history) {
    const int64_t b = k % ctx->B;
    const int64_t k0 = k - b;
    // sub-block of the step (the whole block when there is one level)
    const int64_t b2 = ctx->B2 ? b % ctx->B2 : b;
    const int64_t k1 = k - b2;
    if (s < 1 || s > gl::kMaxFuse || b2 + s > (ctx->B2 ? ctx->B2 : ctx->B))
        return fail(ctx, GL_EINVAL, "internal: %lld in-block steps from step %lld",
                    (long long)s, (long long)k);
    gl_status st;
    if (k0 > 0 && pb.old_k0 != k0) {
        if ((st = block_old(ctx, pb, pb.H, pb.ld, k0, pb.old)) != GL_OK) return st;
        pb.old_k0 = k0;
    }
    if (k1 > k0 && pb.old2_k1 != k1) {
        // Old2 holds Old (rows of the sub-block's steps) + the product over rows k0 .. k1-1
        if ((st = block_sums(ctx, pb, pb.psi_tab, pb.H, pb.ld, ctx->B2, k1,
                             std::max(k0, window_lo(ctx, k1)), k1, pb.old2,
                             k0 > 0 ? pb.old + (k1 - k0) * pb.P : nullptr, GL_KERNEL_SUBBLOCK,
                             GL_KERNEL_SUB_REDUCE)) != GL_OK)
            return st;
        pb.old2_k1 = k1;
    }
    if (pb.p.ndim == 3 && s > gl::kMaxFuse3)
        return fail(ctx, GL_EINVAL, "blocked path: %lld steps per launch on a 3D grid (at most %d)",
                    (long long)s, gl::kMaxFuse3);
    gl::BlockStepArgs args{};
    args.psi = pb.psi_blk;
    args.H = pb.H;
    args.ld = pb.ld;
    args.P = pb.P;
    args.ndim = pb.p.ndim;
    args.nx = pb.p.nx;
    args.ny = pb.p.ny;
    args.nz = pb.p.nz;
    args.rxn = pb.p.rxn;
    args.r = pb.r;
    args.dt = pb.p.dt;
    args.rate = pb.p.rxn_rate;
    args.has_pre = k1 > k0 || k0 > 0;
    args.pre = k1 > k0 ? pb.old2 : pb.old;
    args.pre_row = (int32_t)(k1 > k0 ? b2 : b);
    args.u_cur = u_cur;
    args.u_next = u_next;
    args.u_rows = u_rows;
    args.u_stride = u_stride;
    args.S_out = S_out;
    if (write_history && pb.snap) {
        args.snap = pb.snap;
        for (int64_t i = s - 1; i >= 0; --i)
            if ((k + i + 1) % ctx->C == 0) {
                args.snap_mask |= 1u << i;
                args.snap_row0 = (k + i + 1) / ctx->C;
            }
    }
    args.k = k;
    args.b = (int32_t)b;
    args.b2 = (int32_t)b2;
    args.s = (int32_t)s;
    args.write_history = write_history;
    // chain carries between consecutive launches of a sub-block
    const int64_t sub_len = ctx->B2 ? ctx->B2 : ctx->B;
    int out_buf = 0;
    if (carry_ok(ctx)) {
        if (pb.carry_k == k && s <= pb.carry_n) {
            args.carry_in = pb.carry[pb.carry_cur];
            out_buf = pb.carry_cur ^ 1;
        } else if (b2 == 0 && args.has_pre) {
            // a sub-block's first launch has no rows of its own to sum: its chains start at
            // Old + Old2, which the carry variant of the kernel reads as its carry
            args.carry_in = args.pre + (int64_t)args.pre_row * pb.P;
        }
        if (b2 + s < sub_len) {
            args.carry_out = pb.carry[out_buf];
            args.n_next = (int32_t)std::min<int64_t>(ctx->tune.fuse, sub_len - (b2 + s));
        }
    }
    st = timed(ctx, GL_KERNEL_TRIANGLE, [&] { gl::launch_block_step(args, ctx->stream); });
    if (st != GL_OK) return st;
    if (args.carry_out) {
        pb.carry_k = k + s;
        pb.carry_n = args.n_next;
        pb.carry_cur = out_buf;
    } else {
        pb.carry_k = -1;
    }
    return GL_OK;
}

// Up to `limit` steps on the blocked path (one launch per problem; *done receives the
// count): at the start of each block of B steps the sums over the states before the block
// are formed by the Toeplitz product, at each sub-block start the one over the block's rows
// before it; the in-block steps then run several per kernel.
gl_status step_toeplitz(gl_ctx *ctx, int64_t limit, int64_t *done) {
    const int64_t k = ctx->k;
    const int64_t s = block_run(ctx, k, limit);
    for (gl::Problem &pb : ctx->probs) {
        gl_status st = toeplitz_steps(ctx, pb, k, s, pb.u[pb.cur], pb.u[pb.cur ^ 1], nullptr, 0,
                                      nullptr, 1);
        if (st != GL_OK) return st;
        pb.cur ^= 1;
    }
    HIP_TRY(ctx, hipGetLastError());
    ctx->k = k + s;
    *done = s;
    return GL_OK;
}

// Recomputes u[ks..ke] of one problem from the snapshot u[ks] with the forward's own
// kernels (bit-identical to the forward run), keeping u[k] in adj_u, the step sums S[k]
// in adj_S and the sums G[k] with d psi / d gamma in adj_G (k in [ks, ke)).
gl_status adjoint_recompute(gl_ctx *ctx, gl::Problem &pb, int64_t ks, int64_t ke) {
    const int64_t P = pb.P;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->adj_u, pb.snap + (ks / ctx->C) * P, P * sizeof(double),
                                hipMemcpyDeviceToDevice, ctx->stream));
    const bool toep = ctx->opt.sum_path == GL_SUM_TOEPLITZ_BF16X3;
    gl_status st;
    if (toep) {
        for (int64_t k = ks; k < ke;) {
            const int64_t i = k - ks, s = block_run(ctx, k, ke - k);
            if ((st = toeplitz_steps(ctx, pb, k, s, ctx->adj_u + i * P, ctx->adj_u + (i + s) * P,
                                     ctx->adj_u + (i + 1) * P, P, ctx->adj_S + i * P, 0)) != GL_OK)
                return st;
            k += s;
        }
    }
    for (int64_t k = ks; k < ke && !toep; ++k) {
        const int64_t i = k - ks;
        const double *u = ctx->adj_u + i * P;
        double *un = ctx->adj_u + (i + 1) * P;
        double *S = ctx->adj_S + i * P;
        const int64_t rb = ctx->sched.run_begin[k];
        const int nruns = (int)(ctx->sched.run_begin[k + 1] - rb);
        const int64_t T = ctx->sched.terms[k];
        const int nsplit = gl::gemv_splits(T - 1, P, pb.gemv_groups);
        const bool reverse = ctx->tune.serpentine && (k & 1);
        // S[k] as the forward formed it, and G[k] = sum over the same terms of
        // d psi / d gamma (m) delta[k-m] (the m = 0 weight is 0), in one pass over the rows
        if (nsplit > 0)
            gl::launch_hist_gemv_dual(pb.H, pb.ld, P, pb.psi, pb.dpsi, ctx->d_runs + rb, nruns, k,
                                      1, T, nsplit, reverse, ctx->partial, ctx->adj_partial2,
                                      ctx->stream);
        gl::launch_update(pb, u, nullptr, un, nullptr, S, ctx->partial, nsplit, ctx->stream);
        gl::launch_reduce_partials(ctx->adj_partial2, nsplit, P, nullptr, ctx->adj_G + i * P,
                                   ctx->stream);
    }
    if (toep) {
        // blocked: G for the B steps of each block k_a .. k_a + B - 1 in one matrix-core
        // product with the d psi / d gamma tables over every history row before the block's
        // end: d psi / d gamma (0) = 0 and the tables are zero for m < 0, so row j adds to the
        // steps after it only, and every row is already in the history (the forward wrote
        // rows 0 .. n - 1); the segment's steps are copied out of the block's sums
        const int64_t n = ctx->k;
        for (int64_t ka = ks - ks % ctx->B; ka < ke; ka += ctx->B) {
            if ((st = block_sums(ctx, pb, pb.dpsi_tab, pb.H, pb.ld, ctx->B, ka,
                                 window_lo(ctx, ka), std::min(ka + ctx->B, n), ctx->adj_oldG,
                                 nullptr, GL_KERNEL_TOEPLITZ, GL_KERNEL_OLD_REDUCE)) != GL_OK)
                return st;
            const int64_t k_lo = std::max(ka, ks), k_hi = std::min(ka + ctx->B, ke);
            HIP_TRY(ctx, hipMemcpyAsync(ctx->adj_G + (k_lo - ks) * P,
                                        ctx->adj_oldG + (k_lo - ka) * P,
                                        (size_t)(k_hi - k_lo) * P * sizeof(double),
                                        hipMemcpyDeviceToDevice, ctx->stream));
        }
    }
    HIP_TRY(ctx, hipGetLastError());
    return GL_OK;
}

gl_status adjoint_alloc(gl_ctx *ctx) {
    if (ctx->adj_M) return GL_OK;
    const int64_t C = ctx->C, n = ctx->opt.max_steps;
    const int groups = gl::adjoint_groups(ctx->maxP);
    const bool toep = ctx->opt.sum_path == GL_SUM_TOEPLITZ_BF16X3;
    size_t need = ((size_t)n * ctx->maxld) * sizeof(float) +
                  ((size_t)(3 * C + 1) * ctx->maxP + 2 * (size_t)ctx->maxP +
                   (size_t)n * groups * 3 + 3 * gl::kAdjFinalParts) * sizeof(double);
    if (!toep) need += ctx->part_len * sizeof(double);
    if (toep) {
        need += (2 * (size_t)ctx->B + ctx->B2 + C + 1 + 2 * gl::kMaxFuse) * ctx->maxP *
                sizeof(double);
        for (const gl::Problem &pb : ctx->probs) need += 16 * (size_t)pb.tab_len * sizeof(uint16_t);
    }
    size_t free_b = 0, total_b = 0;
    HIP_TRY(ctx, hipMemGetInfo(&free_b, &total_b));
    if (need + (size_t)(256u << 20) > free_b)
        return fail(ctx, GL_ENOMEM, "gl_adjoint: need %.3f GB of device memory, %.3f GB free",
                    need / 1e9, free_b / 1e9);
    gl_status st;
    if ((st = dev_alloc(ctx, &ctx->adj_M, (size_t)n * ctx->maxld))) return st;
    if ((st = dev_alloc(ctx, &ctx->adj_u, (size_t)(C + 1) * ctx->maxP))) return st;
    if ((st = dev_alloc(ctx, &ctx->adj_S, (size_t)C * ctx->maxP))) return st;
    if ((st = dev_alloc(ctx, &ctx->adj_G, (size_t)C * ctx->maxP))) return st;
    if ((st = dev_alloc(ctx, &ctx->adj_lam[0], ctx->maxP))) return st;
    if ((st = dev_alloc(ctx, &ctx->adj_lam[1], ctx->maxP))) return st;
    if ((st = dev_alloc(ctx, &ctx->adj_grad, (size_t)n * groups * 3))) return st;
    if ((st = dev_alloc(ctx, &ctx->adj_fpart, (size_t)gl::kAdjFinalParts * 3))) return st;
    if (!toep && (st = dev_alloc(ctx, &ctx->adj_partial2, ctx->part_len))) return st;
    if (toep) {
        if ((st = dev_alloc(ctx, &ctx->adj_oldA, (size_t)ctx->B * ctx->maxP))) return st;
        if ((st = dev_alloc(ctx, &ctx->adj_oldG, (size_t)ctx->B * ctx->maxP))) return st;
        if (ctx->B2 && (st = dev_alloc(ctx, &ctx->adj_oldA2, (size_t)ctx->B2 * ctx->maxP)))
            return st;
        if ((st = dev_alloc(ctx, &ctx->adj_lamseg, (size_t)(C + 1) * ctx->maxP))) return st;
        if (carry_ok(ctx))
            for (int c = 0; c < 2; ++c)
                if ((st = dev_alloc(ctx, &ctx->adj_carry[c], (size_t)gl::kMaxFuse * ctx->maxP)))
                    return st;
        // d psi / d gamma tables (zero past a short-memory window, as the psi tables)
        const int64_t npsi = ctx->opt.max_steps + gl::kMaxBlock + 1;
        const int64_t nkeep = ctx->opt.mem_mode == GL_MEM_SHORT
                                  ? std::min(npsi, ctx->opt.short_L + 1)
                                  : npsi;
        for (gl::Problem &pb : ctx->probs) {
            if ((st = dev_alloc(ctx, &pb.dpsi_tab, 16 * (size_t)pb.tab_len))) return st;
            gl::launch_psi_tables(pb.dpsi, nkeep, pb.tab_len, pb.dpsi_tab, ctx->stream);
        }
        HIP_TRY(ctx, hipGetLastError());
    }
    return GL_OK;
}

// The reverse sweep's schedule over the n steps taken: the forward schedule itself for full
// and short memory, its transpose (built on the host, copied to adj_runs) for adaptive memory.
gl_status reverse_schedule(gl_ctx *ctx, int64_t n, gl::Schedule *tsched,
                           const gl::Schedule **ts, const gl::Run **truns) {
    *ts = &ctx->sched;
    *truns = ctx->d_runs;
    if (ctx->opt.mem_mode != GL_MEM_ADAPTIVE) return GL_OK;
    *tsched = gl::transpose_schedule(ctx->sched, n);
    const size_t nruns = tsched->runs.size();
    if (nruns > ctx->adj_runs_cap) {
        if (ctx->adj_runs) {
            ctx->allocs.erase(std::find(ctx->allocs.begin(), ctx->allocs.end(),
                                        (void *)ctx->adj_runs));
            HIP_TRY(ctx, hipFree(ctx->adj_runs));
            ctx->adj_runs = nullptr;
            ctx->adj_runs_cap = 0;
        }
        gl_status st = dev_alloc(ctx, &ctx->adj_runs, nruns);
        if (st != GL_OK) return st;
        ctx->adj_runs_cap = nruns;
    }
    HIP_TRY(ctx, hipMemcpy(ctx->adj_runs, tsched->runs.data(), nruns * sizeof(gl::Run),
                           hipMemcpyHostToDevice));
    *ts = tsched;
    *truns = ctx->adj_runs;
    return GL_OK;
}

// Reverse steps of one segment [ks, ke) of a problem on the blocked path, from lam[ke] in
// adj_lamseg row ke - ks: the sums over the mu rows before each reverse block by the
// matrix-core product (once per block), with sub-blocks those over the block's rows before
// each sub-block by a second product on that base (once per sub-block), and the rows since
// by the in-block kernel, up to the fusion length of reverse steps per launch inside one
// sub-block; then the segment's dot products in one launch.
gl_status adjoint_segment_blocked(gl_ctx *ctx, gl::Problem &pb, int64_t ks, int64_t ke) {
    const int64_t n = ctx->k, P = pb.P;
    const int64_t sub_len = ctx->B2 ? ctx->B2 : ctx->B;
    const int64_t max_s = pb.p.ndim == 3 ? std::min<int64_t>(ctx->tune.fuse, gl::kMaxFuse3)
                                         : ctx->tune.fuse;
    gl_status st;
    for (int64_t k = ke - 1; k >= ks;) {
        const int64_t rho = n - 1 - k;  // reverse step
        const int64_t r0 = rho - rho % ctx->B;
        if (ctx->adj_oldA_r0 != r0) {
            if ((st = block_sums(ctx, pb, pb.psi_tab, ctx->adj_M, pb.ld, ctx->B, r0,
                                 window_lo(ctx, r0), r0, ctx->adj_oldA, nullptr,
                                 GL_KERNEL_TOEPLITZ, GL_KERNEL_OLD_REDUCE)) != GL_OK)
                return st;
            ctx->adj_oldA_r0 = r0;
            ctx->adj_oldA2_r1 = -1;
        }
        const int64_t r1 = rho - rho % sub_len, c = rho - r1;
        if (r1 > r0 && ctx->adj_oldA2_r1 != r1) {
            if ((st = block_sums(ctx, pb, pb.psi_tab, ctx->adj_M, pb.ld, ctx->B2, r1,
                                 std::max(r0, window_lo(ctx, r1)), r1, ctx->adj_oldA2,
                                 ctx->adj_oldA + (r1 - r0) * P, GL_KERNEL_SUBBLOCK,
                                 GL_KERNEL_SUB_REDUCE)) != GL_OK)
                return st;
            ctx->adj_oldA2_r1 = r1;
        }
        const int64_t s = std::max<int64_t>(1, std::min({max_s, sub_len - c, k - ks + 1}));
        gl::BlockStepArgs args{};
        args.psi = pb.psi_blk;
        args.H = ctx->adj_M;
        args.ld = pb.ld;
        args.P = P;
        args.ndim = pb.p.ndim;
        args.nx = pb.p.nx;
        args.ny = pb.p.ny;
        args.nz = pb.p.nz;
        args.rxn = pb.p.rxn;
        args.r = pb.r;
        args.dt = pb.p.dt;
        args.rate = pb.p.rxn_rate;
        args.pre = (r1 > r0 ? ctx->adj_oldA2 : ctx->adj_oldA) + c * P;
        args.pre_row = 0;
        args.has_pre = 1;  // zero sums before the first block
        args.u_cur = ctx->adj_lamseg + (k + 1 - ks) * P;
        args.lam_rows = ctx->adj_lamseg + (k - ks) * P;
        args.u_rev = ctx->adj_u + (k - ks) * P;
        args.k = rho;
        args.b = (int32_t)(rho - r0);
        args.b2 = (int32_t)c;
        args.s = (int32_t)s;
        args.write_history = 1;
        // chain carries between consecutive launches of a sub-block, as on the forward (the
        // sweep runs the sub-block's launches in order, across segment boundaries too: the
        // recomputation in between uses the forward's own carry buffers)
        int out_buf = 0;
        if (carry_ok(ctx)) {
            if (ctx->adj_carry_rho == rho && s <= ctx->adj_carry_n) {
                args.carry_in = ctx->adj_carry[ctx->adj_carry_cur];
                out_buf = ctx->adj_carry_cur ^ 1;
            } else if (c == 0) {
                args.carry_in = args.pre;  // a sub-block's chains start at the sums before it
            }
            if (c + s < sub_len) {
                args.carry_out = ctx->adj_carry[out_buf];
                args.n_next = (int32_t)std::min<int64_t>(max_s, sub_len - (c + s));
            }
        }
        gl::launch_adjoint_steps(args, ctx->stream);
        if (args.carry_out) {
            ctx->adj_carry_rho = rho + s;
            ctx->adj_carry_n = args.n_next;
            ctx->adj_carry_cur = out_buf;
        } else {
            ctx->adj_carry_rho = -1;
        }
        k -= s;
    }
    gl::launch_adjoint_dots(pb, ctx->adj_lamseg, ctx->adj_u, ctx->adj_S, ctx->adj_G, ks, ke - ks,
                            ctx->adj_grad, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GL_OK;
}

// Reverse sweep of every problem over the steps taken so far (see gl_adjoint.hip).
gl_status adjoint_impl(gl_ctx *ctx, const double *dL_duT, double *dL_du0, double *dparams) {
    gl_status st;
    if ((st = adjoint_alloc(ctx)) != GL_OK) return st;
    const int64_t n = ctx->k, C = ctx->C;
    gl::Schedule tsched;
    const gl::Schedule *ts = nullptr;
    const gl::Run *truns = nullptr;
    if ((st = reverse_schedule(ctx, n, &tsched, &ts, &truns)) != GL_OK) return st;
    const bool toep = ctx->opt.sum_path == GL_SUM_TOEPLITZ_BF16X3;
    for (size_t ip = 0; ip < ctx->probs.size(); ++ip) {
        gl::Problem &pb = ctx->probs[ip];
        const int64_t P = pb.P;
        const int groups = gl::adjoint_groups(P);
        const double *lam_top = dL_duT + pb.offset;  // lam at the top of the next segment
        int cur = 0;
        ctx->adj_oldA_r0 = ctx->adj_oldA2_r1 = -1;  // block sums of this problem's mu history
        ctx->adj_carry_rho = -1;
        if (!toep)
            HIP_TRY(ctx, hipMemcpyAsync(ctx->adj_lam[0], lam_top, P * sizeof(double),
                                        hipMemcpyDeviceToDevice, ctx->stream));
        for (int64_t seg = (n - 1) / C; seg >= 0; --seg) {
            const int64_t ks = seg * C, ke = std::min(ks + C, n);
            if ((st = adjoint_recompute(ctx, pb, ks, ke)) != GL_OK) return st;
            if (toep) {
                HIP_TRY(ctx, hipMemcpyAsync(ctx->adj_lamseg + (ke - ks) * P, lam_top,
                                            P * sizeof(double), hipMemcpyDeviceToDevice,
                                            ctx->stream));
                if ((st = adjoint_segment_blocked(ctx, pb, ks, ke)) != GL_OK) return st;
                lam_top = ctx->adj_lamseg;  // lam[ks], row 0
                continue;
            }
            for (int64_t k = ke - 1; k >= ks; --k) {
                const int64_t rho = n - 1 - k;  // reverse step: the reverse schedule at rho
                const int64_t rb = ts->run_begin[rho], T = ts->terms[rho];
                const int nruns = (int)(ts->run_begin[rho + 1] - rb);
                const int nsplit = gl::gemv_splits(T - 1, P, pb.gemv_groups);
                if (nsplit > 0)
                    gl::launch_hist_gemv(ctx->adj_M, pb.ld, P, pb.psi, truns + rb, nruns, rho, 1,
                                         T, nsplit, false, ctx->partial, ctx->stream);
                const int64_t i = k - ks;
                gl::launch_adjoint_update(pb, ctx->adj_lam[cur], ctx->adj_lam[cur ^ 1],
                                          ctx->adj_M + rho * pb.ld, ctx->partial, nsplit,
                                          ctx->adj_u + i * P, ctx->adj_S + i * P,
                                          ctx->adj_G + i * P, ctx->adj_grad + k * groups * 3,
                                          ctx->stream);
                cur ^= 1;
            }
            HIP_TRY(ctx, hipGetLastError());
        }
        HIP_TRY(ctx, hipMemcpyAsync(dL_du0 + pb.offset, toep ? lam_top : ctx->adj_lam[cur],
                                    P * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        gl::launch_adjoint_final(ctx->adj_grad, n * groups, pb.r, pb.p.alpha, std::log(pb.p.dt),
                                 pb.p.dt, ctx->adj_fpart, dparams + 3 * ip, ctx->stream);
        HIP_TRY(ctx, hipGetLastError());
    }
    return GL_OK;
}

gl_status copy_state(gl_ctx *ctx, double *dst) {
    for (gl::Problem &pb : ctx->probs)
        HIP_TRY(ctx, hipMemcpyAsync(dst + pb.offset, pb.u[pb.cur], pb.P * sizeof(double),
                                    hipMemcpyDeviceToDevice, ctx->stream));
    return GL_OK;
}

// Fastest of `reps` timed runs of launch() on the context's stream after one untimed run, in
// milliseconds, from events recorded around it.
template <class F>
gl_status time_best(gl_ctx *ctx, int reps, F launch, float *best) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, GL_EHIP, "hipEventCreate failed");
    }
    gl_status st = GL_OK;
    *best = 0.f;
    for (int r = 0; r <= reps && st == GL_OK; ++r) {
        if ((st = launch()) != GL_OK) break;  // r = 0: the untimed run
        if (r == 0) continue;
        float ms = 0.f;
        if (hipEventRecord(e0, ctx->stream) != hipSuccess || (st = launch()) != GL_OK ||
            hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            if (st == GL_OK) st = fail(ctx, GL_EHIP, "timing a candidate failed");
            break;
        }
        if (r == 1 || ms < *best) *best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

// Candidate launch shapes timed on the context's own problems at step max_steps / 2 (the
// mean depth of a full-memory run), keeping the fastest:
//  - plain path: the GEMV workgroup target (split-K fan-out), one GEMV + update step of
//    every problem per candidate;
//  - blocked path: the product's workgroups per CU (its chunk count), the block product of
//    every problem over the rows before the block at that depth.
// Kernels read the history arena as it stands and write only rows, states and sums that
// the run overwrites before reading them, so the context stays at step 0.
gl_status autotune_impl(gl_ctx *ctx, int32_t what, int64_t *chosen) {
    const bool toep = ctx->opt.sum_path == GL_SUM_TOEPLITZ_BF16X3;
    // a step the run can take (k <= max_steps - 1), so the rows and checkpoint slots the
    // candidates write exist
    const int64_t kmid = ctx->opt.max_steps / 2;
    const int nprob = (int)ctx->probs.size();
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const bool prof = ctx->prof;
    ctx->prof = false;  // no per-kernel events around the candidates
    gl_status st = GL_OK;
    if ((what & GL_TUNE_GEMV) && st == GL_OK) {
        const int64_t rb = ctx->sched.run_begin[kmid];
        const int nruns = (int)(ctx->sched.run_begin[kmid + 1] - rb);
        const int64_t T = ctx->sched.terms[kmid];
        const int cur = ctx->probs[0].cur;
        float best = 0.f;
        int64_t best_g = ctx->tune.gemv_groups;
        for (int64_t g : {int64_t(256), int64_t(512), int64_t(1024), int64_t(2048),
                          kMaxGemvTarget}) {
            HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
            if ((st = apply_gemv_target(ctx, g)) != GL_OK) break;
            float ms = 0.f;
            st = time_best(ctx, 3, [&]() -> gl_status {
                const int64_t wgs = gl::batched_gemv_groups(ctx->probs, T - 1);
                if (wgs > 0)
                    gl::launch_hist_gemv_batched(ctx->d_batch, nprob, wgs, ctx->d_runs + rb,
                                                 nruns, kmid, 1, T, false, ctx->stream);
                gl::launch_update_batched(ctx->d_batch, nprob, ctx->upd_wgs, kmid, cur, T - 1,
                                          ctx->C, ctx->stream);
                HIP_TRY(ctx, hipGetLastError());
                return GL_OK;
            }, &ms);
            if (st != GL_OK) break;
            if (g == 256 || ms < best) {
                best = ms;
                best_g = g;
            }
        }
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        if (st == GL_OK) st = apply_gemv_target(ctx, best_g);
    }
    const int64_t k0 = kmid / ctx->B * ctx->B;
    if ((what & GL_TUNE_PRODUCT) && toep && ctx->tune.kchunk == 0 && k0 >= ctx->B && st == GL_OK) {
        float best = 0.f;
        int64_t best_w = ctx->tune.chunk_wgs;
        for (int64_t w = 1; w <= gl::kMaxChunkWgs && st == GL_OK; w *= 2) {
            ctx->tune.chunk_wgs = w;
            float ms = 0.f;
            st = time_best(ctx, 2, [&]() -> gl_status {
                for (gl::Problem &pb : ctx->probs) {
                    gl_status s2 = block_old(ctx, pb, pb.H, pb.ld, k0, pb.old);
                    if (s2 != GL_OK) return s2;
                }
                HIP_TRY(ctx, hipGetLastError());
                return GL_OK;
            }, &ms);
            if (st == GL_OK && (w == 1 || ms < best)) {
                best = ms;
                best_w = w;
            }
        }
        ctx->tune.chunk_wgs = best_w;
        for (gl::Problem &pb : ctx->probs) {  // the sums written here are not the run's
            pb.old_k0 = pb.old2_k1 = -1;
            pb.carry_k = -1;
        }
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    ctx->prof = prof;
    if (st == GL_OK && chosen) {
        chosen[0] = ctx->tune.gemv_groups;
        chosen[1] = ctx->tune.kchunk > 0 ? 0 : ctx->tune.chunk_wgs;
    }
    return st;
}

}  // namespace

extern "C" {

gl_status gl_init(const gl_problem *probs, int32_t nprob, const gl_options *opt, const double *u0,
                  gl_ctx **out) {
    gl_status st = validate(probs, nprob, opt, u0, out);
    if (st != GL_OK) return st;
    std::unique_ptr<gl_ctx> ctx(new gl_ctx);
    ctx->opt = *opt;
    if (const char *v = env_value("GL_GEMV_GROUPS")) ctx->tune.gemv_groups = std::max(1L, std::atol(v));
    if (const char *v = env_value("GL_GEMV_SERPENTINE")) ctx->tune.serpentine = std::atoi(v) != 0;
    if (const char *v = env_value("GL_SUBBLOCK")) ctx->tune.sub_B = std::atol(v);
    if (const char *v = env_value("GL_FUSE"))
        ctx->tune.fuse = std::min<int64_t>(gl::kMaxFuse, std::max(1L, std::atol(v)));
    for (int32_t i = 0; i < nprob; ++i)  // 3D tiles take fewer steps per in-block launch
        if (probs[i].ndim == 3) ctx->tune.fuse = std::min<int64_t>(ctx->tune.fuse, gl::kMaxFuse3);
    if (const char *v = env_value("GL_TOEPLITZ_KCHUNK"))
        ctx->tune.kchunk = std::max<int64_t>(gl::kMaxTK, std::atol(v) / gl::kMaxTK * gl::kMaxTK);
    ctx->stream = static_cast<hipStream_t>(opt->stream);
    st = init_impl(ctx.get(), probs, nprob, u0);
    if (st != GL_OK) {
        g_thread_err = ctx->err;
        (void)hipStreamSynchronize(ctx->stream);
        release(ctx.get());
        return st;
    }
    *out = ctx.release();
    return GL_OK;
}

gl_status gl_step_n(gl_ctx *ctx, int64_t n, double *uT) {
    if (!ctx) return fail(nullptr, GL_EINVAL, "gl_step_n: ctx is NULL");
    if (n < 0) return fail(ctx, GL_EINVAL, "gl_step_n: n must be >= 0");
    if (ctx->k + n > ctx->opt.max_steps)
        return fail(ctx, GL_ECAPACITY, "gl_step_n: %lld + %lld steps exceed max_steps = %lld",
                    (long long)ctx->k, (long long)n, (long long)ctx->opt.max_steps);
    gl_status st;
    const bool toep = ctx->opt.sum_path == GL_SUM_TOEPLITZ_BF16X3;
    for (int64_t s = 0; s < n;) {
        int64_t done = 1;
        if ((st = toep ? step_toeplitz(ctx, n - s, &done) : step_gemv(ctx)) != GL_OK) return st;
        s += done;
    }
    if (uT && (st = copy_state(ctx, uT)) != GL_OK) return st;
    if (ctx->opt.check_finite) {
        HIP_TRY(ctx, hipMemsetAsync(ctx->d_flag, 0, sizeof(int), ctx->stream));
        for (gl::Problem &pb : ctx->probs)
            gl::launch_check_finite(pb.u[pb.cur], pb.P, ctx->d_flag, ctx->stream);
        int flag = 0;
        HIP_TRY(ctx, hipMemcpyAsync(&flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost,
                                    ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        if (flag) return fail(ctx, GL_ENONFINITE, "gl_step_n: state holds NaN or Inf at step %lld",
                              (long long)ctx->k);
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return resolve_profile(ctx);
}

gl_status gl_reset(gl_ctx *ctx, const double *u0) {
    if (!ctx) return fail(nullptr, GL_EINVAL, "gl_reset: ctx is NULL");
    if (!u0) return fail(ctx, GL_EINVAL, "gl_reset: u0 is NULL");
    return load_initial(ctx, u0);
}

gl_status gl_autotune(gl_ctx *ctx, int32_t what, int64_t *chosen) {
    if (!ctx) return fail(nullptr, GL_EINVAL, "gl_autotune: ctx is NULL");
    if (what & ~(GL_TUNE_GEMV | GL_TUNE_PRODUCT))
        return fail(ctx, GL_EINVAL, "gl_autotune: unknown bits in what = %d", what);
    if (ctx->k != 0)
        return fail(ctx, GL_ESTATE, "gl_autotune: %lld steps taken (tune at step 0)",
                    (long long)ctx->k);
    return autotune_impl(ctx, what ? what : GL_TUNE_GEMV | GL_TUNE_PRODUCT, chosen);
}

gl_status gl_set_profiling(gl_ctx *ctx, int32_t on) {
    if (!ctx) return fail(nullptr, GL_EINVAL, "gl_set_profiling: ctx is NULL");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    gl_status st = resolve_profile(ctx);
    if (st != GL_OK) return st;
    ctx->prof = on != 0;
    for (int i = 0; i < GL_KERNEL_COUNT; ++i) {
        ctx->prof_launches[i] = 0;
        ctx->prof_ms[i] = 0.0;
    }
    return GL_OK;
}

gl_status gl_profile(gl_ctx *ctx, int32_t kernel, int64_t *launches, double *total_ms) {
    if (!ctx) return fail(nullptr, GL_EINVAL, "gl_profile: ctx is NULL");
    if (kernel < 0 || kernel >= GL_KERNEL_COUNT || !launches || !total_ms)
        return fail(ctx, GL_EINVAL, "gl_profile: bad kernel id or NULL output");
    *launches = ctx->prof_launches[kernel];
    *total_ms = ctx->prof_ms[kernel];
    return GL_OK;
}

gl_status gl_adjoint(gl_ctx *ctx, const double *dL_duT, double *dL_du0, double *dparams) {
    if (!ctx) return fail(nullptr, GL_EINVAL, "gl_adjoint: ctx is NULL");
    if (!dL_duT || !dL_du0 || !dparams) return fail(ctx, GL_EINVAL, "gl_adjoint: NULL argument");
    if (ctx->k < 1) return fail(ctx, GL_ESTATE, "gl_adjoint: no forward step taken");
    gl_status st = adjoint_impl(ctx, dL_duT, dL_du0, dparams);
    for (gl::Problem &pb : ctx->probs) {  // sums and carries reused by the recomputation
        pb.old_k0 = pb.old2_k1 = -1;
        pb.carry_k = -1;
    }
    if (st != GL_OK) return st;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return resolve_profile(ctx);
}

void gl_free(gl_ctx *ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    release(ctx);
    delete ctx;
}

const char *gl_last_error(const gl_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_thread_err.c_str();
}

int64_t gl_steps_done(const gl_ctx *ctx) { return ctx ? ctx->k : -1; }

gl_status gl_get_state(gl_ctx *ctx, double *u) {
    if (!ctx) return fail(nullptr, GL_EINVAL, "gl_get_state: ctx is NULL");
    if (!u) return fail(ctx, GL_EINVAL, "gl_get_state: u is NULL");
    gl_status st = copy_state(ctx, u);
    if (st != GL_OK) return st;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return GL_OK;
}

gl_status gl_get_weights(gl_ctx *ctx, int32_t iprob, int64_t count, double *psi, double *dpsi) {
    if (!ctx) return fail(nullptr, GL_EINVAL, "gl_get_weights: ctx is NULL");
    if (iprob < 0 || iprob >= (int32_t)ctx->probs.size() || count < 0 ||
        count > ctx->opt.max_steps + 1)
        return fail(ctx, GL_EINVAL, "gl_get_weights: bad problem index or count");
    const gl::Problem &pb = ctx->probs[iprob];
    if (psi)
        HIP_TRY(ctx, hipMemcpyAsync(psi, pb.psi, count * sizeof(double), hipMemcpyDeviceToDevice,
                                    ctx->stream));
    if (dpsi)
        HIP_TRY(ctx, hipMemcpyAsync(dpsi, pb.dpsi, count * sizeof(double),
                                    hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return GL_OK;
}

int64_t gl_schedule_terms(const gl_ctx *ctx, int64_t k) {
    if (!ctx || k < 0 || k > ctx->opt.max_steps) return -1;
    return ctx->sched.terms[k];
}

gl_status gl_history_sum(gl_ctx *ctx, int32_t iprob, int64_t k, const float *hist, int64_t ld,
                         double *S) {
    if (!ctx) return fail(nullptr, GL_EINVAL, "gl_history_sum: ctx is NULL");
    if (iprob < 0 || iprob >= (int32_t)ctx->probs.size())
        return fail(ctx, GL_EINVAL, "gl_history_sum: bad problem index");
    const gl::Problem &pb = ctx->probs[iprob];
    if (!hist || !S) return fail(ctx, GL_EINVAL, "gl_history_sum: NULL argument");
    if (k < 0 || k > ctx->opt.max_steps)
        return fail(ctx, GL_EINVAL, "gl_history_sum: k out of [0, max_steps]");
    if (ld < pb.P || ld % 4 != 0 || (reinterpret_cast<uintptr_t>(hist) & 15u) != 0)
        return fail(ctx, GL_EINVAL, "gl_history_sum: need ld >= P, ld %% 4 == 0, 16-byte aligned");
    const int64_t rb = ctx->sched.run_begin[k];
    const int nruns = (int)(ctx->sched.run_begin[k + 1] - rb);
    int64_t t_end = ctx->sched.terms[k];
    const double *base = nullptr;
    if (ctx->opt.sum_path == GL_SUM_TOEPLITZ_BF16X3) {
        // rows before the block holding k on the matrix cores, rows k0..k on the plain path
        gl::Problem &pbm = ctx->probs[iprob];
        const int64_t b = k % ctx->B, k0 = k - b;
        if (k0 > 0) {
            pbm.old_k0 = pbm.old2_k1 = -1;  // old[] is reused as scratch here
            pbm.carry_k = -1;
            gl_status st = block_old(ctx, pbm, hist, ld, k0, pbm.old);
            if (st != GL_OK) return st;
            base = pbm.old + b * pbm.P;
        }
        t_end = std::min(b + 1, t_end);  // the schedule's terms m <= b (short memory: <= L)
    }
    const int nsplit = gl::gemv_splits(t_end, pb.P, ctx->tune.gemv_groups);
    gl::launch_hist_gemv(hist, ld, pb.P, pb.psi, ctx->d_runs + rb, nruns, k, 0, t_end, nsplit,
                         false, ctx->partial, ctx->stream);
    gl::launch_reduce_partials(ctx->partial, nsplit, pb.P, base, S, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return GL_OK;
}

}  // extern "C"
