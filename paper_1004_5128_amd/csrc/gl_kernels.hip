// HIP kernels of the plain history-sum path for gfx950 (CDNA4, wave64):
// GL weights, the history GEMV, the stencil + reaction update and helpers.
#include <hip/hip_runtime.h>

#include "gl_internal.h"

// Address spaces of device pointers: global memory, and constant (read-only) memory
// whose wave-uniform loads go through the scalar unit.  The kernels shared by the single
// and batched launches take qualified pointers, because pointers read from a table in
// memory would otherwise become generic (flat) accesses.
#define GL_GLOBAL __attribute__((address_space(1)))
#define GL_CONST __attribute__((address_space(4)))
typedef float f32x4_t __attribute__((ext_vector_type(4)));

namespace gl {

// ------------------------------------------------------------------ weights
//
// psi(gamma, m) = (-1)^m binom(1 - gamma, m) (Sec. 2.1, eq. (8)) by the
// recurrence of eq. (11) written as psi(m) = psi(m-1) (m - 2 + gamma) / m from
// psi(0) = 1 (eq. (12)), and its gamma-derivative by differentiating the same
// product: psi'(m) = psi'(m-1) (m - 2 + gamma) / m + psi(m-1) / m.  A single
// lane walks the recurrence; it runs once per context.
__global__ void weights_kernel(double gamma, int64_t n, double *__restrict__ psi,
                               double *__restrict__ dpsi) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double w = 1.0, dw = 0.0;
    psi[0] = w;
    dpsi[0] = dw;
    for (int64_t m = 1; m <= n; ++m) {
        const double inv_m = 1.0 / (double)m;
        const double ratio = ((double)m - 2.0 + gamma) * inv_m;
        const double dnext = dw * ratio + w * inv_m;
        w = w * ratio;
        dw = dnext;
        psi[m] = w;
        dpsi[m] = dw;
    }
}

void launch_weights(double gamma, int64_t n, double *psi, double *dpsi, hipStream_t s) {
    GL_LAUNCH(weights_kernel, dim3(1), dim3(64), 0, s, gamma, n, psi, dpsi);
}

// ------------------------------------------------------------ history GEMV
//
// Each step's sum sum_t coef_t psi(m_t) H[k - m_t, p] is a weighted reduction
// of whole history rows: a GEMV with a row-major [rows x P] FP32 matrix.  It
// is HBM-bound (4 bytes per multiply-add), so the kernel streams rows with
// 16-byte loads, 1 KB per wave per row, and keeps several rows in flight per
// lane.  A workgroup of 256 lanes owns 1024 consecutive points; the terms are
// split into gridDim.y contiguous ranges (split-K) so that small grids still
// fill the 256 CUs.  Weights are wave-uniform (scalar loads) and the
// accumulation is FP64 in term order: results are deterministic and depend only
// on the term sequence, the term range and the split count.

constexpr int kGemvThreads = 256;
constexpr int kGemvUnroll = 8;

// Terms [ta, tb) of the step-k schedule for the four points col..col+3 (col < P):
// returns their FP64 sums in a[0..3].
// kDual: also the sum with a second weight table psi2 over the same rows (the adjoint's
// d psi / d gamma sums), into b; the first sum's operations are the same either way.
template <bool kDual>
__device__ __forceinline__ void gemv_points(const GL_GLOBAL float *__restrict__ H, int64_t ld,
                                            const GL_CONST double *__restrict__ psi,
                                            const GL_CONST double *__restrict__ psi2,
                                            const GL_CONST Run *__restrict__ runs, int nruns,
                                            int64_t k, int64_t ta, int64_t tb, int64_t col,
                                            int reverse, double a[4], double b[4]) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
    // Runs are visited in order; with `reverse` the terms are walked from the last to the
    // first (oldest row first), so that consecutive steps can traverse the history in
    // opposite directions.
    int64_t tr0 = 0;
    if (reverse)
        for (int r = 0; r < nruns; ++r) tr0 += runs[r].count;
    for (int rr = 0; rr < nruns; ++rr) {
        const int r = reverse ? nruns - 1 - rr : rr;
        const Run run = {runs[r].m0, runs[r].count, runs[r].stride, runs[r].coef};
        int64_t tr1;
        if (reverse) {
            tr1 = tr0;
            tr0 = tr1 - run.count;
            if (tr1 <= ta) break;
        } else {
            tr1 = tr0 + run.count;
            if (tr0 >= tb) break;
        }
        const int64_t lo = ta > tr0 ? ta : tr0;
        const int64_t hi = tb < tr1 ? tb : tr1;
        if (lo < hi) {
            const int64_t stride = reverse ? -(int64_t)run.stride : (int64_t)run.stride;
            const double coef = (double)run.coef;
            int64_t m = run.m0 + ((reverse ? hi - 1 : lo) - tr0) * (int64_t)run.stride;
            const GL_GLOBAL float *row = H + (k - m) * ld + col;
            const int64_t step = stride * ld;
            int64_t cnt = hi - lo;
            while (cnt >= kGemvUnroll) {
                f32x4_t v[kGemvUnroll];
                double w[kGemvUnroll];
#pragma unroll
                for (int u = 0; u < kGemvUnroll; ++u)
                    v[u] = *reinterpret_cast<const GL_GLOBAL f32x4_t *>(row - u * step);
#pragma unroll
                for (int u = 0; u < kGemvUnroll; ++u) w[u] = coef * psi[m + u * stride];
#pragma unroll
                for (int u = 0; u < kGemvUnroll; ++u) {
                    a0 = fma(w[u], (double)v[u].x, a0);
                    a1 = fma(w[u], (double)v[u].y, a1);
                    a2 = fma(w[u], (double)v[u].z, a2);
                    a3 = fma(w[u], (double)v[u].w, a3);
                }
                if constexpr (kDual) {
#pragma unroll
                    for (int u = 0; u < kGemvUnroll; ++u) {
                        const double w2 = coef * psi2[m + u * stride];
                        b0 = fma(w2, (double)v[u].x, b0);
                        b1 = fma(w2, (double)v[u].y, b1);
                        b2 = fma(w2, (double)v[u].z, b2);
                        b3 = fma(w2, (double)v[u].w, b3);
                    }
                }
                row -= kGemvUnroll * step;
                m += kGemvUnroll * stride;
                cnt -= kGemvUnroll;
            }
            for (; cnt > 0; --cnt) {
                const f32x4_t v = *reinterpret_cast<const GL_GLOBAL f32x4_t *>(row);
                const double w = coef * psi[m];
                a0 = fma(w, (double)v.x, a0);
                a1 = fma(w, (double)v.y, a1);
                a2 = fma(w, (double)v.z, a2);
                a3 = fma(w, (double)v.w, a3);
                if constexpr (kDual) {
                    const double w2 = coef * psi2[m];
                    b0 = fma(w2, (double)v.x, b0);
                    b1 = fma(w2, (double)v.y, b1);
                    b2 = fma(w2, (double)v.z, b2);
                    b3 = fma(w2, (double)v.w, b3);
                }
                row -= step;
                m += stride;
            }
        }
        if (!reverse) tr0 = tr1;
    }
    a[0] = a0;
    a[1] = a1;
    a[2] = a2;
    a[3] = a3;
    if constexpr (kDual) {
        b[0] = b0;
        b[1] = b1;
        b[2] = b2;
        b[3] = b3;
    }
}

// Split s of nsplit covers terms [t_begin + T s / nsplit, t_begin + T (s+1) / nsplit).
__device__ __forceinline__ void gemv_split_range(int64_t t_begin, int64_t t_end, int split,
                                                 int nsplit, int64_t *ta, int64_t *tb) {
    const int64_t T = t_end - t_begin;
    *ta = t_begin + (T * split) / nsplit;
    *tb = t_begin + (T * (split + 1)) / nsplit;
}

__device__ __forceinline__ void store4(GL_GLOBAL double *out, int64_t col, int64_t P,
                                       const double a[4]) {
    out[0] = a[0];
    if (col + 1 < P) out[1] = a[1];
    if (col + 2 < P) out[2] = a[2];
    if (col + 3 < P) out[3] = a[3];
}

__global__ __launch_bounds__(kGemvThreads) void hist_gemv_kernel(
    const float *__restrict__ H, int64_t ld, int64_t P, const double *__restrict__ psi,
    const Run *__restrict__ runs, int nruns, int64_t k, int64_t t_begin, int64_t t_end,
    int reverse, double *__restrict__ partial) {
    const int64_t col = ((int64_t)blockIdx.x * kGemvThreads + threadIdx.x) * 4;
    if (col >= P) return;
    int64_t ta, tb;
    gemv_split_range(t_begin, t_end, blockIdx.y, gridDim.y, &ta, &tb);
    double a[4];
    gemv_points<false>((const GL_GLOBAL float *)H, ld, (const GL_CONST double *)psi, nullptr,
                       (const GL_CONST Run *)runs, nruns, k, ta, tb, col, reverse, a, nullptr);
    store4((GL_GLOBAL double *)partial + (int64_t)blockIdx.y * P + col, col, P, a);
}

// Both sums of the adjoint's recomputation (psi and d psi / d gamma) in one pass over the
// history rows: partial receives exactly what hist_gemv_kernel writes, partial2 the second.
__global__ __launch_bounds__(kGemvThreads) void hist_gemv_dual_kernel(
    const float *__restrict__ H, int64_t ld, int64_t P, const double *__restrict__ psi,
    const double *__restrict__ psi2, const Run *__restrict__ runs, int nruns, int64_t k,
    int64_t t_begin, int64_t t_end, int reverse, double *__restrict__ partial,
    double *__restrict__ partial2) {
    const int64_t col = ((int64_t)blockIdx.x * kGemvThreads + threadIdx.x) * 4;
    if (col >= P) return;
    int64_t ta, tb;
    gemv_split_range(t_begin, t_end, blockIdx.y, gridDim.y, &ta, &tb);
    double a[4], b[4];
    gemv_points<true>((const GL_GLOBAL float *)H, ld, (const GL_CONST double *)psi,
                      (const GL_CONST double *)psi2, (const GL_CONST Run *)runs, nruns, k, ta, tb,
                      col, reverse, a, b);
    store4((GL_GLOBAL double *)partial + (int64_t)blockIdx.y * P + col, col, P, a);
    store4((GL_GLOBAL double *)partial2 + (int64_t)blockIdx.y * P + col, col, P, b);
}

__host__ __device__ int gemv_splits(int64_t terms, int64_t P, int64_t target_groups) {
    if (terms <= 0) return 0;
    const int64_t colblocks = (P + kGemvCols - 1) / kGemvCols;
    // aim at target_groups workgroups (default ~4 per CU on 256 CUs), >= 16 terms per split
    int64_t want = (target_groups + colblocks - 1) / colblocks;
    const int64_t by_terms = (terms + 15) / 16;
    if (want > by_terms) want = by_terms;
    if (want > kMaxSplits) want = kMaxSplits;
    if (want < 1) want = 1;
    return (int)want;
}

void launch_hist_gemv(const float *H, int64_t ld, int64_t P, const double *psi, const Run *runs,
                      int nruns, int64_t k, int64_t t_begin, int64_t t_end, int nsplit,
                      bool reverse, double *partial, hipStream_t s) {
    const unsigned colblocks = (unsigned)((P + kGemvCols - 1) / kGemvCols);
    GL_LAUNCH(hist_gemv_kernel, dim3(colblocks, (unsigned)nsplit), dim3(kGemvThreads), 0, s, H, ld,
              P, psi, runs, nruns, k, t_begin, t_end, reverse ? 1 : 0, partial);
}

void launch_hist_gemv_dual(const float *H, int64_t ld, int64_t P, const double *psi,
                           const double *psi2, const Run *runs, int nruns, int64_t k,
                           int64_t t_begin, int64_t t_end, int nsplit, bool reverse,
                           double *partial, double *partial2, hipStream_t s) {
    const unsigned colblocks = (unsigned)((P + kGemvCols - 1) / kGemvCols);
    GL_LAUNCH(hist_gemv_dual_kernel, dim3(colblocks, (unsigned)nsplit), dim3(kGemvThreads), 0, s,
              H, ld, P, psi, psi2, runs, nruns, k, t_begin, t_end, reverse ? 1 : 0, partial,
              partial2);
}

// ---- batched over the problems of an ensemble: one launch for every problem's GEMV.
// Workgroups are laid out problem after problem, each problem's share being
// colblocks x nsplit with nsplit from the same rule as a single problem, so every
// member's sums are bit-identical to its solo run.
__global__ __launch_bounds__(kGemvThreads) void hist_gemv_batched_kernel(
    const BatchEntry *__restrict__ tab, int nprob, const Run *__restrict__ runs, int nruns,
    int64_t k, int64_t t_begin, int64_t t_end, int reverse) {
    int64_t w = blockIdx.x;
    int i = 0, nsplit = 0;
    int64_t cb = 1;
    for (; i < nprob; ++i) {
        cb = (tab[i].P + kGemvCols - 1) / kGemvCols;
        nsplit = gemv_splits(t_end - t_begin, tab[i].P, tab[i].groups);
        const int64_t share = cb * nsplit;
        if (w < share) break;
        w -= share;
    }
    if (i >= nprob) return;
    const BatchEntry &e = tab[i];
    const int split = (int)(w / cb);
    const int64_t col = ((w % cb) * kGemvThreads + threadIdx.x) * 4;
    if (col >= e.P) return;
    int64_t ta, tb;
    gemv_split_range(t_begin, t_end, split, nsplit, &ta, &tb);
    double a[4];
    gemv_points<false>((const GL_GLOBAL float *)e.H, e.ld, (const GL_CONST double *)e.psi,
                       nullptr, (const GL_CONST Run *)runs, nruns, k, ta, tb, col, reverse, a,
                       nullptr);
    store4((GL_GLOBAL double *)e.partial + (int64_t)split * e.P + col, col, e.P, a);
}

int64_t batched_gemv_groups(const std::vector<Problem> &probs, int64_t terms) {
    int64_t total = 0;
    for (const Problem &pb : probs)
        total += ((pb.P + kGemvCols - 1) / kGemvCols) * gemv_splits(terms, pb.P, pb.gemv_groups);
    return total;
}

void launch_hist_gemv_batched(const BatchEntry *tab, int nprob, int64_t wgs, const Run *runs,
                              int nruns, int64_t k, int64_t t_begin, int64_t t_end, bool reverse,
                              hipStream_t s) {
    if (wgs <= 0) return;
    GL_LAUNCH(hist_gemv_batched_kernel, dim3((unsigned)wgs), dim3(kGemvThreads), 0, s, tab, nprob,
              runs, nruns, k, t_begin, t_end, reverse ? 1 : 0);
}

__global__ void reduce_partials_kernel(const double *__restrict__ partial, int nsplit, int64_t P,
                                       const double *__restrict__ base, double *__restrict__ S) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double acc = base ? base[p] : 0.0;
    int q = 0;
    for (; q + 8 <= nsplit; q += 8) {  // loads issued eight at a time, added in split order
        double v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = partial[(int64_t)(q + i) * P + p];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc += v[i];
    }
    for (; q < nsplit; ++q) acc += partial[(int64_t)q * P + p];
    S[p] = acc;
}

void launch_reduce_partials(const double *partial, int nsplit, int64_t P, const double *base,
                            double *S, hipStream_t s) {
    GL_LAUNCH(reduce_partials_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s,
                       partial, nsplit, P, base, S);
}

// ------------------------------------------------------------------ update
//
// One step of eq. (21) once the history sum over m >= 1 is in the GEMV
// partials: delta[k] = the un-normalised stencil of eq. (17) (zero values
// outside the grid) of the FP64 state u[k]; S = psi(0) delta[k] (+ base) +
// sum of the partials in split order; u[k+1] = u[k] + dt f(u[k]) + r S.  The
// history row k receives delta[k] in FP32.  One lane per point; the stencil
// reads the neighbours' FP64 state.

__device__ __forceinline__ double reaction(int rxn, double rate, double u) {
    if (rxn == GL_RXN_LINEAR) return -rate * u;
    if (rxn == GL_RXN_FISHER) return rate * u * (1.0 - u);
    return 0.0;
}

// delta of eq. (17) at point p (3-point in 1D, 7-point in 3D), zero outside the grid.  A
// problem has at most 2^28 points, so the coordinates come from 32-bit divisions.
__device__ __forceinline__ double stencil_at(const GL_GLOBAL double *__restrict__ u, int64_t p,
                                             int ndim, int nx, int ny, int nz) {
    if (ndim == 1) {
        const double e = p + 1 < nx ? u[p + 1] : 0.0;
        const double w = p > 0 ? u[p - 1] : 0.0;
        return e - 2.0 * u[p] + w;
    }
    const uint32_t pp = (uint32_t)p, row = pp / (uint32_t)nx;
    const uint32_t x = pp - row * (uint32_t)nx;
    const uint32_t y = ndim == 2 ? row : row % (uint32_t)ny;
    const double e = x + 1 < (uint32_t)nx ? u[p + 1] : 0.0;
    const double w = x > 0 ? u[p - 1] : 0.0;
    const double n = y + 1 < (uint32_t)ny ? u[p + nx] : 0.0;
    const double s = y > 0 ? u[p - nx] : 0.0;
    if (ndim == 2) return e + w - 4.0 * u[p] + n + s;
    const int64_t layer = (int64_t)nx * ny;
    const uint32_t z = row / (uint32_t)ny;
    const double up = z + 1 < (uint32_t)nz ? u[p + layer] : 0.0;
    const double dn = z > 0 ? u[p - layer] : 0.0;
    return e + w + n + s + up + dn - 6.0 * u[p];
}

// One point of the update; returns nothing, writes unew[p], Hk[p] (nullable), S_out[p]
// (nullable).
__device__ __forceinline__ void update_point(const GL_GLOBAL double *__restrict__ u,
                                             const GL_GLOBAL double *__restrict__ base,
                                             GL_GLOBAL double *__restrict__ unew,
                                             GL_GLOBAL float *__restrict__ Hk,
                                             GL_GLOBAL double *__restrict__ S_out,
                                             const GL_GLOBAL double *__restrict__ partial,
                                             int nsplit, int64_t P, int ndim, int nx, int ny,
                                             int nz, double r, double dt, int rxn, double rate,
                                             int64_t p) {
    const double d = stencil_at(u, p, ndim, nx, ny, nz);
    double s = d;
    if (base) s += base[p];
    int q = 0;
    for (; q + 8 <= nsplit; q += 8) {  // loads issued eight at a time, added in split order
        double v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = partial[(int64_t)(q + i) * P + p];
#pragma unroll
        for (int i = 0; i < 8; ++i) s += v[i];
    }
    for (; q < nsplit; ++q) s += partial[(int64_t)q * P + p];
    const double uk = u[p];
    unew[p] = uk + dt * reaction(rxn, rate, uk) + r * s;
    if (Hk) Hk[p] = (float)d;
    if (S_out) S_out[p] = s;
}

__global__ __launch_bounds__(256) void update_kernel(
    const double *__restrict__ u, const double *__restrict__ base, double *__restrict__ unew,
    float *__restrict__ Hk, double *__restrict__ S_out, const double *__restrict__ partial,
    int nsplit, int64_t P, int ndim, int nx, int ny, int nz, double r, double dt, int rxn,
    double rate) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    update_point((const GL_GLOBAL double *)u, (const GL_GLOBAL double *)base,
                 (GL_GLOBAL double *)unew, (GL_GLOBAL float *)Hk, (GL_GLOBAL double *)S_out,
                 (const GL_GLOBAL double *)partial, nsplit, P, ndim, nx, ny, nz, r, dt, rxn, rate,
                 p);
}

void launch_update(const Problem &pb, const double *u, const double *base, double *unew,
                   float *Hk, double *S_out, const double *partial, int nsplit, hipStream_t s) {
    const gl_problem &p = pb.p;
    GL_LAUNCH(update_kernel, dim3((unsigned)((pb.P + 255) / 256)), dim3(256), 0, s, u, base, unew,
              Hk, S_out, partial, nsplit, pb.P, p.ndim, p.nx, p.ny, p.nz, pb.r, p.dt, p.rxn,
              p.rxn_rate);
}

// Batched update: workgroups laid out problem after problem, ceil(P / 256) each, problem i
// from workgroup tab[i].upd_begin on (found by bisection: a handful of scalar loads, where a
// scan over the table cost each of an ensemble's workgroups up to one load and one 64-bit
// division per problem before it).
__global__ __launch_bounds__(256) void update_batched_kernel(const BatchEntry *__restrict__ tab,
                                                             int nprob, int64_t k, int cur,
                                                             int64_t terms, int64_t C) {
    const int64_t wg = blockIdx.x;
    int lo = 0, hi = nprob - 1;  // the last problem whose first workgroup is <= wg
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].upd_begin <= wg) lo = mid;
        else hi = mid - 1;
    }
    const BatchEntry &e = tab[lo];
    const int64_t w = wg - e.upd_begin;
    if (w >= (e.P + 255) / 256) return;
    const int64_t p = w * 256 + threadIdx.x;
    if (p >= e.P) return;
    const int nsplit = gemv_splits(terms, e.P, e.groups);
    update_point((const GL_GLOBAL double *)e.u[cur], nullptr, (GL_GLOBAL double *)e.u[cur ^ 1],
                 (GL_GLOBAL float *)e.H + k * e.ld, nullptr, (const GL_GLOBAL double *)e.partial,
                 nsplit, e.P, e.ndim, e.nx, e.ny, e.nz, e.r, e.dt, e.rxn, e.rate, p);
    if ((k + 1) % C == 0)  // adjoint checkpoint of u[k+1]
        ((GL_GLOBAL double *)e.snap)[((k + 1) / C) * e.P + p] = ((GL_GLOBAL double *)e.u[cur ^ 1])[p];
}

void launch_update_batched(const BatchEntry *tab, int nprob, int64_t wgs, int64_t k, int cur,
                           int64_t terms, int64_t C, hipStream_t s) {
    GL_LAUNCH(update_batched_kernel, dim3((unsigned)wgs), dim3(256), 0, s, tab, nprob, k, cur,
              terms, C);
}

// ----------------------------------------------------------------- helpers

__global__ void check_finite_kernel(const double *__restrict__ x, int64_t n, int *flag) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(x[i]);
    if (bad) atomicOr(flag, 1);
}

void launch_check_finite(const double *x, int64_t n, int *flag, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    GL_LAUNCH(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, n, flag);
}

}  // namespace gl
