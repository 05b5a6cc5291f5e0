// HIP kernels of the plain history-sum path for gfx950 (CDNA4, wave64):
// GL weights, the history GEMV, the stencil + reaction update and helpers.
#include <hip/hip_runtime.h>

#include "gl_internal.h"

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

__global__ __launch_bounds__(kGemvThreads) void hist_gemv_kernel(
    const float *__restrict__ H, int64_t ld, int64_t P, const double *__restrict__ psi,
    const Run *__restrict__ runs, int nruns, int64_t k, int64_t t_begin, int64_t t_end,
    int reverse, double *__restrict__ partial) {
    const int nsplit = gridDim.y;
    const int split = blockIdx.y;
    const int64_t T = t_end - t_begin;
    const int64_t ta = t_begin + (T * split) / nsplit;
    const int64_t tb = t_begin + (T * (split + 1)) / nsplit;
    const int64_t col = ((int64_t)blockIdx.x * kGemvThreads + threadIdx.x) * 4;

    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (col < P) {
        // Runs are visited in order; with `reverse` each split walks its terms from the
        // last to the first (oldest row first), so that consecutive steps traverse the
        // history in opposite directions and the rows one step read last are still in
        // the last-level cache when the next step starts.
        int64_t tr0 = 0;
        if (reverse)
            for (int r = 0; r < nruns; ++r) tr0 += runs[r].count;
        for (int rr = 0; rr < nruns; ++rr) {
            const int r = reverse ? nruns - 1 - rr : rr;
            const Run run = runs[r];
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
                const float *row = H + (k - m) * ld + col;
                const int64_t step = stride * ld;
                int64_t cnt = hi - lo;
                while (cnt >= kGemvUnroll) {
                    float4 v[kGemvUnroll];
                    double w[kGemvUnroll];
#pragma unroll
                    for (int u = 0; u < kGemvUnroll; ++u)
                        v[u] = *reinterpret_cast<const float4 *>(row - u * step);
#pragma unroll
                    for (int u = 0; u < kGemvUnroll; ++u) w[u] = coef * psi[m + u * stride];
#pragma unroll
                    for (int u = 0; u < kGemvUnroll; ++u) {
                        a0 = fma(w[u], (double)v[u].x, a0);
                        a1 = fma(w[u], (double)v[u].y, a1);
                        a2 = fma(w[u], (double)v[u].z, a2);
                        a3 = fma(w[u], (double)v[u].w, a3);
                    }
                    row -= kGemvUnroll * step;
                    m += kGemvUnroll * stride;
                    cnt -= kGemvUnroll;
                }
                for (; cnt > 0; --cnt) {
                    const float4 v = *reinterpret_cast<const float4 *>(row);
                    const double w = coef * psi[m];
                    a0 = fma(w, (double)v.x, a0);
                    a1 = fma(w, (double)v.y, a1);
                    a2 = fma(w, (double)v.z, a2);
                    a3 = fma(w, (double)v.w, a3);
                    row -= step;
                    m += stride;
                }
            }
            if (!reverse) tr0 = tr1;
        }
        double *out = partial + (int64_t)split * P + col;
        out[0] = a0;
        if (col + 1 < P) out[1] = a1;
        if (col + 2 < P) out[2] = a2;
        if (col + 3 < P) out[3] = a3;
    }
}

int gemv_splits(int64_t terms, int64_t P, int64_t target_groups) {
    if (terms <= 0) return 0;
    const int64_t colblocks = (P + kGemvCols - 1) / kGemvCols;
    // aim at target_groups workgroups (default ~8 per CU on 256 CUs), >= 16 terms per split
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
    GL_LAUNCH(hist_gemv_kernel, dim3(colblocks, (unsigned)nsplit), dim3(kGemvThreads), 0,
                       s, H, ld, P, psi, runs, nruns, k, t_begin, t_end, reverse ? 1 : 0, partial);
}

__global__ void reduce_partials_kernel(const double *__restrict__ partial, int nsplit, int64_t P,
                                       const double *__restrict__ base, double *__restrict__ S) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double acc = base ? base[p] : 0.0;
    for (int q = 0; q < nsplit; ++q) acc += partial[(int64_t)q * P + p];
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

__device__ __forceinline__ double stencil_at(const double *__restrict__ u, int64_t p, int ndim,
                                             int nx, int ny) {
    if (ndim == 1) {
        const double e = p + 1 < nx ? u[p + 1] : 0.0;
        const double w = p > 0 ? u[p - 1] : 0.0;
        return e - 2.0 * u[p] + w;
    }
    const int64_t x = p % nx, y = p / nx;
    const double e = x + 1 < nx ? u[p + 1] : 0.0;
    const double w = x > 0 ? u[p - 1] : 0.0;
    const double n = y + 1 < ny ? u[p + nx] : 0.0;
    const double s = y > 0 ? u[p - nx] : 0.0;
    return e + w - 4.0 * u[p] + n + s;
}

__global__ __launch_bounds__(256) void update_kernel(
    const double *__restrict__ u, const double *__restrict__ base, double *__restrict__ unew,
    float *__restrict__ Hk, double *__restrict__ S_out, const double *__restrict__ partial,
    int nsplit, int64_t P, int ndim, int nx, int ny, double r, double dt, int rxn, double rate) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const double d = stencil_at(u, p, ndim, nx, ny);
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

void launch_update(const Problem &pb, const double *u, const double *base, double *unew,
                   float *Hk, double *S_out, const double *partial, int nsplit, hipStream_t s) {
    const gl_problem &p = pb.p;
    GL_LAUNCH(update_kernel, dim3((unsigned)((pb.P + 255) / 256)), dim3(256), 0, s, u, base, unew,
              Hk, S_out, partial, nsplit, pb.P, p.ndim, p.nx, p.ny, pb.r, p.dt, p.rxn, p.rxn_rate);
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
