// Reverse-time (adjoint) sweep of the explicit GL scheme, eq. (21).
//
// Forward: u[k+1] = u[k] + dt f(u[k]) + r sum_{m} psi(m) delta[k-m], delta = Lap u
// (Lap the stencil of eq. (17), symmetric).  For a loss L(u[n]) with
// lam[k] = dL/du[k] and mu[k] = r Lap lam[k+1]:
//
//   lam[k] = lam[k+1] + dt f'(u[k]) lam[k+1] + sum_{m >= 0} psi(m) mu[k+m],
//
// the forward weights applied in reverse time (full or short memory: the
// window of offsets is the same in both directions), so the sum over the mu
// history is the forward history sum at reverse step n-1-k (adaptive memory
// uses the schedule's transpose instead).  On the blocked path that sum, like
// the forward one, takes the mu rows before its block of reverse steps as one
// matrix-core product per block (the Toeplitz kernel over the mu history) and
// the rows since by the in-block kernel, several reverse steps per launch (the
// in-block source holds it); G below is formed per block with the d psi / d gamma
// tables over the delta history, and the dot products of a segment's steps come
// from one launch of the dots kernel here.  Gradients with dt
// and dx fixed, S[k] = sum psi(m) delta[k-m] and G[k] = sum d psi/d gamma (m)
// delta[k-m]:
//   dL/dalpha = (r/alpha) sum_k <lam[k+1], S[k]>
//   dL/dgamma = sum_k r ln(dt) <lam[k+1], S[k]> + r <lam[k+1], G[k]>
//   dL/drate  = dt sum_k <lam[k+1], df/drate(u[k])>
// Dot products are reduced per workgroup in a fixed tree and summed over steps
// and workgroups in a fixed order: the gradients are deterministic.
#include <hip/hip_runtime.h>

#include "gl_internal.h"

namespace gl {

constexpr int kAdjThreads = 256;

__device__ __forceinline__ double adj_dfdu(int rxn, double rate, double u) {
    if (rxn == GL_RXN_LINEAR) return -rate;
    if (rxn == GL_RXN_FISHER) return rate * (1.0 - 2.0 * u);
    return 0.0;
}

__device__ __forceinline__ double adj_dfdrate(int rxn, double u) {
    if (rxn == GL_RXN_LINEAR) return -u;
    if (rxn == GL_RXN_FISHER) return u * (1.0 - u);
    return 0.0;
}

// Fixed-tree sum of the three per-lane terms over the workgroup into grad[0..2].
__device__ __forceinline__ void adj_group_sums(double t0, double t1, double t2,
                                               double *__restrict__ grad) {
    __shared__ double red[3][kAdjThreads];
    red[0][threadIdx.x] = t0;
    red[1][threadIdx.x] = t1;
    red[2][threadIdx.x] = t2;
    __syncthreads();
    for (int h = kAdjThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
            red[2][threadIdx.x] += red[2][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x < 3) grad[threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kAdjThreads) void adjoint_update_kernel(
    const double *__restrict__ lam1, double *__restrict__ lam0, float *__restrict__ Mrow,
    const double *__restrict__ partial, int nsplit, int64_t P, int ndim, int nx, int ny, int nz,
    double r, double dt, int rxn, double rate, const double *__restrict__ uk,
    const double *__restrict__ Sk, const double *__restrict__ Gk, double *__restrict__ grad) {
    const int64_t p = (int64_t)blockIdx.x * kAdjThreads + threadIdx.x;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    if (p < P) {
        double lap;
        if (ndim == 1) {
            const double e = p + 1 < nx ? lam1[p + 1] : 0.0;
            const double w = p > 0 ? lam1[p - 1] : 0.0;
            lap = e - 2.0 * lam1[p] + w;
        } else {  // at most 2^28 points: 32-bit coordinates
            const uint32_t pp = (uint32_t)p, row = pp / (uint32_t)nx;
            const uint32_t x = pp - row * (uint32_t)nx;
            const uint32_t y = ndim == 2 ? row : row % (uint32_t)ny;
            const double e = x + 1 < (uint32_t)nx ? lam1[p + 1] : 0.0;
            const double w = x > 0 ? lam1[p - 1] : 0.0;
            const double n = y + 1 < (uint32_t)ny ? lam1[p + nx] : 0.0;
            const double s = y > 0 ? lam1[p - nx] : 0.0;
            if (ndim == 2) {
                lap = e + w - 4.0 * lam1[p] + n + s;
            } else {
                const int64_t layer = (int64_t)nx * ny;
                const uint32_t z = row / (uint32_t)ny;
                const double up = z + 1 < (uint32_t)nz ? lam1[p + layer] : 0.0;
                const double dn = z > 0 ? lam1[p - layer] : 0.0;
                lap = e + w + n + s + up + dn - 6.0 * lam1[p];
            }
        }
        const double mu = r * lap;
        double A = mu;
        int q = 0;
        for (; q + 8 <= nsplit; q += 8) {
            double v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = partial[(int64_t)(q + i) * P + p];
#pragma unroll
            for (int i = 0; i < 8; ++i) A += v[i];
        }
        for (; q < nsplit; ++q) A += partial[(int64_t)q * P + p];
        const double l1 = lam1[p];
        const double u = uk[p];
        lam0[p] = l1 + dt * adj_dfdu(rxn, rate, u) * l1 + A;
        Mrow[p] = (float)mu;
        t0 = l1 * Sk[p];
        t1 = l1 * Gk[p];
        t2 = l1 * adj_dfdrate(rxn, u);
    }
    adj_group_sums(t0, t1, t2, grad + (int64_t)blockIdx.x * 3);
}

int adjoint_groups(int64_t P) { return (int)((P + kAdjThreads - 1) / kAdjThreads); }

void launch_adjoint_update(const Problem &pb, const double *lam1, double *lam0, float *Mrow,
                           const double *partial, int nsplit, const double *uk, const double *Sk,
                           const double *Gk, double *grad, hipStream_t s) {
    const gl_problem &p = pb.p;
    GL_LAUNCH(adjoint_update_kernel, dim3((unsigned)adjoint_groups(pb.P)), dim3(kAdjThreads), 0, s,
              lam1, lam0, Mrow, partial, nsplit, pb.P, p.ndim, p.nx, p.ny, p.nz, pb.r, p.dt,
              p.rxn, p.rxn_rate, uk, Sk, Gk, grad);
}

// blockIdx.x: group of 256 points; steps j = blockIdx.y, blockIdx.y + gridDim.y, .. < nk.
// The terms and their tree are the update kernel's, so both paths give the same sums for the
// same lam, u, S and G.
__global__ __launch_bounds__(kAdjThreads) void adjoint_dots_kernel(
    const double *__restrict__ lam, const double *__restrict__ u, const double *__restrict__ S,
    const double *__restrict__ G, int64_t P, int rxn, int64_t k_lo, int64_t nk,
    double *__restrict__ grad) {
    const int64_t p = (int64_t)blockIdx.x * kAdjThreads + threadIdx.x;
    for (int64_t j = blockIdx.y; j < nk; j += gridDim.y) {
        double t0 = 0.0, t1 = 0.0, t2 = 0.0;
        if (p < P) {
            const double l1 = lam[(j + 1) * P + p];
            t0 = l1 * S[j * P + p];
            t1 = l1 * G[j * P + p];
            t2 = l1 * adj_dfdrate(rxn, u[j * P + p]);
        }
        adj_group_sums(t0, t1, t2, grad + ((k_lo + j) * gridDim.x + blockIdx.x) * 3);
        __syncthreads();  // the next step's sums reuse the reduction array
    }
}

void launch_adjoint_dots(const Problem &pb, const double *lam, const double *u, const double *S,
                         const double *G, int64_t k_lo, int64_t nk, double *grad, hipStream_t s) {
    if (nk <= 0) return;
    const dim3 grid((unsigned)adjoint_groups(pb.P), (unsigned)std::min<int64_t>(nk, 65535));
    GL_LAUNCH(adjoint_dots_kernel, grid, dim3(kAdjThreads), 0, s, lam, u, S, G, pb.P, pb.p.rxn,
              k_lo, nk, grad);
}

// The per-step partial sums in two fixed-order stages: workgroup g of kAdjThreads sums the
// entries [g len, (g + 1) len) (lane t: t, t + 256, ... of the range, in order, then the
// tree), then one workgroup sums the kAdjThreads results of the first stage (one per lane,
// then the tree) and forms the gradients.
__global__ __launch_bounds__(kAdjThreads) void adjoint_final_partial_kernel(
    const double *__restrict__ grad, int64_t n, int64_t len, double *__restrict__ part) {
    const int64_t lo = (int64_t)blockIdx.x * len, hi = min(n, lo + len);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kAdjThreads) {
        s0 += grad[i * 3 + 0];
        s1 += grad[i * 3 + 1];
        s2 += grad[i * 3 + 2];
    }
    adj_group_sums(s0, s1, s2, part + (int64_t)blockIdx.x * 3);
}

__global__ __launch_bounds__(kAdjThreads) void adjoint_final_kernel(
    const double *__restrict__ part, double r, double alpha, double lndt, double dt,
    double *__restrict__ dparams) {
    __shared__ double red[3][kAdjThreads];
    red[0][threadIdx.x] = part[threadIdx.x * 3 + 0];
    red[1][threadIdx.x] = part[threadIdx.x * 3 + 1];
    red[2][threadIdx.x] = part[threadIdx.x * 3 + 2];
    __syncthreads();
    for (int h = kAdjThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
            red[2][threadIdx.x] += red[2][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        dparams[0] = (r / alpha) * red[0][0];
        dparams[1] = r * lndt * red[0][0] + r * red[1][0];
        dparams[2] = dt * red[2][0];
    }
}

void launch_adjoint_final(const double *grad, int64_t n, double r, double alpha, double lndt,
                          double dt, double *part, double *dparams, hipStream_t s) {
    static_assert(kAdjFinalParts == kAdjThreads, "one first-stage sum per lane");
    const int64_t len = (n + kAdjFinalParts - 1) / kAdjFinalParts;
    GL_LAUNCH(adjoint_final_partial_kernel, dim3(kAdjFinalParts), dim3(kAdjThreads), 0, s, grad,
              n, len, part);
    GL_LAUNCH(adjoint_final_kernel, dim3(1), dim3(kAdjThreads), 0, s, part, r, alpha, lndt, dt,
              dparams);
}

}  // namespace gl
