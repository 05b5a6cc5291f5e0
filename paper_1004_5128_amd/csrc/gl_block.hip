// One step of the blocked path inside a block, as a single kernel.
//
// The history holds delta[j], the stencil of eq. (17) of each past state, so
// the sum of eq. (21) is taken point by point.  For step k = k0 + b of a block
// starting at k0, inside its sub-block starting at k1 = k - b2:
//   delta[k] = stencil of the FP64 state u[k] (the neighbours' u[k] were
//              written by the previous step's launch);
//   S[p]     = delta[k][p] + Old[b][p] + Old2[b2][p] + sum_{m=1}^{b2} psi(gamma, m) H[k - m][p],
//              Old the Toeplitz product over the rows before the block, Old2 the one
//              over the block's rows before the sub-block (k0 .. k1-1);
//   u[k+1]   = u[k] + dt f(u[k]) + r S;  history row k <- delta[k] (FP32).
// A workgroup owns 64 points (16 lanes x 4 points, 16-byte row loads) and
// splits the sub-block rows m = 1..b2 over 16 row groups, one per 16 lanes; the groups' FP64 partial sums are added
// in group order through LDS.
#include <hip/hip_runtime.h>

#include "gl_internal.h"

namespace gl {

constexpr int kStepThreads = 256;
constexpr int kStepGroups = 16;
constexpr int kStepLanes = kStepThreads / kStepGroups;  // 16
constexpr int kStepPoints = kStepLanes * 4;             // 64 points per workgroup

__device__ __forceinline__ double step_reaction(int rxn, double rate, double u) {
    if (rxn == GL_RXN_LINEAR) return -rate * u;
    if (rxn == GL_RXN_FISHER) return rate * u * (1.0 - u);
    return 0.0;
}

__global__ __launch_bounds__(kStepThreads) void block_step_kernel(BlockStepArgs a) {
    __shared__ double red[kStepGroups][kStepPoints];
    const int tid = threadIdx.x;
    const int grp = tid / kStepLanes;
    const int lane = tid % kStepLanes;
    const int64_t P = a.P;
    const int64_t p0 = (int64_t)blockIdx.x * kStepPoints;
    const int64_t p = p0 + lane * 4;
    const int b = a.b;
    const int64_t k = a.k0 + b;

    // rows m = 1..b2 (those of the sub-block before k) cut into kStepGroups contiguous ranges
    const int b2 = a.b2;
    const int m_lo = 1 + (b2 * grp) / kStepGroups;
    const int m_hi = 1 + (b2 * (grp + 1)) / kStepGroups;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (p < P && m_lo < m_hi) {
        const float *row = a.H + (k - m_lo) * a.ld + p;
        int m = m_lo;
        for (; m + 8 <= m_hi; m += 8) {
            float4 v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = *reinterpret_cast<const float4 *>(row - (int64_t)i * a.ld);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const double w = a.psi[m + i];
                s0 = fma(w, (double)v[i].x, s0);
                s1 = fma(w, (double)v[i].y, s1);
                s2 = fma(w, (double)v[i].z, s2);
                s3 = fma(w, (double)v[i].w, s3);
            }
            row -= 8 * a.ld;
        }
        for (; m < m_hi; ++m) {
            const float4 v = *reinterpret_cast<const float4 *>(row);
            const double w = a.psi[m];
            s0 = fma(w, (double)v.x, s0);
            s1 = fma(w, (double)v.y, s1);
            s2 = fma(w, (double)v.z, s2);
            s3 = fma(w, (double)v.w, s3);
            row -= a.ld;
        }
    }
    red[grp][lane * 4 + 0] = s0;
    red[grp][lane * 4 + 1] = s1;
    red[grp][lane * 4 + 2] = s2;
    red[grp][lane * 4 + 3] = s3;
    __syncthreads();
    if (tid >= kStepPoints) return;
    const int64_t q = p0 + tid;
    if (q >= P) return;

    double d;  // stencil of eq. (17), zero outside the grid
    const double *u = a.u_cur;
    if (a.ndim == 1) {
        const double e = q + 1 < P ? u[q + 1] : 0.0;
        const double w = q > 0 ? u[q - 1] : 0.0;
        d = e - 2.0 * u[q] + w;
    } else {
        const int64_t x = q % a.nx, y = q / a.nx;
        const double e = x + 1 < a.nx ? u[q + 1] : 0.0;
        const double w = x > 0 ? u[q - 1] : 0.0;
        const double n = y + 1 < a.ny ? u[q + a.nx] : 0.0;
        const double s = y > 0 ? u[q - a.nx] : 0.0;
        d = e + w - 4.0 * u[q] + n + s;
    }
    double S = d;
    if (a.old) S += a.old[(int64_t)b * P + q];
    if (a.old2) S += a.old2[(int64_t)b2 * P + q];
#pragma unroll
    for (int g = 0; g < kStepGroups; ++g) S += red[g][tid];
    const double uk = u[q];
    const double un = uk + a.dt * step_reaction(a.rxn, a.rate, uk) + a.r * S;
    a.u_next[q] = un;
    if (a.write_history) a.H[k * a.ld + q] = (float)d;
    if (a.S_out) a.S_out[q] = S;
    if (a.snap && (k + 1) % a.C == 0) a.snap[((k + 1) / a.C) * P + q] = un;  // adjoint checkpoint
}

void launch_block_step(const BlockStepArgs &args, hipStream_t s) {
    const unsigned groups = (unsigned)((args.P + kStepPoints - 1) / kStepPoints);
    GL_LAUNCH(block_step_kernel, dim3(groups), dim3(kStepThreads), 0, s, args);
}

}  // namespace gl
