// The in-block steps of the blocked path as one persistent cooperative launch.
//
// Within a block of B steps starting at k0, step k = k0 + b needs
//   S[p] = u[k][p] + Old[b][p] + sum_{m=1}^{b} psi(gamma, m) H[k - m][p]
// (Old from the Toeplitz product over the states before the block), then the
// update of eq. (21): u[k+1] = u[k] + dt f(u[k]) + r Lap(S).  The sum for a
// point only touches that point's own history, so every workgroup keeps the
// same points for all steps: phase A forms S for its points and stores it, one
// grid-wide barrier makes every S visible, and phase B applies the stencil
// (which reads neighbouring points' S) and writes u[k+1] and the FP32 history
// row k + 1 of its points.  S is double-buffered by step parity, so the next
// step's phase A (own points only) needs no second barrier.  All workgroups run
// the same number of steps and meet every barrier; the launch is cooperative so
// that the runtime guarantees they are all resident.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "gl_internal.h"

namespace gl {

namespace cg = cooperative_groups;

constexpr int kBlkThreads = 256;
constexpr int kBlkGroups = 4;                          // row groups (one per wave)
constexpr int kBlkPoints = (kBlkThreads / kBlkGroups) * 4;  // 256 points per pass

__device__ __forceinline__ double blk_reaction(int rxn, double rate, double u) {
    if (rxn == GL_RXN_LINEAR) return -rate * u;
    if (rxn == GL_RXN_FISHER) return rate * u * (1.0 - u);
    return 0.0;
}

__global__ __launch_bounds__(kBlkThreads) void block_steps_kernel(BlockStepArgs a) {
    cg::grid_group grid = cg::this_grid();
    __shared__ double red[kBlkGroups][kBlkPoints];
    const int tid = threadIdx.x;
    const int rg = tid / (kBlkThreads / kBlkGroups);       // row group of this lane
    const int lane = tid % (kBlkThreads / kBlkGroups);
    const int64_t P = a.P;
    const int64_t npass = (P + (int64_t)gridDim.x * kBlkPoints - 1) / ((int64_t)gridDim.x * kBlkPoints);

    for (int b = a.b_begin; b < a.b_end; ++b) {
        const int64_t k = a.k0 + b;
        const int par = (b - a.b_begin) & 1;
        const double *u = par ? a.u_next : a.u_cur;   // u[k]
        double *un = par ? a.u_cur : a.u_next;        // u[k+1]
        double *S = a.S + (k & 1) * P;
        // rows m = 1..b split into kBlkGroups contiguous ranges, summed in order
        const int m_lo = 1 + (int)(((int64_t)b * rg) / kBlkGroups);
        const int m_hi = 1 + (int)(((int64_t)b * (rg + 1)) / kBlkGroups);

        // ---- phase A: S for this workgroup's points
        for (int64_t pass = 0; pass < npass; ++pass) {
            const int64_t pbase = (pass * gridDim.x + blockIdx.x) * kBlkPoints;
            const int64_t p = pbase + lane * 4;
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            if (p < P) {
                const float *row = a.H + (k - m_lo) * a.ld + p;
                int m = m_lo;
                for (; m + 4 <= m_hi; m += 4) {
                    float4 v[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        v[i] = *reinterpret_cast<const float4 *>(row - (int64_t)i * a.ld);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const double w = a.psi[m + i];
                        s0 = fma(w, (double)v[i].x, s0);
                        s1 = fma(w, (double)v[i].y, s1);
                        s2 = fma(w, (double)v[i].z, s2);
                        s3 = fma(w, (double)v[i].w, s3);
                    }
                    row -= 4 * a.ld;
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
            red[rg][lane * 4 + 0] = s0;
            red[rg][lane * 4 + 1] = s1;
            red[rg][lane * 4 + 2] = s2;
            red[rg][lane * 4 + 3] = s3;
            __syncthreads();
            // one thread per point combines the row groups in order
            const int64_t q = pbase + tid;
            if (q < P) {
                double s = u[q];
                if (a.old) s += a.old[(int64_t)b * P + q];
#pragma unroll
                for (int g = 0; g < kBlkGroups; ++g) s += red[g][tid];
                S[q] = s;
            }
            __syncthreads();
        }

        grid.sync();

        // ---- phase B: stencil + reaction update of this workgroup's points
        for (int64_t pass = 0; pass < npass; ++pass) {
            const int64_t q = (pass * gridDim.x + blockIdx.x) * kBlkPoints + tid;
            if (q < P) {
                double lap;
                if (a.ndim == 1) {
                    const double e = q + 1 < P ? S[q + 1] : 0.0;
                    const double w = q > 0 ? S[q - 1] : 0.0;
                    lap = e - 2.0 * S[q] + w;
                } else {
                    const int64_t x = q % a.nx, y = q / a.nx;
                    const double e = x + 1 < a.nx ? S[q + 1] : 0.0;
                    const double w = x > 0 ? S[q - 1] : 0.0;
                    const double nn = y + 1 < a.ny ? S[q + a.nx] : 0.0;
                    const double ss = y > 0 ? S[q - a.nx] : 0.0;
                    lap = e + w - 4.0 * S[q] + nn + ss;
                }
                const double uk = u[q];
                const double v = uk + a.dt * blk_reaction(a.rxn, a.rate, uk) + a.r * lap;
                un[q] = v;
                a.H[(k + 1) * a.ld + q] = (float)v;
            }
        }
        // the next step's phase A reads u[k+1] and H row k+1 of points this same
        // thread or workgroup wrote; the barrier orders those writes and reads
        __syncthreads();
    }
}

int block_steps_capacity() {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, block_steps_kernel, kBlkThreads, 0) !=
        hipSuccess)
        return 0;
    return cus * per_cu;
}

hipError_t launch_block_steps(const BlockStepArgs &args, int groups, hipStream_t s) {
    BlockStepArgs a = args;
    void *params[] = {&a};
    return hipLaunchCooperativeKernel(reinterpret_cast<void *>(block_steps_kernel), dim3(groups),
                                      dim3(kBlkThreads), params, 0, s);
}

int block_steps_groups(int64_t P, int capacity) {
    int64_t want = (P + kBlkPoints - 1) / kBlkPoints;
    if (want > capacity) want = capacity;
    if (want < 1) want = 1;
    return (int)want;
}

}  // namespace gl
