// In-block steps of the blocked path, several per launch.
//
// The history holds delta[j], the stencil of eq. (17) of each past state, so the sum of
// eq. (21) is taken point by point.  For step kk in a block starting at k0 and a sub-block
// starting at k1 (b = kk - k0, b2 = kk - k1):
//   acc     = Old[b][p] + Old2[b2][p], then acc = fma(psi(gamma, kk - j), delta[j][p], acc)
//             for j = k1 .. kk-1 in ascending order (one chain);
//   S[p]    = acc + delta[kk][p], delta[kk] the FP64 stencil of u[kk] (zero outside the grid);
//   u[kk+1] = u[kk] + dt f(u[kk]) + r S;  history row kk <- (float) delta[kk].
// Old is the Toeplitz product over the rows before the block, Old2 the one over the block's
// rows before the sub-block (either absent when it has no rows); the product kernels hand
// over their sum Old + Old2 as one array.
//
// One launch takes s steps k .. k+s-1 of a sub-block.  A workgroup owns a tile of points
// (16 x 16 in 2D, 256 in 1D, 8 x 8 x 4 in 3D) and recomputes a halo around it: step i is evaluated on the
// tile widened by S-1-i points (S >= s, the compile-time halo), which needs u[k+i] one point
// further out, so u[k] is read on the tile widened by S and the states stay in LDS from step
// to step.  The delta rows of the launch's own steps stay in the registers of the lane that
// owns the point; rows before k come from the history.  A halo point repeats its owner's
// arithmetic in the same order, so all copies of a value are bit-identical, and because the
// chain above does not depend on where a launch starts, any grouping of the steps into
// launches gives the same bits (the adjoint's recomputation relies on this).
//
// Carry: in a sub-block of at most 32 steps a launch also continues, for the points of its
// own tile, the chains of the next launch's steps over every row before that launch
// (Old + Old2, rows k1 .. k-1 from the history, then its own rows k .. k+s-1) and writes them
// out.  The next launch starts its chains there for its whole region (tile and halo, written
// by the neighbouring tiles) instead of re-reading and re-summing the sub-block's rows at
// every halo point; the values are the same chain in the same order, so the bits do not
// change.  A launch without a carry (a sub-block's first, or the first after a restart) sums
// the rows itself.
#include <hip/hip_runtime.h>

#include "gl_internal.h"

namespace gl {

constexpr int kStepThreads = 1024;
constexpr int kTile2 = 16;   // 2D tile side
constexpr int kTile1 = 256;  // 1D tile length
constexpr int kRowBatch = 32; // history rows loaded together (and the most a carry sums)
constexpr int kWin = 16;      // rows per weight window
constexpr int kTilePts = 256; // points of a tile
constexpr int kTile3x = 8, kTile3y = 8, kTile3z = 4;  // 3D tile
static_assert(kTile3x * kTile3y * kTile3z == kTilePts && kTile2 * kTile2 == kTilePts &&
                  kTile1 == kTilePts, "every tile has kTilePts points");

// Region sizes for halo S: the u region (tile widened by S) and the step-0 region (widened
// by S - 1).  1D and 2D share one instantiation sized for 2D; 3D has its own.
template <int S, bool D3>
struct StepGeom {
    static constexpr int kULen = D3 ? (kTile3x + 2 * S) * (kTile3y + 2 * S) * (kTile3z + 2 * S)
                                    : (kTile2 + 2 * S) * (kTile2 + 2 * S);
    static constexpr int kR0 =
        D3 ? (kTile3x + 2 * (S - 1)) * (kTile3y + 2 * (S - 1)) * (kTile3z + 2 * (S - 1))
           : (kTile2 + 2 * (S - 1)) * (kTile2 + 2 * (S - 1));
    static constexpr int kPts = (kR0 + kStepThreads - 1) / kStepThreads;  // per lane
    static_assert(D3 || (kULen >= kTile1 + 2 * S && kR0 >= kTile1 + 2 * (S - 1)),
                  "1D fits 2D sizes");
};

// Workgroups are dispatched to the 8 XCDs in turn (id mod 8), each XCD with its own L2.
// Giving XCD x a contiguous run of tiles (in row-major tile order: a band of the grid) keeps
// the halos its workgroups read mostly inside its own band, so overlapping reads hit its L2
// instead of every XCD fetching most of the grid.  A bijection on 0 .. n-1.
__device__ __forceinline__ int xcd_tile(int id, int n) {
    constexpr int kXcd = 8;
    const int q = n / kXcd, r = n % kXcd;
    const int x = id % kXcd, local = id / kXcd;
    return x * q + min(x, r) + local;
}

__device__ __forceinline__ double step_reaction(int rxn, double rate, double u) {
    if (rxn == GL_RXN_LINEAR) return -rate * u;
    if (rxn == GL_RXN_FISHER) return rate * u * (1.0 - u);
    return 0.0;
}

// f'(u), for the reverse steps
__device__ __forceinline__ double step_reaction_slope(int rxn, double rate, double u) {
    if (rxn == GL_RXN_LINEAR) return -rate;
    if (rxn == GL_RXN_FISHER) return rate * (1.0 - 2.0 * u);
    return 0.0;
}

template <int S, bool D3, bool kFromCarry, bool kRev>
__device__ __forceinline__ void block_steps_body(const BlockStepArgs &a) {
    using G = StepGeom<S, D3>;
    __shared__ double lu[2][G::kULen];
    __shared__ float lrows[kRowBatch][kTilePts];  // carry: the tile's rows k1 .. k+s-1
    __shared__ double lpsi[kRowBatch + 2 * kMaxFuse];  // carry: psi(0 ..)
    const int tid = threadIdx.x;
    const bool two = !D3 && a.ndim == 2;
    const int tx = D3 ? kTile3x : two ? kTile2 : kTile1;
    const int ty = D3 ? kTile3y : two ? kTile2 : 1, tz = D3 ? kTile3z : 1;
    const int hy = D3 || two ? 1 : 0;  // halo along y (and, in 3D, z)
    constexpr int hz = D3 ? 1 : 0;
    const int uw = tx + 2 * S, uh = ty + 2 * S * hy, ud = tz + 2 * S * hz;  // u region
    const int w0 = tx + 2 * (S - 1), h0 = ty + 2 * (S - 1) * hy;            // step-0 region
    const int d0 = tz + 2 * (S - 1) * hz;
    const int uwh = uw * uh, w0h0 = w0 * h0;
    const int64_t nx = a.nx, ny = hy ? a.ny : 1, nz = D3 ? a.nz : 1, P = a.P;
    const int ntx = (int)((nx + tx - 1) / tx), nty = (int)((ny + ty - 1) / ty);
    const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int tix = tile % ntx, trest = tile / ntx;  // tile coordinates, x fastest
    const int tiy = D3 ? trest % nty : trest, tiz = D3 ? trest / nty : 0;
    const int64_t gx0 = (int64_t)tix * tx - S;
    const int64_t gy0 = (int64_t)tiy * ty - S * hy;
    const int64_t gz0 = (int64_t)tiz * tz - S * hz;
    const int s = a.s;
    const int64_t k = a.k;
    // compile-time: a launch that starts from a carry never loads the sub-block's rows into
    // registers, and without them its kernel fits two workgroups per CU
    constexpr bool from_carry = kFromCarry;
    const bool to_carry = a.carry_out != nullptr;  // the host keeps b2 + s <= kRowBatch then

    // u[k] on the u region (zero outside the grid), held in registers until the history
    // loads below are in flight too
    constexpr int kULoads = (G::kULen + kStepThreads - 1) / kStepThreads;
    double uv[kULoads];
    bool uin[kULoads];
#pragma unroll
    for (int c = 0; c < kULoads; ++c) {
        const int idx = tid + c * kStepThreads;
        const int iz = D3 ? idx / uwh : 0, ixy = idx - iz * uwh;
        const int64_t gx = gx0 + ixy % uw, gy = gy0 + ixy / uw, gz = gz0 + iz;
        uin[c] = idx < uwh * ud && gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 &&
                 gz < nz;
        uv[c] = a.u_cur[uin[c] ? (gz * ny + gy) * nx + gx : 0];
    }

    // the lane's points: slot n is point tid + n * 256 of the step-0 region
    int ux[G::kPts];       // index in the u region
    int lvl[G::kPts];      // evaluated at steps i <= lvl (distance to the step-0 region's
                           // edge); -1: no grid point in this slot
    int tl[G::kPts];       // index in the tile (points with lvl >= S - 1)
    int64_t q[G::kPts];    // grid index
#pragma unroll
    for (int n = 0; n < G::kPts; ++n) {
        const int r = tid + n * kStepThreads;
        const int rz = D3 ? r / w0h0 : 0, rxy = r - rz * w0h0;
        const int rx = rxy % w0, ry = rxy / w0;
        const int64_t gx = gx0 + rx + 1, gy = gy0 + ry + hy, gz = gz0 + rz + hz;
        const bool ok = r < w0h0 * d0 && gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 &&
                        gz < nz;
        int l = min(rx, w0 - 1 - rx);
        if (hy) l = min(l, min(ry, h0 - 1 - ry));
        if (D3) l = min(l, min(rz, d0 - 1 - rz));
        lvl[n] = ok ? l : -1;
        ux[n] = ((rz + hz) * uh + ry + hy) * uw + rx + 1;
        tl[n] = (rx - (S - 1)) + (ry - (S - 1) * hy) * tx + (rz - (S - 1) * hz) * tx * ty;
        q[n] = ok ? (gz * ny + gy) * nx + gx : 0;
    }
    // carry work: lane t continues, for tile point pt = t mod 256 (x fastest), the chains of
    // the next launch's steps 2 cp and 2 cp + 1, cp = t / 256 (uniform per wave)
    static_assert(kStepThreads == 4 * kTilePts && kMaxFuse == 8, "four step pairs per point");
    const int pt = tid % kTilePts, cp = tid / kTilePts;
    const int64_t cgx = gx0 + S + pt % tx, cgy = gy0 + S * hy + (pt / tx) % ty;
    const int64_t cgz = gz0 + S * hz + pt / (tx * ty);
    const bool cok = to_carry && cgx < nx && cgy < ny && cgz < nz;
    const int64_t cq = cok ? (cgz * ny + cgy) * nx + cgx : 0;

    // Chains of the s steps up to row k - 1: Old + Old2, then the sub-block's rows.  All loads
    // are issued before any is used and are unconditional: slots without a grid point read
    // point 0, steps past s re-read step s - 1's row, rows past the last re-read it (all
    // unused).  Addresses are a uniform row base plus the lane's 32-bit byte offset.
    uint32_t qb8[G::kPts], qb4[G::kPts];
#pragma unroll
    for (int n = 0; n < G::kPts; ++n) {
        qb8[n] = (uint32_t)q[n] * 8u;
        qb4[n] = (uint32_t)q[n] * 4u;
    }
    // the chains' start: the previous launch's carry, or Old + Old2
    double pv[G::kPts][S];
    const double *cstart = from_carry ? a.carry_in : a.pre;
    const int crow = from_carry ? 0 : a.pre_row;
#pragma unroll
    for (int i = 0; i < S; ++i) {
        const char *o = reinterpret_cast<const char *>(cstart + (int64_t)(crow + min(i, s - 1)) * P);
#pragma unroll
        for (int n = 0; n < G::kPts; ++n) pv[n][i] = *reinterpret_cast<const double *>(o + qb8[n]);
    }
    // reverse steps: u of forward step kf - i, for f' (issued with the other loads)
    double urv[G::kPts][kRev ? S : 1];
    if constexpr (kRev) {
#pragma unroll
        for (int i = 0; i < S; ++i)
#pragma unroll
            for (int n = 0; n < G::kPts; ++n)
                urv[n][i] = *reinterpret_cast<const double *>(
                    reinterpret_cast<const char *>(a.u_rev - (int64_t)min(i, s - 1) * P) + qb8[n]);
    }
    const int nr = a.b2;  // rows k - nr .. k - 1
    const float *rows = a.H + (k - nr) * a.ld;
    float v[G::kPts][kRowBatch];
    // carry: Old + Old2 of the lane's two next steps, and (starting from a carry, when no slot
    // loads rows) rows cp, cp + 4, ... of k - nr .. k - 1 at its tile point, into slot 0's row
    // registers
    double pn[2];
    // step pairs past the next launch's n_next steps (3D launches take at most two) have no
    // carry to form: their waves (cp is uniform per wave) skip the loads and the sums
    const bool cpair = 2 * cp < a.n_next;
    if (to_carry) {
        if (cpair) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
                pn[h] = a.pre[(int64_t)(a.pre_row + s + min(2 * cp + h, a.n_next - 1)) * P + cq];
        }
        if (from_carry) {
#pragma unroll
            for (int e = 0; e < kRowBatch / 4; ++e)
                if (4 * e < nr) v[0][e] = rows[(int64_t)min(4 * e + cp, nr - 1) * a.ld + cq];
        }
    }
    auto load_rows = [&](int j) {
        // groups of 8 rows holding at least one row of the batch (uniform branches, so the
        // loads still issue together)
#pragma unroll
        for (int g8 = 0; g8 < kRowBatch / 8; ++g8) {
            if (j + 8 * g8 < nr) {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int t = 8 * g8 + e;
                    const char *row =
                        reinterpret_cast<const char *>(rows + (int64_t)min(j + t, nr - 1) * a.ld);
#pragma unroll
                    for (int n = 0; n < G::kPts; ++n)
                        v[n][t] = *reinterpret_cast<const float *>(row + qb4[n]);
                }
            }
        }
    };
    if (!from_carry) load_rows(0);
    double acc[G::kPts][S];
#pragma unroll
    for (int n = 0; n < G::kPts; ++n)
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (from_carry) {
                acc[n][i] = pv[n][i];
            } else {
                acc[n][i] = 0.0;
                acc[n][i] += a.has_pre ? pv[n][i] : 0.0;
            }
        }
    for (int j = 0; j < (from_carry ? 0 : nr); j += kRowBatch) {
        if (j > 0) load_rows(j);
#pragma unroll
        for (int h = 0; h < kRowBatch / kWin; ++h) {
            const int j0 = j + h * kWin;
            if (j0 >= nr) continue;
            // row j0 + t is m = nr - j0 - t + i steps back from step k + i: the weights of
            // kWin rows and S steps are psi(nr - j0 - kWin + 1 .. nr - j0 + S - 1)
            double w[kWin + S - 1];
#pragma unroll
            for (int x = 0; x < kWin + S - 1; ++x) w[x] = a.psi[max(nr - j0 - (kWin - 1) + x, 0)];
#pragma unroll
            for (int t = 0; t < kWin; ++t) {
                if (j0 + t < nr) {
#pragma unroll
                    for (int i = 0; i < S; ++i) {
                        if (i < s) {
#pragma unroll
                            for (int n = 0; n < G::kPts; ++n)
                                acc[n][i] = fma(w[kWin - 1 - t + i], (double)v[n][h * kWin + t],
                                                acc[n][i]);
                        }
                    }
                }
            }
        }
    }
    double wl[S];  // psi(1 .. S-1) for this launch's own rows
#pragma unroll
    for (int m = 1; m < S; ++m) wl[m] = m < s ? a.psi[m] : 0.0;
    wl[0] = 0.0;

#pragma unroll
    for (int c = 0; c < kULoads; ++c) {
        const int idx = tid + c * kStepThreads;
        if (idx < uwh * ud) {
            lu[0][idx] = uin[c] ? uv[c] : 0.0;
            lu[1][idx] = 0.0;
        }
    }
    if (to_carry && tid < kRowBatch + 2 * kMaxFuse) lpsi[tid] = a.psi[tid];

    if (to_carry) {  // the tile's rows k - nr .. k - 1 for the carry
        if (from_carry) {
#pragma unroll
            for (int e = 0; e < kRowBatch / 4; ++e)
                if (4 * e + cp < nr) lrows[4 * e + cp][pt] = v[0][e];
        } else {
#pragma unroll
            for (int n = 0; n < G::kPts; ++n)
                if (lvl[n] >= S - 1) {
#pragma unroll
                    for (int t = 0; t < kRowBatch; ++t)
                        if (t < nr) lrows[t][tl[n]] = v[n][t];
                }
        }
    }

    float dl[G::kPts][S];  // the lane's delta rows k .. k + i - 1, FP32 as stored
#pragma unroll
    for (int i = 0; i < S; ++i) {
        if (i >= s) break;
        __syncthreads();  // u[k + i] complete in lu[i & 1]; its readers of step i - 1 done
        const double *uc = lu[i & 1];
        double *un = lu[(i & 1) ^ 1];
        const int64_t kk = k + i;
#pragma unroll
        for (int n = 0; n < G::kPts; ++n) {
            // no contraction of the step's products into sums: every instantiation (S, carry,
            // forward or reverse) then rounds the same operations in the written order, which
            // the bitwise grouping guarantee needs (the chains use explicit fma)
#pragma clang fp contract(off)
            if (lvl[n] < i) continue;
            const int x = ux[n];
            const double u = uc[x];  // lam[kf - i + 1] for reverse steps
            const double lap =
                D3    ? uc[x + 1] + uc[x - 1] + uc[x + uw] + uc[x - uw] + uc[x + uwh] +
                            uc[x - uwh] - 6.0 * u
                : two ? uc[x + 1] + uc[x - 1] - 4.0 * u + uc[x + uw] + uc[x - uw]
                      : uc[x + 1] - 2.0 * u + uc[x - 1];
            // the history row: delta = Lap u, or for reverse steps mu = r Lap lam
            const double d = kRev ? a.r * lap : lap;
            double c = acc[n][i];
#pragma unroll
            for (int i2 = 0; i2 < i; ++i2) c = fma(wl[i - i2], (double)dl[n][i2], c);
            const float df = (float)d;
            dl[n][i] = df;
            const double Sv = c + d;
            double unew;
            if constexpr (kRev)  // lam[kf - i] = lam + dt f'(u[kf - i]) lam + sum psi(m) mu
                unew = u + a.dt * step_reaction_slope(a.rxn, a.rate, urv[n][i]) * u + Sv;
            else
                unew = u + a.dt * step_reaction(a.rxn, a.rate, u) + a.r * Sv;
            un[x] = unew;
            if (lvl[n] >= S - 1) {  // a point of the tile: results go out
                if (to_carry) lrows[nr + i][tl[n]] = df;  // nr + i < nr + s <= kRowBatch
                if (a.write_history) a.H[kk * a.ld + q[n]] = df;
                if constexpr (kRev) {
                    a.lam_rows[q[n] - (int64_t)i * P] = unew;
                } else {
                    if (a.S_out) a.S_out[(int64_t)i * P + q[n]] = Sv;
                    if (i == s - 1) a.u_next[q[n]] = unew;
                    else if (a.u_rows) a.u_rows[(int64_t)i * a.u_stride + q[n]] = unew;
                    if ((a.snap_mask >> i) & 1u)
                        a.snap[(a.snap_row0 +
                                __builtin_popcount(a.snap_mask & ((1u << i) - 1u))) * P +
                               q[n]] = unew;
                }
            }
        }
    }

    // The next launch's chains over rows k1 .. k+s-1 for this tile's points: Old + Old2, then
    // rows k - nr .. k+s-1 in ascending order (LDS row jj = history row k - nr + jj), row jj
    // being m = nr + s - jj + i steps back from the next launch's step i.
    if (to_carry) {
        __syncthreads();
        if (cok && cpair) {
            const int m0 = nr + s, i0 = 2 * cp;
            double c[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                c[h] = 0.0;
                c[h] += a.has_pre ? pn[h] : 0.0;
            }
            // the pair of weights slides down one entry per row
            double w1 = lpsi[m0 + i0 + 1], w0 = lpsi[m0 + i0];
#pragma unroll 8
            for (int jj = 0; jj < m0; ++jj) {
                const double dv = (double)lrows[jj][pt];
                c[0] = fma(w0, dv, c[0]);
                c[1] = fma(w1, dv, c[1]);
                w1 = w0;
                w0 = lpsi[max(m0 + i0 - jj - 1, 0)];
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
                if (i0 + h < a.n_next) a.carry_out[(int64_t)(i0 + h) * P + cq] = c[h];
        }
    }
}

template <int S, bool C>
__global__ __launch_bounds__(kStepThreads) void block_steps_kernel(BlockStepArgs a) {
    block_steps_body<S, false, C, false>(a);
}

template <int S, bool C>
__global__ __launch_bounds__(kStepThreads) void adjoint_steps_kernel(BlockStepArgs a) {
    block_steps_body<S, false, C, true>(a);
}

// A 3D grid has four times the tiles of a 2D grid of the same size: at most 64 VGPRs
// (eight waves per SIMD) keep two workgroups of 16 waves resident per CU.
template <int S, bool C>
__global__ __launch_bounds__(kStepThreads) __attribute__((amdgpu_waves_per_eu(8)))
void block_steps_kernel_3d(BlockStepArgs a) {
    block_steps_body<S, true, C, false>(a);
}

// the reverse steps hold u[kf - i] as well: without the eight-wave bound (one workgroup per
// CU), so that they do not spill
template <int S, bool C>
__global__ __launch_bounds__(kStepThreads) void adjoint_steps_kernel_3d(BlockStepArgs a) {
    block_steps_body<S, true, C, true>(a);
}

int64_t step_tiles(int ndim, int64_t nx, int64_t ny, int64_t nz) {
    return ndim == 3 ? ((nx + kTile3x - 1) / kTile3x) * ((ny + kTile3y - 1) / kTile3y) *
                           ((nz + kTile3z - 1) / kTile3z)
           : ndim == 2 ? ((nx + kTile2 - 1) / kTile2) * ((ny + kTile2 - 1) / kTile2)
                       : (nx + kTile1 - 1) / kTile1;
}

// The in-block kernels for s steps (at most kMaxFuse3 in 3D, checked by the caller), in the
// variant that starts from a carry when the arguments hold one.
template <template <int, bool> class K2, template <int, bool> class K3>
void dispatch_steps(const BlockStepArgs &args, hipStream_t s) {
    const dim3 grid((unsigned)step_tiles(args.ndim, args.nx, args.ny, args.nz)),
        block(kStepThreads);
    static_assert(kMaxFuse3 == 2, "3D instantiations");
    const bool c = args.carry_in != nullptr;
#define GL_STEP_CASE(kern, S)                                                                  \
    do {                                                                                       \
        if (c)                                                                                 \
            GL_LAUNCH((kern<S, true>::fn), grid, block, 0, s, args);                           \
        else                                                                                   \
            GL_LAUNCH((kern<S, false>::fn), grid, block, 0, s, args);                          \
    } while (0)
    if (args.ndim == 3) {
        if (args.s <= 1)
            GL_STEP_CASE(K3, 1);
        else
            GL_STEP_CASE(K3, 2);
    } else if (args.s <= 1) {
        GL_STEP_CASE(K2, 1);
    } else if (args.s <= 2) {
        GL_STEP_CASE(K2, 2);
    } else if (args.s <= 4) {
        GL_STEP_CASE(K2, 4);
    } else {
        GL_STEP_CASE(K2, 8);
    }
#undef GL_STEP_CASE
}

template <int S, bool C> struct Fwd2 { static constexpr auto fn = block_steps_kernel<S, C>; };
template <int S, bool C> struct Fwd3 { static constexpr auto fn = block_steps_kernel_3d<S, C>; };
template <int S, bool C> struct Rev2 { static constexpr auto fn = adjoint_steps_kernel<S, C>; };
template <int S, bool C> struct Rev3 { static constexpr auto fn = adjoint_steps_kernel_3d<S, C>; };

void launch_block_step(const BlockStepArgs &args, hipStream_t s) {
    dispatch_steps<Fwd2, Fwd3>(args, s);
}

void launch_adjoint_steps(const BlockStepArgs &args, hipStream_t s) {
    dispatch_steps<Rev2, Rev3>(args, s);
}

}  // namespace gl
