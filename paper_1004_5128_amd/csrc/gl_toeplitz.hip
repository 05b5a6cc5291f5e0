// Blocked Toeplitz history sum on gfx950 BF16 matrix cores.
//
// With full memory (Sec. 2.2, eq. (21)) step k sums psi(gamma, k - j) delta[j]
// over every past step j <= k, delta[j] the stencil of eq. (17) kept as FP32
// history rows H[j].  For a block of B consecutive steps k = k0 + b
// (b = 0..B-1) the part over the rows before the block,
//
//     Old[b, p] = sum_{j < k0} psi(gamma, k0 + b - j) H[j, p],
//
// is a matrix product T H with the Toeplitz weight matrix T[b, j] =
// psi(k0 + b - j) (B x k0) and the history H (k0 x P).  The kernel takes any row
// window [j_lo, j_hi) with weights psi(k0 + b - j), so the same product also forms
// the sums over the rows of a block that precede one of its sub-blocks.  It is computed once
// per block on the matrix cores with each operand split into two BF16 parts,
// x = hi + lo (hi = x rounded to BF16, lo = the remainder rounded to BF16), and
// three products hi.hi + hi.lo + lo.hi accumulated in FP32; the history rows are
// split on the fly, the weights come from precomputed split tables.  The
// history dimension is cut into chunks whose FP32 partial products are summed in
// FP64, in chunk order, by a second kernel.  The rest of each step's sum (the
// rows inside the block) is added by the in-block step kernel.
#include <hip/hip_runtime.h>

#include "gl_internal.h"

namespace gl {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4v_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// BF16 bits of f rounded to nearest even (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

// ------------------------------------------------------------ weight tables
//
// tab[h][s][i] (h = 0 hi, 1 lo; s = 0..7) holds part h of psi(i - kPsiPad + s),
// zero outside 0..npsi-1.  Eight shifted copies let a lane fetch any eight
// consecutive weights psi(m .. m+7) with one aligned 16-byte load (copy
// s = (m + kPsiPad) mod 8 at index m + kPsiPad - s).
__global__ void psi_tables_kernel(const double *__restrict__ psi, int64_t npsi, int64_t tab_len,
                                  uint16_t *__restrict__ tab) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= tab_len) return;
    const int64_t m = i - kPsiPad + s;
    const double v = (m >= 0 && m < npsi) ? psi[m] : 0.0;
    const uint32_t hb = bf16_bits((float)v);
    const double hv = (double)__uint_as_float(hb << 16);
    const uint32_t lb = bf16_bits((float)(v - hv));
    tab[(int64_t)s * tab_len + i] = (uint16_t)hb;
    tab[(int64_t)(8 + s) * tab_len + i] = (uint16_t)lb;
}

void launch_psi_tables(const double *psi, int64_t npsi, int64_t tab_len, uint16_t *tab,
                       hipStream_t s) {
    dim3 grid((unsigned)((tab_len + 255) / 256), 8);
    GL_LAUNCH(psi_tables_kernel, grid, dim3(256), 0, s, psi, npsi, tab_len, tab);
}

// --------------------------------------------------------------- the GEMM
//
// Workgroup tile: all BM rows of the block x kTN points, 4 waves; K steps of
// kTK history rows staged through LDS.  Each lane loads 8 rows x 4 points of
// FP32 history (16-byte loads), splits them into BF16 hi/lo and stores them
// transposed, [point][row], so that an MFMA B operand (8 consecutive rows of
// one point) is one 16-byte LDS read.  Inside each group of 8 rows the order is
// reversed, which makes the matching A operand (the weights of those rows for
// one output row b) eight consecutive ascending psi values, read from the slice of
// the shifted weight tables the K step needs, staged in LDS beside the history.
// The next K step's history and weight loads are issued before the current step's
// MFMAs.
//
// LDS rows are permuted inside each 32-point block (lds_row below): the transposed stores (a
// lane's four consecutive points, 32 lanes) then hit distinct banks within every 8 and every
// 16 lanes, as do the B reads (consecutive lanes, consecutive rows), and column c of block j
// is point block_point(j, c): one accumulator store instruction still covers the block's 32
// consecutive points.
//
// v_mfma_f32_32x32x16_bf16 lane layout (wave64): A lane l holds row l%32,
// k = 8(l/32)..+7; B lane l holds column l%32, the same k; the accumulator
// lane l holds column l%32, rows 8(r/4) + 4(l/32) + r%4 for r = 0..15.

constexpr int kTN = 128;  // points per workgroup

// LDS row of tile point p, and the tile point of column c of 32-point block j (inverses).
__device__ __forceinline__ int lds_row(int p) {
    return 32 * (p >> 5) + 8 * ((p & 3) ^ ((p >> 5) & 1)) + ((p & 31) >> 2);
}
__device__ __forceinline__ int block_point(int j, int c) {
    return 32 * j + 4 * (c & 7) + ((c >> 3) ^ (j & 1));
}

// Per block length: workgroup size (4 waves, 8 for the 512-row block, which then shares each
// history tile between twice as many output rows), history rows per K step (each lane loads
// 8 rows x 4 points per step), 16-byte LDS words per point (one pad word, odd: conflict-free).
template <int BM> constexpr int gemm_threads() { return BM >= 512 ? 512 : 256; }
template <int BM> constexpr int gemm_tk() { return gemm_threads<BM>() / 4; }
template <int BM> constexpr int gemm_lds_row() { return gemm_tk<BM>() / 8 + 1; }

// Weight words one K step reads from each of the 16 tables (hi/lo x 8 shifts): the table
// indices of a step span BM + TK - 1 entries starting at k0 - jt - (TK - 1) + kPsiPad.
template <int BM>
constexpr int psi_words() {
    return (BM + gemm_tk<BM>() + 6) / 8 + 2;
}

template <int BM>
__global__ __launch_bounds__(gemm_threads<BM>(), BM >= 512 ? 1 : 2) void toeplitz_gemm_kernel(
    const float *__restrict__ H, int64_t ld, int64_t P, const u32x4_t *__restrict__ tab,
    int64_t tab_len, int64_t k0, int64_t j_lo, int64_t j_hi, int64_t kchunk,
    float *__restrict__ out, double *__restrict__ direct, const double *__restrict__ base) {
    constexpr int kThreads = gemm_threads<BM>();
    constexpr int kTK = gemm_tk<BM>();
    constexpr int kLdsRow = gemm_lds_row<BM>();
    constexpr int kWaves = kThreads / 64;
    constexpr int WM = BM / 32 >= kWaves ? kWaves : BM / 32;  // waves along the block rows
    constexpr int WN = kWaves / WM;                             // waves along the points
    constexpr int RB = BM / 32 / WM;                            // 32-row blocks per wave
    constexpr int CB = kTN / 32 / WN;                           // 32-point blocks per wave
    constexpr int NW = psi_words<BM>();
    constexpr int NPSI = 16 * NW;                         // weight words staged per K step
    constexpr int PSI_PER_LANE = (NPSI + kThreads - 1) / kThreads;
    static_assert(kPsiPad >= kTK, "the weight tables' zero pad covers a K step");
    __shared__ u32x4_t lhi[kTN * kLdsRow];
    __shared__ u32x4_t llo[kTN * kLdsRow];
    __shared__ u32x4_t lpsi[NPSI];                        // [table 0..15][NW words]

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int g = lane >> 5;   // which 8-row half of a 16-row MFMA step this lane feeds
    const int64_t n0 = (int64_t)blockIdx.x * kTN;
    const int64_t j_begin = j_lo + (int64_t)blockIdx.y * kchunk;
    const int64_t j_end = j_begin + kchunk < j_hi ? j_begin + kchunk : j_hi;
    const int64_t tab_words = tab_len / 8;  // 16-byte words per table

    // loader: 32 groups of 4 points x kTK / 8 groups of 8 rows
    const int ng = tid & 31, kg = tid >> 5;
    const int64_t col = n0 + ng * 4;
    const bool col_ok = col < P;  // P <= ld, ld % 4 == 0: the 16-byte load stays in the row

    f32x16_t acc[RB][CB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) acc[i][j] = f32x16_t{};

    // the base of a direct (one-chunk) product, fetched at the start for the small row
    // blocks of the sub-block products (registers to spare), at the end otherwise
    constexpr bool kBaseFirst = BM <= 64;
    double bpre[kBaseFirst ? RB : 1][kBaseFirst ? CB : 1][16];
    if constexpr (kBaseFirst) {
        if (direct && base) {
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < CB; ++j) {
                    const int64_t n = n0 + block_point(wn * CB + j, lane & 31);
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        bpre[i][j][r] =
                            n < P ? base[(int64_t)((wm * RB + i) * 32 + 8 * (r / 4) + 4 * g +
                                                   (r % 4)) * P + n]
                                  : 0.0;
                }
        }
    }

    f32x4v_t pre[8];
    u32x4_t ppre[PSI_PER_LANE];
    // first weight word of a K step: word of its lowest table index, less one for slack
    auto psi_w0 = [&](int64_t jt) { return (k0 - jt - (kTK - 1) + kPsiPad) / 8 - 1; };
    auto load_tile = [&](int64_t jt) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t row = jt + kg * 8 + e;
            pre[e] = (col_ok && row < j_end)
                         ? *reinterpret_cast<const f32x4v_t *>(H + row * ld + col)
                         : f32x4v_t{};
        }
    };
    auto load_psi = [&](int64_t jt) {
        const int64_t w0 = psi_w0(jt);
#pragma unroll
        for (int i = 0; i < PSI_PER_LANE; ++i) {
            const int idx = tid + i * kThreads;
            if (idx < NPSI) ppre[i] = tab[(int64_t)(idx / NW) * tab_words + w0 + idx % NW];
        }
    };
    auto stage_tile = [&]() {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = pre[e][c];
            // element p of the group holds row 7 - p: word w packs rows 7 - 2w (low half) and
            // 6 - 2w; hi rounded to nearest even by the packed conversion, lo the same of the
            // (exact) remainder
            u32x4_t h4, l4;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const f32x2_t x = {v[7 - 2 * w], v[6 - 2 * w]};
                const uint32_t hb = __builtin_bit_cast(uint32_t, __builtin_convertvector(x, bf16x2_t));
                const f32x2_t hx = {__uint_as_float(hb << 16), __uint_as_float(hb & 0xffff0000u)};
                h4[w] = hb;
                l4[w] = __builtin_bit_cast(uint32_t, __builtin_convertvector(x - hx, bf16x2_t));
            }
            lhi[lds_row(4 * ng + c) * kLdsRow + kg] = h4;
            llo[lds_row(4 * ng + c) * kLdsRow + kg] = l4;
        }
#pragma unroll
        for (int i = 0; i < PSI_PER_LANE; ++i) {
            const int idx = tid + i * kThreads;
            if (idx < NPSI) lpsi[idx] = ppre[i];
        }
    };

    // The A operand of output row b at K step jt, 16-row step q, lane half g is the 16-byte word
    // of table index idx = k0 + b - jt - 16q - 8g - 7 + kPsiPad: hi copy s = idx mod 8, word
    // (idx - s)/8 - psi_w0(jt) of the staged slice.  With k0, jt (and so every K step start)
    // multiples of 32, s = (b + 1) mod 8 and the word is (b + 1)/8 + kTK/8 - 2q - g, the same
    // for every K step: one LDS word per lane and row block, less 2q.
    int a_word[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        const int b = (wm * RB + i) * 32 + (lane & 31);
        a_word[i] = ((b + 1) & 7) * NW + ((b + 1) >> 3) + kTK / 8 - g;
    }

    if (j_begin < j_end) {
        load_tile(j_begin);
        load_psi(j_begin);
    }
    for (int64_t jt = j_begin; jt < j_end; jt += kTK) {
        __syncthreads();  // the previous step's MFMAs are done with LDS
        stage_tile();
        __syncthreads();
        const bool more = jt + kTK < j_end;
        if (more) load_tile(jt + kTK);
#pragma unroll
        for (int q = 0; q < kTK / 16; ++q) {
            // A operands of this 16-row step for the wave's row blocks: weights of rows
            // jt+16q+8g+7-p, p = 0..7, i.e. psi(mstart + p), from the staged table slice (word
            // a_word[i] - 2q, see below); B operands for all its point blocks; then the three
            // products per accumulator
            bf16x8_t Ah[RB], Al[RB], Bh[CB], Bl[CB];
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                Ah[i] = __builtin_bit_cast(bf16x8_t, lpsi[a_word[i] - 2 * q]);
                Al[i] = __builtin_bit_cast(bf16x8_t, lpsi[a_word[i] + 8 * NW - 2 * q]);
            }
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                const int n = (wn * CB + j) * 32 + (lane & 31);
                Bh[j] = __builtin_bit_cast(bf16x8_t, lhi[n * kLdsRow + 2 * q + g]);
                Bl[j] = __builtin_bit_cast(bf16x8_t, llo[n * kLdsRow + 2 * q + g]);
            }
#pragma unroll
            for (int j = 0; j < CB; ++j)
#pragma unroll
                for (int i = 0; i < RB; ++i) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al[i], Bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah[i], Bl[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah[i], Bh[j], acc[i][j], 0, 0, 0);
                }
        }
        // the next step's weights: in flight across the barrier, not held during the MFMAs
        if (more) load_psi(jt + kTK);
    }

    if (direct) {
        // one chunk: the FP64 sum itself (what the chunk reduction gives for one chunk)
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                const int64_t n = n0 + block_point(wn * CB + j, lane & 31);
                if (n < P) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int64_t e = (int64_t)((wm * RB + i) * 32 + 8 * (r / 4) + 4 * g +
                                                    (r % 4)) * P + n;
                        double v = 0.0;
                        v += (double)acc[i][j][r];
                        if (base) {
                            if constexpr (kBaseFirst)
                                v = bpre[i][j][r] + v;
                            else
                                v = base[e] + v;
                        }
                        direct[e] = v;
                    }
                }
            }
        return;
    }
    float *dst = out + (int64_t)blockIdx.y * BM * P;
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) {
            const int64_t n = n0 + block_point(wn * CB + j, lane & 31);
            if (n < P) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int b = (wm * RB + i) * 32 + 8 * (r / 4) + 4 * g + (r % 4);
                    dst[(int64_t)b * P + n] = acc[i][j][r];
                }
            }
        }
}

int toeplitz_chunks(int64_t rows, int64_t kchunk) {
    return rows <= 0 ? 0 : (int)((rows + kchunk - 1) / kchunk);
}

bool launch_toeplitz_gemm(int BM, const float *H, int64_t ld, int64_t P, const uint16_t *tab,
                          int64_t tab_len, int64_t k0, int64_t j_lo, int64_t j_hi, int64_t kchunk,
                          float *out, double *direct, const double *base, hipStream_t s) {
    // K steps start at j_lo; with k0 and j_lo multiples of 32 and j_hi <= k0 + BM every step
    // has k0 - jt > -BM, which with the zero pad of kPsiPad >= kMaxBlock + kMaxTK + 8 entries
    // keeps the staged weight words inside the tables
    static_assert(kPsiPad >= kMaxBlock + kMaxTK + 8, "the tables' zero pad covers BM + a K step");
    if (k0 % 32 != 0 || j_lo % 32 != 0 || j_hi > k0 + BM || kchunk % kMaxTK != 0) return false;
    const int nchunk = toeplitz_chunks(j_hi - j_lo, kchunk);
    if (nchunk == 0) return true;
    if (nchunk > 1) direct = nullptr;  // the chunk reduction writes the sums
    dim3 grid((unsigned)((P + kTN - 1) / kTN), (unsigned)nchunk);
    const u32x4_t *t = reinterpret_cast<const u32x4_t *>(tab);
#define GL_GEMM_CASE(bm)                                                                       \
    case bm:                                                                                   \
        GL_LAUNCH(toeplitz_gemm_kernel<bm>, grid, dim3(gemm_threads<bm>()), 0, s, H, ld, P, t,  \
                  tab_len, k0, j_lo, j_hi, kchunk, out, direct, base);                          \
        break;
    switch (BM) {
        GL_GEMM_CASE(32)
        GL_GEMM_CASE(64)
        GL_GEMM_CASE(128)
        GL_GEMM_CASE(256)
        GL_GEMM_CASE(512)
        default:
            return false;
    }
#undef GL_GEMM_CASE
    return true;
}

__global__ void old_reduce_kernel(const float *__restrict__ part, int nchunk, int64_t BP,
                                  double *__restrict__ old, const double *__restrict__ base) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= BP) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += (double)part[(int64_t)c * BP + i];
    old[i] = base ? base[i] + s : s;
}

void launch_old_reduce(const float *part, int nchunk, int64_t BM, int64_t P, double *old,
                       const double *base, hipStream_t s) {
    const int64_t BP = BM * P;
    GL_LAUNCH(old_reduce_kernel, dim3((unsigned)((BP + 255) / 256)), dim3(256), 0, s, part,
                       nchunk, BP, old, base);
}

}  // namespace gl
