// Internal declarations of libgl: device data of a context, the per-step
// schedule tables and the kernel launchers.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "gl.h"

namespace gl {

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

// Device-side state of one problem.
struct Problem {
    gl_problem p{};
    int64_t P = 0;        // grid points
    int64_t ld = 0;       // history leading dimension in floats (multiple of 64, >= P)
    double r = 0.0;       // alpha dt^gamma / dx^2
    int64_t offset = 0;   // first point of this problem in concatenated arrays
    double *psi = nullptr;   // [max_steps + 1] FP64 weights
    double *dpsi = nullptr;  // [max_steps + 1] d psi / d gamma
    float *H = nullptr;      // [(max_steps + 1) * ld] FP32 history, row j = u[j]
    double *u[2] = {nullptr, nullptr};  // FP64 state, double-buffered
    int cur = 0;             // u[cur] holds the current step
};

// ---------------------------------------------------------------- kernels

// psi(gamma, m) and d psi / d gamma for m = 0..n.
void launch_weights(double gamma, int64_t n, double *psi, double *dpsi, hipStream_t s);

// Columns per workgroup of the history GEMV.
constexpr int kGemvCols = 1024;

// Number of row splits of the history GEMV for `terms` terms over P points.
int gemv_splits(int64_t terms, int64_t P);
constexpr int kMaxSplits = 64;

// partial[s * P + p] = sum over terms t in split s of [t_begin, t_end) of the
// step-k schedule (runs, nruns) of coef * psi[m] * H[(k - m) * ld + p], FP64.
void launch_hist_gemv(const float *H, int64_t ld, int64_t P, const double *psi, const Run *runs,
                      int nruns, int64_t k, int64_t t_begin, int64_t t_end, int nsplit,
                      double *partial, hipStream_t s);

// S[p] = sum_s partial[s * P + p] (+ base[p] if base != nullptr), fixed order.
void launch_reduce_partials(const double *partial, int nsplit, int64_t P, const double *base,
                            double *S, hipStream_t s);

// One explicit step: S = u + sum_s partial[s]; unew = u + dt f(u) + r Lap(S);
// Hnext = (float) unew.
void launch_update(const Problem &pb, const double *u, double *unew, float *Hnext,
                   const double *partial, int nsplit, hipStream_t s);

// h[p] = (float) u[p]
void launch_to_float(const double *u, float *h, int64_t n, hipStream_t s);

// *flag = 1 if any of x[0..n) is NaN or Inf (flag must start at 0).
void launch_check_finite(const double *x, int64_t n, int *flag, hipStream_t s);

}  // namespace gl
