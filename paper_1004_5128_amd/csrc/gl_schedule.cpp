// Per-step memory schedules as run lists (offset m0, count, stride, coef).
//
// Full memory (Sec. 2.2, eq. (21)) sums offsets 0..k; short memory (Sec. 3.2,
// eq. (22)) the window 0..min(L, k), L in steps; adaptive memory (Sec. 3.2,
// Def. 3.1, Def. 3.2, Prop. 3.1, eq. (24)) the base interval [0, a] and then,
// interval by interval, one sample per increment of 2i-1 points (its median),
// weighted by the increment length.  The PARTITION reading tiles each region
// (a^(i-1), a^i] exactly and takes a short leftover point by point; LITERAL
// takes the paper's medians a^(i-1) + (2i-1)eta - i + 1 up to a^i, in the
// interval holding k only whole increments ending by k, then the tail up to
// k; UNIT_STRIDE is PARTITION with increments of one point.
#include <algorithm>
#include <climits>

#include "gl_internal.h"

namespace gl {
namespace {

// a^e saturated at cap
int64_t pow_capped(int64_t a, int64_t e, int64_t cap) {
    int64_t v = 1;
    for (int64_t i = 0; i < e; ++i) {
        if (v >= (cap + a - 1) / a) return cap;
        v *= a;
    }
    return std::min(v, cap);
}

struct Builder {
    std::vector<Run> *out;
    int64_t terms = 0;
    void add(int64_t m0, int64_t count, int64_t stride, int64_t coef) {
        if (count <= 0) return;
        out->push_back(Run{(int32_t)m0, (int32_t)count, (int32_t)stride, (int32_t)coef});
        terms += count;
    }
};

void adaptive_partition(Builder &b, int64_t k, int64_t a, bool unit) {
    b.add(0, std::min(a, k) + 1, 1, 1);
    int64_t lo = a;
    for (int64_t i = 2; lo < k; ++i) {
        const int64_t hi = pow_capped(a, i, k);
        const int64_t d = unit ? 1 : 2 * i - 1;
        const int64_t whole = (hi - lo) / d;
        b.add(lo + 1 + (d - 1) / 2, whole, d, d);        // medians of whole increments
        b.add(lo + 1 + whole * d, (hi - lo) - whole * d, 1, 1);  // leftover points
        lo = hi;
    }
}

void adaptive_literal(Builder &b, int64_t k, int64_t a) {
    b.add(0, std::min(a, k) + 1, 1, 1);
    if (k <= a) return;
    int64_t reach = a;  // last offset covered by an increment so far
    for (int64_t i = 2;; ++i) {
        const int64_t lo = pow_capped(a, i - 1, INT64_MAX / 4);
        const int64_t hi = pow_capped(a, i, INT64_MAX / 4);
        const int64_t d = 2 * i - 1;
        const int64_t first = lo + i;  // first median of interval I_i
        const bool last = k <= hi;
        // medians first + e d (e >= 0) up to `limit`
        const int64_t limit = last ? k - (i - 1) : hi;
        const int64_t count = limit >= first ? (limit - first) / d + 1 : 0;
        if (count > 0) {
            b.add(first, count, d, d);
            reach = first + (count - 1) * d + (i - 1);
        }
        if (last) {
            b.add(reach + 1, k - reach, 1, 1);
            return;
        }
    }
}

}  // namespace

Schedule build_schedule(const gl_options &opt, int64_t max_steps) {
    Schedule s;
    s.run_begin.reserve(max_steps + 2);
    s.terms.reserve(max_steps + 1);
    Builder b{&s.runs};
    for (int64_t k = 0; k <= max_steps; ++k) {
        s.run_begin.push_back((int64_t)s.runs.size());
        b.terms = 0;
        switch (opt.mem_mode) {
            case GL_MEM_FULL:
                b.add(0, k + 1, 1, 1);
                break;
            case GL_MEM_SHORT:
                b.add(0, std::min<int64_t>(opt.short_L, k) + 1, 1, 1);
                break;
            default:
                if (opt.adapt_rule == GL_ADAPT_LITERAL)
                    adaptive_literal(b, k, opt.adapt_a);
                else
                    adaptive_partition(b, k, opt.adapt_a, opt.adapt_rule == GL_ADAPT_UNIT_STRIDE);
        }
        s.terms.push_back(b.terms);
    }
    s.run_begin.push_back((int64_t)s.runs.size());
    return s;
}

Schedule transpose_schedule(const Schedule &fwd, int64_t n) {
    // entries (m, c) per reverse step rho = n - 1 - j, j = k - m, gathered in CSR form; for a
    // fixed j the steps k = j, j + 1, ... give ascending m, and one step has no repeated offset
    std::vector<int64_t> count(n + 1, 0);
    for (int64_t k = 0; k < n; ++k)
        for (int64_t r = fwd.run_begin[k]; r < fwd.run_begin[k + 1]; ++r) {
            const Run &run = fwd.runs[r];
            for (int64_t t = 0; t < run.count; ++t) ++count[n - 1 - (k - (run.m0 + t * run.stride))];
        }
    std::vector<int64_t> start(n + 1, 0);
    for (int64_t rho = 0; rho < n; ++rho) start[rho + 1] = start[rho] + count[rho];
    std::vector<int32_t> ms(start[n]), cs(start[n]);
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t k = 0; k < n; ++k)
        for (int64_t r = fwd.run_begin[k]; r < fwd.run_begin[k + 1]; ++r) {
            const Run &run = fwd.runs[r];
            for (int64_t t = 0; t < run.count; ++t) {
                const int64_t m = run.m0 + t * run.stride, rho = n - 1 - (k - m);
                ms[fill[rho]] = (int32_t)m;
                cs[fill[rho]++] = run.coef;
            }
        }
    // runs: equal coefficients at a constant stride
    Schedule out;
    out.run_begin.reserve(n + 1);
    out.terms.reserve(n);
    for (int64_t rho = 0; rho < n; ++rho) {
        out.run_begin.push_back((int64_t)out.runs.size());
        out.terms.push_back(count[rho]);
        for (int64_t e = start[rho]; e < start[rho + 1];) {
            Run run{ms[e], 1, 1, cs[e]};
            int64_t f = e + 1;
            if (f < start[rho + 1] && cs[f] == run.coef) {
                run.stride = ms[f] - ms[e];
                while (f < start[rho + 1] && cs[f] == run.coef &&
                       ms[f] - ms[f - 1] == run.stride) {
                    ++run.count;
                    ++f;
                }
            }
            out.runs.push_back(run);
            e = f;
        }
    }
    out.run_begin.push_back((int64_t)out.runs.size());
    return out;
}

}  // namespace gl
