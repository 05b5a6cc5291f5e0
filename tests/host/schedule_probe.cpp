// Host-only probe of libgl's schedule tables (no GPU call): prints, for an n-step run, the
// forward schedule of every step (F lines) and its transpose for the adjoint (T lines) as
// runs m0:count:stride:coef.  Arguments: mem_mode adapt_rule short_L adapt_a n.
#include <cstdio>
#include <cstdlib>

#include "gl_internal.h"

int main(int argc, char **argv) {
    if (argc != 6) return 2;
    gl_options o{};
    o.mem_mode = std::atoi(argv[1]);
    o.adapt_rule = std::atoi(argv[2]);
    o.short_L = std::atol(argv[3]);
    o.adapt_a = std::atoi(argv[4]);
    const int64_t n = std::atol(argv[5]);
    const gl::Schedule f = gl::build_schedule(o, n);
    const gl::Schedule t = gl::transpose_schedule(f, n);
    for (int pass = 0; pass < 2; ++pass) {
        const gl::Schedule &s = pass ? t : f;
        for (int64_t k = 0; k < n; ++k) {
            std::printf("%c %lld %lld", pass ? 'T' : 'F', (long long)k, (long long)s.terms[k]);
            for (int64_t r = s.run_begin[k]; r < s.run_begin[k + 1]; ++r)
                std::printf(" %d:%d:%d:%d", s.runs[r].m0, s.runs[r].count, s.runs[r].stride,
                            s.runs[r].coef);
            std::printf("\n");
        }
    }
    return 0;
}
