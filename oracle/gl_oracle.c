/*
 * gl_oracle.c -- plain FP64 CPU oracle for the explicit Grunwald-Letnikov (GL)
 * fractional reaction-diffusion scheme of Sprouse, MacDonald & Silva,
 * "Computational Efficiency of Fractional Diffusion Using Adaptive Time Step
 * Memory" (arXiv:1004.5128).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The GPU library never
 * links it and shares no code, header, table or constant with it.
 *
 * Everything here is written to be checked against the paper by eye:
 * double precision throughout, no blocking, no fusion, sums in ascending
 * history offset m.  Parallelism (OpenMP) is only over independent grid
 * points, so results do not depend on the thread count.
 *
 * Notation (paper, Sec. 2.2): grid u[k][j,l], k = t/dt, stored as
 * u[l*nx + j] with the x1 index j fastest; nx*ny interior points, the
 * points outside held at zero (zero Dirichlet edge, Sec. 3.1).  A 3D grid
 * u[k][j,l,n] is stored as u[(n*ny + l)*nx + j].
 *
 * Readings of the paper taken here (each one is listed with its reason in the
 * design notes of the repository):
 *  - the weights are psi(gamma,m) = (-1)^m binom(1-gamma, m) (eq. 8), built by
 *    the recurrence of eq. (11) from psi(gamma,0) = 1 (eq. 12);
 *  - the stencil delta is the un-normalised 5-point sum of eq. (17) (3-point in
 *    1D, from the x1 row of eq. (15); 7-point in 3D, the same sum taken over a
 *    third axis, for the N-dimensional model of Sec. 1); dx^2 sits in
 *    r = alpha dt^gamma / dx^2;
 *  - the weights and the scheme are the same for superdiffusion, 1 < gamma <= 2
 *    (the recurrence of eq. (11) holds for any gamma); at gamma = 2 every
 *    weight is 1;
 *  - the reaction term is explicit and outside the GL sum, as in eq. (21):
 *    u[k+1] = u[k] + dt f(u[k]) + r * sum_m psi(gamma,m) delta[k-m];
 *  - short memory (eq. 22) takes the window length L in steps: m = 0..min(L,k);
 *  - adaptive memory (Def. 3.1, 3.2, Prop. 3.1, eq. 24) has two readings,
 *    PARTITION (default: the increments of length 2i-1 tile each region
 *    (a^(i-1), a^i] exactly, a leftover shorter than one increment is taken
 *    point by point) and LITERAL (medians a^(i-1) + (2i-1)eta - i + 1 up to
 *    a^i, the final interval only up to k, then the tail sum of eq. 24 from
 *    the point after the last increment to k); UNIT_STRIDE is PARTITION with
 *    every increment of length 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_FULL = 0, ORC_SHORT = 1, ORC_ADAPTIVE = 2 };
enum { ORC_PARTITION = 0, ORC_LITERAL = 1, ORC_UNIT_STRIDE = 2 };
enum { ORC_RXN_NONE = 0, ORC_RXN_LINEAR = 1, ORC_RXN_FISHER = 2 };

typedef struct {
    int32_t ndim;      /* 1, 2 or 3 */
    int32_t nx, ny, nz; /* interior points per side (ny = 1 in 1D, nz = 1 below 3D) */
    double dx, dt;     /* grid spacing and time step */
    double gamma;      /* anomalous exponent, 0 < gamma <= 2 */
    double alpha;      /* diffusivity */
    int32_t rxn;       /* ORC_RXN_* */
    double rate;       /* beta (linear decay) or rho (Fisher-KPP) */
} orc_problem;

typedef struct {
    int32_t mode;      /* ORC_FULL, ORC_SHORT, ORC_ADAPTIVE */
    int32_t rule;      /* adaptive reading: ORC_PARTITION, ORC_LITERAL, ORC_UNIT_STRIDE */
    int64_t L;         /* short-memory window, in steps */
    int64_t a;         /* adaptive base interval [0, a], a >= 2 */
} orc_memory;

/* ------------------------------------------------------------------ weights */

/* psi(gamma, m) for m = 0..n: Sec. 2.1, eq. (12) psi(gamma,0) = 1 and the
 * recurrence of eq. (11), psi(gamma,m) = -psi(gamma,m-1) (2-gamma-m)/m. */
void orc_psi(double gamma, int64_t n, double *psi)
{
    psi[0] = 1.0;
    for (int64_t m = 1; m <= n; ++m)
        psi[m] = -psi[m - 1] * (2.0 - gamma - (double)m) / (double)m;
}

/* d psi(gamma,m) / d gamma for m = 0..n, by differentiating the recurrence of
 * eq. (11) term by term: psi'(m) = -psi'(m-1)(2-gamma-m)/m + psi(m-1)/m,
 * psi'(0) = 0 (psi(gamma,0) = 1 for every gamma). */
void orc_dpsi(double gamma, int64_t n, double *dpsi)
{
    double prev = 1.0;   /* psi(gamma, m-1) */
    dpsi[0] = 0.0;
    for (int64_t m = 1; m <= n; ++m) {
        double cur = -prev * (2.0 - gamma - (double)m) / (double)m;
        dpsi[m] = -dpsi[m - 1] * (2.0 - gamma - (double)m) / (double)m + prev / (double)m;
        prev = cur;
    }
}

/* --------------------------------------------------------------- schedules */

static int64_t push(int64_t cnt, int64_t cap, int64_t *ms, double *cs, int64_t m, double c)
{
    if (cnt < cap) {
        ms[cnt] = m;
        cs[cnt] = c;
    }
    return cnt + 1;
}

/* a^e, saturated at sat (a >= 2, e >= 0) */
static int64_t pow_sat(int64_t a, int64_t e, int64_t sat)
{
    int64_t v = 1;
    for (int64_t i = 0; i < e; ++i) {
        if (v > sat / a) return sat;
        v *= a;
    }
    return v < sat ? v : sat;
}

/* The (offset m, multiplicity c) pairs that enter the history sum at step k,
 * in ascending m; the term is c * psi(gamma,m) * delta[k-m].
 * Returns the number of pairs (only the first cap are written).
 *
 *  FULL     eq. (21):  m = 0..k, c = 1.
 *  SHORT    eq. (22):  m = 0..min(L, k), c = 1.
 *  ADAPTIVE Def. 3.1-3.2, Prop. 3.1, eq. (24): base interval m = 0..min(a,k)
 *           at c = 1, then for i = 2, 3, ... intervals sampled at stride
 *           d = 2i-1, each sample the median of its increment with c = d. */
int64_t orc_schedule(const orc_memory *mem, int64_t k, int64_t *ms, double *cs, int64_t cap)
{
    int64_t cnt = 0;
    if (mem->mode == ORC_FULL) {
        for (int64_t m = 0; m <= k; ++m) cnt = push(cnt, cap, ms, cs, m, 1.0);
        return cnt;
    }
    if (mem->mode == ORC_SHORT) {
        int64_t top = mem->L < k ? mem->L : k;
        for (int64_t m = 0; m <= top; ++m) cnt = push(cnt, cap, ms, cs, m, 1.0);
        return cnt;
    }

    const int64_t a = mem->a;
    const int64_t base = a < k ? a : k;
    for (int64_t m = 0; m <= base; ++m) cnt = push(cnt, cap, ms, cs, m, 1.0);
    if (k <= a) return cnt;

    if (mem->rule == ORC_LITERAL) {
        /* Medians m_i = a^(i-1) + (2i-1) eta - i + 1, eta = 1, 2, ...; each
         * stands for the 2i-1 points m_i-(i-1) .. m_i+(i-1).  Completed
         * intervals take medians up to a^i; the interval holding k takes those
         * whose increment ends at or before k; the tail sum of eq. (24) then
         * covers the points after the last increment up to k at weight 1. */
        int64_t covered = a;   /* last offset reached by an increment so far */
        for (int64_t i = 2;; ++i) {
            const int64_t lo = pow_sat(a, i - 1, INT64_MAX / 4);
            const int64_t hi = pow_sat(a, i, INT64_MAX / 4);
            const int64_t d = 2 * i - 1;
            const int last = (k <= hi);
            for (int64_t m = lo + i; m <= hi; m += d) {
                if (last && m + (i - 1) > k) break;
                cnt = push(cnt, cap, ms, cs, m, (double)d);
                covered = m + (i - 1);
            }
            if (last) {
                for (int64_t p = covered + 1; p <= k; ++p) cnt = push(cnt, cap, ms, cs, p, 1.0);
                return cnt;
            }
        }
    }

    /* PARTITION (and UNIT_STRIDE, where every increment has length 1): the
     * region (a^(i-1), min(a^i, k)] is cut, from its first point on, into
     * whole increments of d points, each represented by its median with
     * multiplicity d; points left over at the end of the region (fewer than
     * d) enter one by one, as the tail sum of eq. (24) does. */
    int64_t lo = a;
    for (int64_t i = 2; lo < k; ++i) {
        const int64_t hi = pow_sat(a, i, k);
        const int64_t d = (mem->rule == ORC_UNIT_STRIDE) ? 1 : 2 * i - 1;
        int64_t m = lo + 1;
        while (m + d - 1 <= hi) {
            cnt = push(cnt, cap, ms, cs, m + (d - 1) / 2, (double)d);
            m += d;
        }
        for (; m <= hi; ++m) cnt = push(cnt, cap, ms, cs, m, 1.0);
        lo = hi;
    }
    return cnt;
}

/* ----------------------------------------------------------- the scheme */

/* delta of eq. (17): u[j+1,l] + u[j-1,l] - 4u[j,l] + u[j,l+1] + u[j,l-1]
 * (1D: u[j+1] - 2u[j] + u[j-1], the x1 row of eq. 15; 3D: the six neighbours
 * along three axes minus 6u), zero outside the grid. */
static void stencil(const orc_problem *pr, const double *u, double *out)
{
    const int64_t nx = pr->nx, ny = pr->ndim == 1 ? 1 : pr->ny;
    const int64_t nz = pr->ndim == 3 ? pr->nz : 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t n = 0; n < nz; ++n) {
        for (int64_t l = 0; l < ny; ++l) {
            for (int64_t j = 0; j < nx; ++j) {
                const int64_t p = (n * ny + l) * nx + j;
                double east = j + 1 < nx ? u[p + 1] : 0.0;
                double west = j > 0 ? u[p - 1] : 0.0;
                if (pr->ndim == 1) {
                    out[p] = east - 2.0 * u[p] + west;
                } else {
                    double north = l + 1 < ny ? u[p + nx] : 0.0;
                    double south = l > 0 ? u[p - nx] : 0.0;
                    if (pr->ndim == 2) {
                        out[p] = east + west - 4.0 * u[p] + north + south;
                    } else {
                        double up = n + 1 < nz ? u[p + nx * ny] : 0.0;
                        double down = n > 0 ? u[p - nx * ny] : 0.0;
                        out[p] = east + west + north + south + up + down - 6.0 * u[p];
                    }
                }
            }
        }
    }
}

/* f(u): none, the decay -beta u of eq. (18), or Fisher-KPP rho u (1 - u). */
static double reaction(const orc_problem *pr, double u)
{
    if (pr->rxn == ORC_RXN_LINEAR) return -pr->rate * u;
    if (pr->rxn == ORC_RXN_FISHER) return pr->rate * u * (1.0 - u);
    return 0.0;
}

/* f'(u) */
static double reaction_du(const orc_problem *pr, double u)
{
    if (pr->rxn == ORC_RXN_LINEAR) return -pr->rate;
    if (pr->rxn == ORC_RXN_FISHER) return pr->rate * (1.0 - 2.0 * u);
    return 0.0;
}

/* d f / d rate */
static double reaction_drate(const orc_problem *pr, double u)
{
    if (pr->rxn == ORC_RXN_LINEAR) return -u;
    if (pr->rxn == ORC_RXN_FISHER) return u * (1.0 - u);
    return 0.0;
}

/* r = alpha dt^gamma / dx^2: eq. (21) multiplied through by dt. */
double orc_r(const orc_problem *pr)
{
    return pr->alpha * pow(pr->dt, pr->gamma) / (pr->dx * pr->dx);
}

static int64_t npoints(const orc_problem *pr)
{
    return (int64_t)pr->nx * (pr->ndim == 1 ? 1 : (int64_t)pr->ny) *
           (pr->ndim == 3 ? (int64_t)pr->nz : 1);
}

/* Runs nsteps steps of eq. (21) (or its short/adaptive forms, eqs. 22, 24)
 * from u0.  The history holds delta[k] for every past step, as the paper's
 * sum is written.  If store_all, out receives u[0..nsteps] ((nsteps+1)*P
 * values), else only u[nsteps].  Returns 0, or -1 if memory runs out. */
int orc_run(const orc_problem *pr, const orc_memory *mem, const double *u0, int64_t nsteps,
            double *out, int store_all)
{
    const int64_t P = npoints(pr);
    const double r = orc_r(pr);
    const double dt = pr->dt;
    double *psi = malloc(sizeof(double) * (size_t)(nsteps + 1));
    double *delta = malloc(sizeof(double) * (size_t)(nsteps > 0 ? nsteps : 1) * (size_t)P);
    double *u = malloc(sizeof(double) * (size_t)P);
    double *un = malloc(sizeof(double) * (size_t)P);
    int64_t *ms = malloc(sizeof(int64_t) * (size_t)(nsteps + 1));
    double *cs = malloc(sizeof(double) * (size_t)(nsteps + 1));
    if (!psi || !delta || !u || !un || !ms || !cs) {
        free(psi); free(delta); free(u); free(un); free(ms); free(cs);
        return -1;
    }
    orc_psi(pr->gamma, nsteps, psi);
    memcpy(u, u0, sizeof(double) * (size_t)P);
    if (store_all) memcpy(out, u0, sizeof(double) * (size_t)P);

    for (int64_t k = 0; k < nsteps; ++k) {
        stencil(pr, u, delta + k * P);
        const int64_t nt = orc_schedule(mem, k, ms, cs, nsteps + 1);
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < P; ++p) {
            double sum = 0.0;
            for (int64_t t = 0; t < nt; ++t)
                sum += cs[t] * psi[ms[t]] * delta[(k - ms[t]) * P + p];
            un[p] = u[p] + dt * reaction(pr, u[p]) + r * sum;
        }
        double *tmp = u; u = un; un = tmp;
        if (store_all) memcpy(out + (k + 1) * P, u, sizeof(double) * (size_t)P);
    }
    if (!store_all) memcpy(out, u, sizeof(double) * (size_t)P);
    free(psi); free(delta); free(u); free(un); free(ms); free(cs);
    return 0;
}

/* The scheme restricted to one discrete sine mode (linear f only).
 * phi[j,l] = sin(p pi (j+1)/(nx+1)) sin(q pi (l+1)/(ny+1)) satisfies
 * delta(phi) = -lam phi with lam = 4 sin^2(p pi / (2(nx+1))) (+ the same in
 * q, ny in 2D, and in s, nz in 3D), so u[k] = v[k] phi solves eq. (21) exactly
 * when
 *   v[k+1] = v[k] + dt f(v[k]) - r lam sum_m c psi(gamma,m) v[k-m].
 * Writes v[0..n].  Returns 0, -1 on a nonlinear f or no memory. */
int orc_mode_run(const orc_problem *pr, const orc_memory *mem, int32_t p, int32_t q, int32_t s,
                 double v0, int64_t n, double *v)
{
    const double pi = 3.14159265358979323846;
    if (pr->rxn == ORC_RXN_FISHER) return -1;
    double lam = 4.0 * pow(sin(p * pi / (2.0 * (pr->nx + 1))), 2);
    if (pr->ndim >= 2) lam += 4.0 * pow(sin(q * pi / (2.0 * (pr->ny + 1))), 2);
    if (pr->ndim == 3) lam += 4.0 * pow(sin(s * pi / (2.0 * (pr->nz + 1))), 2);
    const double r = orc_r(pr);
    double *psi = malloc(sizeof(double) * (size_t)(n + 1));
    int64_t *ms = malloc(sizeof(int64_t) * (size_t)(n + 1));
    double *cs = malloc(sizeof(double) * (size_t)(n + 1));
    if (!psi || !ms || !cs) {
        free(psi); free(ms); free(cs);
        return -1;
    }
    orc_psi(pr->gamma, n, psi);
    v[0] = v0;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t nt = orc_schedule(mem, k, ms, cs, n + 1);
        double sum = 0.0;
        for (int64_t t = 0; t < nt; ++t) sum += cs[t] * psi[ms[t]] * v[k - ms[t]];
        v[k + 1] = v[k] + pr->dt * reaction(pr, v[k]) - r * lam * sum;
    }
    free(psi); free(ms); free(cs);
    return 0;
}

/* The history sum alone, on a given FP32 history (row j = state j, leading
 * dimension ld): S[p] = sum over the schedule at step k of
 * c * psi(gamma,m) * H[(k-m)*ld + p], for p = 0..P-1, in FP64. */
void orc_history_sum(double gamma, const orc_memory *mem, int64_t k, const float *H, int64_t ld,
                     int64_t P, double *S)
{
    double *psi = malloc(sizeof(double) * (size_t)(k + 1));
    int64_t *ms = malloc(sizeof(int64_t) * (size_t)(k + 1));
    double *cs = malloc(sizeof(double) * (size_t)(k + 1));
    orc_psi(gamma, k, psi);
    const int64_t nt = orc_schedule(mem, k, ms, cs, k + 1);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        double sum = 0.0;
        for (int64_t t = 0; t < nt; ++t) sum += cs[t] * psi[ms[t]] * (double)H[(k - ms[t]) * ld + p];
        S[p] = sum;
    }
    free(psi); free(ms); free(cs);
}

/* -------------------------------------------------------------- adjoint */

/* Loss 0.5 || u[n] - target ||^2 of an n-step run of eq. (21) (any memory
 * mode) and its gradient with respect to u0, alpha, gamma and the reaction
 * rate, with dt and dx held fixed.  Store-all reverse sweep in FP64.
 *
 * The step is u[k+1] = u[k] + dt f(u[k]) + r sum_t c_t psi(m_t) delta[k-m_t]
 * with delta[j] = Lap u[j] (Lap symmetric).  With lam[k] = dL/du[k]:
 *   nu[j]  = sum over steps k that use delta[j] of r c psi(k-j) lam[k+1]
 *            (built by scattering each step's terms, the transpose of the
 *            forward gather);
 *   lam[k] = lam[k+1] + dt f'(u[k]) lam[k+1] + Lap nu[k];
 *   dL/dalpha = sum_k < lam[k+1], (r/alpha) Sigma[k] >,
 *   dL/dgamma = sum_k < lam[k+1], r ln(dt) Sigma[k] + r Sigma'[k] >,
 *   dL/drate  = sum_k < lam[k+1], dt df/drate(u[k]) >,
 * where Sigma[k] = sum_t c psi(m) delta[k-m] and Sigma'[k] the same with
 * d psi / d gamma.  dparams = {dL/dalpha, dL/dgamma, dL/drate}.
 * Returns 0, or -1 if memory runs out. */
int orc_adjoint(const orc_problem *pr, const orc_memory *mem, const double *u0, int64_t n,
                const double *target, double *loss, double *du0, double *dparams)
{
    const int64_t P = npoints(pr);
    const double r = orc_r(pr);
    const double dt = pr->dt;
    double *U = malloc(sizeof(double) * (size_t)(n + 1) * (size_t)P);      /* u[0..n] */
    double *D = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)P);  /* delta[0..n-1] */
    double *NU = calloc((size_t)(n > 0 ? n : 1) * (size_t)P, sizeof(double));
    double *psi = malloc(sizeof(double) * (size_t)(n + 1));
    double *dpsi = malloc(sizeof(double) * (size_t)(n + 1));
    int64_t *ms = malloc(sizeof(int64_t) * (size_t)(n + 1));
    double *cs = malloc(sizeof(double) * (size_t)(n + 1));
    double *lam = malloc(sizeof(double) * (size_t)P);
    double *lamprev = malloc(sizeof(double) * (size_t)P);
    double *lapnu = malloc(sizeof(double) * (size_t)P);
    double *sig = malloc(sizeof(double) * (size_t)P);
    double *dsig = malloc(sizeof(double) * (size_t)P);
    int rc = -1;
    if (!U || !D || !NU || !psi || !dpsi || !ms || !cs || !lam || !lamprev || !lapnu || !sig || !dsig)
        goto done;
    if (orc_run(pr, mem, u0, n, U, 1) != 0) goto done;
    for (int64_t k = 0; k < n; ++k) stencil(pr, U + k * P, D + k * P);
    orc_psi(pr->gamma, n, psi);
    orc_dpsi(pr->gamma, n, dpsi);

    double L = 0.0;
    for (int64_t p = 0; p < P; ++p) {
        double e = U[n * P + p] - target[p];
        L += 0.5 * e * e;
        lam[p] = e;
    }
    double dalpha = 0.0, dgamma = 0.0, drate = 0.0;
    const double lndt = log(dt);
    for (int64_t k = n - 1; k >= 0; --k) {
        /* lam holds lam[k+1] */
        const int64_t nt = orc_schedule(mem, k, ms, cs, n + 1);
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < P; ++p) {
            double s = 0.0, ds = 0.0;
            for (int64_t t = 0; t < nt; ++t) {
                s += cs[t] * psi[ms[t]] * D[(k - ms[t]) * P + p];
                ds += cs[t] * dpsi[ms[t]] * D[(k - ms[t]) * P + p];
            }
            sig[p] = s;
            dsig[p] = ds;
        }
        for (int64_t p = 0; p < P; ++p) {
            dalpha += lam[p] * (r / pr->alpha) * sig[p];
            dgamma += lam[p] * (r * lndt * sig[p] + r * dsig[p]);
            drate += lam[p] * dt * reaction_drate(pr, U[k * P + p]);
        }
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < P; ++p)
            for (int64_t t = 0; t < nt; ++t)
                NU[(k - ms[t]) * P + p] += r * cs[t] * psi[ms[t]] * lam[p];
        stencil(pr, NU + k * P, lapnu);
        for (int64_t p = 0; p < P; ++p)
            lamprev[p] = lam[p] + dt * reaction_du(pr, U[k * P + p]) * lam[p] + lapnu[p];
        double *tmp = lam; lam = lamprev; lamprev = tmp;
    }
    memcpy(du0, lam, sizeof(double) * (size_t)P);
    dparams[0] = dalpha;
    dparams[1] = dgamma;
    dparams[2] = drate;
    *loss = L;
    rc = 0;
done:
    free(U); free(D); free(NU); free(psi); free(dpsi); free(ms); free(cs);
    free(lam); free(lamprev); free(lapnu); free(sig); free(dsig);
    return rc;
}

/* Number of threads the OpenMP runtime will use for the parallel loops. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
