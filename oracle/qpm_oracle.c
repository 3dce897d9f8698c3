/*
 * qpm_oracle.c -- plain CPU oracle for the coupled third-harmonic QPM figure
 * of merit and for the HWSDA optimiser (DE rand/1 + grey-wolf update).
 *
 * TEST INFRASTRUCTURE ONLY. The test-suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only code that loads this library.
 * The HIP library never includes, links or calls it, and the two share no
 * code, header, table or constant generator.
 *
 * Arithmetic contract
 *   - Phases and fitness: long double (x87, 64-bit significand); outputs are
 *     rounded to double once.
 *   - Optimiser (DE, GWO, init): IEEE binary32 with explicit fmaf and
 *     correctly rounded division, built with -ffp-contract=off so that no
 *     other operation is fused. Decisions derived from a float (the +-1 map,
 *     the crossover test) are taken in binary32.
 *
 * Physics (paper Sec. 2.1, the d_eff double integral):
 *   S = int d(z) e^{-i dk2 z} ( int_{z_0}^{z} d(x) e^{-i dk1 x} dx ) dz
 *   f = |S|^2, maximised (paper Sec. 2.1: "find d(x) that makes d_eff
 *   largest"). The crystal is [z_0, z_N]; d(x) = d_n on [z_{n-1}, z_n).
 *   The prefactor of the undepleted-pump derivation is dropped, as the paper
 *   does when it writes the proportionality.
 *
 * Three evaluations of S are provided:
 *   orc_fitness_quad   nested Gauss-Legendre quadrature of the double
 *                      integral itself (the plain definition; small N).
 *   orc_fitness_pairs  the integral split domain by domain:
 *                      S = sum_{m<n} d_m d_n a_m b_n + sum_n d_n^2 c_n with
 *                      a_n = int_{dom n} e^{-i dk1 x} dx,
 *                      b_n = int_{dom n} e^{-i dk2 z} dz,
 *                      c_n = int_{dom n} e^{-i dk2 z} int_{z_{n-1}}^{z}
 *                            e^{-i dk1 x} dx dz   (O(N^2) work).
 *   orc_fitness        the same split evaluated left to right: while the
 *                      outer integral crosses domain n, the inner integral
 *                      equals P_{n-1} = sum_{m<n} d_m a_m plus the partial
 *                      integral inside domain n, so
 *                      S = sum_n d_n b_n P_{n-1} + sum_n c_n   (d_n^2 = 1).
 *
 * Optimiser (paper Sec. 2.2.1 DE, Sec. 2.2.2 GWO, Sec. 3.2 HWSDA steps):
 * see the comments at each function.
 *
 * Parity unpinned (against the paper):
 *   orc_dgwo_step, the improved discrete four-leader GWO of Sec. 3.1.2,
 *   which the paper gives in prose only; it implements a stated reading and
 *   its tests pin the reading, not the paper.
 *   orc_adaptive_F, the adaptive F of Sec. 3.1.1: the paper names its
 *   inputs (standard deviation, fitness range, convergence rate, progress),
 *   the range threshold 10^3, the convergence threshold 0.1, the cosine law
 *   and a quadratic coefficient from 1.0 to 0.8, but not the spread
 *   threshold 0.5, the factors 1.2 and 0.8, the scaling of the cosine law by
 *   0.1, or how s (std / mean) and kappa ((max - mean) / max) are defined;
 *   those are this oracle's readings, pinned by their own branches only.
 *   orc_polish, the gradient polish, is not in the paper at all: its tests
 *   pin mathematical properties of the stated rule (first-order ascent, the
 *   step length, the projection, strict acceptance), not a published
 *   result. Random numbers come from
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11), implemented here from that definition.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double ld;
typedef long double complex cld;

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */

/* e^{-i theta} */
static cld expmi(ld theta) { return cosl(theta) - I * sinl(theta); }

/* sin(x)/x, with its Taylor series near 0 */
static ld sincl_(ld x)
{
    if (fabsl(x) < 1e-5L) {
        ld x2 = x * x;
        return 1.0L - x2 / 6.0L + x2 * x2 / 120.0L;
    }
    return sinl(x) / x;
}

/* E(k, w) = int_0^w e^{-i k t} dt = w sinc(k w / 2) e^{-i k w / 2} */
static cld Ekw(ld k, ld w) { return w * sincl_(0.5L * k * w) * expmi(0.5L * k * w); }

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the parallel regions that follow (n >= 1); timing only, the
   results do not depend on it */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1, 1] (Newton iteration on P_n)            */
/* ------------------------------------------------------------------ */

static void gl_rule(int n, ld *x, ld *w)
{
    const ld pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        ld t = cosl(pi * ((ld)i + 0.75L) / ((ld)n + 0.5L));
        ld dp = 0.0L;
        for (int it = 0; it < 100; ++it) {
            ld p0 = 1.0L, p1 = t;
            for (int k = 2; k <= n; ++k) {
                ld p2 = ((ld)(2 * k - 1) * t * p1 - (ld)(k - 1) * p0) / (ld)k;
                p0 = p1;
                p1 = p2;
            }
            dp = (ld)n * (t * p1 - p0) / (t * t - 1.0L);
            ld dt = p1 / dp;
            t -= dt;
            if (fabsl(dt) < 1e-19L * (1.0L + fabsl(t))) break;
        }
        {
            /* recompute P_n' at the converged node */
            ld p0 = 1.0L, p1 = t;
            for (int k = 2; k <= n; ++k) {
                ld p2 = ((ld)(2 * k - 1) * t * p1 - (ld)(k - 1) * p0) / (ld)k;
                p0 = p1;
                p1 = p2;
            }
            dp = (ld)n * (t * p1 - p0) / (t * t - 1.0L);
        }
        x[i] = t;
        w[i] = 2.0L / ((1.0L - t * t) * dp * dp);
    }
}

void orc_gl_rule(int n, double *x, double *w)
{
    ld *xl = malloc(sizeof(ld) * n), *wl = malloc(sizeof(ld) * n);
    gl_rule(n, xl, wl);
    for (int i = 0; i < n; ++i) { x[i] = (double)xl[i]; w[i] = (double)wl[i]; }
    free(xl);
    free(wl);
}

/* composite Gauss-Legendre on [lo, hi]: npan panels of nq nodes each */
typedef cld (*cfun)(ld t, const void *ctx);
#define GL_NQ 16
static ld g_glx[GL_NQ], g_glw[GL_NQ];
static int g_gl_ready = 0;
static void gl_init(void)
{
    if (!g_gl_ready) {
        gl_rule(GL_NQ, g_glx, g_glw);
        g_gl_ready = 1;
    }
}

static cld gl_integrate(cfun f, const void *ctx, ld lo, ld hi, int npan)
{
    cld acc = 0.0L;
    ld h = (hi - lo) / (ld)npan;
    for (int p = 0; p < npan; ++p) {
        ld a = lo + h * (ld)p;
        ld mid = a + 0.5L * h, half = 0.5L * h;
        for (int q = 0; q < GL_NQ; ++q) acc += half * g_glw[q] * f(mid + half * g_glx[q], ctx);
    }
    return acc;
}

/* panels so that each panel spans at most 1/2 rad of oscillation */
static int panels_for(ld rate, ld len)
{
    ld r = fabsl(rate) * fabsl(len) / 0.5L;
    if (r > 1e6L) r = 1e6L;
    return 1 + (int)r;
}

/* ------------------------------------------------------------------ */
/* per-domain integrals                                                */
/* ------------------------------------------------------------------ */

/* G(k1,k2,w) = int_0^w e^{-i k2 t} E(k1, t) dt  (the diagonal double
 * integral of one domain, shifted to start at 0) */
struct gctx { ld k1, k2; };
static cld g_integrand(ld t, const void *c)
{
    const struct gctx *g = c;
    return expmi(g->k2 * t) * Ekw(g->k1, t);
}

static cld G_domain(ld k1, ld k2, ld w)
{
    if (fabsl(k1 * w) >= 1e-3L) {
        /* closed form: E(k1,t) = (1 - e^{-i k1 t}) / (i k1) */
        return (Ekw(k2, w) - Ekw(k1 + k2, w)) / (I * k1);
    }
    /* small |k1 w|: the closed form cancels; integrate the stable inner
     * expression instead */
    gl_init();
    struct gctx g = {k1, k2};
    return gl_integrate(g_integrand, &g, 0.0L, w, panels_for(fabsl(k1) + fabsl(k2), w));
}

void orc_G(double k1, double k2, double w, double *out2)
{
    cld g = G_domain(k1, k2, w);
    out2[0] = (double)creall(g);
    out2[1] = (double)cimagl(g);
}

/* G by quadrature only (used by tests to pin the closed form) */
void orc_G_quad(double k1, double k2, double w, double *out2)
{
    gl_init();
    struct gctx g = {k1, k2};
    cld r = gl_integrate(g_integrand, &g, 0.0L, w, panels_for(fabsl(k1) + fabsl(k2), w));
    out2[0] = (double)creall(r);
    out2[1] = (double)cimagl(r);
}

/* ------------------------------------------------------------------ */
/* design: domain boundaries and the per-domain integrals               */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    ld dk1, dk2;
    ld *z;
    cld *a, *b, *c;
    cld C;
} orc_design;

void orc_design_free(void *h)
{
    orc_design *d = h;
    if (!d) return;
    free(d->z);
    free(d->a);
    free(d->b);
    free(d->c);
    free(d);
}

/* z: n+1 strictly increasing finite boundaries. Returns NULL when invalid. */
void *orc_design_create(const double *z, int64_t n, double dk1, double dk2)
{
    if (n < 1 || !z || !isfinite(dk1) || !isfinite(dk2)) return NULL;
    for (int64_t i = 0; i <= n; ++i)
        if (!isfinite(z[i])) return NULL;
    for (int64_t i = 0; i < n; ++i)
        if (!(z[i + 1] > z[i])) return NULL;
    gl_init(); /* before the parallel loop below */
    orc_design *d = calloc(1, sizeof(*d));
    d->n = n;
    d->dk1 = dk1;
    d->dk2 = dk2;
    d->z = malloc(sizeof(ld) * (n + 1));
    d->a = malloc(sizeof(cld) * n);
    d->b = malloc(sizeof(cld) * n);
    d->c = malloc(sizeof(cld) * n);
    for (int64_t i = 0; i <= n; ++i) d->z[i] = z[i];
    cld C = 0.0L;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        ld lo = d->z[i], hi = d->z[i + 1];
        ld w = hi - lo, m = 0.5L * (lo + hi);
        /* int_{lo}^{hi} e^{-i k x} dx = e^{-i k m} w sinc(k w / 2) */
        d->a[i] = expmi(d->dk1 * m) * w * sincl_(0.5L * d->dk1 * w);
        d->b[i] = expmi(d->dk2 * m) * w * sincl_(0.5L * d->dk2 * w);
        d->c[i] = expmi(d->dk1 * lo) * expmi(d->dk2 * lo) * G_domain(d->dk1, d->dk2, w);
    }
    for (int64_t i = 0; i < n; ++i) C += d->c[i];
    d->C = C;
    return d;
}

int64_t orc_design_n(const void *h) { return ((const orc_design *)h)->n; }

/* a, b, c: 2n doubles (re, im interleaved); C: 2 doubles */
void orc_design_phases(const void *h, double *a, double *b, double *c, double *C)
{
    const orc_design *d = h;
    for (int64_t i = 0; i < d->n; ++i) {
        if (a) { a[2 * i] = (double)creall(d->a[i]); a[2 * i + 1] = (double)cimagl(d->a[i]); }
        if (b) { b[2 * i] = (double)creall(d->b[i]); b[2 * i + 1] = (double)cimagl(d->b[i]); }
        if (c) { c[2 * i] = (double)creall(d->c[i]); c[2 * i + 1] = (double)cimagl(d->c[i]); }
    }
    if (C) { C[0] = (double)creall(d->C); C[1] = (double)cimagl(d->C); }
}

/* ------------------------------------------------------------------ */
/* fitness                                                              */
/* ------------------------------------------------------------------ */

/* d: np x n int8 (+1 / -1). S: 2*np doubles, f: np doubles (either NULL ok) */
void orc_fitness(const void *h, const int8_t *dd, int64_t np, double *S, double *f)
{
    const orc_design *d = h;
    const int64_t n = d->n;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t g = 0; g < np; ++g) {
        const int8_t *dg = dd + g * n;
        cld P = 0.0L, Q = 0.0L;
        for (int64_t k = 0; k < n; ++k) {
            ld s = (ld)dg[k];
            Q += s * d->b[k] * P; /* outer integral over domain k with the inner prefix */
            P += s * d->a[k];
        }
        cld Sg = Q + d->C;
        if (S) { S[2 * g] = (double)creall(Sg); S[2 * g + 1] = (double)cimagl(Sg); }
        if (f) f[g] = (double)(creall(Sg) * creall(Sg) + cimagl(Sg) * cimagl(Sg));
    }
}

/* O(N^2) pair sum with a real-valued d (np x n doubles); includes d_n^2 c_n */
void orc_fitness_pairs(const void *h, const double *dd, int64_t np, double *S, double *f)
{
    const orc_design *d = h;
    const int64_t n = d->n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < np; ++g) {
        const double *dg = dd + g * n;
        cld acc = 0.0L;
        for (int64_t nn = 0; nn < n; ++nn) {
            cld inner = 0.0L;
            for (int64_t m = 0; m < nn; ++m) inner += (ld)dg[m] * d->a[m];
            acc += (ld)dg[nn] * d->b[nn] * inner;
            acc += (ld)dg[nn] * (ld)dg[nn] * d->c[nn];
        }
        if (S) { S[2 * g] = (double)creall(acc); S[2 * g + 1] = (double)cimagl(acc); }
        if (f) f[g] = (double)(creall(acc) * creall(acc) + cimagl(acc) * cimagl(acc));
    }
}

/* Nested Gauss-Legendre quadrature of the double integral for one genome,
 * straight from the boundaries (uses none of the per-domain closed forms). */
struct ectx { ld k; };
static cld e_integrand(ld x, const void *c) { return expmi(((const struct ectx *)c)->k * x); }

int orc_fitness_quad(const double *z, int64_t n, double dk1, double dk2, const int8_t *dg, double *S)
{
    if (n < 1) return -1;
    gl_init();
    struct ectx e1 = {dk1};
    cld P = 0.0L, acc = 0.0L;
    for (int64_t k = 0; k < n; ++k) {
        ld lo = z[k], hi = z[k + 1];
        ld s = (ld)dg[k];
        int npan = panels_for(fabsl((ld)dk1) + fabsl((ld)dk2), hi - lo);
        ld h = (hi - lo) / (ld)npan;
        for (int p = 0; p < npan; ++p) {
            ld pa = lo + h * (ld)p, mid = pa + 0.5L * h, half = 0.5L * h;
            for (int q = 0; q < GL_NQ; ++q) {
                ld zz = mid + half * g_glx[q];
                /* inner integral from the start of this domain to zz */
                cld part = gl_integrate(e_integrand, &e1, lo, zz, panels_for(dk1, zz - lo));
                cld inner = P + s * part;
                acc += half * g_glw[q] * s * expmi((ld)dk2 * zz) * inner;
            }
        }
        P += s * gl_integrate(e_integrand, &e1, lo, hi, panels_for(dk1, hi - lo));
    }
    S[0] = (double)creall(acc);
    S[1] = (double)cimagl(acc);
    return 0;
}

/* Exhaustive search over d with d_1 = +1 (f is invariant under d -> -d).
 * n <= 26. Writes the best d, its f, and the second-best distinct f. */
int orc_bruteforce(const void *h, int8_t *d_best, double *f_best, double *f_second)
{
    const orc_design *d = h;
    const int64_t n = d->n;
    if (n > 26 || n < 1) return -1;
    const int64_t count = (int64_t)1 << (n - 1);
    ld best = -1.0L, second = -1.0L;
    int64_t best_p = 0;
    for (int64_t p = 0; p < count; ++p) {
        cld P = 0.0L, Q = 0.0L;
        for (int64_t k = 0; k < n; ++k) {
            ld s = (k == 0) ? 1.0L : (((p >> (k - 1)) & 1) ? -1.0L : 1.0L);
            Q += s * d->b[k] * P;
            P += s * d->a[k];
        }
        cld Sg = Q + d->C;
        ld fv = creall(Sg) * creall(Sg) + cimagl(Sg) * cimagl(Sg);
        if (fv > best) { second = best; best = fv; best_p = p; }
        else if (fv > second) second = fv;
    }
    for (int64_t k = 0; k < n; ++k)
        d_best[k] = (k == 0) ? 1 : (((best_p >> (k - 1)) & 1) ? -1 : 1);
    *f_best = (double)best;
    *f_second = (double)second;
    return 0;
}

/* ------------------------------------------------------------------ */
/* differentiable relaxation d = tanh(theta) (not in the paper)         */
/* ------------------------------------------------------------------ */

/* theta: B x n. For real d the double integral is
 *   S = sum_{m<n} d_m d_n a_m b_n + sum_n d_n^2 c_n,
 * and dS/dd_k = b_k P_{k-1} + a_k R_{k+1} + 2 c_k d_k with
 * P_{k-1} = sum_{m<k} d_m a_m, R_{k+1} = sum_{n>k} d_n b_n.
 * df/dtheta_k = 2 Re(conj(S) dS/dd_k) (1 - d_k^2). */
void orc_relax(const void *h, const double *theta, int64_t B, double *S, double *f, double *grad)
{
    const orc_design *d = h;
    const int64_t n = d->n;
#pragma omp parallel
    {
        ld *dv = malloc(sizeof(ld) * n);
        cld *R = malloc(sizeof(cld) * (n + 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t bb = 0; bb < B; ++bb) {
            const double *th = theta + bb * n;
            for (int64_t k = 0; k < n; ++k) dv[k] = tanhl((ld)th[k]);
            cld P = 0.0L, Q = 0.0L, D = 0.0L;
            for (int64_t k = 0; k < n; ++k) {
                Q += dv[k] * d->b[k] * P;
                P += dv[k] * d->a[k];
                D += dv[k] * dv[k] * d->c[k];
            }
            cld Sg = Q + D;
            if (S) { S[2 * bb] = (double)creall(Sg); S[2 * bb + 1] = (double)cimagl(Sg); }
            if (f) f[bb] = (double)(creall(Sg) * creall(Sg) + cimagl(Sg) * cimagl(Sg));
            if (grad) {
                R[n] = 0.0L;
                for (int64_t k = n - 1; k >= 0; --k) R[k] = R[k + 1] + dv[k] * d->b[k];
                cld Pk = 0.0L;
                for (int64_t k = 0; k < n; ++k) {
                    cld dS = d->b[k] * Pk + d->a[k] * R[k + 1] + 2.0L * d->c[k] * dv[k];
                    ld df = 2.0L * creall(conjl(Sg) * dS);
                    grad[bb * n + k] = (double)(df * (1.0L - dv[k] * dv[k]));
                    Pk += dv[k] * d->a[k];
                }
            }
        }
        free(dv);
        free(R);
    }
}

/* f at real-valued d (long double), used for finite differences in tests */
void orc_relax_f_at(const void *h, const double *theta, int64_t B, double *f)
{
    orc_relax(h, theta, B, NULL, f, NULL);
}

/* Gradient polish of a few rows through the relaxation (not in the paper; a
 * use of the relaxation above to refine +-1 designs): each row of genes x
 * (binary32, rows x n) starts theta = x, so tanh(theta) has the signs of the
 * row's +-1 design. Then `steps` steps of normalised gradient ascent on the
 * relaxed fitness,
 *   g = df/dtheta (orc_relax),  m = max_k |g_k|,  theta += eta g / m
 * (no step when m = 0), so every step moves theta by exactly eta in the
 * largest coordinate. The result is projected back to a gene row
 * y = clamp(theta, -1, 1) (same signs as theta) and scored by the exact +-1
 * fitness of its signs (d = -1 exactly when y < 0), f1; the row is
 * accepted when f1 > f0 (strictly), f0 being the exact fitness the caller
 * holds for the row. theta in double; outputs: theta_out (rows x n, the
 * final theta, may be NULL), f1 (rows), accept (rows: 1 or 0). */
void orc_polish(const void *h, const float *x, int64_t rows, const double *f0, int steps, double eta,
                double *theta_out, double *f1, int32_t *accept)
{
    const orc_design *d = h;
    const int64_t n = d->n;
    double *th = malloc(sizeof(double) * rows * n);
    double *g = malloc(sizeof(double) * rows * n);
    int8_t *sg = malloc((size_t)(rows * n));
    for (int64_t k = 0; k < rows * n; ++k) th[k] = (double)x[k];
    for (int st = 0; st < steps; ++st) {
        orc_relax(h, th, rows, NULL, NULL, g);
        for (int64_t r = 0; r < rows; ++r) {
            double m = 0.0;
            for (int64_t k = 0; k < n; ++k) m = fmax(m, fabs(g[r * n + k]));
            if (m == 0.0) continue;
            for (int64_t k = 0; k < n; ++k) th[r * n + k] += eta * g[r * n + k] / m;
        }
    }
    for (int64_t k = 0; k < rows * n; ++k) {
        const double y = fmin(fmax(th[k], -1.0), 1.0);
        sg[k] = y < 0.0 ? -1 : 1;
    }
    orc_fitness(h, sg, rows, NULL, f1);
    for (int64_t r = 0; r < rows; ++r) accept[r] = f1[r] > f0[r] ? 1 : 0;
    if (theta_out) memcpy(theta_out, th, sizeof(double) * rows * n);
    free(th);
    free(g);
    free(sg);
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11 definition)                                     */
/* ------------------------------------------------------------------ */

void orc_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    /* round multipliers and Weyl key increments from the Philox paper */
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * x0;
        uint64_t p1 = (uint64_t)M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* stream tags (counter word 3, low byte); high 24 bits = instance */
enum { TAG_INIT = 1, TAG_DE_IDX = 2, TAG_DE_CR = 3, TAG_GWO = 4, TAG_DGWO = 5 };

static uint32_t draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t inst,
                     uint32_t tag, int lane)
{
    uint32_t ctr[4] = {c0, c1, c2, (inst << 8) | tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox(ctr, key, out);
    return out[lane];
}

/* maps from a 32-bit word; every one is exact in binary32 */
static float u24f(uint32_t u) { return (float)(u >> 8) * 0x1p-24f; }        /* [0, 1) */
static float symf(uint32_t u) { return (float)(u >> 8) * 0x1p-23f - 1.0f; } /* [-1, 1) */
static uint32_t bnd(uint32_t u, uint32_t m) { return (uint32_t)(((uint64_t)u * m) >> 32); }

/* the +-1 map: d = -1 exactly when the gene is below zero (-0.0 maps to +1) */
void orc_sign_map(const float *x, int64_t count, int8_t *d)
{
    for (int64_t i = 0; i < count; ++i) d[i] = (x[i] < 0.0f) ? -1 : 1;
}

/* ------------------------------------------------------------------ */
/* DE (paper Sec. 2.2.1)                                                */
/* ------------------------------------------------------------------ */

/* Step 1, initialisation: x_ij uniform on the box, here [-1, 1). */
void orc_init_pop(int64_t np, int64_t D, uint64_t seed, uint32_t inst, float *x)
{
    for (int64_t i = 0; i < np; ++i)
        for (int64_t j = 0; j < D; ++j)
            x[i * D + j] = symf(draw(seed, (uint32_t)(j >> 2), (uint32_t)i, 0u, inst, TAG_INIT, (int)(j & 3)));
}

/* the k-th (0-based) member of {0..np-1} minus the excluded indices */
static int64_t kth_not_excluded(int64_t k, int64_t np, const int64_t *ex, int nex)
{
    int64_t seen = 0;
    for (int64_t r = 0; r < np; ++r) {
        int skip = 0;
        for (int e = 0; e < nex; ++e)
            if (ex[e] == r) skip = 1;
        if (skip) continue;
        if (seen == k) return r;
        ++seen;
    }
    return -1;
}

/* Steps 2-3, rand/1 mutation and binomial crossover, synchronous (every
 * trial reads the population x of generation g).
 *   r1, r2, r3: mutually distinct and different from i (needs np >= 4),
 *     drawn uniformly without replacement;
 *   v = x_r1 + F (x_r2 - x_r3), clamped to [-1, 1];
 *   u_ij = v_j when randb(j) <= CR or j == jrand, else x_ij.
 * idx (may be NULL): np x 4 int32 = r1, r2, r3, jrand. */
void orc_de_step(const float *x, int64_t np, int64_t D, float F, float CR, uint64_t seed,
                 uint32_t g, uint32_t inst, float *u, int32_t *idx)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < np; ++i) {
        uint32_t o[4];
        for (int l = 0; l < 4; ++l) o[l] = draw(seed, 0u, (uint32_t)i, g, inst, TAG_DE_IDX, l);
        int64_t ex[3];
        ex[0] = i;
        int64_t r1 = kth_not_excluded(bnd(o[0], (uint32_t)(np - 1)), np, ex, 1);
        ex[1] = r1;
        int64_t r2 = kth_not_excluded(bnd(o[1], (uint32_t)(np - 2)), np, ex, 2);
        ex[2] = r2;
        int64_t r3 = kth_not_excluded(bnd(o[2], (uint32_t)(np - 3)), np, ex, 3);
        int64_t jrand = bnd(o[3], (uint32_t)D);
        if (idx) {
            idx[4 * i + 0] = (int32_t)r1;
            idx[4 * i + 1] = (int32_t)r2;
            idx[4 * i + 2] = (int32_t)r3;
            idx[4 * i + 3] = (int32_t)jrand;
        }
        for (int64_t j = 0; j < D; ++j) {
            uint32_t q = draw(seed, (uint32_t)(j >> 2), (uint32_t)i, g, inst, TAG_DE_CR, (int)(j & 3));
            int take = (u24f(q) <= CR) || (j == jrand);
            float diff = x[r2 * D + j] - x[r3 * D + j];
            float v = fmaf(F, diff, x[r1 * D + j]);
            v = fminf(fmaxf(v, -1.0f), 1.0f);
            u[i * D + j] = take ? v : x[i * D + j];
        }
    }
}

/* ------------------------------------------------------------------ */
/* GWO (paper Sec. 2.2.2)                                               */
/* ------------------------------------------------------------------ */

/* Per gene j of a non-leader wolf x, for each leader k in (alpha, beta,
 * delta) with its own random pair (r1, r2) in [0, 1):
 *   A = 2 a r1 - a,  C = 2 r2,
 *   D_k = |C X_k - x|,  Y_k = X_k - A D_k;
 * then the magnitude-weighted combination
 *   y = (sum_k w_k Y_k) / 3,  w_k = |Y_k| / sum |Y|   (variant 0, as printed)
 *   y = (Y_1 + Y_2 + Y_3) / 3                         (variant 1, textbook)
 * clamped to [-1, 1]; y = 0 when all three Y_k are 0. Leaders keep their
 * positions. The pair (r1, r2) of (gene j, leader k) is the low / high
 * 16-bit half of one Philox word. */
void orc_gwo_step(const float *x, int64_t np, int64_t D, const int32_t *leaders, float a,
                  uint64_t seed, uint32_t g, uint32_t inst, int variant, float *y)
{
    const float two_a = 2.0f * a;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < np; ++i) {
        int is_leader = (i == leaders[0] || i == leaders[1] || i == leaders[2]);
        for (int64_t j = 0; j < D; ++j) {
            if (is_leader) { y[i * D + j] = x[i * D + j]; continue; }
            float xi = x[i * D + j];
            float Y[3];
            for (int k = 0; k < 3; ++k) {
                int64_t t = 3 * (j & 3) + k; /* word index within the gene quad */
                uint32_t c0 = (uint32_t)(3 * (j >> 2) + t / 4);
                uint32_t o = draw(seed, c0, (uint32_t)i, g, inst, TAG_GWO, (int)(t % 4));
                float r1 = (float)(o & 0xFFFFu) * 0x1p-16f;
                float r2 = (float)(o >> 16) * 0x1p-16f;
                float A = fmaf(two_a, r1, -a);
                float Cc = 2.0f * r2;
                float Xk = x[(int64_t)leaders[k] * D + j];
                float Dk = fabsf(fmaf(Cc, Xk, -xi));
                Y[k] = fmaf(-A, Dk, Xk);
            }
            float yv;
            if (variant == 1) {
                yv = ((Y[0] + Y[1]) + Y[2]) / 3.0f;
            } else {
                float s = (fabsf(Y[0]) + fabsf(Y[1])) + fabsf(Y[2]);
                if (s == 0.0f) {
                    yv = 0.0f;
                } else {
                    float num = fmaf(fabsf(Y[2]), Y[2], fmaf(fabsf(Y[1]), Y[1], fabsf(Y[0]) * Y[0]));
                    yv = (num / s) / 3.0f;
                }
            }
            y[i * D + j] = fminf(fmaxf(yv, -1.0f), 1.0f);
        }
    }
}

/* ------------------------------------------------------------------ */
/* improved discrete grey-wolf step (Sec. 3.1.2)                        */
/* ------------------------------------------------------------------ */

/* PARITY UNPINNED against the paper: Sec. 3.1.2 describes the discrete
 * variant in words only (four leaders, +-1 states, a transition
 * probability from the leaders' state counts, a perturbation that is
 * strong early and a small flip probability late, a dispersion parameter,
 * social learning at a falling rate) and gives no formula or rate. The
 * rule below is this oracle's reading; its tests pin the implementation to
 * the rule (special cases, frequencies), not the rule to the paper.
 *
 * Generation parameters, t = g / G in double, each rounded to float once:
 *   par[0] = t
 *   par[1] = 1 - 2 eps, eps = 0.1 (1 - t) + 0.01 t    (perturbation)
 *   par[2] = eps
 *   par[3] = lambda = 0.2 (1 - t)                      (social learning) */
void orc_dgwo_params(int64_t g, int64_t G, float *par)
{
    double t = (double)g / (double)G;
    float eps = (float)(0.1 * (1.0 - t) + 0.01 * t);
    par[0] = (float)t;
    par[1] = (float)(1.0 - 2.0 * (double)eps);
    par[2] = eps;
    par[3] = (float)(0.2 * (1.0 - t));
}

/* One step. L4: the four best (alpha, beta, delta, then the fourth); the
 * first three keep their rows, every other wolf (the fourth included)
 * gets new +-1 genes. For gene j of wolf i, with one Philox word w
 * (tag DGWO, word j % 4 of counter j / 4):
 *   n     = how many of the four leaders hold state +1 (gene >= 0) at j;
 *   dist  = n / 4                  (the leaders' state distribution),
 *   maj   = 1, 0 or 1/2 as n > 2, n < 2 or n = 2  (the dominant state),
 *   p     = fmaf(t, maj - dist, dist)   (distribution early, majority late),
 *   p'    = fmaf(1 - 2 eps, p, eps)     (perturbation towards 1/2),
 *   social learning when (w >> 16 & 0x3FFF) 2^-14 < lambda: the state of
 *   leader w >> 30; otherwise +1 when (w & 0xFFFF) 2^-16 < p', else -1.
 * All of it in binary32. */
void orc_dgwo_step(const float *x, int64_t np, int64_t D, const int32_t *L4, const float *par, uint64_t seed,
                   uint32_t g, uint32_t inst, float *y)
{
    const float t = par[0], c1 = par[1], eps = par[2], lam = par[3];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < np; ++i) {
        int keep = (i == L4[0] || i == L4[1] || i == L4[2]);
        for (int64_t j = 0; j < D; ++j) {
            if (keep) {
                y[i * D + j] = x[i * D + j];
                continue;
            }
            int plus[4], n = 0;
            for (int k = 0; k < 4; ++k) {
                plus[k] = !(x[(int64_t)L4[k] * D + j] < 0.0f);
                n += plus[k];
            }
            uint32_t w = draw(seed, (uint32_t)(j >> 2), (uint32_t)i, g, inst, TAG_DGWO, (int)(j & 3));
            float dist = (float)n * 0.25f;
            float maj = n > 2 ? 1.0f : (n < 2 ? 0.0f : 0.5f);
            float p = fmaf(t, maj - dist, dist);
            float p2 = fmaf(c1, p, eps);
            float us = (float)((w >> 16) & 0x3FFFu) * 0x1p-14f;
            float up = (float)(w & 0xFFFFu) * 0x1p-16f;
            int state = us < lam ? plus[w >> 30] : (up < p2);
            y[i * D + j] = state ? 1.0f : -1.0f;
        }
    }
}

/* ------------------------------------------------------------------ */
/* leaders and the HWSDA loop (paper Sec. 3.2)                          */
/* ------------------------------------------------------------------ */

static const double *g_sort_f;
static int cmp_desc(const void *pa, const void *pb)
{
    int64_t ia = *(const int64_t *)pa, ib = *(const int64_t *)pb;
    double fa = g_sort_f[ia], fb = g_sort_f[ib];
    if (fa > fb) return -1;
    if (fa < fb) return 1;
    return (ia < ib) ? -1 : (ia > ib);
}

/* Step 3: sort all fitness values, best first (ties: lower index first),
 * and take the first three as alpha, beta, delta. */
static void topk(const double *f, int64_t np, int k, int32_t *out)
{
    int64_t *ord = malloc(sizeof(int64_t) * np);
    for (int64_t i = 0; i < np; ++i) ord[i] = i;
    g_sort_f = f;
    qsort(ord, np, sizeof(int64_t), cmp_desc);
    for (int m = 0; m < k; ++m) out[m] = (int32_t)ord[m];
    free(ord);
}

void orc_top3(const double *f, int64_t np, int32_t *out) { topk(f, np, 3, out); }

/* the four best (Sec. 3.1.2: a fourth leader joins alpha, beta, delta) */
void orc_top4(const double *f, int64_t np, int32_t *out) { topk(f, np, 4, out); }

/* a decreases linearly from 2 towards 0 over the run */
float orc_a_schedule(int64_t g, int64_t G) { return (float)(2.0 * (1.0 - (double)g / (double)G)); }

/* ------------------------------------------------------------------ */
/* parameter control (Sec. 3.1.1; the parameter settings of Sec. 4)     */
/* ------------------------------------------------------------------ */

/* The GWO coefficient a_g of generation g under each control:
 *   0  the textbook schedule above, a from 2 towards 0 (Sec. 2.2.2); F is
 *      the caller's constant;
 *   1  F = a, starting at 0.1 and falling to 0.01 over the run (Sec. 4,
 *      parameter settings). The paper gives no decay law; linear in g / G
 *      is this oracle's reading;
 *   2  a as in 1, F adaptive (orc_adaptive_F). */
float orc_a_control(int control, int64_t g, int64_t G)
{
    if (control == 0) return orc_a_schedule(g, G);
    double t = (double)g / (double)G;
    return (float)(0.1 * (1.0 - t) + 0.01 * t);
}

/* The adaptive DE scale factor of Sec. 3.1.1, kept in [0.01, 0.1], from
 * the fitness of the population that enters generation g:
 *   s     = std(f) / mean(f)          relative spread (population std),
 *   kappa = (max f - mean f) / max f  how far the mean trails the best
 *                                     (small once the population has
 *                                     converged: the convergence measure),
 *   range = max f - min f             (f in um^2).
 * Low diversity, s < 0.1 or kappa < 0.1: F is raised by the exploration
 * factor 1.2. Else too much spread or a narrow range, s > 0.5 or
 * range < 10^3: F is lowered by the exploitation factor 0.8. Else the
 * factor is 1. The factor scales the decay law of the intermediate state,
 *   base(g) = 0.1 (cos(pi g / (2G)) + 1) / 2 (1 - 0.2 (g / G)^2),
 * the paper's cosine decay times a quadratic coefficient falling from 1.0
 * to 0.8, scaled so that F starts at the top of the interval; the product
 * is clamped to [0.01, 0.1] and rounded to float once. Readings (the paper
 * names the quantities but not these values): the definitions of s and
 * kappa, the threshold 0.5 on s, the factors 1.2 and 0.8, the scaling by
 * 0.1, and that the factor applies to base(g) rather than to the previous
 * F. */
float orc_adaptive_F(const double *f, int64_t np, int64_t g, int64_t G)
{
    double sum = 0.0, mx = f[0], mn = f[0];
    for (int64_t i = 0; i < np; ++i) {
        sum += f[i];
        if (f[i] > mx) mx = f[i];
        if (f[i] < mn) mn = f[i];
    }
    double mean = sum / (double)np;
    double ss = 0.0;
    for (int64_t i = 0; i < np; ++i) ss += (f[i] - mean) * (f[i] - mean);
    double sd = sqrt(ss / (double)np);
    double s = mean > 0.0 ? sd / mean : 0.0;
    double kappa = mx > 0.0 ? (mx - mean) / mx : 0.0;
    double m = 1.0;
    if (s < 0.1 || kappa < 0.1)
        m = 1.2;
    else if (s > 0.5 || mx - mn < 1e3)
        m = 0.8;
    double t = (double)g / (double)G;
    double base = 0.1 * (0.5 * (cos(0.5 * M_PI * t) + 1.0)) * (1.0 - 0.2 * t * t);
    double F = base * m;
    if (F < 0.01) F = 0.01;
    if (F > 0.1) F = 0.1;
    return (float)F;
}

/* ------------------------------------------------------------------ */
/* multi-wavelength objective (the multi-wavelength SHG and coupled THG  */
/* designs of the paper's last section)                                 */
/* ------------------------------------------------------------------ */

/* K designs on the same boundaries z, one per wavelength (its dk1, dk2),
 * L = z_N - z_0. Per genome and wavelength k:
 *   SHG (kind 0): G_k = |int d(z) e^{-i dk1_k z} dz| / L
 *                     = |sum_n d_n a_n^(k)| / L, the single-integral
 *                 coupling of second-harmonic generation;
 *   THG (kind 1): G_k = |S_k| / L^2, the coupled double integral of
 *                 Sec. 2.1 with the k-th (dk1, dk2).
 * The paper's objective h = sum_k |G0 - G_k| + beta (max_k G_k - min_k G_k)
 * is minimised; the optimiser maximises f = -h. Normalising G by L (SHG)
 * and L^2 (THG) makes G dimensionless (at most 1), so G0 and beta are too:
 * a reading, the paper does not state its scale.
 * dd: np x n int8; G (may be NULL): np x K; f: np. Returns -1 when the
 * designs differ in their boundaries or an argument is out of range. */
static int multi_valid(const void *const *designs, int K, int kind)
{
    if (K < 1 || (kind != 0 && kind != 1)) return 0;
    const orc_design *d0 = designs[0];
    for (int k = 1; k < K; ++k) {
        const orc_design *dk = designs[k];
        if (dk->n != d0->n) return 0;
        for (int64_t i = 0; i <= d0->n; ++i)
            if (dk->z[i] != d0->z[i]) return 0;
    }
    return 1;
}

int orc_multi_objective(const void *const *designs, int K, int kind, double G0, double beta, const int8_t *dd,
                        int64_t np, double *G, double *f)
{
    if (!multi_valid(designs, K, kind)) return -1;
    const orc_design *d0 = designs[0];
    const int64_t n = d0->n;
    const ld L = d0->z[n] - d0->z[0];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t g = 0; g < np; ++g) {
        const int8_t *dg = dd + g * n;
        ld sum = 0.0L, gmax = 0.0L, gmin = 0.0L;
        for (int k = 0; k < K; ++k) {
            const orc_design *dk = designs[k];
            cld P = 0.0L, Q = 0.0L;
            for (int64_t m = 0; m < n; ++m) {
                ld s = (ld)dg[m];
                Q += s * dk->b[m] * P;
                P += s * dk->a[m];
            }
            ld Gk = kind == 0 ? cabsl(P) / L : cabsl(Q + dk->C) / (L * L);
            if (G) G[g * K + k] = (double)Gk;
            sum += fabsl((ld)G0 - Gk);
            if (k == 0 || Gk > gmax) gmax = Gk;
            if (k == 0 || Gk < gmin) gmin = Gk;
        }
        f[g] = (double)(-(sum + (ld)beta * (gmax - gmin)));
    }
    return 0;
}

/* the fitness the optimiser maximises: |d_eff|^2 of one design, or the
 * negated multi-wavelength objective */
typedef struct {
    const orc_design *d;       /* single design (K == 0) */
    const void *const *ds;     /* K designs */
    int K, kind;
    double G0, beta;
} orc_target;

static void fitness_of_genes(const orc_target *t, int64_t D, const float *x, int64_t np, int8_t *scratch, double *f)
{
    orc_sign_map(x, np * D, scratch);
    if (t->K == 0)
        orc_fitness(t->d, scratch, np, NULL, f);
    else
        orc_multi_objective(t->ds, t->K, t->kind, t->G0, t->beta, scratch, np, NULL, f);
}

/* The whole optimiser. x_out: np x n final genes, f_out: np final fitness,
 * trace (may be NULL): best fitness after each generation; params (may be
 * NULL): F_g and a_g of each generation (2 G floats).
 * Per generation g of HWSDA (algo 0, Sec. 3.2): F_g and a_g from the
 * control (orc_a_control; orc_adaptive_F on the current fitness under
 * control 2), DE trials, evaluation, greedy selection (strict >); leaders
 * from the sorted fitness; GWO candidates for the other wolves (variants 0
 * and 1), or the discrete four-leader step (variant 2, orc_dgwo_step,
 * guided by the four best), evaluation, greedy selection again (alpha,
 * beta, delta kept). CR stays fixed (step 6 of Sec. 3.2 updates "F, CR and
 * others"; the paper gives a rule for F only).
 * The two optimisers HWSDA is compared with (Tables 3-7):
 *   algo 1, DE alone (Sec. 2.2.1): per generation only the DE trials,
 *           their evaluation and the greedy selection;
 *   algo 2, GWO alone (Sec. 2.2.2): per generation the leaders from the
 *           sorted fitness, the omega wolves move to their GWO candidates
 *           unconditionally (the basic GWO has no greedy selection; it is
 *           DE's operator, which HWSDA adds back as its step 5), alpha,
 *           beta and delta keep their positions, evaluation. */
static int hwsda_loop(const orc_target *t, int64_t D, int64_t np, int64_t G, float F, float CR, uint64_t seed,
                      uint32_t inst, int variant, int control, int algo, float *x_out, double *f_out, double *trace,
                      float *params)
{
    if (np < 4 || G < 1 || control < 0 || control > 2 || variant < 0 || variant > 2 || algo < 0 || algo > 2)
        return -1;
    float *x = x_out;
    float *u = malloc(sizeof(float) * np * D);
    int8_t *sg = malloc((size_t)(np * D));
    double *f = f_out;
    double *fu = malloc(sizeof(double) * np);
    orc_init_pop(np, D, seed, inst, x);
    fitness_of_genes(t, D, x, np, sg, f);
    for (int64_t g = 0; g < G; ++g) {
        const float a_g = orc_a_control(control, g, G);
        const float F_g = control == 0 ? F : (control == 1 ? a_g : orc_adaptive_F(f, np, g, G));
        if (params) {
            params[2 * g] = F_g;
            params[2 * g + 1] = a_g;
        }
        if (algo != 2) {
            orc_de_step(x, np, D, F_g, CR, seed, (uint32_t)g, inst, u, NULL);
            fitness_of_genes(t, D, u, np, sg, fu);
            for (int64_t i = 0; i < np; ++i)
                if (fu[i] > f[i]) {
                    memcpy(x + i * D, u + i * D, sizeof(float) * D);
                    f[i] = fu[i];
                }
        }
        if (algo != 1) {
            int32_t L[4];
            if (variant == 2) {
                float par[4];
                orc_top4(f, np, L);
                orc_dgwo_params(g, G, par);
                orc_dgwo_step(x, np, D, L, par, seed, (uint32_t)g, inst, u);
            } else {
                orc_top3(f, np, L);
                orc_gwo_step(x, np, D, L, a_g, seed, (uint32_t)g, inst, variant, u);
            }
            fitness_of_genes(t, D, u, np, sg, fu);
            for (int64_t i = 0; i < np; ++i) {
                if (i == L[0] || i == L[1] || i == L[2]) continue;
                if (algo == 2 || fu[i] > f[i]) {
                    memcpy(x + i * D, u + i * D, sizeof(float) * D);
                    f[i] = fu[i];
                }
            }
        }
        if (trace) {
            double best = f[0];
            for (int64_t i = 1; i < np; ++i)
                if (f[i] > best) best = f[i];
            trace[g] = best;
        }
    }
    free(u);
    free(sg);
    free(fu);
    return 0;
}

int orc_hwsda_run_ctl(const void *h, int64_t np, int64_t G, float F, float CR, uint64_t seed,
                      uint32_t inst, int variant, int control, float *x_out, double *f_out,
                      double *trace, float *params)
{
    const orc_target t = {h, NULL, 0, 0, 0.0, 0.0};
    return hwsda_loop(&t, ((const orc_design *)h)->n, np, G, F, CR, seed, inst, variant, control, 0, x_out, f_out,
                      trace, params);
}

/* The loop with the optimiser chosen by algo: 0 HWSDA, 1 DE alone, 2 GWO
 * alone (see hwsda_loop). */
int orc_run_algo(const void *h, int64_t np, int64_t G, float F, float CR, uint64_t seed, uint32_t inst, int variant,
                 int control, int algo, float *x_out, double *f_out, double *trace, float *params)
{
    const orc_target t = {h, NULL, 0, 0, 0.0, 0.0};
    return hwsda_loop(&t, ((const orc_design *)h)->n, np, G, F, CR, seed, inst, variant, control, algo, x_out,
                      f_out, trace, params);
}

/* The optimiser chosen by algo (as orc_run_algo) on the multi-wavelength
 * objective (f = -h of orc_multi_objective); controls 0 and 1 (the
 * adaptive rule's thresholds are stated for |d_eff|^2). */
int orc_run_obj_algo(const void *const *designs, int K, int kind, double G0, double beta, int64_t np, int64_t G,
                     float F, float CR, uint64_t seed, uint32_t inst, int variant, int control, int algo,
                     float *x_out, double *f_out, double *trace, float *params)
{
    if (!multi_valid(designs, K, kind) || control == 2) return -1;
    const orc_target t = {NULL, designs, K, kind, G0, beta};
    const int64_t D = ((const orc_design *)designs[0])->n;
    return hwsda_loop(&t, D, np, G, F, CR, seed, inst, variant, control, algo, x_out, f_out, trace, params);
}

/* HWSDA on the multi-wavelength objective. */
int orc_hwsda_run_obj(const void *const *designs, int K, int kind, double G0, double beta, int64_t np, int64_t G,
                      float F, float CR, uint64_t seed, uint32_t inst, int variant, int control, float *x_out,
                      double *f_out, double *trace, float *params)
{
    return orc_run_obj_algo(designs, K, kind, G0, beta, np, G, F, CR, seed, inst, variant, control, 0, x_out, f_out,
                            trace, params);
}

/* The optimiser with the textbook parameters (control 0). */
int orc_hwsda_run(const void *h, int64_t np, int64_t G, float F, float CR, uint64_t seed,
                  uint32_t inst, int variant, float *x_out, double *f_out, double *trace)
{
    return orc_hwsda_run_ctl(h, np, G, F, CR, seed, inst, variant, 0, x_out, f_out, trace, NULL);
}
