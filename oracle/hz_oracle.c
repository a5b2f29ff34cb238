/*
 * hz_oracle.c -- plain, unblocked, one-sided implicit Hari-Zimmermann GSVD
 * of a real (double) or complex (double complex) matrix pair (F, G).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the CPU oracle against which the GPU
 * library is checked.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the GPU library never links, calls or
 * includes anything from here, and this file includes nothing from the
 * library.  It is written for obviousness, not speed: one column pair at a
 * time, sequential dot products, no blocking.
 *
 * What it computes (Novakovic & Singer, "Implicit Hari-Zimmermann algorithm
 * for the generalized SVD on the GPUs"):
 *   Section 1   : F Z = U Sigma_F, G Z = V Sigma_G, U^*U = V^*V = I,
 *                 Sigma_F^2 + Sigma_G^2 = I, Sigma = Sigma_G^{-1} Sigma_F,
 *                 output sorted descendingly by a symmetric permutation.
 *   Section 2   : n = 1 closed form; prescaling by Z_0 = diag(1/||g_j||).
 *   Section 2.1 : pointwise step on the pivot pair (i, j): 2x2 pivot
 *                 matrices from dot products, relative-orthogonality skip
 *                 test, the 2x2 transformation (2.1.1 complex, 2.1.2 real,
 *                 each with its exception), application to the columns of
 *                 F, G, Z, and the column-sorting heuristic.
 *   Section 2.2 : sweeps under a sequential or parallel strategy.
 *   Section 2.4 : final rescaling and extraction of U, V, Sigma_F, Sigma_G,
 *                 Sigma, Z.
 *   Section 2.5 : big/small classification (criteria C1 and C2) and the stop rule
 *                 "no big transformation in a sweep".
 *   Table 1     : variant 0 (C1, prescaled, ordinary dot products),
 *                 variant 4 (the same with criterion C2), and variants 1
 *                 and 5 (0 and 4 with the enhanced dot products of
 *                 Appendix A: for real pairs all the pivot entries a_ii,
 *                 a_jj, a_ij, b_ij; for complex pairs the squared norms
 *                 a_ii, a_jj by the appendix's simpler procedure, the
 *                 off-diagonal entries, for which it defines none,
 *                 ordinary).
 *
 * Readings of passages that are silent, garbled or inconsistent (each one is
 * also listed in the design notes of the repository):
 *   - The prescale factor is 1/||g_j||_2 (Section 3.3 and the requirement
 *     diag(B) = I); the 1/sqrt(||g_j||) printed in Section 2 is a typo.
 *   - cos(theta) = 1/sqrt(1 + tan^2(theta)) (the printed 1/(1 + tan^2) would
 *     not give a rotation), sin(theta) = tan(theta) cos(theta).
 *   - Real exception (A' proportional to B'): the printed matrix with |x| is
 *     a congruence to I only for x >= 0; the sign of x is carried onto the
 *     off-diagonal entries, which is the complex exception with zeta in
 *     {0, pi}.
 *   - Complex case, h = 0 and v != 0: tan(gamma) = +-inf, cos(gamma) = 0 and
 *     sin(gamma) = sign(v) (the printed "sin = 1" holds only for v > 0).
 *   - sign(a, b) is |a| with the sign of b (copysign), also for b = +-0.
 *   - The orthogonality threshold eps*sqrt(n) is a parameter tol (default
 *     eps*sqrt(n), eps = DBL_EPSILON = 2^-52); criterion C1 compares the
 *     computed scaled cosines with 1 exactly.
 *   - Stop rule: after a sweep with no big transformation (the outer-level
 *     rule of Section 2.5), or after max_sweeps sweeps.
 *   - The output is sorted by a stable descending sort on sigma.
 *
 * Matrices are column-major (Fortran order) with leading dimensions; F and G
 * are overwritten by U and V.  Complex matrices are interleaved
 * (re, im) double complex.
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex zdouble;

/* ---------------------------------------------------------------- helpers */

static double sign1(double b) { return copysign(1.0, b); }

static double dot_rr(const double *x, const double *y, int64_t m)
{
    double s = 0.0;
    for (int64_t r = 0; r < m; ++r)
        s += x[r] * y[r];
    return s;
}

/* The product a*b rounded toward -infinity, from the round-to-nearest
 * product p and its exact error e = a*b - p (one FMA): the exact product
 * is p + e, so it rounds down to p when e >= 0 and otherwise to the next
 * double below p (the one the exact value lies above).  Normal range. */
static double mul_rd(double a, double b)
{
    const double p = a * b;
    const double e = fma(a, b, -p);
    return (e < 0.0) ? nextafter(p, -INFINITY) : p;
}

/* Enhanced dot product (Appendix A): for each pair of entries the product
 * rounded down, c, and its rounding error d = fma(a, b, -c) >= 0, summed
 * separately; the result is (sum of c) + (sum of d). */
static double dot_rr_enh(const double *x, const double *y, int64_t m)
{
    double sc = 0.0, sd = 0.0;
    for (int64_t r = 0; r < m; ++r) {
        const double c = mul_rd(x[r], y[r]);
        sc += c;
        sd += fma(x[r], y[r], -c);
    }
    return sc + sd;
}

/* Exported for the tests: the enhanced dot product of x and y (n entries),
 * and the rounded-down product with its error term. */
double hzo_edot(int64_t n, const double *x, const double *y) { return dot_rr_enh(x, y, n); }

void hzo_mul_rd(double a, double b, double *c, double *d)
{
    *c = mul_rd(a, b);
    *d = fma(a, b, -*c);
}

/* x^* y for complex columns. */
static zdouble dot_zz(const zdouble *x, const zdouble *y, int64_t m)
{
    zdouble s = 0.0;
    for (int64_t r = 0; r < m; ++r)
        s += conj(x[r]) * y[r];
    return s;
}

/* Squared norm of a complex column by the simpler procedure of Appendix A:
 * per entry the rounded-down squares of the real and the imaginary part,
 * c_r and c_i, and the sum e of their errors, combined as (e + min) + max
 * of the two squares, and these summed. */
static double enh_abs2(zdouble a)
{
    const double re = creal(a), im = cimag(a);
    const double cr = mul_rd(re, re), ci = mul_rd(im, im);
    const double e = fma(re, re, -cr) + fma(im, im, -ci);
    return (cr <= ci) ? (e + cr) + ci : (e + ci) + cr;
}

static double nrm2sq_z_enh(const zdouble *x, int64_t m)
{
    double s = 0.0;
    for (int64_t r = 0; r < m; ++r)
        s += enh_abs2(x[r]);
    return s;
}

/* Exported for the tests: enh_abs2 of re + i im. */
double hzo_enh_abs2(double re, double im) { return enh_abs2(CMPLX(re, im)); }

static double nrm2sq_z(const zdouble *x, int64_t m)
{
    double s = 0.0;
    for (int64_t r = 0; r < m; ++r)
        s += creal(x[r]) * creal(x[r]) + cimag(x[r]) * cimag(x[r]);
    return s;
}

/* cos and sin of an angle in (-pi/2, pi/2] from its tangent (Section 2.1.1:
 * the tangent identities, with the infinite-tangent case). */
static void cos_sin_from_tan(double tn, double *c, double *s)
{
    if (isinf(tn)) {
        *c = 0.0;
        *s = sign1(tn);
    } else {
        *c = 1.0 / sqrt(1.0 + tn * tn);
        *s = tn * (*c);
    }
}

/* ------------------------------------------------------- 2x2, real case */

/*
 * Section 2.1.2: the real transformation Zhat' = (1/t) [[cos phi, sin phi],
 * [-sin psi, cos psi]] that makes Zhat'^T A' Zhat' diagonal and
 * Zhat'^T B' Zhat' = I for A' = [[aii, aij], [aij, ajj]],
 * B' = [[1, x], [x, 1]].  Z is returned column-major: Z[0]=Z11, Z[1]=Z21,
 * Z[2]=Z12, Z[3]=Z22.  *exc is set when the exception (A' proportional to B')
 * is taken.
 */
void hzo_real_2x2_c(double aii, double ajj, double aij, double x, double Z[4], int *exc,
                    double cc[2]);

void hzo_real_2x2(double aii, double ajj, double aij, double x, double Z[4], int *exc)
{
    double cc[2];
    hzo_real_2x2_c(aii, ajj, aij, x, Z, exc, cc);
}

/*
 * As hzo_real_2x2, also returning the unscaled cosines cc = (cos phi,
 * cos psi) that criterion C2 of Section 2.5 tests (both NaN for the
 * exception, whose matrix is not of that form).
 */
void hzo_real_2x2_c(double aii, double ajj, double aij, double x, double Z[4], int *exc,
                    double cc[2])
{
    const double t = sqrt(fma(-x, x, 1.0));
    const double num = t * (ajj - aii);
    const double den = 2.0 * aij - (aii + ajj) * x;
    *exc = 0;
    if (ajj - aii == 0.0 && den == 0.0) {
        /* Exception: cot(2 theta) = 0/0. */
        const double ax = fabs(x);
        const double s = (x < 0.0) ? -1.0 : 1.0;
        const double r2 = 1.0 / sqrt(2.0);
        const double p = 1.0 / sqrt(1.0 + ax), q = 1.0 / sqrt(1.0 - ax);
        Z[0] = r2 * p;
        Z[1] = r2 * s * p;
        Z[2] = -r2 * s * q;
        Z[3] = r2 * q;
        *exc = 1;
        cc[0] = cc[1] = NAN;
        return;
    }
    const double xi = x / (sqrt(1.0 + x) + sqrt(1.0 - x));
    const double eta = x / ((1.0 + sqrt(1.0 + x)) * (1.0 + sqrt(1.0 - x)));
    const double cot2 = num / den;
    const double tn = sign1(cot2) / (fabs(cot2) + sqrt(1.0 + cot2 * cot2));
    double c, s;
    cos_sin_from_tan(tn, &c, &s);
    const double cphi = c + xi * (s - eta * c);
    const double cpsi = c - xi * (s + eta * c);
    const double sphi = s - xi * (c + eta * s);
    const double spsi = s + xi * (c - eta * s);
    Z[0] = cphi / t;
    Z[1] = -spsi / t;
    Z[2] = sphi / t;
    Z[3] = cpsi / t;
    cc[0] = cphi;
    cc[1] = cpsi;
}

/* ---------------------------------------------------- 2x2, complex case */

/*
 * Section 2.1.1: Zhat' = (1/t) [[cos phi, e^{i alpha} sin phi],
 * [-e^{-i beta} sin psi, cos psi]] for A' = [[aii, aij], [conj(aij), ajj]],
 * B' = [[1, b], [conj(b), 1]].  Column-major Z as in the real case.
 */
void hzo_cplx_2x2_c(double aii, double ajj, zdouble aij, zdouble b, zdouble Z[4], int *exc,
                    double cc[2]);

void hzo_cplx_2x2(double aii, double ajj, zdouble aij, zdouble b, zdouble Z[4], int *exc)
{
    double cc[2];
    hzo_cplx_2x2_c(aii, ajj, aij, b, Z, exc, cc);
}

/* As hzo_cplx_2x2, also returning cc = (cos phi, cos psi) (NaN for the
 * exception). */
void hzo_cplx_2x2_c(double aii, double ajj, zdouble aij, zdouble b, zdouble Z[4], int *exc,
                    double cc[2])
{
    const double x = hypot(creal(b), cimag(b));
    const double zeta = (b == 0.0) ? 0.0 : carg(b);
    const zdouble ez = cexp(I * zeta);      /* e^{i zeta} */
    const zdouble emz = cexp(-I * zeta);    /* e^{-i zeta} */
    const zdouble z = emz * aij;
    const double t = sqrt(fma(-x, x, 1.0));
    const double u = creal(z), v = cimag(z);
    const double h = ajj - aii;
    *exc = 0;
    if (v == 0.0 && h == 0.0) {
        const double r2 = 1.0 / sqrt(2.0);
        const double p = 1.0 / sqrt(1.0 + x), q = 1.0 / sqrt(1.0 - x);
        Z[0] = r2 * p;
        Z[1] = r2 * emz * p;
        Z[2] = -r2 * ez * q;
        Z[3] = r2 * q;
        *exc = 1;
        cc[0] = cc[1] = NAN;
        return;
    }
    const double tau = sign1(h);
    const double tan2 = tau * (2.0 * u - (aii + ajj) * x) / (t * sqrt(h * h + 4.0 * v * v));
    const double tang = 2.0 * v / h;
    double c2, s2, cg, sg;
    cos_sin_from_tan(tan2, &c2, &s2);
    cos_sin_from_tan(tang, &cg, &sg);
    const double r2 = 1.0 / sqrt(2.0);
    const double cphi = r2 * sqrt(1.0 + x * s2 + t * cg * c2);
    const double cpsi = r2 * sqrt(1.0 - x * s2 + t * cg * c2);
    const zdouble ea_sphi = ez * ((s2 - x) + I * (t * sg * c2)) / (2.0 * cpsi);
    const zdouble eb_spsi = emz * ((s2 + x) - I * (t * sg * c2)) / (2.0 * cphi);
    Z[0] = cphi / t;
    Z[1] = -eb_spsi / t;
    Z[2] = ea_sphi / t;
    Z[3] = cpsi / t;
    cc[0] = cphi;
    cc[1] = cpsi;
}

/* Interleaved-argument wrapper of hzo_cplx_2x2_c for foreign callers. */
void hzo_cplx_2x2_v(double aii, double ajj, const double *aij, const double *b,
                    double *Zout, int *exc, double cc[2])
{
    zdouble Z[4];
    hzo_cplx_2x2_c(aii, ajj, aij[0] + I * aij[1], b[0] + I * b[1], Z, exc, cc);
    for (int k = 0; k < 4; ++k) {
        Zout[2 * k] = creal(Z[k]);
        Zout[2 * k + 1] = cimag(Z[k]);
    }
}

/* ------------------------------------------------------------ orderings */

/*
 * Parallel strategies of Section 2.2 on N (even) indices, as tables of
 * steps x (N/2) pairs (p < q):
 *  kind 1, modified modulus (quasi-cyclic, N steps): step k pairs every
 *          p < q with p + q = k (mod N); for even k the two fixed points
 *          k/2 and k/2 + N/2 are paired with each other.
 *  kind 2, round robin (cyclic, N - 1 steps): index N - 1 is fixed and the
 *          others rotate; step k pairs (k, N-1) and ((k-i) mod (N-1),
 *          (k+i) mod (N-1)) for i = 1 .. N/2 - 1.
 * Kind 0 is the sequential row-cyclic order (1,2),(1,3),...,(n-1,n), one
 * pair per step.  Returns the number of steps; table holds steps*ppairs*2
 * ints, where ppairs = 1 for kind 0 and N/2 otherwise.
 */
int hzo_ordering(int kind, int n, int *table)
{
    if (kind == 0) {
        int s = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                table[2 * s] = i;
                table[2 * s + 1] = j;
                ++s;
            }
        return s;
    }
    const int N = n + (n & 1);
    const int half = N / 2;
    if (kind == 1) {
        for (int k = 0; k < N; ++k) {
            int c = 0;
            for (int p = 0; p < N; ++p) {
                const int q = ((k - p) % N + N) % N;
                if (p < q) {
                    table[2 * (k * half + c)] = p;
                    table[2 * (k * half + c) + 1] = q;
                    ++c;
                }
            }
            if ((k & 1) == 0) {
                table[2 * (k * half + c)] = k / 2;
                table[2 * (k * half + c) + 1] = k / 2 + half;
                ++c;
            }
        }
        return N;
    }
    if (kind == 2) {
        const int M = N - 1;
        for (int k = 0; k < M; ++k) {
            table[2 * (k * half)] = k;
            table[2 * (k * half) + 1] = M;
            for (int i = 1; i < half; ++i) {
                int p = ((k - i) % M + M) % M, q = (k + i) % M;
                if (p > q) { const int tmp = p; p = q; q = tmp; }
                table[2 * (k * half + i)] = p;
                table[2 * (k * half + i) + 1] = q;
            }
        }
        return M;
    }
    return -1;
}

static int ordering_steps(int kind, int n, int *ppairs)
{
    const int N = n + (n & 1);
    if (kind == 0) { *ppairs = 1; return n * (n - 1) / 2; }
    *ppairs = N / 2;
    return kind == 1 ? N : N - 1;
}

/* ---------------------------------------------------- shared finishing */

typedef struct { double key; int64_t idx; } sortrec;

static int cmp_desc(const void *a, const void *b)
{
    const sortrec *x = a, *y = b;
    if (x->key > y->key) return -1;
    if (x->key < y->key) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);   /* stable */
}

/* Stable descending sort of sigma, permuting the columns of the es-byte
 * element matrices U, V, Z and the entries of sigma, sigma_f, sigma_g. */
static void sort_desc(int64_t m_f, int64_t m_g, int64_t n, size_t es,
                      char *F, int64_t ldf, char *G, int64_t ldg, char *Z, int64_t ldz,
                      double *sigma, double *sigma_f, double *sigma_g)
{
    sortrec *rec = malloc(sizeof(sortrec) * n);
    for (int64_t j = 0; j < n; ++j) { rec[j].key = sigma[j]; rec[j].idx = j; }
    qsort(rec, n, sizeof(sortrec), cmp_desc);
    const int64_t rows[3] = {m_f, m_g, n}, lds[3] = {ldf, ldg, ldz};
    char *mats[3] = {F, G, Z};
    for (int w = 0; w < 3; ++w) {
        char *tmp = malloc(es * rows[w] * n);
        for (int64_t j = 0; j < n; ++j)
            memcpy(tmp + es * rows[w] * j, mats[w] + es * lds[w] * rec[j].idx, es * rows[w]);
        for (int64_t j = 0; j < n; ++j)
            memcpy(mats[w] + es * lds[w] * j, tmp + es * rows[w] * j, es * rows[w]);
        free(tmp);
    }
    double *vec[3] = {sigma, sigma_f, sigma_g};
    double *tmpv = malloc(sizeof(double) * n);
    for (int w = 0; w < 3; ++w) {
        for (int64_t j = 0; j < n; ++j) tmpv[j] = vec[w][rec[j].idx];
        memcpy(vec[w], tmpv, sizeof(double) * n);
    }
    free(tmpv);
    free(rec);
}

/* ------------------------------------------------------------ real GSVD */

static void swap_cols_r(double *Y, int64_t ld, int64_t m, int64_t i, int64_t j)
{
    for (int64_t r = 0; r < m; ++r) {
        const double t = Y[i * ld + r];
        Y[i * ld + r] = Y[j * ld + r];
        Y[j * ld + r] = t;
    }
}

static void rot_cols_r(double *Y, int64_t ld, int64_t m, int64_t i, int64_t j, const double Zh[4])
{
    double *yi = Y + i * ld, *yj = Y + j * ld;
    for (int64_t r = 0; r < m; ++r) {
        const double a = yi[r], b = yj[r];
        yi[r] = a * Zh[0] + b * Zh[1];
        yj[r] = a * Zh[2] + b * Zh[3];
    }
}

/*
 * Section 2.5: a transformation is small under criterion C1 (variant 0)
 * when both scaled cosines (cos phi)/t and (cos psi)/t, the diagonal of
 * Zhat', equal 1, and under criterion C2 (variant 4) when the unscaled
 * cosines cos phi and cos psi equal 1; every other transformation is big.
 */
static int is_big(int variant, double z11, double z22, const double cc[2])
{
    if (variant == 4 || variant == 5) return !(cc[0] == 1.0 && cc[1] == 1.0);
    return !(z11 == 1.0 && z22 == 1.0);
}

/*
 * Section 3.5.3, real case: the sort decision of a transformed pivot pair
 * compares the diagonal of Zhat'^T A' Zhat', i.e. the squared norms the two
 * columns of F will have after the transformation, computed from the pivot
 * entries without touching the columns:
 *   a''_11 = Z11^2 a_ii + 2 Z11 Z21 a_ij + Z21^2 a_jj,
 *   a''_22 = Z12^2 a_ii + 2 Z12 Z22 a_ij + Z22^2 a_jj
 * (Zh column-major: Z11, Z21, Z12, Z22).  Exported for the tests.
 */
void hzo_real_sort_keys(double aii, double ajj, double aij, const double Zh[4], double *a11,
                        double *a22)
{
    *a11 = Zh[0] * Zh[0] * aii + 2.0 * Zh[0] * Zh[1] * aij + Zh[1] * Zh[1] * ajj;
    *a22 = Zh[2] * Zh[2] * aii + 2.0 * Zh[2] * Zh[3] * aij + Zh[3] * Zh[3] * ajj;
}

/*
 * One pointwise step on the pivot pair (i, j), i < j (Section 2.1, variant
 * 0, 1, 4 or 5).  Adds to *all and *big and returns nothing else.
 */
static void step_real(int64_t m_f, int64_t m_g, int64_t n, double *F, int64_t ldf,
                      double *G, int64_t ldg, double *Z, int64_t ldz,
                      int64_t i, int64_t j, double tol, int sort, int variant,
                      int64_t *all, int64_t *big)
{
    const double *fi = F + i * ldf, *fj = F + j * ldf;
    double (*dot)(const double *, const double *, int64_t) =
        (variant == 1 || variant == 5) ? dot_rr_enh : dot_rr;
    const double aii = dot(fi, fi, m_f);
    const double ajj = dot(fj, fj, m_f);
    const double aij = dot(fi, fj, m_f);
    const double bij = dot(G + i * ldg, G + j * ldg, m_g);
    if (fabs(aij) < sqrt(aii) * sqrt(ajj) * tol && fabs(bij) < tol) {
        if (sort && aii < ajj) {
            swap_cols_r(F, ldf, m_f, i, j);
            swap_cols_r(G, ldg, m_g, i, j);
            swap_cols_r(Z, ldz, n, i, j);
        }
        return;
    }
    double Zh[4], cc[2];
    int exc;
    hzo_real_2x2_c(aii, ajj, aij, bij, Zh, &exc, cc);
    *all += 1;
    if (is_big(variant, Zh[0], Zh[3], cc))
        *big += 1;
    if (sort) {
        double a11, a22;
        hzo_real_sort_keys(aii, ajj, aij, Zh, &a11, &a22);
        if (a11 < a22) {
            double t;
            t = Zh[0]; Zh[0] = Zh[2]; Zh[2] = t;
            t = Zh[1]; Zh[1] = Zh[3]; Zh[3] = t;
        }
    }
    rot_cols_r(F, ldf, m_f, i, j, Zh);
    rot_cols_r(G, ldg, m_g, i, j, Zh);
    rot_cols_r(Z, ldz, n, i, j, Zh);
}

/*
 * Real GSVD.  ordering: 0 row-cyclic, 1 modified modulus, 2 round robin
 * (kinds 1 and 2 run the disjoint pairs of each step on OpenMP threads; the
 * result does not depend on the thread count).  tol <= 0 selects
 * sqrt(n)*DBL_EPSILON.  info[0..3] = sweeps, all transformations, big
 * transformations, converged flag.  Returns 0, or 1 if not converged within
 * max_sweeps, or -1 on a bad argument.
 */
int hzo_dgsvd(int64_t m_f, int64_t m_g, int64_t n,
              double *F, int64_t ldf, double *G, int64_t ldg, double *Z, int64_t ldz,
              double *sigma, double *sigma_f, double *sigma_g,
              int ordering, double tol, int max_sweeps, int sort, int variant, int threads,
              int64_t *info)
{
    if (n < 1 || m_f < n || m_g < n || ldf < m_f || ldg < m_g || ldz < n ||
        (variant != 0 && variant != 1 && variant != 4 && variant != 5))
        return -1;
    info[0] = info[1] = info[2] = 0;
    info[3] = 1;
    if (n == 1) {
        /* Section 2: closed form for n = 1. */
        const double nf = sqrt(dot_rr(F, F, m_f)), ng = sqrt(dot_rr(G, G, m_g));
        const double r = sqrt(nf * nf + ng * ng);
        for (int64_t k = 0; k < m_f; ++k) F[k] /= nf;
        for (int64_t k = 0; k < m_g; ++k) G[k] /= ng;
        Z[0] = 1.0 / r;
        sigma_f[0] = nf / r;
        sigma_g[0] = ng / r;
        sigma[0] = nf / ng;
        return 0;
    }
    if (tol <= 0.0) tol = sqrt((double)n) * DBL_EPSILON;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
    /* Section 2: prescaling, Z_0 = diag(1/||g_j||). */
    for (int64_t j = 0; j < n; ++j) {
        const double d = 1.0 / sqrt(dot_rr(G + j * ldg, G + j * ldg, m_g));
        for (int64_t r = 0; r < m_f; ++r) F[j * ldf + r] *= d;
        for (int64_t r = 0; r < m_g; ++r) G[j * ldg + r] *= d;
        for (int64_t r = 0; r < n; ++r) Z[j * ldz + r] = (r == j) ? d : 0.0;
    }
    int ppairs;
    const int steps = ordering_steps(ordering, (int)n, &ppairs);
    int *table = malloc(sizeof(int) * 2 * (size_t)steps * ppairs);
    if (hzo_ordering(ordering, (int)n, table) < 0) { free(table); return -1; }
    int converged = 0, sw = 0;
    while (sw < max_sweeps) {
        int64_t all = 0, big = 0;
        for (int s = 0; s < steps; ++s) {
            const int *row = table + 2 * (size_t)s * ppairs;
            #pragma omp parallel for schedule(dynamic, 1) reduction(+:all, big) if (ppairs > 1)
            for (int l = 0; l < ppairs; ++l) {
                const int64_t i = row[2 * l], j = row[2 * l + 1];
                if (j >= n) continue;   /* padding index of odd n */
                step_real(m_f, m_g, n, F, ldf, G, ldg, Z, ldz, i, j, tol, sort, variant, &all, &big);
            }
        }
        ++sw;
        info[1] += all;
        info[2] += big;
        if (big == 0) { converged = 1; break; }
    }
    free(table);
    info[0] = sw;
    info[3] = converged;
    /* Section 2.4: extraction. */
    for (int64_t j = 0; j < n; ++j) {
        double *fj = F + j * ldf, *gj = G + j * ldg, *zj = Z + j * ldz;
        const double sf = sqrt(dot_rr(fj, fj, m_f));
        const double sg = sqrt(dot_rr(gj, gj, m_g));
        const double th = 1.0 / sqrt(sf * sf + sg * sg);
        sigma_f[j] = sf * th;
        sigma_g[j] = sg * th;
        sigma[j] = sf / sg;
        for (int64_t r = 0; r < m_f; ++r) fj[r] /= sf;
        for (int64_t r = 0; r < m_g; ++r) gj[r] /= sg;
        for (int64_t r = 0; r < n; ++r) zj[r] *= th;
    }
    sort_desc(m_f, m_g, n, sizeof(double), (char *)F, ldf, (char *)G, ldg, (char *)Z, ldz,
              sigma, sigma_f, sigma_g);
    return converged ? 0 : 1;
}

/* --------------------------------------------------------- complex GSVD */

static void swap_cols_z(zdouble *Y, int64_t ld, int64_t m, int64_t i, int64_t j)
{
    for (int64_t r = 0; r < m; ++r) {
        const zdouble t = Y[i * ld + r];
        Y[i * ld + r] = Y[j * ld + r];
        Y[j * ld + r] = t;
    }
}

static void rot_cols_z(zdouble *Y, int64_t ld, int64_t m, int64_t i, int64_t j, const zdouble Zh[4])
{
    zdouble *yi = Y + i * ld, *yj = Y + j * ld;
    for (int64_t r = 0; r < m; ++r) {
        const zdouble a = yi[r], b = yj[r];
        yi[r] = a * Zh[0] + b * Zh[1];
        yj[r] = a * Zh[2] + b * Zh[3];
    }
}

static void step_cplx(int64_t m_f, int64_t m_g, int64_t n, zdouble *F, int64_t ldf,
                      zdouble *G, int64_t ldg, zdouble *Z, int64_t ldz,
                      int64_t i, int64_t j, double tol, int sort, int variant,
                      int64_t *all, int64_t *big)
{
    zdouble *fi = F + i * ldf, *fj = F + j * ldf;
    double (*nrm)(const zdouble *, int64_t) =
        (variant == 1 || variant == 5) ? nrm2sq_z_enh : nrm2sq_z;
    const double aii = nrm(fi, m_f);
    const double ajj = nrm(fj, m_f);
    const zdouble aij = dot_zz(fi, fj, m_f);
    const zdouble bij = dot_zz(G + i * ldg, G + j * ldg, m_g);
    const double abs_a = hypot(creal(aij), cimag(aij));
    const double abs_b = hypot(creal(bij), cimag(bij));
    if (abs_a < sqrt(aii) * sqrt(ajj) * tol && abs_b < tol) {
        if (sort && aii < ajj) {
            swap_cols_z(F, ldf, m_f, i, j);
            swap_cols_z(G, ldg, m_g, i, j);
            swap_cols_z(Z, ldz, n, i, j);
        }
        return;
    }
    zdouble Zh[4];
    double cc[2];
    int exc;
    hzo_cplx_2x2_c(aii, ajj, aij, bij, Zh, &exc, cc);
    *all += 1;
    if (is_big(variant, creal(Zh[0]), creal(Zh[3]), cc))   /* the diagonal of Zhat' is real */
        *big += 1;
    rot_cols_z(F, ldf, m_f, i, j, Zh);
    rot_cols_z(G, ldg, m_g, i, j, Zh);
    rot_cols_z(Z, ldz, n, i, j, Zh);
    /* Section 3.5.3: in the complex case the sort decision uses the
     * recomputed norms of the transformed columns of F. */
    if (sort && nrm2sq_z(fi, m_f) < nrm2sq_z(fj, m_f)) {
        swap_cols_z(F, ldf, m_f, i, j);
        swap_cols_z(G, ldg, m_g, i, j);
        swap_cols_z(Z, ldz, n, i, j);
    }
}

/*
 * Exported for the tests: one pointwise step (Section 2.1) on the pivot pair
 * (i, j), i < j, of the real or the interleaved complex pair (F, G, Z), exactly
 * as a sweep takes it (skip test, transformation, counters, sorting).
 * counts[0] and counts[1] receive the transformation and the big
 * transformation the step applied (0 or 1 each).
 */
void hzo_step_real(int64_t m_f, int64_t m_g, int64_t n, double *F, int64_t ldf, double *G,
                   int64_t ldg, double *Z, int64_t ldz, int64_t i, int64_t j, double tol,
                   int sort, int variant, int64_t counts[2])
{
    counts[0] = counts[1] = 0;
    step_real(m_f, m_g, n, F, ldf, G, ldg, Z, ldz, i, j, tol, sort, variant, &counts[0],
              &counts[1]);
}

void hzo_step_cplx(int64_t m_f, int64_t m_g, int64_t n, double *F, int64_t ldf, double *G,
                   int64_t ldg, double *Z, int64_t ldz, int64_t i, int64_t j, double tol,
                   int sort, int variant, int64_t counts[2])
{
    counts[0] = counts[1] = 0;
    step_cplx(m_f, m_g, n, (zdouble *)F, ldf, (zdouble *)G, ldg, (zdouble *)Z, ldz, i, j, tol,
              sort, variant, &counts[0], &counts[1]);
}

/* Complex GSVD; arguments as hzo_dgsvd, with interleaved complex F, G, Z. */
int hzo_zgsvd(int64_t m_f, int64_t m_g, int64_t n,
              double *Fd, int64_t ldf, double *Gd, int64_t ldg, double *Zd, int64_t ldz,
              double *sigma, double *sigma_f, double *sigma_g,
              int ordering, double tol, int max_sweeps, int sort, int variant, int threads,
              int64_t *info)
{
    zdouble *F = (zdouble *)Fd, *G = (zdouble *)Gd, *Z = (zdouble *)Zd;
    if (n < 1 || m_f < n || m_g < n || ldf < m_f || ldg < m_g || ldz < n ||
        (variant != 0 && variant != 1 && variant != 4 && variant != 5))
        return -1;
    info[0] = info[1] = info[2] = 0;
    info[3] = 1;
    if (n == 1) {
        const double nf = sqrt(nrm2sq_z(F, m_f)), ng = sqrt(nrm2sq_z(G, m_g));
        const double r = sqrt(nf * nf + ng * ng);
        for (int64_t k = 0; k < m_f; ++k) F[k] /= nf;
        for (int64_t k = 0; k < m_g; ++k) G[k] /= ng;
        Z[0] = 1.0 / r;
        sigma_f[0] = nf / r;
        sigma_g[0] = ng / r;
        sigma[0] = nf / ng;
        return 0;
    }
    if (tol <= 0.0) tol = sqrt((double)n) * DBL_EPSILON;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
    for (int64_t j = 0; j < n; ++j) {
        const double d = 1.0 / sqrt(nrm2sq_z(G + j * ldg, m_g));
        for (int64_t r = 0; r < m_f; ++r) F[j * ldf + r] *= d;
        for (int64_t r = 0; r < m_g; ++r) G[j * ldg + r] *= d;
        for (int64_t r = 0; r < n; ++r) Z[j * ldz + r] = (r == j) ? d : 0.0;
    }
    int ppairs;
    const int steps = ordering_steps(ordering, (int)n, &ppairs);
    int *table = malloc(sizeof(int) * 2 * (size_t)steps * ppairs);
    if (hzo_ordering(ordering, (int)n, table) < 0) { free(table); return -1; }
    int converged = 0, sw = 0;
    while (sw < max_sweeps) {
        int64_t all = 0, big = 0;
        for (int s = 0; s < steps; ++s) {
            const int *row = table + 2 * (size_t)s * ppairs;
            #pragma omp parallel for schedule(dynamic, 1) reduction(+:all, big) if (ppairs > 1)
            for (int l = 0; l < ppairs; ++l) {
                const int64_t i = row[2 * l], j = row[2 * l + 1];
                if (j >= n) continue;
                step_cplx(m_f, m_g, n, F, ldf, G, ldg, Z, ldz, i, j, tol, sort, variant, &all, &big);
            }
        }
        ++sw;
        info[1] += all;
        info[2] += big;
        if (big == 0) { converged = 1; break; }
    }
    free(table);
    info[0] = sw;
    info[3] = converged;
    for (int64_t j = 0; j < n; ++j) {
        zdouble *fj = F + j * ldf, *gj = G + j * ldg, *zj = Z + j * ldz;
        const double sf = sqrt(nrm2sq_z(fj, m_f));
        const double sg = sqrt(nrm2sq_z(gj, m_g));
        const double th = 1.0 / sqrt(sf * sf + sg * sg);
        sigma_f[j] = sf * th;
        sigma_g[j] = sg * th;
        sigma[j] = sf / sg;
        for (int64_t r = 0; r < m_f; ++r) fj[r] /= sf;
        for (int64_t r = 0; r < m_g; ++r) gj[r] /= sg;
        for (int64_t r = 0; r < n; ++r) zj[r] *= th;
    }
    sort_desc(m_f, m_g, n, sizeof(zdouble), (char *)F, ldf, (char *)G, ldg, (char *)Z, ldz,
              sigma, sigma_f, sigma_g);
    return converged ? 0 : 1;
}
