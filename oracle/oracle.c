/*
 * oracle.c -- CPU reference for the polynomial conversion matvec  beta = A alpha.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle: a plain, slow, obviously
 * correct O(N^2) evaluation of beta_j = sum_k A_jk alpha_k from the closed-form
 * entries of each conversion matrix printed in the paper (Townsend, Webb, Olver,
 * "Fast polynomial transforms based on Toeplitz and Hankel matrices",
 * arXiv:1604.07486).  It shares no code, table or constant with the GPU library.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may build,
 * load or call it; the product path never does.
 *
 * Precision: special-function tables are built in binary128 (__float128,
 * libquadmath), the matrix entries are formed in x87 extended precision and each
 * row is summed with Neumaier's compensated summation in extended precision.
 * The result is rounded to double once.
 *
 * Kinds (the "plain definition" the fast method approximates):
 *   0 leg2cheb   Sec. 1, eq. (M)           (Alpert-Rokhlin closed form)
 *   1 cheb2leg   Sec. 5.1, eq. (FormulaL)
 *   2 ultra2ultra Sec. 5.2, eq. (UltraSconversion), params (lambda1, lambda2)
 *   3 jac2jac    Sec. 5.3, case-2 closed form (beta = delta), params (a, b, g)
 *   4 lag2lag    Sec. 5.4, NIST 18.18.18 closed form, params (a1, a2)
 * plus the unit steps of the Jacobi case 1 (orc_jacobi_step), O(N).
 *
 * Readings of the paper taken here (each pinned by tests/test_oracle_pins.py):
 *   - eq. (M), first case: the condition "j even" at j = 0 is read as "k even"
 *     (the entry is zero when k - j is odd, as in the second case).
 *   - eq. (UltraSconversion) is used as printed; the Gamma ratio with argument
 *     (k-j)/2 + lambda1 - lambda2 over Gamma(lambda1 - lambda2) Gamma((k-j)/2+1)
 *     is evaluated as the Pochhammer quotient (lambda1-lambda2)_m / m!, which is
 *     the same number and stays finite when lambda1 - lambda2 is an integer.
 *   - Jacobi, row j = 0 when gamma + beta + 1 = 0: the product
 *     (2j+gamma+beta+1) Gamma(j+gamma+beta+1) is taken at its limit
 *     Gamma(gamma+beta+2).
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __float128 f128;
typedef long double ldbl;

enum { ORC_LEG2CHEB = 0, ORC_CHEB2LEG = 1, ORC_ULTRA2ULTRA = 2, ORC_JAC2JAC = 3, ORC_LAG2LAG = 4 };

/* ------------------------------------------------------------------------- */
/* Special-function tables (binary128)                                        */
/* ------------------------------------------------------------------------- */

/* Lambda(n) = Gamma(n+1/2)/Gamma(n+1) for integers n = 0..M (the function the
 * paper calls Lambda, defined under eq. (M)).  For integer n,
 * Gamma(n+1/2)/Gamma(n+1) = sqrt(pi) * prod_{i=1..n} (2i-1)/(2i), i.e. sqrt(pi)
 * times the central binomial coefficient C(2n,n) over 4^n. */
static void lambda_int_table(int64_t M, f128 *out)
{
    const f128 sqrtpi = sqrtq(M_PIq);
    f128 c = 1;
    out[0] = sqrtpi;
    for (int64_t i = 1; i <= M; ++i) {
        c = c * (f128)(2 * i - 1) / (f128)(2 * i);
        out[i] = sqrtpi * c;
    }
}

/* (x)_m / m!  for m = 0..M (rising factorial over factorial).  For x not a
 * non-positive integer this is Gamma(m+x)/(Gamma(x) Gamma(m+1)). */
static void poch_over_fact_table(f128 x, int64_t M, f128 *out)
{
    f128 p = 1;
    out[0] = 1;
    for (int64_t m = 0; m < M; ++m) {
        p = p * (x + (f128)m) / (f128)(m + 1);
        out[m + 1] = p;
    }
}

/* log|(x)_n| for n >= 0 and its sign; (x)_n = x (x+1) ... (x+n-1).
 * Returns 0 in *is_zero when a factor vanishes. */
static f128 log_poch(f128 x, int64_t n, int *sign, int *is_zero)
{
    *sign = 1;
    *is_zero = 0;
    f128 acc = 0;
    int64_t i = 0;
    /* explicit product over the factors that are <= 0 */
    while (i < n && x + (f128)i <= 0) {
        f128 f = x + (f128)i;
        if (f == 0) { *is_zero = 1; return 0; }
        *sign = -*sign;
        acc += logq(-f);
        ++i;
    }
    if (i < n) {
        f128 y = x + (f128)i; /* > 0 */
        acc += lgammaq(y + (f128)(n - i)) - lgammaq(y);
    }
    return acc;
}

/* ------------------------------------------------------------------------- */
/* Row evaluation                                                              */
/* ------------------------------------------------------------------------- */

typedef struct {
    int kind;
    int64_t N;
    /* extended-precision tables used by the inner loops */
    ldbl *lam;      /* Lambda(n), n = 0..N+1 (leg2cheb, cheb2leg)                 */
    ldbl *lamh;     /* Lambda(n + 1/2) = Gamma(n+1)/Gamma(n+3/2), n = 0..N+1        */
    ldbl *pt;       /* Toeplitz-type Pochhammer quotient table, index k - j or m   */
    ldbl *ph;       /* ultra: (l1)_s/(l2)_{s+1}, s = 0..N                           */
    /* Jacobi tables (log-space, binary128): see jacobi_entry                      */
    f128 *jb_logB;  /* log (beta+1)_k,  k = 0..N                                    */
    f128 *jb_logC;  /* log (c+1)_s, c = gamma+beta+1, s = 0..2N                     */
    f128 *jb_logE;  /* log|(e)_s|, e = alpha+beta+1, s = 0..2N                      */
    int8_t *jb_sgnE;
    int8_t *jb_zeroE;
    ldbl *jb_D;     /* row prefactor, j = 0..N                                      */
    double p[4];
    int absmode;    /* row sums of |A_jk| |alpha_k| instead of A_jk alpha_k (bar scales) */
} orc_ctx;

static inline void neumaier_add(ldbl *s, ldbl *c, ldbl t)
{
    ldbl u = *s + t;
    if (fabsl(*s) >= fabsl(t)) *c += (*s - u) + t;
    else *c += (t - u) + *s;
    *s = u;
}

/* Entry A_jk, 0 <= j <= k <= N. */
static ldbl entry(const orc_ctx *C, int64_t j, int64_t k)
{
    switch (C->kind) {
    case ORC_LEG2CHEB: {
        /* eq. (M): M_0k = Lambda(k/2)^2 / pi (k even); M_jk = (2/pi) Lambda((k-j)/2)
         * Lambda((k+j)/2) for 0 < j <= k, k - j even; zero otherwise. */
        if ((k - j) & 1) return 0;
        const ldbl invpi = 1.0L / 3.14159265358979323846264338327950288L;
        if (j == 0) return invpi * C->lam[k / 2] * C->lam[k / 2];
        return 2.0L * invpi * C->lam[(k - j) / 2] * C->lam[(k + j) / 2];
    }
    case ORC_CHEB2LEG: {
        /* eq. (FormulaL): L_00 = 1; L_jj = sqrt(pi)/(2 Lambda(j)); for j < k, k - j
         * even: -k (j+1/2) (Lambda((k-j-2)/2)/(k-j)) (Lambda((j+k-1)/2)/(j+k+1)). */
        if ((k - j) & 1) return 0;
        if (j == k) {
            if (j == 0) return 1.0L;
            const ldbl sqrtpi = 1.77245385090551602729816748334114518L;
            return sqrtpi / (2.0L * C->lam[j]);
        }
        int64_t m = (k - j - 2) / 2;      /* (k-j-2)/2 >= 0 */
        int64_t s = (j + k) / 2;          /* (j+k-1)/2 = s - 1/2, s >= 1 */
        ldbl lam_half = C->lamh[s - 1];   /* Lambda(s - 1/2) */
        return -(ldbl)k * ((ldbl)j + 0.5L) * (C->lam[m] / (ldbl)(k - j)) *
               (lam_half / (ldbl)(j + k + 1));
    }
    case ORC_ULTRA2ULTRA: {
        /* eq. (UltraSconversion), k - j even:
         * (j + l2) * (l1-l2)_m/m! * Gamma(s+l1) Gamma(l2) / (Gamma(l1) Gamma(s+l2+1)),
         * m = (k-j)/2, s = (k+j)/2; the last factor is (l1)_s / (l2)_{s+1}. */
        if ((k - j) & 1) return 0;
        ldbl l2 = (ldbl)C->p[1];
        return ((ldbl)j + l2) * C->pt[(k - j) / 2] * C->ph[(k + j) / 2];
    }
    case ORC_LAG2LAG:
        /* NIST 18.18.18: A_jk = (a1-a2)_{k-j}/(k-j)!, j <= k. */
        return C->pt[k - j];
    }
    return 0;
}

static double row(const orc_ctx *C, int64_t j, const double *alpha)
{
    ldbl s = 0, c = 0;
    int64_t step = (C->kind == ORC_JAC2JAC || C->kind == ORC_LAG2LAG) ? 1 : 2;
    for (int64_t k = j; k <= C->N; k += step) {
        if (alpha[k] == 0.0) continue;
        if (C->absmode) neumaier_add(&s, &c, fabsl(entry(C, j, k)) * fabsl((ldbl)alpha[k]));
        else neumaier_add(&s, &c, entry(C, j, k) * (ldbl)alpha[k]);
    }
    return (double)(s + c);
}

static void ctx_free(orc_ctx *C)
{
    free(C->lam); free(C->lamh); free(C->pt); free(C->ph);
    free(C->jb_logB); free(C->jb_logC); free(C->jb_logE); free(C->jb_sgnE);
    free(C->jb_zeroE); free(C->jb_D);
    memset(C, 0, sizeof(*C));
}

static int ctx_init(orc_ctx *C, int kind, const double *params, int64_t N)
{
    memset(C, 0, sizeof(*C));
    C->kind = kind;
    C->N = N;
    for (int i = 0; i < 4 && params; ++i) C->p[i] = params[i];
    if (kind == ORC_LEG2CHEB || kind == ORC_CHEB2LEG) {
        int64_t M = N + 2;
        f128 *t = (f128 *)malloc(sizeof(f128) * (size_t)(M + 1));
        C->lam = (ldbl *)malloc(sizeof(ldbl) * (size_t)(M + 1));
        C->lamh = (ldbl *)malloc(sizeof(ldbl) * (size_t)(M + 1));
        if (!t || !C->lam || !C->lamh) { free(t); ctx_free(C); return -2; }
        lambda_int_table(M, t);
        for (int64_t n = 0; n <= M; ++n) {
            C->lam[n] = (ldbl)t[n];
            /* Lambda(n + 1/2) = Gamma(n+1)/Gamma(n+3/2) = 1/((n + 1/2) Lambda(n)) */
            C->lamh[n] = (ldbl)(1 / (((f128)n + (f128)0.5) * t[n]));
        }
        free(t);
        return 0;
    }
    if (kind == ORC_ULTRA2ULTRA) {
        f128 l1 = params[0], l2 = params[1];
        if (!(params[0] > 0) || !(params[1] > 0)) return -1;
        f128 *a = (f128 *)malloc(sizeof(f128) * (size_t)(N + 1));
        C->pt = (ldbl *)malloc(sizeof(ldbl) * (size_t)(N + 1));
        C->ph = (ldbl *)malloc(sizeof(ldbl) * (size_t)(N + 1));
        if (!a || !C->pt || !C->ph) { free(a); ctx_free(C); return -2; }
        poch_over_fact_table(l1 - l2, N, a);
        for (int64_t m = 0; m <= N; ++m) C->pt[m] = (ldbl)a[m];
        /* (l1)_s / (l2)_{s+1}: s = 0 gives 1/l2; next = prev (s+l1)/(s+1+l2) */
        f128 h = 1 / l2;
        for (int64_t s = 0; s <= N; ++s) {
            C->ph[s] = (ldbl)h;
            h = h * ((f128)s + l1) / ((f128)s + 1 + l2);
        }
        free(a);
        return 0;
    }
    if (kind == ORC_LAG2LAG) {
        if (!(params[0] > -1) || !(params[1] > -1)) return -1;
        f128 *a = (f128 *)malloc(sizeof(f128) * (size_t)(N + 1));
        C->pt = (ldbl *)malloc(sizeof(ldbl) * (size_t)(N + 1));
        if (!a || !C->pt) { free(a); ctx_free(C); return -2; }
        poch_over_fact_table((f128)params[0] - (f128)params[1], N, a);
        for (int64_t m = 0; m <= N; ++m) C->pt[m] = (ldbl)a[m];
        free(a);
        return 0;
    }
    if (kind == ORC_JAC2JAC) {
        f128 a = params[0], b = params[1], g = params[2];
        if (!(params[0] > -1) || !(params[1] > -1) || !(params[2] > -1)) return -1;
        f128 c = g + b + 1, e = a + b + 1;
        int64_t S = 2 * N;
        f128 *pq = (f128 *)malloc(sizeof(f128) * (size_t)(N + 1));
        C->pt = (ldbl *)malloc(sizeof(ldbl) * (size_t)(N + 1));
        C->jb_logB = (f128 *)malloc(sizeof(f128) * (size_t)(N + 1));
        C->jb_logC = (f128 *)malloc(sizeof(f128) * (size_t)(S + 1));
        C->jb_logE = (f128 *)malloc(sizeof(f128) * (size_t)(S + 1));
        C->jb_sgnE = (int8_t *)malloc((size_t)(S + 1));
        C->jb_zeroE = (int8_t *)malloc((size_t)(S + 1));
        C->jb_D = (ldbl *)malloc(sizeof(ldbl) * (size_t)(N + 1));
        if (!pq || !C->pt || !C->jb_logB || !C->jb_logC || !C->jb_logE || !C->jb_sgnE ||
            !C->jb_zeroE || !C->jb_D) { free(pq); ctx_free(C); return -2; }
        poch_over_fact_table(a - g, N, pq);
        for (int64_t m = 0; m <= N; ++m) C->pt[m] = (ldbl)pq[m];
        free(pq);
        /* log (b+1)_k and log (c+1)_s: positive arguments, cumulative sums of logs */
        f128 acc = 0;
        for (int64_t k = 0; k <= N; ++k) {
            C->jb_logB[k] = acc;
            acc += logq(b + 1 + (f128)k);
        }
        acc = 0;
        for (int64_t s = 0; s <= S; ++s) {
            C->jb_logC[s] = acc;
            acc += logq(c + 1 + (f128)s);
        }
        /* log|(e)_s| with sign; once a factor vanishes every later one is zero */
        acc = 0;
        int sg = 1, zero = 0;
        for (int64_t s = 0; s <= S; ++s) {
            C->jb_logE[s] = acc;
            C->jb_sgnE[s] = (int8_t)sg;
            C->jb_zeroE[s] = (int8_t)zero;
            f128 f = e + (f128)s;
            if (f == 0) zero = 1;
            else { if (f < 0) sg = -sg; acc += logq(fabsq(f)); }
        }
        /* D_j = (2j + c)(c+1)_{j-1} for j > 0 and D_0 = 1 (the limit of
         * (2j+c) Gamma(j+c)/Gamma(c+1) at j = 0, valid also when c = 0).  Only its
         * sign is stored; row_jacobi() adds log|D_j| = log|2j+c| + log (c+1)_{j-1}. */
        C->jb_D[0] = 1.0L;
        for (int64_t j = 1; j <= N; ++j) C->jb_D[j] = (2 * (f128)j + c) >= 0 ? 1.0L : -1.0L;
        return 0;
    }
    return -1;
}

/* Jacobi entry, Sec. 5.3 case-2 closed form (beta = delta) written with
 * Pochhammer symbols so that every factor stays finite:
 *   A_jk = D_j (e+k)_j/(b+1)_j (b+1)_k/(c+1)_{k+j} (a-g)_{k-j}/(k-j)!,
 *   c = g+b+1, e = a+b+1, D_j = (2j+c)(c+1)_{j-1} (j > 0), D_0 = 1.
 * Magnitudes are combined in log space (binary128) before one exp.  lgD is
 * log|D_j| (jacobi_lgD).  Sets *zero when the entry vanishes. */
static f128 jacobi_lgD(const orc_ctx *C, int64_t j)
{
    f128 c = (f128)C->p[2] + (f128)C->p[1] + 1;
    return j > 0 ? logq(fabsq(2 * (f128)j + c)) + C->jb_logC[j - 1] : 0;
}

static ldbl jacobi_entry(const orc_ctx *C, int64_t j, int64_t k, f128 lgD, int *zero)
{
    int64_t sidx = k + j;
    f128 lg;
    int sg;
    *zero = 0;
    if (C->jb_zeroE[k]) {
        int z;
        lg = log_poch((f128)C->p[0] + (f128)C->p[1] + 1 + (f128)k, j, &sg, &z);
        if (z) { *zero = 1; return 0; }
    } else {
        if (C->jb_zeroE[sidx]) { *zero = 1; return 0; }
        lg = C->jb_logE[sidx] - C->jb_logE[k];
        sg = C->jb_sgnE[sidx] * C->jb_sgnE[k];
    }
    lg += C->jb_logB[k] - C->jb_logB[j] - C->jb_logC[sidx] + lgD;
    return (ldbl)sg * C->jb_D[j] * expl((ldbl)lg) * C->pt[k - j];
}

static double row_jacobi(const orc_ctx *C, int64_t j, const double *alpha)
{
    const f128 lgD = jacobi_lgD(C, j);
    ldbl s = 0, cc = 0;
    for (int64_t k = j; k <= C->N; ++k) {
        if (alpha[k] == 0.0) continue;
        int z;
        ldbl a = jacobi_entry(C, j, k, lgD, &z);
        if (z) continue;
        if (C->absmode) neumaier_add(&s, &cc, fabsl(a) * fabsl((ldbl)alpha[k]));
        else neumaier_add(&s, &cc, a * (ldbl)alpha[k]);
    }
    return (double)(s + cc);
}

/* ------------------------------------------------------------------------- */
/* Public entry points (loaded with ctypes by the tests)                      */
/* ------------------------------------------------------------------------- */

/* beta = A alpha for rows `rows[0..nrows)` (all rows 0..N when rows == NULL).
 * alpha: N+1 doubles.  beta: N+1 doubles when rows == NULL, else nrows doubles.
 * nthreads <= 0 uses the OpenMP default.  Returns 0 on success. */
static int matvec_mode(int kind, const double *params, int64_t N, const double *alpha, double *beta,
                       const int64_t *rows, int64_t nrows, int nthreads, int absmode)
{
    if (N < 0 || !alpha || !beta) return -1;
    orc_ctx C;
    int rc = ctx_init(&C, kind, params, N);
    if (rc) return rc;
    C.absmode = absmode;
    int64_t R = rows ? nrows : N + 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < R; ++i) {
        int64_t j = rows ? rows[i] : i;
        if (j < 0 || j > N) { bad = 1; continue; }
        beta[i] = (kind == ORC_JAC2JAC) ? row_jacobi(&C, j, alpha) : row(&C, j, alpha);
    }
    ctx_free(&C);
    return bad ? -1 : 0;
}

int orc_matvec(int kind, const double *params, int64_t N, const double *alpha, double *beta,
               const int64_t *rows, int64_t nrows, int nthreads)
{
    return matvec_mode(kind, params, N, alpha, beta, rows, nrows, nthreads, 0);
}

/* (|A| |alpha|)_j = sum_k |A_jk| |alpha_k| for the same rows: the scale of the
 * rounding error of any evaluation of row j (test bars only). */
int orc_matvec_abs(int kind, const double *params, int64_t N, const double *alpha, double *beta,
                   const int64_t *rows, int64_t nrows, int nthreads)
{
    return matvec_mode(kind, params, N, alpha, beta, rows, nrows, nthreads, 1);
}

/* Dense matrix A (row-major, (N+1)^2 doubles), entry by entry. */
int orc_dense(int kind, const double *params, int64_t N, double *A)
{
    if (N < 0 || !A) return -1;
    orc_ctx C;
    int rc = ctx_init(&C, kind, params, N);
    if (rc) return rc;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j <= N; ++j) {
        const f128 lgD = kind == ORC_JAC2JAC ? jacobi_lgD(&C, j) : 0;
        for (int64_t k = 0; k <= N; ++k) {
            double v = 0.0;
            if (k >= j) {
                if (kind == ORC_JAC2JAC) {
                    int z;
                    ldbl e = jacobi_entry(&C, j, k, lgD, &z);
                    v = z ? 0.0 : (double)e;
                } else {
                    v = (double)entry(&C, j, k);
                }
            }
            A[j * (N + 1) + k] = v;
        }
    }
    ctx_free(&C);
    return 0;
}

/* max_{j,k} |A_jk| over the (N+1)x(N+1) matrix (O(N^2); used to scale error bars
 * for conversions whose entries grow with N). */
double orc_absmax(int kind, const double *params, int64_t N)
{
    orc_ctx C;
    if (N < 0 || ctx_init(&C, kind, params, N)) return -1.0;
    double best = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(max : best)
    for (int64_t j = 0; j <= N; ++j) {
        const f128 lgD = kind == ORC_JAC2JAC ? jacobi_lgD(&C, j) : 0;
        for (int64_t k = j; k <= N; ++k) {
            double v;
            if (kind == ORC_JAC2JAC) {
                int z;
                v = fabs((double)jacobi_entry(&C, j, k, lgD, &z));
            } else {
                v = fabs((double)entry(&C, j, k));
            }
            if (v > best) best = v;
        }
    }
    ctx_free(&C);
    return best;
}

/* Jacobi case 1 of Sec. 5.3 (a whole-number change of the first parameter),
 * one unit step in O(N), binary128.  The step up is the upper-bidiagonal factor
 * S_(a,b) that maps coefficients in P^(a,b) to coefficients in P^(a+1,b); its
 * entries come from the textbook connection relation (a consequence of the
 * three-term recurrence, DLMF 18.9.5 with the reflection of Tab. 18.6.1)
 *   (2n+a+b+1) P_n^(a,b) = (n+a+b+1) P_n^(a+1,b) - (n+b) P_{n-1}^(a+1,b):
 *   S_nn = (n+a+b+1)/(2n+a+b+1),  S_{n,n+1} = -(n+b+1)/(2n+a+b+3)
 * (the factor printed in the paper carries a+1, a+2, ... in the second
 * diagonal; the relation above, checked against exact bases, has b+1, b+2, ...).
 * dir = +1: out = S_(a,b) alpha (the result is in P^(a+1,b));
 * dir = -1: out solves S_(a-1,b) out = alpha by backward substitution, as the
 * paper prescribes for a decrease (the result is in P^(a-1,b)).
 * S_00 = 1 also when a+b+1 = 0 (the n = 0 limit).  Returns 0 on success. */
int orc_jacobi_step(double a_, double b_, int64_t N, const double *alpha, double *out, int dir)
{
    if (N < 0 || !alpha || !out || (dir != 1 && dir != -1)) return -1;
    const f128 b = b_, a = dir == 1 ? (f128)a_ : (f128)a_ - 1;  /* the factor S_(a,b) */
    if (!(a > -1) || !(b > -1)) return -1;
    f128 *x = (f128 *)malloc(sizeof(f128) * (size_t)(N + 2));
    if (!x) return -2;
    x[N + 1] = 0;
    for (int64_t n = N; n >= 0; --n) {
        const f128 fn = (f128)n;
        const f128 dnn = n == 0 ? (f128)1 : (fn + a + b + 1) / (2 * fn + a + b + 1);
        const f128 up = -(fn + b + 1) / (2 * fn + a + b + 3);
        if (dir == 1) x[n] = dnn * (f128)alpha[n] + (n < N ? up * (f128)alpha[n + 1] : 0);
        else x[n] = ((f128)alpha[n] - up * x[n + 1]) / dnn;
    }
    for (int64_t n = 0; n <= N; ++n) out[n] = (double)x[n];
    free(x);
    return 0;
}

/* Lambda(n) = Gamma(n+1/2)/Gamma(n+1), n = 0..M, rounded to double. */
int orc_lambda(int64_t M, double *out)
{
    if (M < 0 || !out) return -1;
    f128 *t = (f128 *)malloc(sizeof(f128) * (size_t)(M + 1));
    if (!t) return -2;
    lambda_int_table(M, t);
    for (int64_t n = 0; n <= M; ++n) out[n] = (double)t[n];
    free(t);
    return 0;
}

/* Lambda(n) as a decimal string with 34 significant digits (for pins). */
int orc_lambda_str(int64_t n, char *buf, int len)
{
    if (n < 0 || !buf || len < 48) return -1;
    f128 *t = (f128 *)malloc(sizeof(f128) * (size_t)(n + 1));
    if (!t) return -2;
    lambda_int_table(n, t);
    quadmath_snprintf(buf, (size_t)len, "%.34Qe", t[n]);
    free(t);
    return 0;
}
