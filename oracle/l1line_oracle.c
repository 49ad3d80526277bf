/*
 * l1line_oracle.c -- exact CPU oracle for the sparse robust l1 best-fit line
 * (Ling & Brooks, "l1-Norm Regularized l1-Norm Best-Fit Lines").
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file.  It shares no code with the
 * GPU library and is written to be checked against the paper by eye: plain
 * loops, a library sort, no blocking or fusion.
 *
 * WHAT IT COMPUTES
 *   X is n x m, column-major (x(i,k) = X[i + k*ld]); rows i are points,
 *   columns are coordinates.  For a preserved coordinate j (the paper's
 *   j-hat) the LP (3) of Sec. 2 splits, by the proof of Lemma 1, into one
 *   problem per other column k:
 *       g_jk(v) = sum_{i: x_ij != 0} |x_ij| * |r_i - v|  +  lambda |v|
 *                 + sum_{i: x_ij == 0} |x_ik|,      r_i = x_ik / x_ij.
 *   g_jk is convex and piecewise linear; its minimisers are weighted medians
 *   of the points r_i (weights |x_ij|) together with the point 0 (weight
 *   lambda).  Algorithm 1 then sets v_j = 1, takes every v_k, scores
 *       z_j = sum_i sum_k |x_ik - v_k x_ij|  +  lambda sum_k |v_k|
 *   (the penalty includes |v_j| = 1) and keeps the j with the smallest z_j,
 *   the first one on ties (strict "<" over ascending j).
 *
 * READINGS WHERE THE PAPER LEAVES A CHOICE
 *   ratios   r_i = fl(x_ik / x_ij) + 0.0: IEEE double division, round to
 *            nearest, then -0 turned into +0.  Points are ordered by
 *            (r_i, i) ascending.
 *   exact    every sum of weights and every comparison of such sums with
 *            lambda is EXACT: a finite double is an integer multiple of
 *            2^-1074, so sums are held as big integers in those units.  The
 *            selection is therefore the real-number weighted median, free of
 *            any summation order.
 *   tie rule Lemma 1 accepts every point that meets its condition
 *            (solncond); several points (or 0) can be minimisers when
 *            g_jk has a flat piece.  Rule R3: v_k = 0 when 0 minimises g_jk,
 *            else the minimiser closest to 0.  With S_p the exact sum of the
 *            first p weights in sorted order, W = S_n', A = S_N (N points
 *            below 0), B = S_{N+Z} (Z points equal to 0):
 *              zero      if 2A <= W + lambda  and  W <= 2B + lambda
 *              negative  if 2A >  W + lambda: first p <= N with 2 S_p > W + lambda
 *              positive  otherwise:           first p >  N+Z with 2 S_p + lambda >= W
 *            tie_rule = 1 instead runs the test of Algorithm 1 verbatim
 *            (half-open interval, last match wins, default 0), reading the
 *            unbound index in its sgn(.) as the tested point.
 *   zero column  a column j with no nonzero entry gives v = e_j (v_j = 1,
 *            every other v_k = 0), as Algorithm 1 does.
 *   floating sums  the reported sums (column mass, residual e_jk, E_j, P_j)
 *            use the fixed order R64: term t goes to partial t mod 64 (each
 *            partial summed in increasing t from +0.0), then
 *            p[l] = p[l] + p[l+d] for d = 32,16,8,4,2,1 and l < d; result p[0].
 *            The residual term is |x_ik - fl(v_k * x_ij)| with three separate
 *            roundings (no fused multiply-add).
 *
 * STATUS CODES (returned by every entry point)
 *    0  ok
 *   -1  invalid argument (n < 1, m < 1, ld < n, L < 1, lambda < 0 or NaN,
 *       null pointer, j or k out of range)
 *   -3  X holds a NaN or an infinity
 *   -4  a selected ratio overflowed to +-inf (results then unspecified)
 *   -5  out of host memory
 *
 * ALGORITHM 2 (oracle_breakpoints): the breakpoints of every segment's
 *   solution path v_k(lambda) and the lambda_max beyond which v_k = 0, from
 *   the paper's loop over the sorted points with exact sums (see the
 *   function's comment for the one reading it takes).
 *
 * ALGORITHM 3 lives in oracle.py (solution_path, exact rationals); from this
 *   file it uses oracle_breakpoints and oracle_residual (the score of one
 *   breakpoint entry, as Algorithm 1 computes it).
 *
 * PINS (tests/test_oracle_*.py): the worked example of Sec. 3.1 (Table I,
 * Fig. 1 lines, the breakpoints and the maximum useful lambda), exact
 * rational brute force over every breakpoint on tiny inputs, an LP solver on
 * LP (4), the dual certificate of Lemma 1's proof, the closed form for the
 * smallest lambda that zeroes v_k (Lemma 1's proof, Algorithm 2), lambda = 0
 * as plain weighted-median (LAD) regression, and exact invariances.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENONFINITE (-3)
#define OR_ERANGE (-4)
#define OR_ENOMEM (-5)

/* ------------------------------------------------------------------ big */
/* Non-negative integers in units of 2^-1074, 64-bit limbs, little endian.
 * A finite double is below 2^1024 = 2^2098 units; sums of up to 2^31 terms
 * and their doubles stay below 2^2131, so 36 limbs (2304 bits) suffice. */
#define NLIMB 36
typedef struct { uint64_t d[NLIMB]; } big;

static void big_zero(big *a) { memset(a, 0, sizeof *a); }

/* a += |x| for a finite double x */
static void big_add_double(big *a, double x)
{
    uint64_t bits;
    memcpy(&bits, &x, sizeof bits);
    uint64_t bexp = (bits >> 52) & 0x7ff;
    uint64_t mant = bits & ((1ull << 52) - 1);
    uint64_t shift;
    if (bexp == 0) {              /* subnormal or zero: mant * 2^-1074 */
        shift = 0;
    } else {                      /* normal: (2^52 + mant) * 2^(bexp-1075) */
        mant |= 1ull << 52;
        shift = bexp - 1;
    }
    if (mant == 0) return;
    unsigned limb = (unsigned)(shift / 64), off = (unsigned)(shift % 64);
    uint64_t lo = mant << off;
    uint64_t hi = off ? (mant >> (64 - off)) : 0;
    unsigned __int128 c = (unsigned __int128)a->d[limb] + lo;
    a->d[limb] = (uint64_t)c;
    c = (unsigned __int128)a->d[limb + 1] + hi + (uint64_t)(c >> 64);
    a->d[limb + 1] = (uint64_t)c;
    uint64_t carry = (uint64_t)(c >> 64);
    for (unsigned t = limb + 2; carry && t < NLIMB; ++t) {
        c = (unsigned __int128)a->d[t] + carry;
        a->d[t] = (uint64_t)c;
        carry = (uint64_t)(c >> 64);
    }
}

/* r = a + b */
static void big_add(big *r, const big *a, const big *b)
{
    uint64_t carry = 0;
    for (int t = 0; t < NLIMB; ++t) {
        unsigned __int128 c = (unsigned __int128)a->d[t] + b->d[t] + carry;
        r->d[t] = (uint64_t)c;
        carry = (uint64_t)(c >> 64);
    }
}

/* r = 2a */
static void big_twice(big *r, const big *a) { big_add(r, a, a); }

static int big_cmp(const big *a, const big *b)
{
    for (int t = NLIMB - 1; t >= 0; --t) {
        if (a->d[t] != b->d[t]) return a->d[t] < b->d[t] ? -1 : 1;
    }
    return 0;
}

/* ------------------------------------------------------------------ R64 */
static double r64_sum(const double *terms, int64_t count)
{
    double p[64];
    for (int l = 0; l < 64; ++l) p[l] = 0.0;
    for (int64_t t = 0; t < count; ++t) p[t % 64] = p[t % 64] + terms[t];
    for (int d = 32; d >= 1; d /= 2)
        for (int l = 0; l < d; ++l) p[l] = p[l] + p[l + d];
    return p[0];
}

/* --------------------------------------------------------------- points */
typedef struct {
    double r;      /* fl(x_ik / x_ij) + 0.0 */
    int64_t row;   /* i */
    double w;      /* |x_ij| */
} point;

static int point_cmp(const void *pa, const void *pb)
{
    const point *a = (const point *)pa, *b = (const point *)pb;
    if (a->r < b->r) return -1;
    if (a->r > b->r) return 1;
    if (a->row < b->row) return -1;
    if (a->row > b->row) return 1;
    return 0;
}

#define XAT(X, ld, i, k) ((X)[(i) + (k) * (ld)])

/* Sorted ratio list of segment (j, k): fills pts (capacity n), returns n'. */
static int64_t build_points(const double *X, int64_t n, int64_t ld, int64_t j,
                           int64_t k, point *pts)
{
    int64_t np = 0;
    for (int64_t i = 0; i < n; ++i) {
        double xj = XAT(X, ld, i, j);
        if (xj == 0.0) continue;
        double r = XAT(X, ld, i, k) / xj;
        pts[np].r = r + 0.0;
        pts[np].row = i;
        pts[np].w = fabs(xj);
        ++np;
    }
    qsort(pts, (size_t)np, sizeof(point), point_cmp);
    return np;
}

/* Selection for one lambda on a sorted list (rule R3 or Algorithm 1).
 * Returns the position (0-based) of the chosen point, or -1 for v = 0. */
static int64_t select_point(const point *pts, int64_t np, double lambda,
                            int tie_rule)
{
    big W, lam, S, twoS, rhs, lhs;
    big_zero(&W);
    for (int64_t p = 0; p < np; ++p) big_add_double(&W, pts[p].w);
    big_zero(&lam);
    big_add_double(&lam, lambda);

    if (tie_rule == 1) {
        /* Algorithm 1 verbatim: for each point in sorted order, accept it when
         * sgn(r) * lambda lies in (W - 2 S_p, W - 2 S_{p-1}]; last one wins. */
        int64_t chosen = -1;
        big Sprev;
        big_zero(&Sprev);
        for (int64_t p = 0; p < np; ++p) {
            S = Sprev;
            big_add_double(&S, pts[p].w);          /* S = S_p, p 1-based */
            big twoSprev;
            big_twice(&twoSprev, &Sprev);
            big_twice(&twoS, &S);
            int ok;
            if (pts[p].r > 0.0) {          /* 2 S_{p-1} + lam <= W < 2 S_p + lam */
                big_add(&lhs, &twoSprev, &lam);
                big_add(&rhs, &twoS, &lam);
                ok = big_cmp(&lhs, &W) <= 0 && big_cmp(&W, &rhs) < 0;
            } else if (pts[p].r < 0.0) {   /* 2 S_{p-1} <= W + lam < 2 S_p */
                big_add(&rhs, &W, &lam);
                ok = big_cmp(&twoSprev, &rhs) <= 0 && big_cmp(&rhs, &twoS) < 0;
            } else {                       /* 2 S_{p-1} <= W < 2 S_p */
                ok = big_cmp(&twoSprev, &W) <= 0 && big_cmp(&W, &twoS) < 0;
            }
            if (ok) chosen = p;
            Sprev = S;
        }
        return chosen;
    }

    /* Rule R3. */
    int64_t N = 0, Z = 0;
    while (N < np && pts[N].r < 0.0) ++N;
    while (N + Z < np && pts[N + Z].r == 0.0) ++Z;
    big A, B, twoA, twoB, WpL;
    big_zero(&A);
    for (int64_t p = 0; p < N; ++p) big_add_double(&A, pts[p].w);
    B = A;
    for (int64_t p = N; p < N + Z; ++p) big_add_double(&B, pts[p].w);
    big_twice(&twoA, &A);
    big_twice(&twoB, &B);
    big_add(&WpL, &W, &lam);
    big twoBpL;
    big_add(&twoBpL, &twoB, &lam);

    if (big_cmp(&twoA, &WpL) <= 0 && big_cmp(&W, &twoBpL) <= 0)
        return -1;                                   /* 0 is a minimiser */
    big_zero(&S);
    if (big_cmp(&twoA, &WpL) > 0) {                  /* minimiser below 0 */
        for (int64_t p = 0; p < N; ++p) {
            big_add_double(&S, pts[p].w);
            big_twice(&twoS, &S);
            if (big_cmp(&twoS, &WpL) > 0) return p;
        }
        return -2;                                   /* unreachable */
    }
    S = B;                                           /* minimiser above 0 */
    for (int64_t p = N + Z; p < np; ++p) {
        big_add_double(&S, pts[p].w);
        big_twice(&twoS, &S);
        big_add(&lhs, &twoS, &lam);
        if (big_cmp(&lhs, &W) >= 0) return p;
    }
    return -2;                                       /* unreachable */
}

/* e_jk = R64 over i of |x_ik - fl(v * x_ij)|; terms is scratch of length n */
static double residual(const double *X, int64_t n, int64_t ld, int64_t j,
                       int64_t k, double v, double *terms)
{
    for (int64_t i = 0; i < n; ++i) {
        double prod = v * XAT(X, ld, i, j);
        double diff = XAT(X, ld, i, k) - prod;
        terms[i] = fabs(diff);
    }
    return r64_sum(terms, n);
}

static int check_x(const double *X, int64_t n, int64_t m, int64_t ld)
{
    if (!X || n < 1 || m < 1 || ld < n) return OR_EINVAL;
    for (int64_t k = 0; k < m; ++k)
        for (int64_t i = 0; i < n; ++i)
            if (!isfinite(XAT(X, ld, i, k))) return OR_ENONFINITE;
    return OR_OK;
}

static int check_lambdas(const double *lam, int64_t L)
{
    if (!lam || L < 1) return OR_EINVAL;
    for (int64_t t = 0; t < L; ++t)
        if (!(lam[t] >= 0.0) || isinf(lam[t])) return OR_EINVAL;
    return OR_OK;
}

/* ============================================================ entry points */

/* Column mass W_j = R64_i |x_ij| and zero count Z_j = #{i : x_ij == 0}. */
int oracle_column_stats(const double *X, int64_t n, int64_t m, int64_t ld,
                        double *W, int64_t *zeros)
{
    int st = check_x(X, n, m, ld);
    if (st) return st;
    double *terms = (double *)malloc((size_t)n * sizeof(double));
    if (!terms) return OR_ENOMEM;
    for (int64_t k = 0; k < m; ++k) {
        int64_t z = 0;
        for (int64_t i = 0; i < n; ++i) {
            terms[i] = fabs(XAT(X, ld, i, k));
            if (XAT(X, ld, i, k) == 0.0) ++z;
        }
        if (W) W[k] = r64_sum(terms, n);
        if (zeros) zeros[k] = z;
    }
    free(terms);
    return OR_OK;
}

/* One segment (j, k != j) for L penalties: v[t], row[t] (-1 when v = 0) and
 * e[t] = e_jk(lambda_t).  Sorts once and reuses the list for every lambda. */
int oracle_segment(const double *X, int64_t n, int64_t m, int64_t ld,
                   int64_t j, int64_t k, const double *lambdas, int64_t L,
                   int tie_rule, double *v, int32_t *row, double *e)
{
    int st = check_x(X, n, m, ld);
    if (st) return st;
    st = check_lambdas(lambdas, L);
    if (st) return st;
    if (j < 0 || j >= m || k < 0 || k >= m || j == k || !v) return OR_EINVAL;
    point *pts = (point *)malloc((size_t)n * sizeof(point));
    double *terms = (double *)malloc((size_t)n * sizeof(double));
    if (!pts || !terms) { free(pts); free(terms); return OR_ENOMEM; }
    int64_t np = build_points(X, n, ld, j, k, pts);
    int status = OR_OK;
    for (int64_t t = 0; t < L; ++t) {
        int64_t p = select_point(pts, np, lambdas[t], tie_rule);
        double vk = p >= 0 ? pts[p].r : 0.0;
        if (isinf(vk)) status = OR_ERANGE;
        v[t] = vk;
        if (row) row[t] = p >= 0 ? (int32_t)pts[p].row : -1;
        if (e) e[t] = residual(X, n, ld, j, k, vk, terms);
    }
    free(pts);
    free(terms);
    return status;
}

/* Everything for one preserved coordinate j and L penalties:
 *   V[t*m + k] = v_k, ROW[t*m + k] (-1 for v_k = 0 and for k = j),
 *   EJK[t*m + k] = e_jk (e_jj = +0), and per lambda
 *   EJ[t] = R64_k e_jk, PJ[t] = R64_k |v_k|, ZJ[t] = EJ + fl(lambda * PJ).
 * Any output pointer may be NULL. */
int oracle_fit_j(const double *X, int64_t n, int64_t m, int64_t ld, int64_t j,
                 const double *lambdas, int64_t L, int tie_rule, double *V,
                 int32_t *ROW, double *EJK, double *EJ, double *PJ, double *ZJ)
{
    int st = check_x(X, n, m, ld);
    if (st) return st;
    st = check_lambdas(lambdas, L);
    if (st) return st;
    if (j < 0 || j >= m) return OR_EINVAL;
    point *pts = (point *)malloc((size_t)n * sizeof(point));
    double *terms = (double *)malloc((size_t)(n > m ? n : m) * sizeof(double));
    double *vv = (double *)malloc((size_t)(L * m) * sizeof(double));
    double *ee = (double *)malloc((size_t)(L * m) * sizeof(double));
    int32_t *rr = (int32_t *)malloc((size_t)(L * m) * sizeof(int32_t));
    if (!pts || !terms || !vv || !ee || !rr) {
        free(pts); free(terms); free(vv); free(ee); free(rr);
        return OR_ENOMEM;
    }
    int status = OR_OK;
    for (int64_t k = 0; k < m; ++k) {
        if (k == j) {
            for (int64_t t = 0; t < L; ++t) {
                vv[t * m + k] = 1.0;
                ee[t * m + k] = 0.0;
                rr[t * m + k] = -1;
            }
            continue;
        }
        int64_t np = build_points(X, n, ld, j, k, pts);
        for (int64_t t = 0; t < L; ++t) {
            int64_t p = select_point(pts, np, lambdas[t], tie_rule);
            double vk = p >= 0 ? pts[p].r : 0.0;
            if (isinf(vk)) status = OR_ERANGE;
            vv[t * m + k] = vk;
            rr[t * m + k] = p >= 0 ? (int32_t)pts[p].row : -1;
            ee[t * m + k] = residual(X, n, ld, j, k, vk, terms);
        }
    }
    for (int64_t t = 0; t < L; ++t) {
        double E = r64_sum(ee + t * m, m);
        for (int64_t k = 0; k < m; ++k) terms[k] = fabs(vv[t * m + k]);
        double P = r64_sum(terms, m);
        double pen = lambdas[t] * P;
        double z = E + pen;
        if (EJ) EJ[t] = E;
        if (PJ) PJ[t] = P;
        if (ZJ) ZJ[t] = z;
    }
    if (V) memcpy(V, vv, (size_t)(L * m) * sizeof(double));
    if (EJK) memcpy(EJK, ee, (size_t)(L * m) * sizeof(double));
    if (ROW) memcpy(ROW, rr, (size_t)(L * m) * sizeof(int32_t));
    free(pts); free(terms); free(vv); free(ee); free(rr);
    return status;
}

/* Algorithm 1 over a path of L penalties (L = 1 is a single fit):
 *   V[t*m + k] = v*_k(lambda_t), J[t] = j*, OBJ[t] = z_{j*},
 *   ROW[t*m + k] = sorted-point row that gave v*_k (-1 if v*_k = 0 or k = j*),
 *   ZALL[t*m + j] = z_j(lambda_t) for every j.
 * Candidates j run in parallel (OpenMP, `nthreads` threads, <= 0: default);
 * each j is computed independently and the argmin is taken serially. */
int oracle_fit_path(const double *X, int64_t n, int64_t m, int64_t ld,
                    const double *lambdas, int64_t L, int tie_rule,
                    int nthreads, double *V, int64_t *J, double *OBJ,
                    int32_t *ROW, double *ZALL)
{
    int st = check_x(X, n, m, ld);
    if (st) return st;
    st = check_lambdas(lambdas, L);
    if (st) return st;
    if (!V || !J || !OBJ) return OR_EINVAL;
    double *Vall = (double *)malloc((size_t)(m * L * m) * sizeof(double));
    int32_t *Rall = (int32_t *)malloc((size_t)(m * L * m) * sizeof(int32_t));
    double *Z = (double *)malloc((size_t)(m * L) * sizeof(double));
    int *stj = (int *)calloc((size_t)m, sizeof(int));
    if (!Vall || !Rall || !Z || !stj) {
        free(Vall); free(Rall); free(Z); free(stj);
        return OR_ENOMEM;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t j = 0; j < m; ++j) {
        stj[j] = oracle_fit_j(X, n, m, ld, j, lambdas, L, tie_rule,
                              Vall + j * L * m, Rall + j * L * m, NULL, NULL,
                              NULL, Z + j * L);
    }
    int status = OR_OK;
    for (int64_t j = 0; j < m; ++j)
        if (stj[j] && (status == OR_OK || stj[j] != OR_ERANGE)) status = stj[j];
    if (status != OR_OK && status != OR_ERANGE) {
        free(Vall); free(Rall); free(Z); free(stj);
        return status;
    }
    for (int64_t t = 0; t < L; ++t) {
        int64_t best = 0;
        for (int64_t j = 1; j < m; ++j)
            if (Z[j * L + t] < Z[best * L + t]) best = j;
        J[t] = best;
        OBJ[t] = Z[best * L + t];
        memcpy(V + t * m, Vall + best * L * m + t * m, (size_t)m * sizeof(double));
        if (ROW) memcpy(ROW + t * m, Rall + best * L * m + t * m, (size_t)m * sizeof(int32_t));
        if (ZALL)
            for (int64_t j = 0; j < m; ++j) ZALL[t * m + j] = Z[j * L + t];
    }
    free(Vall); free(Rall); free(Z); free(stj);
    return status;
}

/* ------------------------------------------------------- components */
/* Successive components (Sec. 2, after Algorithm 3: a component is found by
 * Algorithm 1 on the data projected onto the null space of the components
 * derived so far).  With X_0 = X and the same lambda for every component:
 *   v_c    = Algorithm 1 on X_c (j_c, z_c its preserved column and objective)
 *   w_c    = v_c made orthogonal to w_0 .. w_{c-1} (classical Gram-Schmidt,
 *            unnormalised): w = v_c; for l < c:
 *            w_k = fl(w_k - fl(fl(R64_k(w_lk * v_ck) / R64_k(w_lk^2)) * w_lk))
 *   X_c+1  = X_c projected off w_c:  s_i = R64_k fl(x_ik * w_ck),
 *            u_k = fl(w_ck / R64_k(w_ck^2)),  x_ik = fl(x_ik - fl(s_i * u_k))
 * (every product rounded on its own, no fused multiply-add; R64 as above).
 *   V [p*m], J [p], OBJ [p]; Xout (n x m, ld = n, nullable): X_p-1, the data
 *   the last component was fitted on. */
static double r64_dot(const double *a, const double *b, int64_t m, double *terms)
{
    for (int64_t k = 0; k < m; ++k) terms[k] = a[k] * b[k];
    return r64_sum(terms, m);
}

int oracle_components(const double *X, int64_t n, int64_t m, int64_t ld, double lambda,
                      int64_t p, double *V, int64_t *J, double *OBJ, double *Xout)
{
    int st = check_x(X, n, m, ld);
    if (st) return st;
    st = check_lambdas(&lambda, 1);
    if (st) return st;
    if (p < 1 || p > m || !V || !J || !OBJ) return OR_EINVAL;
    double *Xc = (double *)malloc((size_t)(n * m) * sizeof(double));
    double *Wb = (double *)malloc((size_t)(p * m) * sizeof(double));
    double *cw = (double *)malloc((size_t)p * sizeof(double));
    double *terms = (double *)malloc((size_t)(m > n ? m : n) * sizeof(double));
    double *row = (double *)malloc((size_t)m * sizeof(double));
    if (!Xc || !Wb || !cw || !terms || !row) {
        free(Xc); free(Wb); free(cw); free(terms); free(row);
        return OR_ENOMEM;
    }
    for (int64_t k = 0; k < m; ++k)
        for (int64_t i = 0; i < n; ++i) Xc[i + k * n] = XAT(X, ld, i, k);
    int status = OR_OK;
    for (int64_t c = 0; c < p; ++c) {
        st = oracle_fit_path(Xc, n, m, n, &lambda, 1, 0, 0, V + c * m, J + c, OBJ + c, NULL, NULL);
        if (st && st != OR_ERANGE) { status = st; break; }
        if (st) status = st;
        if (c == p - 1) break;
        const double *v = V + c * m;
        double *w = Wb + c * m;
        for (int64_t k = 0; k < m; ++k) w[k] = v[k];
        for (int64_t l = 0; l < c; ++l) {
            const double coef = r64_dot(Wb + l * m, v, m, terms) / cw[l];
            for (int64_t k = 0; k < m; ++k) w[k] = w[k] - coef * Wb[l * m + k];
        }
        cw[c] = r64_dot(w, w, m, terms);
        if (!(cw[c] > 0.0)) { status = OR_EINVAL; break; }
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t k = 0; k < m; ++k) row[k] = Xc[i + k * n];
            const double si = r64_dot(row, w, m, terms);
            for (int64_t k = 0; k < m; ++k) {
                const double uk = w[k] / cw[c];
                const double prod = si * uk;
                Xc[i + k * n] = Xc[i + k * n] - prod;
            }
        }
    }
    if (Xout) memcpy(Xout, Xc, (size_t)(n * m) * sizeof(double));
    free(Xc); free(Wb); free(cw); free(terms); free(row);
    return status;
}

/* Threads OpenMP will use for oracle_fit_path (1 without OpenMP). */
/* ------------------------------------------------------------ Algorithm 2 */
/* r = a - b for a >= b */
static void big_sub(big *r, const big *a, const big *b)
{
    uint64_t borrow = 0;
    for (int t = 0; t < NLIMB; ++t) {
        unsigned __int128 d = (unsigned __int128)a->d[t] - b->d[t] - borrow;
        r->d[t] = (uint64_t)d;
        borrow = (uint64_t)(d >> 64) ? 1 : 0;
    }
}

/* The double nearest to a * 2^-1074 (ties to even). */
static double big_to_double(const big *a)
{
    int top = -1;
    for (int t = NLIMB - 1; t >= 0 && top < 0; --t)
        if (a->d[t]) top = t * 64 + 63 - __builtin_clzll(a->d[t]);
    if (top < 0) return 0.0;
    if (top <= 52) {                         /* exact: at most 53 bits */
        uint64_t v = a->d[0];
        return ldexp((double)v, -1074);
    }
    int lo = top - 52;                       /* keep bits top..lo */
    uint64_t q = 0;
    for (int b = top; b >= lo; --b) q = (q << 1) | ((a->d[b / 64] >> (b % 64)) & 1u);
    int half = (a->d[(lo - 1) / 64] >> ((lo - 1) % 64)) & 1u;
    int sticky = 0;
    for (int b = lo - 2; b >= 0 && !sticky; --b) sticky = (a->d[b / 64] >> (b % 64)) & 1u;
    if (half && (sticky || (q & 1u))) ++q;  /* q may become 2^53: still exact */
    return ldexp((double)q, lo - 1074);
}

/* Algorithm 2 for one segment (preserved j, column k), in the paper's
 * notation: over the sorted points r_p (weights w_p = |x_pj|),
 *   lambda_p = sgn(r_p) (sum of the weights after p - sum before p) - w_p,
 * a breakpoint max(0, lambda_p) with v_k = r_p wherever lambda_p + 2 w_p > 0,
 * and lambda_max = the largest lambda_p + 2 w_p (at least 0), where v_k
 * becomes 0.  Every sum is exact (big integers); each lambda is then rounded
 * once to the nearest double.
 * Reading: zero ratios (sgn 0) are left out of the loop -- by Lemma 1 a
 * point at 0 never moves the minimiser away from 0 and v_k = 0 is the
 * terminal entry -- so lambda_max is Lemma 1's exact threshold
 * max(0, 2A - W, W - 2B).  The entries are returned in increasing lambda:
 * on the negative side the sorted order, on the positive side its reverse,
 * and then the terminal entry (lambda_max, 0, row -1).  With the R3 rule the
 * solution on [lam[t], lam[t+1]) is (v[t], row[t]).
 *   cap      capacity of lam, v, row (nullable when cap = 0)
 *   count    entries of the segment (the terminal one included)
 *   lmax     lambda_max */
int oracle_breakpoints(const double *X, int64_t n, int64_t m, int64_t ld, int64_t j,
                       int64_t k, int64_t cap, double *lam, double *v, int32_t *row,
                       int64_t *count, double *lmax)
{
    int st = check_x(X, n, m, ld);
    if (st) return st;
    if (j < 0 || j >= m || k < 0 || k >= m || j == k || !count || !lmax) return OR_EINVAL;
    point *pts = (point *)malloc((size_t)n * sizeof(point) + 1);
    big *prefix = (big *)malloc(((size_t)n + 1) * sizeof(big));   /* weight before p */
    if (!pts || !prefix) { free(pts); free(prefix); return OR_ENOMEM; }
    int64_t np = build_points(X, n, ld, j, k, pts);
    big_zero(&prefix[0]);
    for (int64_t p = 0; p < np; ++p) {
        prefix[p + 1] = prefix[p];
        big_add_double(&prefix[p + 1], pts[p].w);
    }
    big W = prefix[np], before, after, lp, lp2, best;
    big_zero(&best);
    int64_t c = 0;
    /* visit the points in the order the entries are listed: negative side in
     * sorted order, positive side from 0 outwards */
    int64_t N = 0, Z = 0;
    while (N < np && pts[N].r < 0.0) ++N;
    while (N + Z < np && pts[N + Z].r == 0.0) ++Z;
    for (int pass = 0; pass < 2; ++pass) {
        int64_t first = pass == 0 ? 0 : np - 1, last = pass == 0 ? N : N + Z - 1, step = pass == 0 ? 1 : -1;
        for (int64_t p = first; p != last; p += step) {
            /* weight before p and after p in sorted order */
            before = prefix[p];
            big_sub(&after, &W, &before);
            big wp;
            big_zero(&wp);
            big_add_double(&wp, pts[p].w);
            big_sub(&after, &after, &wp);
            /* lambda_p + 2 w_p = sgn (after - before) + w_p, kept as a signed
             * pair (positive part, negative part) */
            big pos, neg;
            if (pts[p].r < 0.0) { pos = before; neg = after; }    /* before - after */
            else { pos = after; neg = before; }                   /* after - before */
            big_add(&lp2, &pos, &wp);                             /* lambda_p + 2 w_p = pos + w_p - neg */
            if (big_cmp(&lp2, &neg) <= 0) continue;               /* not > 0 */
            big_sub(&lp2, &lp2, &neg);
            if (big_cmp(&lp2, &best) > 0) best = lp2;
            /* max(0, lambda_p) = max(0, pos - neg - w_p) */
            big negw;
            big_add(&negw, &neg, &wp);
            if (big_cmp(&pos, &negw) > 0) big_sub(&lp, &pos, &negw); else big_zero(&lp);
            if (c < cap) {
                lam[c] = big_to_double(&lp);
                v[c] = pts[p].r;
                row[c] = (int32_t)pts[p].row;
            }
            ++c;
        }
    }
    if (c < cap) { lam[c] = big_to_double(&best); v[c] = 0.0; row[c] = -1; }
    ++c;
    *count = c;
    *lmax = big_to_double(&best);
    free(pts);
    free(prefix);
    return OR_OK;
}

/* The residual e_jk = R64 over i of |x_ik - fl(v * x_ij)| at a given v, as
 * Algorithm 1 scores it; Algorithm 3 scores every breakpoint entry with it. */
int oracle_residual(const double *X, int64_t n, int64_t m, int64_t ld, int64_t j,
                    int64_t k, double v, double *e)
{
    if (!X || n < 1 || m < 1 || ld < n || j < 0 || j >= m || k < 0 || k >= m || !e || !isfinite(v))
        return OR_EINVAL;
    double *terms = (double *)malloc((size_t)n * sizeof(double));
    if (!terms) return OR_ENOMEM;
    *e = residual(X, n, ld, j, k, v, terms);
    free(terms);
    return OR_OK;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
