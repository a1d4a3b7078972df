/*
 * Body of the plain cyclic Jacobi oracle, instantiated twice by oracle.c:
 * once with REAL=double (unit roundoff 2^-53) and once with REAL=float
 * (2^-24).  TEST INFRASTRUCTURE ONLY -- see the header of oracle.c.
 *
 * Everything here is written from Section 3.1 of Zhang & Bai (the rotation
 * J(i,j;c,s), Lemma "offa-jr" for the angle, Algorithm 3.2 for the cyclic
 * sweep) and Remark "dc" (Section 3.2) for the negligible-entry rule.
 * Matrices are column-major: element (i,j) of X is X[i + j*ldx].
 */

/* Lemma offa-jr: mu = (a_jj - a_ii) / (2 a_ij); t is the smaller root of
 * t^2 + 2 mu t - 1 = 0, c = 1/sqrt(1+t^2), s = t c.  (c,s) = (1,0) if a_ij = 0.
 * For |mu| so large that mu^2 overflows, t = 1/(2 mu) is the limit of both
 * branches. */
static void FN(angle)(REAL aii, REAL ajj, REAL aij, REAL *c, REAL *s, REAL *t)
{
    if (aij == (REAL)0) { *c = 1; *s = 0; *t = 0; return; }
    REAL mu = (ajj - aii) / ((REAL)2 * aij);
    REAL tt;
    if (FABS(mu) > BIGMU) {
        tt = (REAL)0.5 / mu;
    } else if (mu >= (REAL)0) {
        tt = (REAL)1 / (mu + SQRT((REAL)1 + mu * mu));
    } else {
        tt = (REAL)1 / (mu - SQRT((REAL)1 + mu * mu));
    }
    REAL cc = (REAL)1 / SQRT((REAL)1 + tt * tt);
    *c = cc; *s = tt * cc; *t = tt;
}

/* Remark dc: a_pq may be treated as zero when |a_pq| <= u sqrt(|a_pp a_qq|).
 * The rule is additionally capped by skip_abs (= tol ||A||_F / n), so that
 * the entries it leaves behind can never by themselves keep
 * ||off(T)||_F above tol ||A||_F. */
static int FN(negligible)(REAL app, REAL aqq, REAL apq, REAL skip_abs)
{
    if (apq == (REAL)0) return 1;
    REAL a = FABS(apq);
    REAL lim = UNIT * SQRT(FABS(app * aqq));
    if (skip_abs < lim) lim = skip_abs;
    return a <= lim;
}

/* One rotation J(p,q;c,s) applied as T <- J^T T J and P <- P J
 * (Algorithm 3.2, third step).  Off-diagonal entries of rows/columns p,q and
 * the columns of P use the tau = s/(1+c) form of the same rotation; the
 * diagonal pair uses b_pp = a_pp - t a_pq, b_qq = a_qq + t a_pq, and b_pq is
 * set to zero (the value the exact rotation produces, Lemma offa-jr). */
static void FN(rotate)(int n, REAL *T, int ldt, REAL *P, int ldp, int np,
                       int p, int q, REAL c, REAL s, REAL t)
{
    REAL tau = s / ((REAL)1 + c);
    REAL apq = T[p + (size_t)q * ldt];
    for (int j = 0; j < n; ++j) {
        if (j == p || j == q) continue;
        REAL x = T[p + (size_t)j * ldt];
        REAL y = T[q + (size_t)j * ldt];
        REAL nx = x - s * (y + tau * x);
        REAL ny = y + s * (x - tau * y);
        T[p + (size_t)j * ldt] = nx; T[j + (size_t)p * ldt] = nx;
        T[q + (size_t)j * ldt] = ny; T[j + (size_t)q * ldt] = ny;
    }
    T[p + (size_t)p * ldt] -= t * apq;
    T[q + (size_t)q * ldt] += t * apq;
    T[p + (size_t)q * ldt] = 0;
    T[q + (size_t)p * ldt] = 0;
    if (P) {
        for (int i = 0; i < np; ++i) {
            REAL x = P[i + (size_t)p * ldp];
            REAL y = P[i + (size_t)q * ldp];
            P[i + (size_t)p * ldp] = x - s * (y + tau * x);
            P[i + (size_t)q * ldp] = y + s * (x - tau * y);
        }
    }
}

/* ||off(T)||_F summed directly over i != j (Section 1 notation: off(G) is
 * G minus its diagonal). */
static double FN(offnorm)(int n, const REAL *T, int ldt)
{
    double acc = 0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            if (i != j) { double v = T[i + (size_t)j * ldt]; acc += v * v; }
    return sqrt(acc);
}

static double FN(fro)(int m, int n, const REAL *A, int lda)
{
    double acc = 0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) { double v = A[i + (size_t)j * lda]; acc += v * v; }
    return sqrt(acc);
}

/* Handle one index pair (p<q) of a cyclic sweep; returns 1 if a rotation was
 * applied. */
static int FN(do_pair)(int n, REAL *T, int ldt, REAL *P, int ldp, int np,
                       int p, int q, REAL skip_abs)
{
    REAL app = T[p + (size_t)p * ldt], aqq = T[q + (size_t)q * ldt];
    REAL apq = T[p + (size_t)q * ldt];
    if (FN(negligible)(app, aqq, apq, skip_abs)) {
        T[p + (size_t)q * ldt] = 0; T[q + (size_t)p * ldt] = 0;
        return 0;
    }
    REAL c, s, t;
    FN(angle)(app, aqq, apq, &c, &s, &t);
    FN(rotate)(n, T, ldt, P, ldp, np, p, q, c, s, t);
    return 1;
}

/* Algorithm 3.2 (and step 4 of Algorithm 4.1): starting from the current T
 * and P, sweep until ||off(T)||_F <= tol * nrmA or max_sweeps sweeps ran.
 * order 0 = row cyclic (i = 1..n-1, j = i+1..n), order 1 = the round-robin
 * order of or_round_robin, one parallel step after another; inside a step the
 * rotations are disjoint and are applied one after the other.
 * Returns 0 on convergence, 1 if max_sweeps was reached first. */
static int FN(sweeps)(int n, REAL *T, int ldt, REAL *P, int ldp, int np,
                      double tol, double nrmA, int max_sweeps, int order,
                      int *sweeps_out, long long *rot_out,
                      double *off_hist, int hist_len)
{
    int sweeps = 0;
    long long rot = 0;
    REAL skip_abs = (REAL)(tol * nrmA / (n > 0 ? n : 1));
    int ne = n + (n & 1);
    int *pp = NULL, *qq = NULL;
    if (order == 1 && n > 1) {
        pp = (int *)malloc(sizeof(int) * (ne / 2));
        qq = (int *)malloc(sizeof(int) * (ne / 2));
    }
    double off = FN(offnorm)(n, T, ldt);
    if (off_hist && hist_len > 0) off_hist[0] = off;
    while (off > tol * nrmA && sweeps < max_sweeps) {
        if (order == 0) {
            for (int p = 0; p < n - 1; ++p)
                for (int q = p + 1; q < n; ++q)
                    rot += FN(do_pair)(n, T, ldt, P, ldp, np, p, q, skip_abs);
        } else {
            for (int r = 0; r < ne - 1; ++r) {
                or_round_robin(ne, r, pp, qq);
                for (int k = 0; k < ne / 2; ++k) {
                    if (qq[k] >= n) continue; /* pair with the padding index */
                    rot += FN(do_pair)(n, T, ldt, P, ldp, np, pp[k], qq[k], skip_abs);
                }
            }
        }
        ++sweeps;
        off = FN(offnorm)(n, T, ldt);
        if (off_hist && sweeps < hist_len) off_hist[sweeps] = off;
    }
    free(pp); free(qq);
    if (sweeps_out) *sweeps_out = sweeps;
    if (rot_out) *rot_out = rot;
    return off > tol * nrmA ? 1 : 0;
}
