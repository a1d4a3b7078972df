/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the
 * mixed-precision preconditioned Jacobi eigensolver of Zhang & Bai,
 * "A mixed precision preconditioned Jacobi method for the symmetric
 * eigenvalue problem" (arXiv 2211.03339).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library, and neither includes nor
 * links the other.
 *
 * What each function follows:
 *   or_syev            Algorithm 3.2 (cyclic Jacobi), FP64: the plain method;
 *                      the preconditioned Algorithm 4.1 reaches the same
 *                      eigendecomposition, so this is the end-to-end oracle.
 *   or_syev_f32        the same algorithm in FP32 (unit roundoff 2^-24), the
 *                      reference for the low-precision step 1 of Algorithm 4.1.
 *   or_jacobi_from     step 4 of Algorithm 4.1: sweeps from a given T and P.
 *   or_round_robin     the non-overlapping parallel ordering of Section 6.2
 *                      (circle method; reading of the garbled list there).
 *   or_parallel_step   one step of n/2 disjoint rotations, all angles taken
 *                      from T before the step (they commute, Section 3.1).
 *   or_angle           Lemma offa-jr.
 *   or_mgs             modified Gram-Schmidt, step 2 of Algorithm 4.1
 *                      (Lemma MGS, Section 2).
 *   or_gemm            C = op(A) op(B), naive triple loop (step 3 of
 *                      Algorithm 4.1: T = Q^T A Q).
 *   or_svd_onesided    Algorithm 5.1 sweeps (Lemma ortho-2c) on given C, V.
 *   or_svd_finish      final steps of Algorithm 5.2: order by column norm,
 *                      sigma_j = ||c_j||, u_j = c_j / sigma_j.
 * All matrices are column-major.  Nothing here is blocked, fused or
 * reordered beyond what the cited algorithm states.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

void or_round_robin(int n, int r, int *p, int *q);

/* ---------------------------------------------------------------- FP64 */
#define REAL double
#define FN(x) or_d_##x
#define FABS fabs
#define SQRT sqrt
#define UNIT 1.1102230246251565e-16 /* 2^-53 */
#define BIGMU 1e150
#include "jacobi_body.h"
#undef REAL
#undef FN
#undef FABS
#undef SQRT
#undef UNIT
#undef BIGMU

/* ---------------------------------------------------------------- FP32 */
#define REAL float
#define FN(x) or_s_##x
#define FABS fabsf
#define SQRT sqrtf
#define UNIT 5.9604644775390625e-08f /* 2^-24 */
#define BIGMU 1e18f
#include "jacobi_body.h"

/* Section 6.2 ordering, read as the circle (round-robin) method: for an even
 * number of indices n and step r = 0..n-2, ring position 0 holds index 0 and
 * ring position k >= 1 holds index 1 + ((k - 1 + r) mod (n - 1)); position i
 * is paired with position n-1-i.  Each pair is returned as (min, max), so
 * that p < q as in Lemma offa-jr.  Over r = 0..n-2 every pair i<j occurs
 * exactly once (one sweep). */
void or_round_robin(int n, int r, int *p, int *q)
{
    for (int i = 0; i < n / 2; ++i) {
        int ka = i, kb = n - 1 - i;
        int a = ka == 0 ? 0 : 1 + (ka - 1 + r) % (n - 1);
        int b = kb == 0 ? 0 : 1 + (kb - 1 + r) % (n - 1);
        p[i] = a < b ? a : b;
        q[i] = a < b ? b : a;
    }
}

void or_angle(double aii, double ajj, double aij, double *c, double *s, double *t)
{
    or_d_angle(aii, ajj, aij, c, s, t);
}

double or_fro(int m, int n, const double *A, int lda) { return or_d_fro(m, n, A, lda); }
double or_off(int n, const double *T, int ldt) { return or_d_offnorm(n, T, ldt); }

/* One parallel step: every angle is computed from T as it is before the
 * step, then the disjoint rotations are applied in list order.  Pairs whose
 * q is >= n (padding index) are ignored.  Returns the number applied. */
long long or_parallel_step(int n, double *T, int ldt, double *P, int ldp, int np,
                           int npairs, const int *p, const int *q, double skip_abs)
{
    double *cs = (double *)malloc(sizeof(double) * 3 * (npairs > 0 ? npairs : 1));
    int *act = (int *)malloc(sizeof(int) * (npairs > 0 ? npairs : 1));
    for (int k = 0; k < npairs; ++k) {
        act[k] = 0;
        if (q[k] >= n) continue;
        int a = p[k], b = q[k];
        double app = T[a + (size_t)a * ldt], aqq = T[b + (size_t)b * ldt];
        double apq = T[a + (size_t)b * ldt];
        if (or_d_negligible(app, aqq, apq, skip_abs)) { act[k] = 2; continue; }
        or_d_angle(app, aqq, apq, &cs[3 * k], &cs[3 * k + 1], &cs[3 * k + 2]);
        act[k] = 1;
    }
    long long applied = 0;
    for (int k = 0; k < npairs; ++k) {
        int a = p[k], b = q[k];
        if (act[k] == 2) {
            T[a + (size_t)b * ldt] = 0; T[b + (size_t)a * ldt] = 0;
        } else if (act[k] == 1) {
            or_d_rotate(n, T, ldt, P, ldp, np, a, b, cs[3 * k], cs[3 * k + 1], cs[3 * k + 2]);
            ++applied;
        }
    }
    free(cs); free(act);
    return applied;
}

int or_jacobi_from(int n, double *T, int ldt, double *P, int ldp, int np,
                   double tol, double nrmA, int max_sweeps, int order,
                   int *sweeps, long long *rot, double *off_hist, int hist_len)
{
    return or_d_sweeps(n, T, ldt, P, ldp, np, tol, nrmA, max_sweeps, order,
                       sweeps, rot, off_hist, hist_len);
}

/* Sort eigenpairs: W ascending, columns of V permuted alongside (a stable
 * insertion of indices, ties kept in working order). */
static void sort_pairs_d(int n, const double *d, int *idx)
{
    for (int i = 0; i < n; ++i) idx[i] = i;
    for (int i = 1; i < n; ++i) {
        int v = idx[i], j = i - 1;
        while (j >= 0 && d[idx[j]] > d[v]) { idx[j + 1] = idx[j]; --j; }
        idx[j + 1] = v;
    }
}

/* Algorithm 3.2 from T = A, P = I.  Outputs W (ascending) and V (n x n,
 * leading dimension ldv).  Returns 0 converged, 1 not converged, -1 bad
 * arguments. */
int or_syev(int n, const double *A, int lda, double tol, int max_sweeps, int order,
            double *W, double *V, int ldv, int *sweeps, long long *rot,
            double *off_hist, int hist_len)
{
    if (n < 0 || lda < (n > 1 ? n : 1) || ldv < (n > 1 ? n : 1)) return -1;
    if (n == 0) { if (sweeps) *sweeps = 0; if (rot) *rot = 0; return 0; }
    double *T = (double *)malloc(sizeof(double) * n * n);
    double *P = (double *)malloc(sizeof(double) * n * n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            T[i + (size_t)j * n] = A[i + (size_t)j * lda];
            P[i + (size_t)j * n] = i == j ? 1.0 : 0.0;
        }
    double nrmA = or_d_fro(n, n, A, lda);
    int info = or_d_sweeps(n, T, n, P, n, n, tol, nrmA, max_sweeps, order,
                           sweeps, rot, off_hist, hist_len);
    double *d = (double *)malloc(sizeof(double) * n);
    int *idx = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) d[i] = T[i + (size_t)i * n];
    sort_pairs_d(n, d, idx);
    for (int k = 0; k < n; ++k) {
        W[k] = d[idx[k]];
        for (int i = 0; i < n; ++i) V[i + (size_t)k * ldv] = P[i + (size_t)idx[k] * n];
    }
    free(T); free(P); free(d); free(idx);
    return info;
}

/* The same algorithm carried out entirely in FP32 (A given in FP32).
 * W ascending, V its eigenvectors. */
int or_syev_f32(int n, const float *A, int lda, double tol, int max_sweeps, int order,
                float *W, float *V, int ldv, int *sweeps, long long *rot)
{
    if (n < 0 || lda < (n > 1 ? n : 1) || ldv < (n > 1 ? n : 1)) return -1;
    if (n == 0) { if (sweeps) *sweeps = 0; if (rot) *rot = 0; return 0; }
    float *T = (float *)malloc(sizeof(float) * n * n);
    float *P = (float *)malloc(sizeof(float) * n * n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            T[i + (size_t)j * n] = A[i + (size_t)j * lda];
            P[i + (size_t)j * n] = i == j ? 1.0f : 0.0f;
        }
    double nrmA = or_s_fro(n, n, A, lda);
    int info = or_s_sweeps(n, T, n, P, n, n, tol, nrmA, max_sweeps, order,
                           sweeps, rot, NULL, 0);
    double *d = (double *)malloc(sizeof(double) * n);
    int *idx = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) d[i] = T[i + (size_t)i * n];
    sort_pairs_d(n, d, idx);
    for (int k = 0; k < n; ++k) {
        W[k] = (float)d[idx[k]];
        for (int i = 0; i < n; ++i) V[i + (size_t)k * ldv] = P[i + (size_t)idx[k] * n];
    }
    free(T); free(P); free(d); free(idx);
    return info;
}

/* Modified Gram-Schmidt (step 2 of Algorithm 4.1, Lemma MGS): Z (m x n,
 * full column rank) = Q R with Q^T Q = I, R upper triangular with positive
 * diagonal.  Column k is normalised, then removed from every later column.
 * R may be NULL.  Returns 0, or k+1 if column k has zero norm (breakdown). */
int or_mgs(int m, int n, const double *Z, int ldz, double *Q, int ldq, double *R, int ldr)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) Q[i + (size_t)j * ldq] = Z[i + (size_t)j * ldz];
    if (R)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) R[i + (size_t)j * ldr] = 0;
    for (int k = 0; k < n; ++k) {
        double *qk = Q + (size_t)k * ldq;
        double nn = 0;
        for (int i = 0; i < m; ++i) nn += qk[i] * qk[i];
        double rkk = sqrt(nn);
        if (!(rkk > 0)) return k + 1;
        for (int i = 0; i < m; ++i) qk[i] /= rkk;
        if (R) R[k + (size_t)k * ldr] = rkk;
        for (int j = k + 1; j < n; ++j) {
            double *qj = Q + (size_t)j * ldq;
            double rkj = 0;
            for (int i = 0; i < m; ++i) rkj += qk[i] * qj[i];
            for (int i = 0; i < m; ++i) qj[i] -= rkj * qk[i];
            if (R) R[k + (size_t)j * ldr] = rkj;
        }
    }
    return 0;
}

/* C (m x n) = op(A) op(B), op = transpose when the flag is set.  Naive
 * k-inner triple loop in FP64. */
void or_gemm(int ta, int tb, int m, int n, int k, const double *A, int lda,
             const double *B, int ldb, double *C, int ldc)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            double acc = 0;
            for (int l = 0; l < k; ++l) {
                double a = ta ? A[l + (size_t)i * lda] : A[i + (size_t)l * lda];
                double b = tb ? B[j + (size_t)l * ldb] : B[l + (size_t)j * ldb];
                acc += a * b;
            }
            C[i + (size_t)j * ldc] = acc;
        }
}

/* Algorithm 5.1 sweeps on a given C (m x n, m >= n) and V (n x n, updated in
 * place; identity for the plain method, Q for Algorithm 5.2).  For each pair
 * (i<j): alpha = c_i.c_i, beta = c_j.c_j, gamma = c_i.c_j; the rotation of
 * Lemma ortho-2c uses mu = (beta - alpha) / (2 gamma) and is applied to the
 * columns of C and V.  A pair is rotated only when
 * |gamma| > m u sqrt(alpha beta).  Stops when
 * ||off(C^T C)||_F <= tol ||C^T C||_F, or after a sweep that applied fewer
 * than ratio_stop * N rotations (N = n(n-1)/2; the paper's rule with
 * ratio 2e-4), or after max_sweeps.  order as in or_syev.  Returns 0 when a
 * stopping rule fired, 1 on max_sweeps. */
int or_svd_onesided(int m, int n, double *C, int ldc, double *V, int ldv,
                    double tol, double ratio_stop, int max_sweeps, int order,
                    int *sweeps_out, long long *rot_out)
{
    int sweeps = 0;
    long long rot = 0;
    int ne = n + (n & 1);
    int *pp = (int *)malloc(sizeof(int) * (ne / 2 + 1));
    int *qq = (int *)malloc(sizeof(int) * (ne / 2 + 1));
    double *G = (double *)malloc(sizeof(double) * n * (size_t)n);
    long long N = (long long)n * (n - 1) / 2;
    int info = 1;
    while (sweeps < max_sweeps) {
        or_gemm(1, 0, n, n, m, C, ldc, C, ldc, G, n);
        double offg = or_d_offnorm(n, G, n), nrmg = or_d_fro(n, n, G, n);
        if (offg <= tol * nrmg) { info = 0; break; }
        long long applied = 0;
        int nsteps = order == 0 ? 1 : ne - 1;
        for (int r = 0; r < nsteps; ++r) {
            int npairs;
            if (order == 0) npairs = 0; else { or_round_robin(ne, r, pp, qq); npairs = ne / 2; }
            int total = order == 0 ? (int)N : npairs;
            int pi = 0, pj = 1;
            for (int e = 0; e < total; ++e) {
                int i, j;
                if (order == 0) {
                    i = pi; j = pj;
                    if (++pj == n) { ++pi; pj = pi + 1; }
                } else {
                    i = pp[e]; j = qq[e];
                    if (j >= n) continue;
                }
                double *ci = C + (size_t)i * ldc, *cj = C + (size_t)j * ldc;
                double al = 0, be = 0, ga = 0;
                for (int t = 0; t < m; ++t) { al += ci[t] * ci[t]; be += cj[t] * cj[t]; ga += ci[t] * cj[t]; }
                if (!(fabs(ga) > m * 1.1102230246251565e-16 * sqrt(al * be))) continue;
                double c, s, t;
                or_d_angle(al, be, ga, &c, &s, &t);
                double tau = s / (1 + c);
                for (int k = 0; k < m; ++k) {
                    double x = ci[k], y = cj[k];
                    ci[k] = x - s * (y + tau * x);
                    cj[k] = y + s * (x - tau * y);
                }
                double *vi = V + (size_t)i * ldv, *vj = V + (size_t)j * ldv;
                for (int k = 0; k < n; ++k) {
                    double x = vi[k], y = vj[k];
                    vi[k] = x - s * (y + tau * x);
                    vj[k] = y + s * (x - tau * y);
                }
                ++applied;
            }
        }
        rot += applied;
        ++sweeps;
        if ((double)applied < ratio_stop * (double)N) { info = 0; break; }
    }
    free(pp); free(qq); free(G);
    if (sweeps_out) *sweeps_out = sweeps;
    if (rot_out) *rot_out = rot;
    return info;
}

/* Last three steps of Algorithm 5.2: reorder the columns of [C; V] so that
 * ||c_1|| >= ... >= ||c_n||, then sigma_j = ||c_j||, u_j = c_j / sigma_j. */
void or_svd_finish(int m, int n, const double *C, int ldc, const double *Vin, int ldvi,
                   double *S, double *U, int ldu, double *V, int ldv)
{
    double *nr = (double *)malloc(sizeof(double) * n);
    int *idx = (int *)malloc(sizeof(int) * n);
    for (int j = 0; j < n; ++j) {
        double a = 0;
        for (int i = 0; i < m; ++i) a += C[i + (size_t)j * ldc] * C[i + (size_t)j * ldc];
        nr[j] = sqrt(a);
        idx[j] = j;
    }
    for (int i = 1; i < n; ++i) {
        int v = idx[i], j = i - 1;
        while (j >= 0 && nr[idx[j]] < nr[v]) { idx[j + 1] = idx[j]; --j; }
        idx[j + 1] = v;
    }
    for (int k = 0; k < n; ++k) {
        int j = idx[k];
        S[k] = nr[j];
        for (int i = 0; i < m; ++i) U[i + (size_t)k * ldu] = C[i + (size_t)j * ldc] / nr[j];
        for (int i = 0; i < n; ++i) V[i + (size_t)k * ldv] = Vin[i + (size_t)j * ldvi];
    }
    free(nr); free(idx);
}
