/*
 * tridiag.c -- plain FP64 reference of a tridiagonalization-based symmetric
 * eigensolver, the kind of solver the paper takes for the low-precision
 * step 1 of Algorithm 4.1.
 *
 * TEST INFRASTRUCTURE ONLY (the same rules as oracle.c): only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load this code; it
 * shares nothing with the GPU library.
 *
 * The paper's step 1 is a LAPACK-style FP32 eigensolver (ssyev / ssyevd on the
 * CPU, a cuSOLVER syevd on the GPU; Section 6 setup).  The analysis uses only
 * its backward stability (Lemma symeig).  Such a solver reduces A to
 * tridiagonal form by Householder similarity transforms, solves the
 * tridiagonal eigenproblem and transforms its eigenvectors back.  Each routine
 * below is the textbook form of one of those parts, in FP64, one element or one
 * vector at a time:
 *
 *   or_sytrd            Householder tridiagonalization A = Q T Q^T.  Column k
 *                       (k = 0 .. n-3) gets one reflector H_k = I - tau u u^T
 *                       with u(k+1) = 1 and u(i) = 0 for i <= k, chosen so that
 *                       H_k maps the entries below the diagonal of column k to
 *                       (beta, 0, ..., 0), beta = -sign(alpha) ||x|| where
 *                       x = A(k+1:n, k), alpha = x(0) (sign(0) = +1); when the
 *                       entries below the subdiagonal are already zero, tau = 0
 *                       (H_k = I) and beta = alpha.  The trailing block B is
 *                       replaced by H_k B H_k as the symmetric rank-2 update
 *                       B - u w^T - w u^T with p = tau B u and
 *                       w = p - (tau (p^T u) / 2) u.  Q = H_0 H_1 ... H_{n-3}.
 *   or_sturm_count      number of eigenvalues of T below x: the number of
 *                       negative pivots of the LDL^T factorization of T - x I
 *                       (Sylvester's law of inertia; Sturm sequence), with
 *                       pivots of magnitude below pivmin replaced by -pivmin.
 *   or_tridiag_eigvals  each eigenvalue by bisection on the Sturm count,
 *                       starting from the Gershgorin interval.
 *   or_tridiag_vector   an eigenvector by inverse iteration: three solves with
 *                       T - lambda I by Gaussian elimination with partial
 *                       pivoting, normalised after each.
 *   or_apply_reflectors Z = H_0 H_1 ... H_{n-3} Y, one reflector at a time
 *                       (H_{n-3} first).
 * Matrices are column-major.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

int or_sytrd(int n, const double *A0, int lda, double *d, double *e, double *tau, double *U, int ldu)
{
    if (n <= 0) return 0;
    double *A = malloc(sizeof(double) * (size_t)n * n);
    double *p = malloc(sizeof(double) * (size_t)n);
    double *w = malloc(sizeof(double) * (size_t)n);
    if (!A || !p || !w) { free(A); free(p); free(w); return -1; }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) A[i + (size_t)j * n] = A0[i + (size_t)j * lda];
    for (int k = 0; k < n; ++k) {
        tau[k] = 0.0;
        for (int i = 0; i < n; ++i) U[i + (size_t)k * ldu] = 0.0;
    }
    for (int k = 0; k + 2 < n; ++k) {
        const int r0 = k + 1;            /* first row of x and of the trailing block */
        const int m = n - r0;            /* length of x */
        double *x = A + r0 + (size_t)k * n;
        d[k] = A[k + (size_t)k * n];
        double alpha = x[0];
        double tail = 0.0;
        for (int i = 1; i < m; ++i) tail += x[i] * x[i];
        U[r0 + (size_t)k * ldu] = 1.0;
        if (tail == 0.0) {               /* already reduced: H_k = I */
            tau[k] = 0.0;
            e[k] = alpha;
            continue;
        }
        double r = sqrt(alpha * alpha + tail);
        double beta = alpha >= 0.0 ? -r : r;
        tau[k] = (beta - alpha) / beta;
        double scal = 1.0 / (alpha - beta);
        for (int i = 1; i < m; ++i) U[r0 + i + (size_t)k * ldu] = x[i] * scal;
        e[k] = beta;
        const double *u = U + r0 + (size_t)k * ldu;
        double t = tau[k];
        /* p = tau B u, B = A(r0:n, r0:n) */
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += A[r0 + i + (size_t)(r0 + j) * n] * u[j];
            p[i] = t * s;
        }
        double pu = 0.0;
        for (int i = 0; i < m; ++i) pu += p[i] * u[i];
        for (int i = 0; i < m; ++i) w[i] = p[i] - 0.5 * t * pu * u[i];
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i)
                A[r0 + i + (size_t)(r0 + j) * n] -= u[i] * w[j] + w[i] * u[j];
        /* column k (and row k) of the reduced matrix */
        x[0] = beta;
        for (int i = 1; i < m; ++i) x[i] = 0.0;
    }
    if (n >= 2) {
        d[n - 2] = A[(n - 2) + (size_t)(n - 2) * n];
        e[n - 2] = A[(n - 1) + (size_t)(n - 2) * n];
    }
    d[n - 1] = A[(n - 1) + (size_t)(n - 1) * n];
    free(A); free(p); free(w);
    return 0;
}

static double pivmin_of(int n, const double *e)
{
    double m = 1.0;
    for (int i = 0; i + 1 < n; ++i)
        if (e[i] * e[i] > m) m = e[i] * e[i];
    return DBL_MIN * m;
}

int or_sturm_count(int n, const double *d, const double *e, double x)
{
    const double pivmin = pivmin_of(n, e);
    int c = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++c;
    for (int i = 1; i < n; ++i) {
        q = (d[i] - x) - e[i - 1] * e[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0) ++c;
    }
    return c;
}

/* w(k) = the k-th smallest eigenvalue (k = 0 .. n-1). */
void or_tridiag_eigvals(int n, const double *d, const double *e, double *w)
{
    if (n <= 0) return;
    double gl = d[0], gu = d[0];
    for (int i = 0; i < n; ++i) {
        double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
        if (d[i] - r < gl) gl = d[i] - r;
        if (d[i] + r > gu) gu = d[i] + r;
    }
    double span = gu - gl;
    gl -= 2.0 * DBL_EPSILON * span + 1e-300;
    gu += 2.0 * DBL_EPSILON * span + 1e-300;
    for (int k = 0; k < n; ++k) {
        double lo = gl, hi = gu;
        for (int it = 0; it < 400; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;   /* no representable point in between */
            if (or_sturm_count(n, d, e, mid) <= k) lo = mid;
            else hi = mid;
        }
        w[k] = 0.5 * (lo + hi);
    }
}

/* Inverse iteration for the eigenvalue lam: z (length n, unit 2-norm). */
int or_tridiag_vector(int n, const double *d, const double *e, double lam, double *z)
{
    if (n <= 0) return 0;
    if (n == 1) { z[0] = 1.0; return 0; }
    double tnorm = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
        if (r > tnorm) tnorm = r;
    }
    double tiny = DBL_EPSILON * (tnorm > 0 ? tnorm : 1.0);
    double *U0 = malloc(sizeof(double) * n), *U1 = malloc(sizeof(double) * n);
    double *U2 = malloc(sizeof(double) * n), *L = malloc(sizeof(double) * n);
    int *piv = malloc(sizeof(int) * n);
    if (!U0 || !U1 || !U2 || !L || !piv) { free(U0); free(U1); free(U2); free(L); free(piv); return -1; }
    /* LU with partial pivoting of T - lam I: row i of U has entries in columns i, i+1, i+2 */
    double r0 = d[0] - lam, r1 = e[0], r2 = 0.0;
    for (int i = 0; i + 1 < n; ++i) {
        double s0 = e[i], s1 = d[i + 1] - lam, s2 = (i + 2 < n) ? e[i + 1] : 0.0;
        if (fabs(s0) > fabs(r0)) {
            double t0 = r0, t1 = r1, t2 = r2;
            r0 = s0; r1 = s1; r2 = s2;
            s0 = t0; s1 = t1; s2 = t2;
            piv[i] = 1;
        } else {
            piv[i] = 0;
        }
        if (r0 == 0.0) r0 = tiny;
        double mult = s0 / r0;
        L[i] = mult;
        U0[i] = r0; U1[i] = r1; U2[i] = r2;
        r0 = s1 - mult * r1;
        r1 = s2 - mult * r2;
        r2 = 0.0;
    }
    if (fabs(r0) < tiny) r0 = r0 < 0 ? -tiny : tiny;
    U0[n - 1] = r0; U1[n - 1] = 0.0; U2[n - 1] = 0.0;
    if (n >= 2) U2[n - 2] = 0.0;
    /* start vector: fixed, with no special relation to any eigenvector */
    for (int i = 0; i < n; ++i) z[i] = 1.0 + 0.5 * sin(1.0 + 0.37 * i);
    for (int it = 0; it < 3; ++it) {
        /* forward: the row operations of the factorization applied to z */
        double carry = z[0];
        for (int i = 0; i + 1 < n; ++i) {
            double other = z[i + 1];
            double pivot = carry;
            if (piv[i]) { pivot = other; other = carry; }
            z[i] = pivot;
            carry = other - L[i] * pivot;
        }
        z[n - 1] = carry;
        /* back substitution with U */
        for (int i = n - 1; i >= 0; --i) {
            double s = z[i];
            if (i + 1 < n) s -= U1[i] * z[i + 1];
            if (i + 2 < n) s -= U2[i] * z[i + 2];
            z[i] = s / U0[i];
        }
        double nrm = 0.0;
        for (int i = 0; i < n; ++i) nrm += z[i] * z[i];
        nrm = sqrt(nrm);
        for (int i = 0; i < n; ++i) z[i] /= nrm;
    }
    free(U0); free(U1); free(U2); free(L); free(piv);
    return 0;
}

/* Z = H_0 H_1 ... H_{n-3} Y in place (Y: n x ncol); U, tau as from or_sytrd. */
void or_apply_reflectors(int n, const double *U, int ldu, const double *tau, double *Y, int ldy, int ncol)
{
    for (int k = n - 3; k >= 0; --k) {
        if (tau[k] == 0.0) continue;
        const double *u = U + (size_t)k * ldu;
        for (int j = 0; j < ncol; ++j) {
            double *y = Y + (size_t)j * ldy;
            double s = 0.0;
            for (int i = k + 1; i < n; ++i) s += u[i] * y[i];
            s *= tau[k];
            for (int i = k + 1; i < n; ++i) y[i] -= s * u[i];
        }
    }
}
