/*
 * CPU FP64 ORACLE -- test infrastructure only (see oracle.h).
 *
 * Dense symmetric-indefinite LDL^T with Bunch-Kaufman partial pivoting
 * (Bunch & Kaufman 1977, alpha = (1 + sqrt 17)/8, lowest index on ties).  The
 * paper factors the augmented KKT matrix of eq. (7) with an LDL^T that also
 * reports the inertia (n_+, n_-, n_0), Sec. IV "Step direction"; this is the
 * plain unblocked textbook form of that factorization, with the inertia taken
 * from the 1x1 and 2x2 pivot blocks (Sylvester's law of inertia).  Only the
 * lower triangle of the row-major matrix is read or written.
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

#define AT(i, j) A[(size_t)(i) * n + (j)]
/* symmetric element (i, j) through the lower triangle */
#define SYM(i, j) ((i) >= (j) ? AT(i, j) : AT(j, i))

static void swap_d(double* a, double* b) { double t = *a; *a = *b; *b = t; }

/* symmetric interchange of rows/columns a < b, lower-triangle storage */
static void sym_swap(int n, double* A, int a, int b) {
    if (a == b) return;
    if (a > b) { int t = a; a = b; b = t; }
    for (int j = 0; j < a; ++j) swap_d(&AT(a, j), &AT(b, j));
    for (int j = a + 1; j < b; ++j) swap_d(&AT(j, a), &AT(b, j));
    for (int j = b + 1; j < n; ++j) swap_d(&AT(j, a), &AT(j, b));
    swap_d(&AT(a, a), &AT(b, b));
}

static void count_1x1(double d, int inertia[3]) {
    if (d > 0) inertia[0]++;
    else if (d < 0) inertia[1]++;
    else inertia[2]++;
}

int bk_factor(int n, double* A, int* perm, int* blk, int inertia[3]) {
    const double alpha = (1.0 + sqrt(17.0)) / 8.0;
    inertia[0] = inertia[1] = inertia[2] = 0;
    for (int k = 0; k < n; ++k) perm[k] = k;
    int k = 0;
    while (k < n) {
        double akk = fabs(AT(k, k));
        int r = -1;
        double colmax = 0.0;
        for (int i = k + 1; i < n; ++i) {
            double v = fabs(AT(i, k));
            if (v > colmax) { colmax = v; r = i; }
        }
        if (akk == 0.0 && colmax == 0.0) {          /* zero column: exact zero pivot */
            blk[k] = 1;
            inertia[2]++;
            k += 1;
            continue;
        }
        int size = 1, kp = k;
        if (akk < alpha * colmax) {
            double rowmax = 0.0;                     /* off-diagonal max of row/column r */
            for (int j = k; j < n; ++j)
                if (j != r) { double v = fabs(SYM(r, j)); if (v > rowmax) rowmax = v; }
            if (akk * rowmax >= alpha * colmax * colmax) {
                kp = k;
            } else if (fabs(AT(r, r)) >= alpha * rowmax) {
                kp = r;
            } else {
                size = 2;
                kp = r;
            }
        }
        if (size == 1) {
            sym_swap(n, A, k, kp);
            { int t = perm[k]; perm[k] = perm[kp]; perm[kp] = t; }
            double d = AT(k, k);
            blk[k] = 1;
            count_1x1(d, inertia);
            if (d != 0.0) {
                /* trailing update A_ij -= A_ik A_jk / d, then scale the column */
                for (int i = k + 1; i < n; ++i) {
                    double li = AT(i, k) / d;
                    if (li == 0.0) continue;
                    for (int j = k + 1; j <= i; ++j) AT(i, j) -= li * AT(j, k);
                }
                for (int i = k + 1; i < n; ++i) AT(i, k) /= d;
            }
            k += 1;
        } else {
            sym_swap(n, A, k + 1, kp);
            { int t = perm[k + 1]; perm[k + 1] = perm[kp]; perm[kp] = t; }
            double a = AT(k, k), b = AT(k + 1, k), c = AT(k + 1, k + 1);
            double det = a * c - b * b;
            blk[k] = 2;
            blk[k + 1] = 0;
            if (det < 0) { inertia[0]++; inertia[1]++; }
            else if (det > 0) { if (a + c > 0) inertia[0] += 2; else inertia[1] += 2; }
            else { inertia[2]++; count_1x1(a + c, inertia); }
            if (det != 0.0) {
                /* trailing update A_ij -= [A_ik A_ik1] D^{-1} [A_jk A_jk1]^T */
                for (int i = k + 2; i < n; ++i) {
                    double u = AT(i, k), v = AT(i, k + 1);
                    double l0 = (c * u - b * v) / det;
                    double l1 = (a * v - b * u) / det;
                    for (int j = k + 2; j <= i; ++j) AT(i, j) -= l0 * AT(j, k) + l1 * AT(j, k + 1);
                }
                /* L rows: [l_i0 l_i1] = [A_ik A_ik1] D^{-1} */
                for (int i = k + 2; i < n; ++i) {
                    double u = AT(i, k), v = AT(i, k + 1);
                    AT(i, k) = (c * u - b * v) / det;
                    AT(i, k + 1) = (a * v - b * u) / det;
                }
            }
            k += 2;
        }
    }
    return 0;
}

void bk_solve(int n, const double* A, const int* perm, const int* blk, double* b, double* w) {
    /* P A P^T = L D L^T ;  A x = b  <=>  L D L^T (P x) = P b */
    for (int i = 0; i < n; ++i) w[i] = b[perm[i]];
    /* forward: L z = w (L unit lower; a 2x2 block's sub-diagonal entry belongs to D) */
    for (int k = 0; k < n;) {
        int s = blk[k] == 2 ? 2 : 1;
        for (int i = k + s; i < n; ++i) {
            w[i] -= AT(i, k) * w[k];
            if (s == 2) w[i] -= AT(i, k + 1) * w[k + 1];
        }
        k += s;
    }
    /* block diagonal */
    for (int k = 0; k < n;) {
        if (blk[k] == 2) {
            double a = AT(k, k), bb = AT(k + 1, k), c = AT(k + 1, k + 1);
            double det = a * c - bb * bb;
            double u = w[k], v = w[k + 1];
            w[k] = det != 0.0 ? (c * u - bb * v) / det : 0.0;
            w[k + 1] = det != 0.0 ? (a * v - bb * u) / det : 0.0;
            k += 2;
        } else {
            double d = AT(k, k);
            w[k] = d != 0.0 ? w[k] / d : 0.0;
            k += 1;
        }
    }
    /* backward: L^T y = z */
    for (int k = n - 1; k >= 0;) {
        int first = (blk[k] == 0) ? k - 1 : k;
        int s = (blk[first] == 2) ? 2 : 1;
        for (int c = first; c < first + s; ++c) {
            double acc = w[c];
            for (int i = first + s; i < n; ++i) acc -= AT(i, c) * w[i];
            w[c] = acc;
        }
        k = first - 1;
    }
    for (int i = 0; i < n; ++i) b[perm[i]] = w[i];
}
