/*
 * CPU oracle for the dense generalized Hermitian eigenproblem H C = eps S C
 * (the paper's Eq. (2), reduced to standard form by the three steps of its
 * section "Solving the generalized eigenproblem").
 *
 * TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  The GPU solver never includes, links or calls
 * anything here, and nothing here is shared with it.
 *
 * Plain C, FP64 throughout, OpenMP over independent rows/columns only.
 * Build: gcc -O2 -fopenmp -shared -fPIC oracle.c -o liboracle.so -lm
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_E_NONFINITE (-101)
#define ORACLE_E_NOCONV (-102)

static double oracle_now(void) { return omp_get_wtime(); }

int oracle_threads(void) { return omp_get_max_threads(); }

/* Symmetric tridiagonal eigenproblem by the implicit QL iteration with the
 * shift taken as the eigenvalue of the leading 2x2 block nearest to its top
 * diagonal entry (Bowdler, Martin, Reinsch, Wilkinson 1968).
 *
 * d[0..n-1]: diagonal, overwritten by the eigenvalues in ascending order.
 * e[0..n-1]: e[i] = T[i+1, i] for i < n-1; e[n-1] is scratch; destroyed.
 * z: if not NULL, n x n (ldz) receives the orthonormal eigenvectors as
 *    columns (it is initialised to the identity here).
 * A block is split where |e[i]| <= eps (|d[i]| + |d[i+1]|).  Returns 0, or
 * -1 when one eigenvalue needs more than 30 iterations. */
int oracle_tql(int n, double *d, double *e, double *z, int ldz)
{
    if (n <= 0) return 0;
    if (z) {
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) z[(size_t)i + (size_t)j * ldz] = (i == j) ? 1.0 : 0.0;
    }
    e[n - 1] = 0.0;
    for (int l = 0; l < n; ++l) {
        int iters = 0;
        for (;;) {
            int m = l;
            while (m < n - 1) {
                double scale = fabs(d[m]) + fabs(d[m + 1]);
                if (fabs(e[m]) <= DBL_EPSILON * scale) break;
                ++m;
            }
            if (m == l) break; /* d[l] has converged */
            if (++iters > 30) return -1;
            /* shift mu: eigenvalue of [[d_l, e_l], [e_l, d_{l+1}]] nearest d_l */
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            double mu = d[l] - e[l] / (g + copysign(r, g));
            /* chase from the bottom of the block [l, m] to its top */
            double sn = 1.0, cs = 1.0, p = 0.0;
            g = d[m] - mu;
            int restart = 0;
            for (int i = m - 1; i >= l; --i) {
                double f = sn * e[i];
                double b = cs * e[i];
                r = hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) { /* exact split inside the block */
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    restart = 1;
                    break;
                }
                sn = f / r;
                cs = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * sn + 2.0 * cs * b;
                p = sn * r;
                d[i + 1] = g + p;
                g = cs * r - b;
                if (z) {
                    double *zi = z + (size_t)i * ldz, *zi1 = z + (size_t)(i + 1) * ldz;
#pragma omp parallel for schedule(static) if (n >= 512)
                    for (int k = 0; k < n; ++k) {
                        double t = zi1[k];
                        zi1[k] = sn * zi[k] + cs * t;
                        zi[k] = cs * zi[k] - sn * t;
                    }
                }
            }
            if (restart) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    /* ascending order; eigenvector columns follow their eigenvalues */
    for (int i = 0; i < n - 1; ++i) {
        int kmin = i;
        for (int j = i + 1; j < n; ++j)
            if (d[j] < d[kmin]) kmin = j;
        if (kmin != i) {
            double t = d[i];
            d[i] = d[kmin];
            d[kmin] = t;
            if (z) {
                double *a = z + (size_t)i * ldz, *b = z + (size_t)kmin * ldz;
                for (int k = 0; k < n; ++k) {
                    double s = a[k];
                    a[k] = b[k];
                    b[k] = s;
                }
            }
        }
    }
    return 0;
}

/* Number of eigenvalues of the symmetric tridiagonal (d, e) that are
 * strictly below x: the count of negative pivots of the LDL^T
 * factorisation of T - x I (Sylvester's law of inertia). */
int oracle_sturm_count(int n, const double *d, const double *e, double x)
{
    double emax2 = 1.0;
    for (int i = 0; i + 1 < n; ++i)
        if (e[i] * e[i] > emax2) emax2 = e[i] * e[i];
    double pivmin = DBL_MIN * emax2;
    int count = 0;
    double q = 1.0;
    for (int i = 0; i < n; ++i) {
        double off2 = i > 0 ? e[i - 1] * e[i - 1] : 0.0;
        q = (d[i] - x) - (i > 0 ? off2 / q : 0.0);
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++count;
    }
    return count;
}

#include "oracle_core.inc"
#define ORACLE_COMPLEX
#include "oracle_core.inc"
#undef ORACLE_COMPLEX
