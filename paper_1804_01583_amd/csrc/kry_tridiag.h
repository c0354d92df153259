// Eigenvalues of a symmetric tridiagonal matrix and the first and last
// components of its eigenvectors, by the implicit QL iteration with a
// Wilkinson shift (deflating from the top; Givens rotations chase the bulge
// up from the bottom of the active block).  Only two rows of the
// eigenvector matrix are carried, so the cost is O(m) per sweep.  Used by
// the error bound of Lemma 1, which needs (e^{tT})_{m,1} = sum_i q_{m,i}
// q_{1,i} e^{theta_i t}.  Callable from host and device code.
#pragma once

#include <cmath>

#if defined(__HIPCC__)
#define KRY_HD __host__ __device__
#else
#define KRY_HD
#endif

namespace kry {

// d[0..m-1]: diagonal in, eigenvalues out.  e[0..m-1]: e[i] couples rows i
// and i+1 (e[m-1] is scratch).  q1, qm: on return the first and last row of
// the orthogonal eigenvector matrix.  Returns false when a block needs more
// than max_iter sweeps.
KRY_HD inline bool tridiag_eig_rows(int m, double* d, double* e, double* q1, double* qm, int max_iter = 64) {
    for (int i = 0; i < m; ++i) {
        q1[i] = i == 0 ? 1.0 : 0.0;
        qm[i] = i == m - 1 ? 1.0 : 0.0;
    }
    if (m <= 0) return true;
    e[m - 1] = 0.0;
    const double eps = 2.220446049250313e-16;
    for (int l = 0; l < m; ++l) {
        int iter = 0;
        while (true) {
            // the first negligible coupling at or below l closes the active block [l, mm]
            int mm = l;
            for (; mm < m - 1; ++mm) {
                const double dd = fabs(d[mm]) + fabs(d[mm + 1]);
                if (fabs(e[mm]) <= eps * dd) break;
            }
            if (mm == l) break;
            if (++iter > max_iter) return false;
            // shift: the eigenvalue of the leading 2 x 2 block nearer d[l]
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[mm] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = mm - 1;
            bool split = false;
            for (; i >= l; --i) {
                const double f = s * e[i];
                const double b = c * e[i];
                r = hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {            // underflow: the block splits here
                    d[i + 1] -= p;
                    e[mm] = 0.0;
                    split = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                // columns i and i+1 of the eigenvector matrix, rows 1 and m
                double t = q1[i + 1];
                q1[i + 1] = s * q1[i] + c * t;
                q1[i] = c * q1[i] - s * t;
                t = qm[i + 1];
                qm[i + 1] = s * qm[i] + c * t;
                qm[i] = c * qm[i] - s * t;
            }
            if (split) continue;
            d[l] -= p;
            e[l] = g;
            e[mm] = 0.0;
        }
    }
    return true;
}

}  // namespace kry
