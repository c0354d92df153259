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

// 1/sqrt(x) for x > 0: a single-precision start (the hardware reciprocal root
// on the device) refined by two Newton steps y <- y (3/2 - x y^2 / 2), which
// take its ~2^-23 relative error below double rounding.  Far-out x falls back
// to the plain root.
KRY_HD inline double rsqrt_refined(double x) {
    if (!(x > 1e-30 && x < 1e30)) return 1.0 / sqrt(x);
#if defined(__HIP_DEVICE_COMPILE__)
    double y = (double)__builtin_amdgcn_rsqf((float)x);
#else
    double y = (double)(1.0f / sqrtf((float)x));
#endif
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}

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
            // the first negligible coupling at or below l closes the active
            // block [l, mm]; checked 8 at a time so the loads go out together
            int mm = l;
            while (mm < m - 1) {
                int hit = -1;
#pragma unroll
                for (int u = 7; u >= 0; --u) {
                    const int q = mm + u;
                    const int qc = q < m - 1 ? q : m - 2;
                    const double dd = fabs(d[qc]) + fabs(d[qc + 1]);
                    if (q < m - 1 && fabs(e[qc]) <= eps * dd) hit = q;
                }
                if (hit >= 0) {
                    mm = hit;
                    break;
                }
                mm += 8;
            }
            if (mm > m - 1) mm = m - 1;
            if (mm == l) break;
            if (++iter > max_iter) return false;
            // shift: the eigenvalue of the leading 2 x 2 block nearer d[l]
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[mm] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            bool split = false;
            // The chase runs from i = mm - 1 down to l.  Step i reads e[i],
            // d[i], d[i+1] (not yet changed) and rows 1 and m at i; it
            // writes e[i+1], d[i+1] and the rows at i+1.  The rows' entry
            // at i+1 is carried in a register from the step before, and
            // step i-1's inputs are loaded during step i.
            double q1c = q1[mm], qmc = qm[mm];
            double ei = e[mm - 1], di = d[mm - 1], dn = d[mm], q1i = q1[mm - 1], qmi = qm[mm - 1];
            for (int i = mm - 1; i >= l; --i) {
                const int ip = i - 1 >= l ? i - 1 : i;      // prefetch index (a harmless reload at the end)
                const double e_nx = e[ip], d_nx = d[ip], q1_nx = q1[ip], qm_nx = qm[ip];
                const double f = s * ei;
                const double b = c * ei;
                // |f|, |g| are of the size of T's entries here, so f^2 + g^2
                // neither overflows nor loses range; one refined reciprocal
                // root gives r, s and c (a root plus a division would double
                // this dependent chain, which is the solver's latency)
                const double x = fma(f, f, g * g);
                if (x == 0.0) {            // underflow: the block splits here
                    e[i + 1] = 0.0;
                    d[i + 1] = dn - p;
                    q1[i + 1] = q1c;
                    qm[i + 1] = qmc;
                    e[mm] = 0.0;
                    split = true;
                    break;
                }
                const double inv = rsqrt_refined(x);
                e[i + 1] = x * inv;
                s = f * inv;
                c = g * inv;
                g = dn - p;
                r = (di - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                // columns i and i+1 of the eigenvector matrix, rows 1 and m
                q1[i + 1] = s * q1i + c * q1c;
                q1c = c * q1i - s * q1c;
                qm[i + 1] = s * qmi + c * qmc;
                qmc = c * qmi - s * qmc;
                dn = di;                   // d[i] is step i-1's d[i+1], unchanged so far
                ei = e_nx;
                di = d_nx;
                q1i = q1_nx;
                qmi = qm_nx;
            }
            if (split) continue;
            q1[l] = q1c;
            qm[l] = qmc;
            d[l] -= p;
            e[l] = g;
            e[mm] = 0.0;
        }
    }
    return true;
}

}  // namespace kry
