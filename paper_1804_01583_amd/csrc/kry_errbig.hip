// Lemma 1's integrand for Lanczos runs at large Krylov dimension (paper
// Section 4.2; the checks of Algorithm 4), without the serial QL sweep of
// kry_errctl.hip: the eigenvalues theta_i of T_m by bisection with Sturm
// counts, one lane per eigenvalue, and the first and last components of each
// unit eigenvector by the twisted factorisation of T_m - theta_i I (the
// top-down pivots dp, the bottom-up pivots dm, the twist index r where
// |gamma_r| = |dp_r + dm_r - (a_r - theta)| is least, z_r = 1 and the two
// one-sided recurrences), one lane per eigenvalue again.  Then
//     (e^{t T_m})_{m,1} = sum_i q_{1,i} q_{m,i} e^{theta_i t}
// at the nodes of the composite rule, as in kry_errctl.hip.  Every step is
// O(m) per eigenvalue and the eigenvalues are independent, so the work
// spreads over the chip instead of one lane.
//
// The sums along the recurrences are kept as ratios to the current
// component, W_i = z_0 / z_i and Y_i = sum_{l <= i} (z_l / z_i)^2 (forward),
// U_t = z_{m-1} / z_t and V_t = sum_{l >= t} (z_l / z_t)^2 (backward), so the
// unit vector's end components are z_0 = W_r, z_{m-1} = U_r with
// |z|^2 = Y_r + V_r - 1.  A non-finite weight (an eigenvector with a valley
// deeper than the double range between its end and its peak) makes the
// bound infinite: that checkpoint does not stop the run.
#include "kry_device.h"

#include <cfloat>
#include <cmath>

namespace kry {

namespace {

using namespace dev;

constexpr int kQuadLevels = 40;
constexpr int kQuadSplit = 8;
constexpr int kQuadNodes = (kQuadLevels + 1) * kQuadSplit * 8;
constexpr int kBigThreads = 256;

__device__ __forceinline__ const double* run_sc(const BatchArgs& B, int p) {
    return B.scal + (int64_t)(B.run0 + p) * B.L.stride;
}

// Same state rules as k_lemma1 (kry_errctl.hip): 0 evaluate, 1 stopped,
// 2 exact (breakdown), 4 past the augmented run's cap.
__device__ __forceinline__ int big_state(const BatchArgs& B, const ErrArgs& X, const double* sc, int p, int j) {
    if (sc[B.L.misc + MISC_STOPPED] != 0.0) return 1;
    if ((int)sc[B.L.misc + MISC_KEFF] <= j) return 2;
    if (X.role[B.run0 + p] == 2 && j > B.L.k - 1) return 4;
    return 0;
}

__device__ __forceinline__ bool all_done(const ErrArgs& X, int P) {
    bool all = true;
    for (int q = 0; q < P; ++q) all = all && X.flags[q] != 0.0;
    return all;
}

__device__ __forceinline__ double diag_of(const BatchArgs& B, const ErrArgs& X, const double* sc, int i) {
    return X.hess ? sc[B.L.hess + i * B.L.k + i] : sc[B.L.alpha + i + 1];
}

// Sturm count: eigenvalues of T (diagonal a, squared off-diagonal b2) below x
__device__ __forceinline__ int sturm_below(const double* a, const double* b2, int m, double x, double pivmin) {
    double d = a[0] - x;
    if (fabs(d) < pivmin) d = -pivmin;
    int cnt = d < 0.0 ? 1 : 0;
    for (int i = 1; i < m; ++i) {
        d = (a[i] - x) - b2[i - 1] / d;
        if (fabs(d) < pivmin) d = -pivmin;
        cnt += d < 0.0 ? 1 : 0;
    }
    return cnt;
}

// T of run p staged in LDS: a[0..m), b2[0..m-1) (squares of the off-diagonal)
__device__ __forceinline__ void stage_t(const BatchArgs& B, const ErrArgs& X, const double* sc, int m, double* a,
                                        double* b2) {
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        a[i] = diag_of(B, X, sc, i);
        const double b = i + 1 < m ? sc[B.L.beta + i + 1] : 0.0;
        b2[i] = b * b;
    }
    __syncthreads();
}

// Grid (ceil(m / kBigThreads), P): theta[p][i], the i-th smallest eigenvalue
// of T_m, by 64 bisection steps from the Gershgorin interval.
__global__ __launch_bounds__(kBigThreads) void k_big_bisect(BatchArgs B, ErrArgs X, int m, BigErrArgs G) {
    extern __shared__ double lds[];
    const int p = blockIdx.y;
    if (all_done(X, (int)gridDim.y)) return;
    const double* sc = run_sc(B, p);
    if (big_state(B, X, sc, p, m) != 0) return;
    double* a = lds;
    double* b2 = lds + m;
    stage_t(B, X, sc, m, a, b2);
    // Gershgorin interval and the pivot floor (as LAPACK's bisection takes it)
    __shared__ double s_lo, s_hi, s_piv;
    if (threadIdx.x == 0) {
        double lo = INFINITY, hi = -INFINITY, bmax = 0.0;
        for (int i = 0; i < m; ++i) {
            const double r = (i > 0 ? sqrt(b2[i - 1]) : 0.0) + (i + 1 < m ? sqrt(b2[i]) : 0.0);
            lo = fmin(lo, a[i] - r);
            hi = fmax(hi, a[i] + r);
            if (i + 1 < m) bmax = fmax(bmax, b2[i]);
        }
        const double w = fmax(hi - lo, DBL_MIN);
        s_lo = lo - 2.0 * DBL_EPSILON * w;
        s_hi = hi + 2.0 * DBL_EPSILON * w;
        s_piv = DBL_MIN * fmax(1.0, bmax);
    }
    __syncthreads();
    const int i = blockIdx.x * kBigThreads + threadIdx.x;
    if (i >= m) return;
    double lo = s_lo, hi = s_hi;
    for (int it = 0; it < 64; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_below(a, b2, m, mid, s_piv) > i) hi = mid;
        else lo = mid;
    }
    G.theta[(int64_t)p * G.ld + i] = 0.5 * (lo + hi);
}

// Grid (ceil(nc / kBigThreads), P) for eigenvalues i0 .. i0 + nc - 1:
// w[p][i] = q_{1,i} q_{m,i} by the twisted factorisation; dp kept in
// G.work[p][t][i - i0] (step-major, so a wavefront's lanes read one line).
__global__ __launch_bounds__(kBigThreads) void k_big_ends(BatchArgs B, ErrArgs X, int m, BigErrArgs G, int i0,
                                                          int nc) {
    extern __shared__ double lds[];
    const int p = blockIdx.y;
    if (all_done(X, (int)gridDim.y)) return;
    const double* sc = run_sc(B, p);
    if (big_state(B, X, sc, p, m) != 0) return;
    double* a = lds;
    double* b2 = lds + m;
    stage_t(B, X, sc, m, a, b2);
    const int li = blockIdx.x * kBigThreads + threadIdx.x;
    if (li >= nc) return;
    const int i = i0 + li;
    const double lam = G.theta[(int64_t)p * G.ld + i];
    const double piv = DBL_MIN * 4.0;
    double* dp = G.work + (int64_t)p * G.ld * G.chunk;
    auto at = [&](int t) -> double& { return dp[(int64_t)t * G.chunk + li]; };
    // top-down pivots of T - lam I
    double d = a[0] - lam;
    if (fabs(d) < piv) d = -piv;
    at(0) = d;
    for (int t = 1; t < m; ++t) {
        d = (a[t] - lam) - b2[t - 1] / d;
        if (fabs(d) < piv) d = -piv;
        at(t) = d;
    }
    // bottom-up pivots, the twist index, U_t and V_t at the best index
    double dm = a[m - 1] - lam;
    if (fabs(dm) < piv) dm = -piv;
    double U = 1.0, V = 1.0;
    int r = m - 1;
    double best = fabs(at(m - 1) + dm - (a[m - 1] - lam));
    double Ur = U, Vr = V;
    for (int t = m - 1; t >= 1; --t) {
        // step from t to t - 1: c = -b_{t-1} / dm_t
        const double c = -sqrt(b2[t - 1]) / dm;
        U *= c;
        V = c * c * V + 1.0;
        dm = (a[t - 1] - lam) - b2[t - 1] / dm;
        if (fabs(dm) < piv) dm = -piv;
        const double g = fabs(at(t - 1) + dm - (a[t - 1] - lam));
        if (g < best) {
            best = g;
            r = t - 1;
            Ur = U;
            Vr = V;
        }
    }
    // W_r = z_0 / z_r and Y_r from the top: c = -b_t / dp_t for t < r
    double W = 1.0, Y = 1.0;
    for (int t = 0; t < r; ++t) {
        const double c = -sqrt(b2[t]) / at(t);
        W *= c;
        Y = c * c * Y + 1.0;
    }
    const double nz2 = Y + Vr - 1.0;
    double w = W * Ur / nz2;
    if (!isfinite(w)) w = __builtin_nan("");
    G.w[(int64_t)p * G.ld + i] = w;
}

// One workgroup per run: the integral over the composite rule of
// |sum_i w_i e^{theta_i t}|, the bound and the stop, as k_lemma1 does.
__global__ __launch_bounds__(kBigThreads) void k_big_integral(BatchArgs B, ErrArgs X, int m, BigErrArgs G) {
    __shared__ double s_red[kBigThreads / 64];
    const int p = blockIdx.x;
    if (all_done(X, (int)gridDim.x)) return;
    double* sc = B.scal + (int64_t)(B.run0 + p) * B.L.stride;
    const int st = big_state(B, X, sc, p, m);
    if (st != 0) {
        if (threadIdx.x == 0) {
            if (st == 2) {
                sc[B.L.misc + MISC_BOUND] = 0.0;
                sc[B.L.misc + MISC_STOPPED] = 1.0;
                sc[B.L.misc + MISC_KSTOP] = sc[B.L.misc + MISC_KEFF];
            }
            X.flags[p] = 1.0;
        }
        return;
    }
    const bool affine = X.role[B.run0 + p] == 2;
    const double* th = G.theta + (int64_t)p * G.ld;
    const double* wv = G.w + (int64_t)p * G.ld;
    const double tau = X.tau;
    double acc = 0.0;
    for (int idx = threadIdx.x; idx < kQuadNodes; idx += kBigThreads) {
        const int g = idx % 8;
        const int part = (idx / 8) % kQuadSplit;
        const int lev = idx / (8 * kQuadSplit);
        const double a0 = lev == 0 ? 0.0 : tau * ldexp(1.0, -(kQuadLevels - lev + 1));
        const double b0 = tau * ldexp(1.0, -(kQuadLevels - lev));
        const double h = (b0 - a0) / kQuadSplit;
        const double lo = a0 + part * h;
        const double t = lo + 0.5 * h * (X.gl_x[g] + 1.0);
        double v = 0.0;
        for (int i = 0; i < m; ++i) v = fma(wv[i], exp(th[i] * t), v);
        double wgt = 0.5 * h * X.gl_w[g];
        if (affine) wgt *= tau - t;
        acc = fma(wgt, fabs(v), acc);
    }
    double vals[1] = {acc};
    const double integral = block_sum<1>(vals, s_red);
    if (threadIdx.x == 0) {
        const double bound = isfinite(integral) ? sc[B.L.beta + m] * exp(X.lam_plus * tau) * integral : INFINITY;
        sc[B.L.misc + MISC_BOUND] = bound;
        const bool stop = bound < X.eps;
        if (stop) {
            sc[B.L.misc + MISC_STOPPED] = 1.0;
            sc[B.L.misc + MISC_KSTOP] = (double)m;
        }
        X.flags[p] = stop ? 1.0 : 0.0;
    }
}

}  // namespace

size_t big_lds_bytes(int m) { return (size_t)2 * m * sizeof(double); }

hipError_t big_prepare() {
    const int bytes = (int)big_lds_bytes(kMaxKP);
    hipError_t e = hipFuncSetAttribute((const void*)k_big_bisect, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_big_ends, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e;
}

hipError_t launch_lemma1_big(int P, const BatchArgs& B, const ErrArgs& X, int j, const BigErrArgs& G, hipStream_t s) {
    if (j < 1 || j > G.ld || P < 1 || P > kMaxP) return hipErrorInvalidValue;
    const size_t lds = big_lds_bytes(j);
    const unsigned nb = (unsigned)((j + kBigThreads - 1) / kBigThreads);
    hipLaunchKernelGGL(k_big_bisect, dim3(nb, P), dim3(kBigThreads), lds, s, B, X, j, G);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int i0 = 0; i0 < j; i0 += G.chunk) {
        const int nc = j - i0 < G.chunk ? j - i0 : G.chunk;
        const unsigned nbc = (unsigned)((nc + kBigThreads - 1) / kBigThreads);
        hipLaunchKernelGGL(k_big_ends, dim3(nbc, P), dim3(kBigThreads), lds, s, B, X, j, G, i0, nc);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_big_integral, dim3(P), dim3(kBigThreads), 0, s, B, X, j, G);
    return hipGetLastError();
}

}  // namespace kry
