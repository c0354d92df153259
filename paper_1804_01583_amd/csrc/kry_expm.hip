// Small dense stage on gfx950: e^{H t} e_1 for every time step (paper
// Section 4.2, Eq. approx-formula), the basis matrix of Section 3.2 and the
// per-step box check that stands in for the LP of Section 2.1.
//
// For the symmetric tridiagonal H of Lanczos, H = Q diag(theta) Q^T is
// computed once per run by a parallel cyclic Jacobi method (Golub & Van Loan,
// Matrix Computations, Sec. 8.5: symmetric 2x2 Schur rotations applied to
// disjoint pairs chosen by a round-robin ordering), held in LDS by one
// workgroup.  Then every step is independent:
//   generator / center run:  y_s = beta0 * P Q diag(e^{theta s dt}) Q^T e_1
//   augmented run [0;1]:     H~ = [[0, 0], [|b| e_1, T]] gives
//                            y_s = |b| * P Q diag((e^{theta t} - 1)/theta) Q^T e_1
// so no step depends on the previous one and no error accumulates over steps.
#include "kry_internal.h"

#include <cmath>

namespace kry {

namespace {

constexpr int kLd = kMaxK + 1;   // padded LDS row length

__device__ __forceinline__ double* run_scal(const ExpmArgs& E, int r) {
    return E.scal + (int64_t)r * E.L.stride;
}

// One workgroup per run.
__global__ __launch_bounds__(kBlock) void k_eig_coeffs(ExpmArgs E) {
    __shared__ double A[kMaxK * kLd];
    __shared__ double Q[kMaxK * kLd];
    __shared__ double s_c[kMaxK / 2], s_s[kMaxK / 2];
    __shared__ int s_p[kMaxK / 2], s_q[kMaxK / 2];
    __shared__ double s_red[2 * (kBlock / 64)];
    __shared__ int s_stop;

    const int run = blockIdx.x;
    const double* sc = run_scal(E, run);
    const int k = E.L.k, o = E.L.o;
    const int keff = (int)sc[E.L.misc + MISC_KEFF];
    int m = keff;
    if (E.role[run] == 2 && m > k - 1) m = k - 1;   // augmented run: k-1 Lanczos steps + border
    if (threadIdx.x == 0) E.msize[run] = m;
    if (m <= 0) return;
    const int mm = m + (m & 1);        // even size for the round-robin pairing
    const int half = mm / 2;
    const int tid = threadIdx.x;

    for (int idx = tid; idx < mm * mm; idx += kBlock) {
        const int i = idx / mm, c = idx % mm;
        double a = 0.0;
        if (i < m && c < m) {
            if (i == c) a = sc[E.L.alpha + i + 1];
            else if (c == i + 1) a = sc[E.L.beta + i + 1];
            else if (i == c + 1) a = sc[E.L.beta + c + 1];
        }
        A[i * kLd + c] = a;
        Q[i * kLd + c] = (i == c) ? 1.0 : 0.0;
    }
    __syncthreads();

    const double eps = 2.220446049250313e-16;
    const int N = mm - 1;              // rotating players 0..N-1, fixed player N
    for (int sweep = 0; sweep < 60; ++sweep) {
        // convergence: off(A) <= eps * |A|_F
        double v[2] = {0.0, 0.0};
        for (int idx = tid; idx < mm * mm; idx += kBlock) {
            const int i = idx / mm, c = idx % mm;
            const double a = A[i * kLd + c];
            v[1] = fma(a, a, v[1]);
            if (i != c) v[0] = fma(a, a, v[0]);
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            v[0] += __shfl_xor(v[0], off, 64);
            v[1] += __shfl_xor(v[1], off, 64);
        }
        if ((tid & 63) == 0) { s_red[2 * (tid >> 6)] = v[0]; s_red[2 * (tid >> 6) + 1] = v[1]; }
        __syncthreads();
        if (tid == 0) {
            double off2 = 0.0, fro2 = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) { off2 += s_red[2 * w]; fro2 += s_red[2 * w + 1]; }
            s_stop = (off2 <= eps * eps * fro2) ? 1 : 0;
        }
        __syncthreads();
        if (s_stop) break;

        for (int round = 0; round < N; ++round) {
            if (tid < half) {
                int p, q;
                if (tid == 0) { p = round; q = N; }
                else { p = (round + tid) % N; q = (round - tid + N) % N; }
                if (p > q) { const int t = p; p = q; q = t; }
                const double apq = A[p * kLd + q];
                double c = 1.0, s = 0.0;
                if (apq != 0.0) {
                    const double tau = (A[q * kLd + q] - A[p * kLd + p]) / (2.0 * apq);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                s_p[tid] = p; s_q[tid] = q; s_c[tid] = c; s_s[tid] = s;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int idx = tid; idx < half * mm; idx += kBlock) {
                const int pr = idx / mm, x = idx % mm;
                const int p = s_p[pr], q = s_q[pr];
                const double c = s_c[pr], s = s_s[pr];
                const double ap = A[p * kLd + x], aq = A[q * kLd + x];
                A[p * kLd + x] = c * ap - s * aq;
                A[q * kLd + x] = s * ap + c * aq;
            }
            __syncthreads();
            // columns: A <- A J, Q <- Q J
            for (int idx = tid; idx < half * mm; idx += kBlock) {
                const int pr = idx / mm, x = idx % mm;
                const int p = s_p[pr], q = s_q[pr];
                const double c = s_c[pr], s = s_s[pr];
                const double ap = A[x * kLd + p], aq = A[x * kLd + q];
                A[x * kLd + p] = c * ap - s * aq;
                A[x * kLd + q] = s * ap + c * aq;
                const double qp = Q[x * kLd + p], qq = Q[x * kLd + q];
                Q[x * kLd + p] = c * qp - s * qq;
                Q[x * kLd + q] = s * qp + c * qq;
            }
            __syncthreads();
            if (tid < half) {
                const int p = s_p[tid], q = s_q[tid];
                A[p * kLd + q] = 0.0;
                A[q * kLd + p] = 0.0;
            }
            __syncthreads();
        }
    }

    // theta_i and coef[q][i] = beta0 * (P Q)[q,i] * Q[0,i]
    const double beta0 = sc[E.L.beta + 0];
    double* theta = E.theta + (int64_t)run * k;
    double* coef = E.coef + (int64_t)run * o * k;
    for (int i = tid; i < m; i += kBlock) theta[i] = A[i * kLd + i];
    for (int idx = tid; idx < o * m; idx += kBlock) {
        const int q = idx / m, i = idx % m;
        const double* Prow = sc + E.L.proj + q * (k + 1);
        double s = 0.0;
        for (int l = 0; l < m; ++l) s = fma(Prow[l], Q[l * kLd + i], s);
        coef[q * k + i] = beta0 * s * Q[0 * kLd + i];
    }
}

// basis[s][q][run] = sum_i coef[q][i] f(theta_i, s dt), one thread per (s, run)
__global__ __launch_bounds__(kBlock) void k_assemble(AssembleArgs A) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (A.steps + 1) * A.nruns;
    if (idx >= total) return;
    const int64_t s = idx / A.nruns;
    const int run = (int)(idx % A.nruns);
    const int m = A.msize[run];
    const double t = (double)s * A.dt;
    const bool bordered = A.role[run] == 2;
    const double* theta = A.theta + (int64_t)run * A.k;
    const double* coef = A.coef + (int64_t)run * A.o * A.k;
    double y[kMaxO];
#pragma unroll
    for (int q = 0; q < kMaxO; ++q) y[q] = 0.0;
    for (int i = 0; i < m; ++i) {
        const double th = theta[i];
        double f;
        if (bordered) f = (th != 0.0) ? expm1(th * t) / th : t;
        else f = exp(th * t);
#pragma unroll
        for (int q = 0; q < kMaxO; ++q)
            if (q < A.o) y[q] = fma(coef[q * A.k + i], f, y[q]);
    }
#pragma unroll
    for (int q = 0; q < kMaxO; ++q)
        if (q < A.o) A.basis[(s * A.o + q) * A.nruns + run] = y[q];
}

// a9: first violated (step, row) and its counter-example.  One workgroup.
__global__ __launch_bounds__(kBlock) void k_check(CheckArgs C) {
    __shared__ long long s_min[kBlock / 64];
    __shared__ int s_bad[kBlock / 64];
    const int64_t total = (C.steps + 1) * C.o;
    long long best = total;
    int bad = 0;
    for (int64_t e = threadIdx.x; e < total; e += kBlock) {
        const int64_t s = e / C.o;
        const int q = (int)(e % C.o);
        const double* M = C.basis + (s * C.o + q) * C.nruns;
        double mid = 0.0, rad = 0.0;
        for (int r = 0; r < C.nruns; ++r) {
            mid = fma(M[r], C.zc[r], mid);
            rad = fma(fabs(M[r]), C.radius[r], rad);
        }
        if (!isfinite(mid) || !isfinite(rad)) { bad = 1; continue; }
        const bool hit = (mid - rad <= C.uhi[q]) && (mid + rad >= C.ulo[q]);
        if (hit && e < best) best = e;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const long long o2 = __shfl_xor(best, off, 64);
        best = o2 < best ? o2 : best;
        bad |= __shfl_xor(bad, off, 64);
    }
    if ((threadIdx.x & 63) == 0) { s_min[threadIdx.x >> 6] = best; s_bad[threadIdx.x >> 6] = bad; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 1; w < kBlock / 64; ++w) {
        best = s_min[w] < best ? s_min[w] : best;
        bad |= s_bad[w];
    }
    best = s_min[0] < best ? s_min[0] : best;
    bad |= s_bad[0];
    double* out = C.verdict;
    out[5] = bad ? 4.0 : 0.0;    // KRY_ENUMERIC
    if (best >= total) {
        out[0] = -1.0; out[1] = -1.0; out[2] = 0.0; out[3] = 0.0; out[4] = 0.0;
        for (int r = 0; r < C.nruns; ++r) out[6 + r] = C.zc[r];
        return;
    }
    const int64_t s = best / C.o;
    const int q = (int)(best % C.o);
    const double* M = C.basis + (s * C.o + q) * C.nruns;
    double mid = 0.0, rad = 0.0;
    for (int r = 0; r < C.nruns; ++r) {
        mid = fma(M[r], C.zc[r], mid);
        rad = fma(fabs(M[r]), C.radius[r], rad);
    }
    double lam = 0.0, dir = 0.0;
    if (mid < C.ulo[q]) { lam = (C.ulo[q] - mid) / rad; dir = 1.0; }
    else if (mid > C.uhi[q]) { lam = (mid - C.uhi[q]) / rad; dir = -1.0; }
    for (int r = 0; r < C.nruns; ++r) {
        const double sg = (M[r] > 0.0) ? 1.0 : ((M[r] < 0.0) ? -1.0 : 0.0);
        out[6 + r] = C.zc[r] + dir * lam * sg * C.radius[r];
    }
    out[0] = (double)s;
    out[1] = (double)q;
    out[2] = mid + dir * lam * rad;
    out[3] = mid - rad;
    out[4] = mid + rad;
}

}  // namespace

hipError_t launch_eig_coeffs(const ExpmArgs& E, int32_t nruns, hipStream_t s) {
    if (nruns <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eig_coeffs, dim3(nruns), dim3(kBlock), 0, s, E);
    return hipGetLastError();
}

hipError_t launch_assemble(const AssembleArgs& A, hipStream_t s) {
    const int64_t total = (A.steps + 1) * A.nruns;
    const int64_t blocks = (total + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_check(const CheckArgs& C, hipStream_t s) {
    hipLaunchKernelGGL(k_check, dim3(1), dim3(kBlock), 0, s, C);
    return hipGetLastError();
}

}  // namespace kry
