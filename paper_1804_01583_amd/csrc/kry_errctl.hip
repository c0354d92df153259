// A-posteriori error control of the Krylov dimension (paper Section 4.2:
// Lemma 1 and the checks of Algorithms 2 and 4) for Lanczos runs.
//
// At a checkpoint j (4, then ceil(1.1 j) with 1.1 j a double product) each
// run of the batch evaluates, for its normalised start vector (the
// algorithms take v / |v| and the bound sees T only),
//     bound = h e^{max(lambda,0) tau} int_0^tau w(t) |(e^{t T_j})_{j,1}| dt
// (h = beta_j, lambda >= lambda_max of the symmetric part of A, w = 1, or
// w = tau - t for the augmented run, which integrates the approximation of
// e^{As} b / |b|) and stops at the first checkpoint below the target.  T_j is
// diagonalised (kry_tridiag.h) so the integrand is a sum of j exponentials;
// the integral uses a fixed composite rule: 8-point Gauss-Legendre on
// [0, tau 2^-L] and [tau 2^-(i+1), tau 2^-i], i < L, each split into U equal
// parts.  One workgroup per run.
#include "kry_device.h"
#include "kry_tridiag.h"

#include <cmath>

namespace kry {

namespace {

using namespace dev;

constexpr int kQuadLevels = 40;
constexpr int kQuadSplit = 8;
constexpr int kQuadNodes = (kQuadLevels + 1) * kQuadSplit * 8;

// Stage j's norms -> beta_j, sigma_{j+1} (and k_eff on breakdown), as the
// next mat-vec would record them; one block.
template <int P>
__global__ __launch_bounds__(kBlock) void k_record_stage(BatchArgs B, int j) {
    if (batch_stopped<P>(B)) return;   // the batch met its error target
    __shared__ double s_lds[(kBlock / 64) * P];
    __shared__ double s_nrm[P];
    const double* part = stage_part(B, j);
    double acc[P];
#pragma unroll
    for (int p = 0; p < P; ++p) acc[p] = 0.0;
    add_strided_partials<P>(part, B.nblocks, 0, acc);
    const double t = block_sum<P>(acc, s_lds);
    if (threadIdx.x < P) s_nrm[threadIdx.x] = t;
    __syncthreads();
    record_stage(B, P, j + 1, s_nrm);
}

__global__ __launch_bounds__(kBlock) void k_lemma1(BatchArgs B, ErrArgs X, int j) {
    {
        // the whole batch stopped at an earlier checkpoint (a block that sees
        // its own run's flag already set may skip: it would change nothing)
        bool all = true;
        for (int q = 0; q < (int)gridDim.x; ++q) all = all && X.flags[q] != 0.0;
        if (all) return;
    }
    __shared__ double s_d[kMaxKE], s_e[kMaxKE], s_q1[kMaxKE], s_qm[kMaxKE];
    __shared__ double s_red[kBlock / 64];
    __shared__ int s_state;   // 0 evaluate, 1 already stopped, 2 exact (breakdown), 3 no eigenvalues, 4 past k - 1
    const int p = blockIdx.x;
    double* sc = run_scal(B, p);
    const int m = j;                       // Lanczos steps so far
    const bool affine = X.role[B.run0 + p] == 2;
    if (threadIdx.x == 0) {
        int st = 0;
        if (sc[B.L.misc + MISC_STOPPED] != 0.0) st = 1;
        else if ((int)sc[B.L.misc + MISC_KEFF] <= j) st = 2;
        else if (affine && j > B.L.k - 1) st = 4;   // the bordered matrix holds k - 1 Lanczos steps at most
        if (st == 2) {
            // the Krylov space became invariant: the result is exact
            sc[B.L.misc + MISC_BOUND] = 0.0;
            sc[B.L.misc + MISC_STOPPED] = 1.0;
            sc[B.L.misc + MISC_KSTOP] = sc[B.L.misc + MISC_KEFF];
        }
        if (st == 0) {
            for (int i = 0; i < m; ++i) {
                s_d[i] = X.hess ? sc[B.L.hess + i * B.L.k + i] : sc[B.L.alpha + i + 1];
                s_e[i] = i + 1 < m ? sc[B.L.beta + i + 1] : 0.0;
            }
            if (!tridiag_eig_rows(m, s_d, s_e, s_q1, s_qm)) st = 3;
        }
        s_state = st;
    }
    __syncthreads();
    const int st = s_state;
    if (st == 1 || st == 2 || st == 4) {
        if (threadIdx.x == 0) X.flags[p] = 1.0;
        return;
    }
    const double tau = X.tau;
    double acc = 0.0;
    if (st == 0) {
        for (int idx = threadIdx.x; idx < kQuadNodes; idx += kBlock) {
            const int g = idx % 8;
            const int part = (idx / 8) % kQuadSplit;
            const int lev = idx / (8 * kQuadSplit);          // 0: [0, tau 2^-L]; i > 0: [tau 2^-(L-i+1), tau 2^-(L-i)]
            const double a = lev == 0 ? 0.0 : tau * ldexp(1.0, -(kQuadLevels - lev + 1));
            const double b = tau * ldexp(1.0, -(kQuadLevels - lev));
            const double h = (b - a) / kQuadSplit;
            const double lo = a + part * h;
            const double t = lo + 0.5 * h * (X.gl_x[g] + 1.0);
            double v = 0.0;
            for (int i = 0; i < m; ++i) v = fma(s_qm[i] * s_q1[i], exp(s_d[i] * t), v);
            double wgt = 0.5 * h * X.gl_w[g];
            if (affine) wgt *= tau - t;
            acc = fma(wgt, fabs(v), acc);
        }
    }
    double vals[1] = {acc};
    const double integral = block_sum<1>(vals, s_red);
    if (threadIdx.x == 0) {
        double bound;
        if (st == 3) bound = INFINITY;                       // eigen-iteration failed: do not stop here
        else bound = sc[B.L.beta + m] * exp(X.lam_plus * tau) * integral;
        sc[B.L.misc + MISC_BOUND] = bound;
        const bool stop = bound < X.eps;
        if (stop) {
            sc[B.L.misc + MISC_STOPPED] = 1.0;
            sc[B.L.misc + MISC_KSTOP] = (double)j;
        }
        X.flags[p] = stop ? 1.0 : 0.0;
    }
}

// max_r (a_rr + sum_{c != r} |a_rc|): a Gershgorin upper bound of the
// largest eigenvalue of a symmetric CSR matrix; block maxima then one block.
__global__ __launch_bounds__(kBlock) void k_row_gersh(CsrArgs A, int64_t n, int64_t rows_per_block, double* part) {
    __shared__ double s_m[kBlock / 64];
    const int lb = logical_block((int)gridDim.x);
    const int64_t r0 = (int64_t)lb * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    double v = -INFINITY;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        double s = 0.0;
        for (int64_t e = A.rowptr[r]; e < A.rowptr[r + 1]; ++e) s += A.colidx[e] == r ? A.vals[e] : fabs(A.vals[e]);
        v = s > v ? s : v;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) v = s_m[w] > v ? s_m[w] : v;
        part[lb] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce_gersh(const double* part, int nb, double* out) {
    __shared__ double s_m[kBlock / 64];
    double v = -INFINITY;
    for (int b = threadIdx.x; b < nb; b += kBlock) v = part[b] > v ? part[b] : v;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) v = s_m[w] > v ? s_m[w] : v;
        *out = v;
    }
}

}  // namespace

hipError_t launch_record_stage(int P, const BatchArgs& B, int j, hipStream_t s) {
    switch (P) {
        case 1: hipLaunchKernelGGL((k_record_stage<1>), dim3(1), dim3(kBlock), 0, s, B, j); break;
        case 2: hipLaunchKernelGGL((k_record_stage<2>), dim3(1), dim3(kBlock), 0, s, B, j); break;
        case 4: hipLaunchKernelGGL((k_record_stage<4>), dim3(1), dim3(kBlock), 0, s, B, j); break;
        case 8: hipLaunchKernelGGL((k_record_stage<8>), dim3(1), dim3(kBlock), 0, s, B, j); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lemma1(int P, const BatchArgs& B, const ErrArgs& X, int j, hipStream_t s) {
    if (j < 1 || j > kMaxKE) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lemma1, dim3(P), dim3(kBlock), 0, s, B, X, j);
    return hipGetLastError();
}

hipError_t launch_row_gersh(const CsrArgs& A, int64_t n, double* partials, int32_t nblocks, int64_t rows_per_block,
                            double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_row_gersh, dim3(nblocks), dim3(kBlock), 0, s, A, n, rows_per_block, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_gersh, dim3(1), dim3(kBlock), 0, s, partials, nblocks, out);
    return hipGetLastError();
}

}  // namespace kry
