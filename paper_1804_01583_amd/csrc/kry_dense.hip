// Dense stage for Krylov dimensions too large for the one-workgroup LDS
// exponential (m = pk up to 512): e^{H dt} and the time grid
//     y_s = P e^{H s dt} S0,   s = 0..steps,
// with P = C V (o x m) and S0 the m x w start coefficients (E_1 R_0 for a
// block run, beta_0 e_1 for a single vector).
//
// Phi = e^{H dt} by scaling and squaring of the degree-18 Taylor polynomial
// (the paper names library methods without choosing one, Section 4.1): with X = H dt / 2^s and
// |X|_1 <= 1 the remainder is below 1/19! * e < 2e-17 relative.  The
// polynomial is evaluated by Paterson-Stockmeyer in powers of X^5
// (4 + 3 products), then s squarings.  Steps s = b B + r then use
//     y_s = (P Phi^r) (Psi^b S0),     Psi = Phi^B,
// i.e. B - 1 products for the chain P Phi^r and ceil((steps+1)/B) - 1 for the
// anchors, all as small GEMMs, and one assembly kernel.  All FP64.
#include "kry_device.h"

#include <cmath>

namespace kry {

namespace {

constexpr int kT = 32;   // GEMM tile

// C = alpha A B + beta C (row-major; A M x K, B K x N).  beta == 0 never reads C.
__global__ __launch_bounds__(256) void k_dgemm(int M, int N, int K, double alpha, const double* __restrict__ A,
                                               int lda, const double* __restrict__ Bm, int ldb, double beta,
                                               double* __restrict__ C, int ldc) {
    __shared__ double sA[kT][kT + 1];
    __shared__ double sB[kT][kT + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;      // 2 x 2 outputs per thread
    const int row0 = blockIdx.y * kT, col0 = blockIdx.x * kT;
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int k0 = 0; k0 < K; k0 += kT) {
        for (int t = threadIdx.x; t < kT * kT; t += 256) {
            const int r = t / kT, c = t % kT;
            const int ar = row0 + r, ac = k0 + c;
            sA[r][c] = (ar < M && ac < K) ? A[(int64_t)ar * lda + ac] : 0.0;
            const int br = k0 + r, bc = col0 + c;
            sB[r][c] = (br < K && bc < N) ? Bm[(int64_t)br * ldb + bc] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < kT; ++kk) {
            const double a0 = sA[2 * ty][kk], a1 = sA[2 * ty + 1][kk];
            const double b0 = sB[kk][2 * tx], b1 = sB[kk][2 * tx + 1];
            acc[0][0] = fma(a0, b0, acc[0][0]);
            acc[0][1] = fma(a0, b1, acc[0][1]);
            acc[1][0] = fma(a1, b0, acc[1][0]);
            acc[1][1] = fma(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int r = row0 + 2 * ty + a, c = col0 + 2 * tx + b;
            if (r < M && c < N) {
                double v = alpha * acc[a][b];
                if (beta != 0.0) v = fma(beta, C[(int64_t)r * ldc + c], v);
                C[(int64_t)r * ldc + c] = v;
            }
        }
    }
}

// Out = c0 I + c1 X1 + c2 X2 + c3 X3 + c4 X4 (m x m, ld m).
struct Lin {
    const double* X[4];
    double c[5];
};
__global__ __launch_bounds__(256) void k_lincomb(int m, Lin L, double* __restrict__ out) {
    const int64_t mm = (int64_t)m * m;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < mm; t += (int64_t)gridDim.x * 256) {
        const int64_t r = t / m, c = t % m;
        double v = r == c ? L.c[0] : 0.0;
        for (int q = 0; q < 4; ++q)
            if (L.c[q + 1] != 0.0) v = fma(L.c[q + 1], L.X[q][t], v);
        out[t] = v;
    }
}

// dst (m x m, ld m) = scale * src (ld lds); also used as a plain copy
__global__ __launch_bounds__(256) void k_scopy(int m, const double* __restrict__ src, int lds, double scale,
                                               double* __restrict__ dst, int cols, int ldd) {
    const int64_t tot = (int64_t)m * cols;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < tot; t += (int64_t)gridDim.x * 256) {
        const int64_t r = t / cols, c = t % cols;
        dst[r * ldd + c] = scale * src[r * lds + c];
    }
}

// max column sum of |H| over the leading m x m block (one workgroup)
__global__ __launch_bounds__(256) void k_norm1(int m, const double* __restrict__ H, int ldh, double* out) {
    __shared__ double s[256];
    double best = 0.0;
    for (int c = threadIdx.x; c < m; c += 256) {
        double t = 0.0;
        for (int r = 0; r < m; ++r) t += fabs(H[(int64_t)r * ldh + c]);
        best = t > best ? t : best;
    }
    s[threadIdx.x] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int t = 0; t < 256; ++t) v = s[t] > v ? s[t] : v;
        *out = v;
    }
}

// basis[s][q][run0 + c] = sum_i Z[s % B][q][i] anch[s / B][i][c], c < w
__global__ __launch_bounds__(128) void k_dassemble(const double* __restrict__ Z, const double* __restrict__ anch,
                                                   int m, int o, int w, int B, int64_t steps,
                                                   double* __restrict__ basis, int nruns, int run0) {
    const int64_t s = blockIdx.x;
    if (s > steps) return;
    const int t = threadIdx.x;
    if (t >= o * w) return;
    const int q = t / w, c = t % w;
    const double* z = Z + ((int64_t)(s % B) * o + q) * m;
    const double* a = anch + (int64_t)(s / B) * m * w;
    double v = 0.0;
    for (int i = 0; i < m; ++i) v = fma(z[i], a[(int64_t)i * w + c], v);
    basis[(s * o + q) * nruns + run0 + c] = v;
}

hipError_t gemm(int M, int N, int K, double alpha, const double* A, int lda, const double* Bm, int ldb, double beta,
                double* C, int ldc, hipStream_t s) {
    const dim3 grid((N + kT - 1) / kT, (M + kT - 1) / kT);
    hipLaunchKernelGGL(k_dgemm, grid, dim3(256), 0, s, M, N, K, alpha, A, lda, Bm, ldb, beta, C, ldc);
    return hipGetLastError();
}

int grid_for(int64_t count) { return (int)std::min<int64_t>((count + 255) / 256, 2048); }

}  // namespace

namespace {
__global__ __launch_bounds__(256) void k_fill(double* p, int64_t count, double v) {
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < count; t += (int64_t)gridDim.x * 256) p[t] = v;
}
// basis[s][r][run0 + c] = v for every step, row and c < w: NaN when the
// run's exponential is undefined (non-finite H), which the box check
// reports; 0 for a run whose start vector is zero.
__global__ __launch_bounds__(256) void k_fill_columns(double* basis, int64_t steps, int o, int nruns, int run0, int w,
                                                      double v) {
    const int64_t total = (steps + 1) * o * w;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i % w;
        const int64_t sr = i / w;
        basis[sr * nruns + run0 + c] = v;
    }
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t* p, int64_t count, int32_t v) {
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < count; t += (int64_t)gridDim.x * 256) p[t] = v;
}
}  // namespace

namespace {
// The same H, P and start scale as k_expm_chain forms in LDS (tridiagonal from
// alpha/beta for Lanczos, Hessenberg store for a stored basis, bordered by
// the augmented variable for the affine run).
__global__ __launch_bounds__(256) void k_build_dense(ExpmArgs E, int run, int m, double* __restrict__ H,
                                                     double* __restrict__ P, double* __restrict__ S0) {
    const double* sc = E.scal + (int64_t)run * E.L.stride;
    const int k = E.L.k, o = E.L.o;
    const bool bordered = E.role[run] == 2;
    const int sh = bordered ? 1 : 0;
    for (int idx = threadIdx.x + blockIdx.x * 256; idx < m * m; idx += gridDim.x * 256) {
        const int i = idx / m, c = idx % m;
        double h = 0.0;
        if (bordered && i == 1 && c == 0) h = sc[E.L.beta + 0];
        else if (i >= sh && c >= sh) {
            const int a = i - sh, b = c - sh;
            if (E.hess_mode) {
                if (a <= b) h = sc[E.L.hess + a * k + b];
                else if (a == b + 1) h = sc[E.L.beta + b + 1];
            } else {
                if (a == b) h = sc[E.L.alpha + a + 1];
                else if (b == a + 1) h = sc[E.L.beta + a + 1];
                else if (a == b + 1) h = sc[E.L.beta + b + 1];
            }
        }
        H[idx] = h;
    }
    for (int idx = threadIdx.x + blockIdx.x * 256; idx < o * m; idx += gridDim.x * 256) {
        const int q = idx / m, c = idx % m;
        const int col = c - sh;
        P[idx] = col >= 0 ? sc[E.L.proj + q * (k + 1) + col] : 0.0;
    }
    for (int idx = threadIdx.x + blockIdx.x * 256; idx < m; idx += gridDim.x * 256)
        S0[idx] = idx == 0 ? (bordered ? 1.0 : sc[E.L.beta + 0]) : 0.0;
}
}  // namespace

hipError_t launch_build_dense(const ExpmArgs& E, int run, int m, double* H, double* P, double* S0, hipStream_t s) {
    if (m <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_build_dense, dim3(grid_for((int64_t)m * m)), dim3(256), 0, s, E, run, m, H, P, S0);
    return hipGetLastError();
}

// plain fill kernels (not memset nodes, so the work stays capturable)
hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(count)), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(count)), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

size_t dense_workspace_doubles(int m, int o, int w, int B, int nanch) {
    return (size_t)10 * m * m + (size_t)B * o * m + (size_t)nanch * m * w + 8;
}

hipError_t dense_expm_steps(const DenseJob& J, double* ws, double* host_norm, hipStream_t s) {
    const int m = J.m;
    if (J.o * J.w > 128) return hipErrorInvalidValue;
    if (m <= 0) {
        // a run with a zero start vector: its basis columns are zero
        hipLaunchKernelGGL(k_dassemble, dim3((unsigned)(J.steps + 1)), dim3(128), 0, s, ws, ws, 0, J.o, J.w, J.B,
                           J.steps, J.basis, J.nruns, J.run0);
        return hipGetLastError();
    }
    const int64_t mm = (int64_t)m * m;
    double* X = ws;
    double* X2 = X + mm;
    double* X3 = X2 + mm;
    double* X4 = X3 + mm;
    double* X5 = X4 + mm;
    double* L0 = X5 + mm;
    double* L1 = L0 + mm;
    double* L2 = L1 + mm;
    double* L3 = L2 + mm;
    double* T = L3 + mm;
    double* Z = T + mm;
    double* anch = Z + (int64_t)J.B * J.o * m;
    double* nrm = anch + (int64_t)J.nanch * m * J.w;
    hipError_t e;
    if (J.nonfinite || J.m == 0) {
        hipLaunchKernelGGL(k_fill_columns, dim3(256), dim3(256), 0, s, J.basis, J.steps, J.o, J.nruns, J.run0, J.w,
                           J.nonfinite ? __builtin_nan("") : 0.0);
        return hipGetLastError();
    }
    // |H dt|_1 -> the number of halvings
    hipLaunchKernelGGL(k_norm1, dim3(1), dim3(256), 0, s, m, J.H, J.ldh, nrm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(host_norm, nrm, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    const double nx = *host_norm * J.dt;
    if (!std::isfinite(nx)) {
        // a non-finite value reached H: the run's basis columns become NaN
        // and the box check reports KRY_ENUMERIC in its verdict
        hipLaunchKernelGGL(k_fill_columns, dim3(256), dim3(256), 0, s, J.basis, J.steps, J.o, J.nruns, J.run0, J.w,
                           __builtin_nan(""));
        return hipGetLastError();
    }
    int sq = 0;
    while (nx / std::ldexp(1.0, sq) > 1.0) ++sq;
    hipLaunchKernelGGL(k_scopy, dim3(grid_for(mm)), dim3(256), 0, s, m, J.H, J.ldh, J.dt / std::ldexp(1.0, sq), X, m,
                       m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // powers
    if ((e = gemm(m, m, m, 1.0, X, m, X, m, 0.0, X2, m, s)) != hipSuccess) return e;
    if ((e = gemm(m, m, m, 1.0, X2, m, X, m, 0.0, X3, m, s)) != hipSuccess) return e;
    if ((e = gemm(m, m, m, 1.0, X2, m, X2, m, 0.0, X4, m, s)) != hipSuccess) return e;
    if ((e = gemm(m, m, m, 1.0, X4, m, X, m, 0.0, X5, m, s)) != hipSuccess) return e;
    // chunks L_q = sum_{i=0..4} X^i / (5q + i)!
    double f[19];
    f[0] = 1.0;
    for (int i = 1; i <= 18; ++i) f[i] = f[i - 1] / i;
    double* Lq[4] = {L0, L1, L2, L3};
    for (int q = 0; q < 4; ++q) {
        Lin L{{X, X2, X3, X4}, {0, 0, 0, 0, 0}};
        for (int i = 0; i < 5; ++i) L.c[i] = (5 * q + i <= 18) ? f[5 * q + i] : 0.0;
        hipLaunchKernelGGL(k_lincomb, dim3(grid_for(mm)), dim3(256), 0, s, m, L, Lq[q]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // Horner in X^5: ((L3 X5 + L2) X5 + L1) X5 + L0
    if ((e = gemm(m, m, m, 1.0, L3, m, X5, m, 1.0, L2, m, s)) != hipSuccess) return e;
    if ((e = gemm(m, m, m, 1.0, L2, m, X5, m, 1.0, L1, m, s)) != hipSuccess) return e;
    if ((e = gemm(m, m, m, 1.0, L1, m, X5, m, 1.0, L0, m, s)) != hipSuccess) return e;
    double* Phi = L0;
    double* spare = T;
    for (int i = 0; i < sq; ++i) {
        if ((e = gemm(m, m, m, 1.0, Phi, m, Phi, m, 0.0, spare, m, s)) != hipSuccess) return e;
        std::swap(Phi, spare);
    }
    // Psi = Phi^B (B a power of two) in two free buffers
    double* Psi = X;
    double* tmp = X2;
    hipLaunchKernelGGL(k_scopy, dim3(grid_for(mm)), dim3(256), 0, s, m, Phi, m, 1.0, Psi, m, m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int b = 1; b < J.B; b <<= 1) {
        if ((e = gemm(m, m, m, 1.0, Psi, m, Psi, m, 0.0, tmp, m, s)) != hipSuccess) return e;
        std::swap(Psi, tmp);
    }
    // chain Z_r = P Phi^r
    hipLaunchKernelGGL(k_scopy, dim3(grid_for((int64_t)J.o * m)), dim3(256), 0, s, J.o, J.P, J.ldp, 1.0, Z, m, m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int r = 1; r < J.B; ++r) {
        double* zp = Z + (int64_t)(r - 1) * J.o * m;
        if ((e = gemm(J.o, m, m, 1.0, zp, m, Phi, m, 0.0, zp + (int64_t)J.o * m, m, s)) != hipSuccess) return e;
    }
    // anchors a_b = Psi^b S0
    hipLaunchKernelGGL(k_scopy, dim3(grid_for((int64_t)m * J.w)), dim3(256), 0, s, m, J.S0, J.lds0, 1.0, anch, J.w,
                       J.w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int b = 1; b < J.nanch; ++b) {
        double* ap = anch + (int64_t)(b - 1) * m * J.w;
        if ((e = gemm(m, J.w, m, 1.0, Psi, m, ap, J.w, 0.0, ap + (int64_t)m * J.w, J.w, s)) != hipSuccess) return e;
    }
    if (J.o * J.w > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dassemble, dim3((unsigned)(J.steps + 1)), dim3(128), 0, s, Z, anch, m, J.o, J.w, J.B,
                       J.steps, J.basis, J.nruns, J.run0);
    return hipGetLastError();
}

}  // namespace kry
