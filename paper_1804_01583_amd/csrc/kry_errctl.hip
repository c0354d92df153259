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
//
// Arnoldi runs (Algorithm 2) have an upper Hessenberg H_j, so the integrand
// (e^{t H_j})_{j,1} comes from exponentials instead.  The nodes of level i + 1
// are exactly twice those of level i (the intervals double and the rule is
// the same), so one chain per (part, Gauss point) pair covers the levels
// 1..L: F(t) = e^{t H} - I at the level-1 node by the Taylor polynomial in LDS
// (kry_ldsmm.h), then F(2t) = 2 F(t) + F(t)^2 for each further level, which
// keeps the relative accuracy of the small-t values that e^{tH} itself would
// round away against I.  The level-0 node takes its own Taylor polynomial.
// One workgroup per (run, chain) writes its weighted sum; a second kernel
// adds the 64 sums in a fixed order and decides the stop.
#include "kry_device.h"
#include "kry_ldsmm.h"
#include "kry_tridiag.h"

#include <algorithm>
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

// the whole batch stopped at an earlier checkpoint (a block that sees its
// own run's flag already set may skip: it would change nothing)
__device__ __forceinline__ bool batch_done(const ErrArgs& X, int P) {
    bool all = true;
    for (int q = 0; q < P; ++q) all = all && X.flags[q] != 0.0;
    return all;
}

// State of run p at checkpoint j: 0 evaluate, 1 already stopped, 2 exact
// (breakdown), 4 past k - 1 (the bordered matrix of the augmented run holds
// k - 1 Krylov steps at most); 3 (no eigenvalues) is set by the caller.
__device__ __forceinline__ int lemma1_state(const BatchArgs& B, const ErrArgs& X, const double* sc, int p, int j) {
    if (sc[B.L.misc + MISC_STOPPED] != 0.0) return 1;
    if ((int)sc[B.L.misc + MISC_KEFF] <= j) return 2;
    if (X.role[B.run0 + p] == 2 && j > B.L.k - 1) return 4;
    return 0;
}

// the Krylov space became invariant: the result is exact
__device__ __forceinline__ void mark_exact(const BatchArgs& B, double* sc) {
    sc[B.L.misc + MISC_BOUND] = 0.0;
    sc[B.L.misc + MISC_STOPPED] = 1.0;
    sc[B.L.misc + MISC_KSTOP] = sc[B.L.misc + MISC_KEFF];
}

// the bound from the integral, recorded with the stop decision
__device__ __forceinline__ void lemma1_decide(const BatchArgs& B, const ErrArgs& X, double* sc, int p, int j,
                                              double integral, bool failed) {
    const double bound = failed ? INFINITY : sc[B.L.beta + j] * exp(X.lam_plus * X.tau) * integral;
    sc[B.L.misc + MISC_BOUND] = bound;
    const bool stop = bound < X.eps;
    if (stop) {
        sc[B.L.misc + MISC_STOPPED] = 1.0;
        sc[B.L.misc + MISC_KSTOP] = (double)j;
    }
    X.flags[p] = stop ? 1.0 : 0.0;
}

// Node t of the composite rule: Gauss point g of part u on level lev, and
// its weight (0.5 h w_g, times tau - t for the augmented run).
__device__ __forceinline__ void quad_node(const ErrArgs& X, int lev, int u, int g, bool affine, double& t,
                                          double& wgt) {
    const double tau = X.tau;
    const double a = lev == 0 ? 0.0 : tau * ldexp(1.0, -(kQuadLevels - lev + 1));
    const double b = tau * ldexp(1.0, -(kQuadLevels - lev));
    const double h = (b - a) / kQuadSplit;
    const double lo = a + u * h;
    t = lo + 0.5 * h * (X.gl_x[g] + 1.0);
    wgt = 0.5 * h * X.gl_w[g];
    if (affine) wgt *= tau - t;
}

__global__ __launch_bounds__(kBlock) void k_lemma1(BatchArgs B, ErrArgs X, int j) {
    if (batch_done(X, (int)gridDim.x)) return;
    __shared__ double s_d[kMaxKE], s_e[kMaxKE], s_q1[kMaxKE], s_qm[kMaxKE];
    __shared__ double s_red[kBlock / 64];
    __shared__ int s_state;   // lemma1_state, or 3: no eigenvalues
    const int p = blockIdx.x;
    double* sc = run_scal(B, p);
    const int m = j;                       // Lanczos steps so far
    const bool affine = X.role[B.run0 + p] == 2;
    if (threadIdx.x == 0) {
        int st = lemma1_state(B, X, sc, p, j);
        if (st == 2) mark_exact(B, sc);
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
    double acc = 0.0;
    if (st == 0) {
        for (int idx = threadIdx.x; idx < kQuadNodes; idx += kBlock) {
            // level 0: [0, tau 2^-L]; level i > 0: [tau 2^-(L-i+1), tau 2^-(L-i)]
            double t, wgt;
            quad_node(X, idx / (8 * kQuadSplit), (idx / 8) % kQuadSplit, idx % 8, affine, t, wgt);
            double v = 0.0;
            for (int i = 0; i < m; ++i) v = fma(s_qm[i] * s_q1[i], exp(s_d[i] * t), v);
            acc = fma(wgt, fabs(v), acc);
        }
    }
    double vals[1] = {acc};
    const double integral = block_sum<1>(vals, s_red);
    // an eigen-iteration that failed gives an infinite bound: no stop here
    if (threadIdx.x == 0) lemma1_decide(B, X, sc, p, m, integral, st == 3);
}

// Slot 4 <- e^{t H} - I for the j x j Hessenberg matrix of run sc (mm = j
// rounded up to even, zero padded): X = t H / 2^s with |X|_1 <= 1, the
// Taylor polynomial without its constant term, then s doublings
// F <- 2 F + F^2 ping-ponging between slots 4 and 5; returns the final slot.
__device__ __forceinline__ int hess_expm1(double* lds, const BatchArgs& B, const double* sc, int m, int mm, double t,
                                          double* s_red) {
    const int k = B.L.k;
    for (int idx = threadIdx.x; idx < mm * mm; idx += blockDim.x) {
        const int a = idx / mm, c = idx % mm;
        double h = 0.0;
        if (a < m && c < m) {
            if (a <= c) h = sc[B.L.hess + a * k + c];
            else if (a == c + 1) h = sc[B.L.beta + c + 1];
        }
        lds[a * ldsmm::kLd + c] = h * t;
    }
    __syncthreads();
    const double nrm = ldsmm::norm1_slot0(lds, mm, s_red);
    int sq = 0;
    while (isfinite(nrm) && nrm > ldexp(1.0, sq) && sq < 1100) ++sq;
    if (sq > 0) {
        const double shrink = ldexp(1.0, -sq);
        for (int idx = threadIdx.x; idx < mm * mm; idx += blockDim.x) {
            const int a = idx / mm, c = idx % mm;
            lds[a * ldsmm::kLd + c] *= shrink;
        }
        __syncthreads();
    }
    ldsmm::taylor18(lds, mm, 0.0);
    int cur = 4;
    for (int i = 0; i < sq; ++i) {
        const double* F = lds + cur * ldsmm::kSlot;
        ldsmm::mm_mfma(lds, cur, cur, 9 - cur, mm, [=](int r, int c) { return 2.0 * F[r * ldsmm::kLd + c]; });
        cur = 9 - cur;
    }
    return cur;
}

// (e^{tH})_{m,1} from F = e^{tH} - I in slot `slot`
__device__ __forceinline__ double corner(const double* lds, int slot, int m) {
    return lds[slot * ldsmm::kSlot + (m - 1) * ldsmm::kLd] + (m == 1 ? 1.0 : 0.0);
}

constexpr int kHessChains = kQuadSplit * 8;   // (part, Gauss point) pairs
constexpr int kHessThreads = 512;

// grid (kHessChains, P): workgroup (c, p) integrates chain c of run p over
// every level and writes its weighted sum to part[p * kHessChains + c].
__global__ __launch_bounds__(kHessThreads) void k_lemma1_hess(BatchArgs B, ErrArgs X, int j, double* part) {
    extern __shared__ double lds[];
    __shared__ double s_red[kHessThreads / 64];
    const int p = blockIdx.y, chain = blockIdx.x;
    double* out = part + p * kHessChains + chain;
    if (batch_done(X, (int)gridDim.y)) return;
    const double* sc = run_scal(B, p);
    if (lemma1_state(B, X, sc, p, j) != 0) {
        if (threadIdx.x == 0) *out = 0.0;
        return;
    }
    const bool affine = X.role[B.run0 + p] == 2;
    const int m = j, mm = m + (m & 1);
    const int g = chain % 8, u = chain / 8;
    double acc = 0.0, t, wgt;
    // level 0: [0, tau 2^-L]
    quad_node(X, 0, u, g, affine, t, wgt);
    int slot = hess_expm1(lds, B, sc, m, mm, t, s_red);
    acc = fma(wgt, fabs(corner(lds, slot, m)), acc);
    __syncthreads();
    // level 1, then each level's node is twice the previous one
    quad_node(X, 1, u, g, affine, t, wgt);
    slot = hess_expm1(lds, B, sc, m, mm, t, s_red);
    acc = fma(wgt, fabs(corner(lds, slot, m)), acc);
    for (int lev = 2; lev <= kQuadLevels; ++lev) {
        const double* F = lds + slot * ldsmm::kSlot;
        ldsmm::mm_mfma(lds, slot, slot, 9 - slot, mm, [=](int r, int c) { return 2.0 * F[r * ldsmm::kLd + c]; });
        slot = 9 - slot;
        quad_node(X, lev, u, g, affine, t, wgt);
        acc = fma(wgt, fabs(corner(lds, slot, m)), acc);
    }
    if (threadIdx.x == 0) *out = acc;
}

// one wave per run: the chains' sums in order, then the bound and the stop
__global__ __launch_bounds__(64) void k_lemma1_hess_finish(BatchArgs B, ErrArgs X, int j, const double* part) {
    if (batch_done(X, (int)gridDim.x)) return;
    const int p = blockIdx.x;
    if (threadIdx.x != 0) return;
    double* sc = run_scal(B, p);
    const int st = lemma1_state(B, X, sc, p, j);
    if (st == 2) mark_exact(B, sc);
    if (st != 0) {
        X.flags[p] = 1.0;
        return;
    }
    double integral = 0.0;
    for (int c = 0; c < kHessChains; ++c) integral += part[p * kHessChains + c];
    lemma1_decide(B, X, sc, p, j, integral, !isfinite(integral));
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

// Upper bound of lambda_max((A + A^T)/2) for a general CSR matrix: Gershgorin
// on the symmetric part with |a_rc + a_cr| / 2 <= (|a_rc| + |a_cr|) / 2, i.e.
// max_r a_rr + (R_r + C_r) / 2 with R_r, C_r the absolute off-diagonal sums
// of row r and column r.  The column sums are scattered as fixed-point
// integers (unit u, a power of two >= 2^-40 max|a|, each entry rounded up),
// so they add up exactly in any order and the bound stays an upper bound.

// block maxima of |a| (a non-finite entry gives infinity)
__global__ __launch_bounds__(kBlock) void k_abs_max(const double* vals, int64_t nnz, double* part) {
    __shared__ double s_m[kBlock / 64];
    double v = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kBlock) {
        const double x = fabs(vals[e]);
        v = isfinite(x) ? (x > v ? x : v) : INFINITY;
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
        part[blockIdx.x] = v;
    }
}

// colfix[c] += ceil-ish(|a_rc| / (2u)) for every off-diagonal entry; the
// integer part plus one is at least the quotient, and overflow of a column
// (more than 2^23 entries) sets *overflow
__global__ __launch_bounds__(kBlock) void k_col_scatter(CsrArgs A, int64_t n, double inv_2u,
                                                        unsigned long long* colfix, int* overflow) {
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kBlock) {
        for (int64_t e = A.rowptr[r]; e < A.rowptr[r + 1]; ++e) {
            const int64_t c = A.colidx[e];
            const double x = fabs(A.vals[e]);
            if (c == r || x == 0.0) continue;
            const unsigned long long q = (unsigned long long)(x * inv_2u) + 1ull;
            const unsigned long long old = atomicAdd(colfix + c, q);
            if (old + q < old) *overflow = 1;
        }
    }
}

// block maxima of a_rr + R_r / 2 + colfix[r] u
__global__ __launch_bounds__(kBlock) void k_gersh_general(CsrArgs A, int64_t n, int64_t rows_per_block, double u,
                                                          const unsigned long long* colfix, double* part) {
    __shared__ double s_m[kBlock / 64];
    const int lb = logical_block((int)gridDim.x);
    const int64_t r0 = (int64_t)lb * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    double v = -INFINITY;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        double d = 0.0, off = 0.0;
        for (int64_t e = A.rowptr[r]; e < A.rowptr[r + 1]; ++e) {
            if (A.colidx[e] == r) d += A.vals[e];
            else off += fabs(A.vals[e]);
        }
        const double s = d + 0.5 * off + (double)colfix[r] * u;
        v = s > v ? s : v;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) v = s_m[w] > v ? s_m[w] : v;
        part[lb] = v;
    }
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

}  // namespace

size_t lemma1_hess_lds_bytes() { return (size_t)6 * ldsmm::kSlot * sizeof(double); }

hipError_t errctl_prepare() {
    return hipFuncSetAttribute((const void*)k_lemma1_hess, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lemma1_hess_lds_bytes());
}

hipError_t launch_lemma1_hess(int P, const BatchArgs& B, const ErrArgs& X, int j, double* part, hipStream_t s) {
    if (j < 1 || j > kMaxK || P < 1 || P > kMaxP) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lemma1_hess, dim3(kHessChains, P), dim3(kHessThreads), lemma1_hess_lds_bytes(), s, B, X, j,
                       part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lemma1_hess_finish, dim3(P), dim3(64), 0, s, B, X, j, (const double*)part);
    return hipGetLastError();
}

int lemma1_hess_partials() { return kMaxP * kHessChains; }

hipError_t launch_abs_max(const double* vals, int64_t nnz, double* part, int32_t nblocks, double* out,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_abs_max, dim3(nblocks), dim3(kBlock), 0, s, vals, nnz, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_gersh, dim3(1), dim3(kBlock), 0, s, (const double*)part, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_gersh_general(const CsrArgs& A, int64_t n, double u, unsigned long long* colfix, int* overflow,
                                double* partials, int32_t nblocks, int64_t rows_per_block, double* out,
                                hipStream_t s) {
    const int zb = (int)std::min<int64_t>(4096, (n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_zero_u64, dim3(zb), dim3(kBlock), 0, s, colfix, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_col_scatter, dim3(zb), dim3(kBlock), 0, s, A, n, 0.5 / u, colfix, overflow);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gersh_general, dim3(nblocks), dim3(kBlock), 0, s, A, n, rows_per_block, u,
                       (const unsigned long long*)colfix, partials);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_gersh, dim3(1), dim3(kBlock), 0, s, (const double*)partials, nblocks, out);
    return hipGetLastError();
}

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
