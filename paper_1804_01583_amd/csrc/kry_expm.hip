// Small dense stage on gfx950: e^{H t} e_1 for every time step (paper
// Section 4.2, Eq. approx-formula), the basis matrix of Section 3.2 and the
// per-step box check that stands in for the LP of Section 2.1.
//
// Per run, one workgroup keeps H in LDS and computes
//   Phi = e^{H dt}   by Pade [13/13] with scaling and squaring
//                    (N. J. Higham, SIAM J. Matrix Anal. Appl. 26(4), 2005),
//   Psi = Phi^B      by squaring (B a power of two near sqrt(steps + 1)),
// then two short chains, Z_r = P Phi^r (r < B) and a_b = Psi^b e_1, so that
//   y_s = beta0 * Z_{s mod B} a_{s div B},   s = 0..steps,
// is assembled for all steps in parallel by k_assemble.  The chains are
// at most B and (steps+1)/B long, instead of one recurrence over all steps.
// The augmented run uses the bordered matrix H~ = [[0, 0], [|b| e_1, T]] and
// P~ = [0, C Q] with scale 1; generator and center runs use T itself.
#include "kry_internal.h"

#include <cmath>

namespace kry {

namespace {

constexpr int kLd = kMaxK + 1;          // padded LDS row length
constexpr int kSlot = kMaxK * kLd;      // one matrix in LDS
constexpr double kTheta13 = 5.371920351148152;   // Higham 2005: degree-13 limit of |X|_1

__device__ __forceinline__ const double* run_scal(const ExpmArgs& E, int r) {
    return E.scal + (int64_t)r * E.L.stride;
}

// C = A * B(l, j) for mm x mm matrices in LDS (mm even); `extra(i, j)` is
// added to each entry.  Each thread owns 2x2 output blocks.  C must not
// alias A or the storage B reads.
template <class FB, class FE>
__device__ __forceinline__ void mm_lds(const double* A, FB Bf, double* C, int mm, FE extra) {
    const int nb = mm >> 1;
    for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
        const int i = 2 * (t / nb), j = 2 * (t % nb);
        double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
        for (int l = 0; l < mm; ++l) {
            const double a0 = A[i * kLd + l], a1 = A[(i + 1) * kLd + l];
            const double b0 = Bf(l, j), b1 = Bf(l, j + 1);
            c00 = fma(a0, b0, c00);
            c01 = fma(a0, b1, c01);
            c10 = fma(a1, b0, c10);
            c11 = fma(a1, b1, c11);
        }
        C[i * kLd + j] = c00 + extra(i, j);
        C[i * kLd + j + 1] = c01 + extra(i, j + 1);
        C[(i + 1) * kLd + j] = c10 + extra(i + 1, j);
        C[(i + 1) * kLd + j + 1] = c11 + extra(i + 1, j + 1);
    }
    __syncthreads();
}

__device__ __forceinline__ void square_lds(const double* A, double* C, int mm) {
    mm_lds(A, [A](int l, int j) { return A[l * kLd + j]; }, C, mm, [](int, int) { return 0.0; });
}

// Solve M F = R in place (F overwrites R) by Gauss-Jordan elimination with
// partial pivoting; M is destroyed.  mm <= 64 so one wave finds the pivot.
__device__ void solve_lds(double* M, double* R, int mm, int* s_piv, double* s_f) {
    for (int c = 0; c < mm; ++c) {
        if (threadIdx.x < 64) {
            const int r = c + threadIdx.x;
            double v = (r < mm) ? fabs(M[r * kLd + c]) : -1.0;
            int at = r;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(v, off, 64);
                const int oa = __shfl_xor(at, off, 64);
                if (ov > v || (ov == v && oa < at)) { v = ov; at = oa; }
            }
            if (threadIdx.x == 0) *s_piv = at;
        }
        __syncthreads();
        const int piv = *s_piv;
        if (piv != c) {
            for (int j = threadIdx.x; j < 2 * mm; j += blockDim.x) {
                double* X = (j < mm) ? M : R;
                const int jj = (j < mm) ? j : j - mm;
                const double t = X[c * kLd + jj];
                X[c * kLd + jj] = X[piv * kLd + jj];
                X[piv * kLd + jj] = t;
            }
            __syncthreads();
        }
        if (threadIdx.x < mm) s_f[threadIdx.x] = M[threadIdx.x * kLd + c];
        __syncthreads();
        const double inv = 1.0 / s_f[c];
        for (int j = threadIdx.x; j < 2 * mm; j += blockDim.x) {
            double* X = (j < mm) ? M : R;
            const int jj = (j < mm) ? j : j - mm;
            X[c * kLd + jj] *= inv;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < mm * 2 * mm; e += blockDim.x) {
            const int r = e / (2 * mm), j = e % (2 * mm);
            if (r == c) continue;
            double* X = (j < mm) ? M : R;
            const int jj = (j < mm) ? j : j - mm;
            X[r * kLd + jj] = fma(-s_f[r], X[c * kLd + jj], X[r * kLd + jj]);
        }
        __syncthreads();
    }
}

// One workgroup per run: Phi, Psi and the two chains.
__global__ __launch_bounds__(kExpmThreads) void k_expm_chain(ExpmArgs E) {
    extern __shared__ double lds[];
    double* S0 = lds;
    double* S1 = lds + 1 * kSlot;
    double* S2 = lds + 2 * kSlot;
    double* S3 = lds + 3 * kSlot;
    double* S4 = lds + 4 * kSlot;
    double* S5 = lds + 5 * kSlot;
    __shared__ double s_f[kMaxK];
    __shared__ double s_red[kExpmThreads / 64];
    __shared__ int s_piv;

    const int run = blockIdx.x;
    const double* sc = run_scal(E, run);
    const int k = E.L.k, o = E.L.o;
    const int keff = min((int)sc[E.L.misc + MISC_KEFF], (int)sc[E.L.misc + MISC_KSTOP]);
    const bool bordered = E.role[run] == 2;
    int m = keff;                            // size of H
    if (bordered) m = (keff > k - 1 ? k - 1 : keff) + 1;
    if (keff <= 0) m = 0;                    // zero start vector: the run contributes nothing
    if (threadIdx.x == 0) {
        E.msize[run] = m;
        E.scale[run] = bordered ? 1.0 : sc[E.L.beta + 0];
    }
    if (m == 0) return;
    const int mm = m + (m & 1);
    const int tid = threadIdx.x;

    // X = H dt (zero padded to mm)
    for (int idx = tid; idx < mm * mm; idx += blockDim.x) {
        const int i = idx / mm, c = idx % mm;
        double h = 0.0;
        if (i < m && c < m) {
            // row/column 0 of the bordered matrix is the augmented variable;
            // the Krylov matrix of A occupies 1..m-1 there
            const int sh = bordered ? 1 : 0;
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
        }
        S0[i * kLd + c] = h * E.dt;
    }
    __syncthreads();

    // scaling: |X|_1 <= theta_13 after dividing by 2^sq
    double colsum = 0.0;
    if (tid < mm) {
        for (int i = 0; i < mm; ++i) colsum += fabs(S0[i * kLd + tid]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) colsum = fmax(colsum, __shfl_xor(colsum, off, 64));
    if ((tid & 63) == 0) s_red[tid >> 6] = colsum;
    __syncthreads();
    double nrm = 0.0;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) nrm = fmax(nrm, s_red[w]);
    int sq = 0;
    if (nrm > kTheta13) sq = (int)ceil(log2(nrm / kTheta13));
    const double shrink = ldexp(1.0, -sq);
    __syncthreads();
    for (int idx = tid; idx < mm * mm; idx += blockDim.x) {
        const int i = idx / mm, c = idx % mm;
        S0[i * kLd + c] *= shrink;
    }
    __syncthreads();

    // Pade [13/13]: U = X (X6 (b13 X6 + b11 X4 + b9 X2) + b7 X6 + b5 X4 + b3 X2 + b1 I)
    //               V =    X6 (b12 X6 + b10 X4 + b8 X2) + b6 X6 + b4 X4 + b2 X2 + b0 I
    const double* b = E.pade;
    square_lds(S0, S1, mm);                                                    // X2
    square_lds(S1, S2, mm);                                                    // X4
    mm_lds(S2, [S1](int l, int j) { return S1[l * kLd + j]; }, S3, mm,
           [](int, int) { return 0.0; });                                      // X6
    mm_lds(S3, [=](int l, int j) {
               const int e = l * kLd + j;
               return b[13] * S3[e] + b[11] * S2[e] + b[9] * S1[e];
           }, S4, mm, [=](int i, int j) {
               const int e = i * kLd + j;
               return b[7] * S3[e] + b[5] * S2[e] + b[3] * S1[e] + (i == j ? b[1] : 0.0);
           });                                                                 // U' in S4
    mm_lds(S3, [=](int l, int j) {
               const int e = l * kLd + j;
               return b[12] * S3[e] + b[10] * S2[e] + b[8] * S1[e];
           }, S5, mm, [=](int i, int j) {
               const int e = i * kLd + j;
               return b[6] * S3[e] + b[4] * S2[e] + b[2] * S1[e] + (i == j ? b[0] : 0.0);
           });                                                                 // V in S5
    mm_lds(S0, [S4](int l, int j) { return S4[l * kLd + j]; }, S1, mm,
           [](int, int) { return 0.0; });                                      // U in S1
    for (int idx = tid; idx < mm * mm; idx += blockDim.x) {
        const int e = (idx / mm) * kLd + idx % mm;
        const double u = S1[e], v = S5[e];
        S5[e] = v - u;
        S1[e] = v + u;
    }
    __syncthreads();
    solve_lds(S5, S1, mm, &s_piv, s_f);                                        // r13(X) in S1

    // LDS matrices below are addressed as lds + slot * kSlot with an integer
    // slot, never through stored pointers, so the accesses stay ds_* (LDS)
    // instructions instead of generic flat ones.
    // undo the scaling: Phi = r13(X)^(2^sq), ping-pong between slots 1 and 2
    int phi = 1;
    for (int i = 0; i < sq; ++i) {
        square_lds(lds + phi * kSlot, lds + (3 - phi) * kSlot, mm);
        phi = 3 - phi;
    }
    // Psi = Phi^B, ping-pong between slots 3 and 4
    int psi = phi;
    for (int e = 1, nxt = 3; e < E.B; e <<= 1) {
        square_lds(lds + psi * kSlot, lds + nxt * kSlot, mm);
        psi = nxt;
        nxt = 7 - nxt;
    }
    const double* Phi = lds + phi * kSlot;
    const double* Psi = lds + psi * kSlot;

    // chains: Z_{r+1} = Z_r Phi (r + 1 < B), a_{b+1} = Psi a_b (b + 1 < nanch);
    // slot 0 holds the ping-pong buffers: Z at [cur * kMaxO * kLd], a at [2 * kMaxO * kLd + cur * kLd]
    constexpr int kZ = kMaxO * kLd;
    for (int idx = tid; idx < o * mm; idx += blockDim.x) {
        const int q = idx / mm, c = idx % mm;
        double pv = 0.0;
        if (c < m) {
            const int col = bordered ? c - 1 : c;
            pv = (col >= 0) ? sc[E.L.proj + q * (k + 1) + col] : 0.0;
        }
        lds[q * kLd + c] = pv;
    }
    if (tid < mm) lds[2 * kZ + tid] = (tid == 0) ? 1.0 : 0.0;
    __syncthreads();
    double* Zg = E.Z + (int64_t)run * E.B * kMaxO * kMaxK;
    double* Ag = E.anch + (int64_t)run * E.nanch * kMaxK;
    const int iters = max(E.B, E.nanch);
    for (int r = 0; r < iters; ++r) {
        const int cur = r & 1, nxt = cur ^ 1;
        const double* zc = lds + cur * kZ;
        const double* ac = lds + 2 * kZ + cur * kLd;
        // publish step r
        if (r < E.B) {
            for (int idx = tid; idx < o * mm; idx += blockDim.x) {
                const int q = idx / mm, c = idx % mm;
                Zg[((int64_t)r * kMaxO + q) * kMaxK + c] = zc[q * kLd + c];
            }
        }
        if (r < E.nanch) {
            for (int c = tid; c < mm; c += blockDim.x) Ag[(int64_t)r * kMaxK + c] = ac[c];
        }
        // advance
        if (tid < o * mm) {
            if (r + 1 < E.B) {
                const int q = tid / mm, c = tid % mm;
                double acc = 0.0;
                for (int l = 0; l < mm; ++l) acc = fma(zc[q * kLd + l], Phi[l * kLd + c], acc);
                lds[nxt * kZ + q * kLd + c] = acc;
            }
        } else if (tid < o * mm + mm) {
            if (r + 1 < E.nanch) {
                const int i = tid - o * mm;
                double acc = 0.0;
                for (int l = 0; l < mm; ++l) acc = fma(Psi[i * kLd + l], ac[l], acc);
                lds[2 * kZ + nxt * kLd + i] = acc;
            }
        }
        __syncthreads();
    }
}

// basis[s][q][run] = scale * Z_{s mod B}[q] . a_{s div B}; one thread per (s, run)
__global__ __launch_bounds__(kBlock) void k_assemble(AssembleArgs A) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (A.steps + 1) * A.nruns;
    if (idx >= total) return;
    const int64_t s = idx / A.nruns;
    const int run = (int)(idx % A.nruns);
    const int m = A.msize[run];
    double y[kMaxO];
#pragma unroll
    for (int q = 0; q < kMaxO; ++q) y[q] = 0.0;
    if (m > 0) {
        const double* z = A.Z + (((int64_t)run * A.B + (s % A.B)) * kMaxO) * kMaxK;
        const double* a = A.anch + ((int64_t)run * A.nanch + (s / A.B)) * kMaxK;
        for (int i = 0; i < m; ++i) {
            const double ai = a[i];
#pragma unroll
            for (int q = 0; q < kMaxO; ++q)
                if (q < A.o) y[q] = fma(z[q * kMaxK + i], ai, y[q]);
        }
        const double sc = A.scale[run];
#pragma unroll
        for (int q = 0; q < kMaxO; ++q) y[q] *= sc;
    }
#pragma unroll
    for (int q = 0; q < kMaxO; ++q)
        if (q < A.o) A.basis[(s * A.o + q) * A.nruns + run] = y[q];
}

// a9, part 1: each block finds the first violated (step, row) among its
// entries (step-major order) and whether a non-finite range was met.
__global__ __launch_bounds__(kBlock) void k_check_blocks(CheckArgs C) {
    __shared__ long long s_min[kBlock / 64];
    __shared__ int s_bad[kBlock / 64];
    const int64_t total = (C.steps + 1) * C.o;
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    long long best = total;
    int bad = 0;
    if (e < total) {
        const int64_t s = e / C.o;
        const int q = (int)(e % C.o);
        const double* M = C.basis + (s * C.o + q) * C.nruns;
        double mid = 0.0, rad = 0.0;
        for (int r = 0; r < C.nruns; ++r) {
            mid = fma(M[r], C.zc[r], mid);
            rad = fma(fabs(M[r]), C.radius[r], rad);
        }
        if (!isfinite(mid) || !isfinite(rad)) bad = 1;
        else if ((mid - rad <= C.uhi[q]) && (mid + rad >= C.ulo[q])) best = e;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const long long o2 = __shfl_xor(best, off, 64);
        best = o2 < best ? o2 : best;
        bad |= __shfl_xor(bad, off, 64);
    }
    if ((threadIdx.x & 63) == 0) { s_min[threadIdx.x >> 6] = best; s_bad[threadIdx.x >> 6] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            best = s_min[w] < best ? s_min[w] : best;
            bad |= s_bad[w];
        }
        C.part[2 * blockIdx.x] = (double)best;
        C.part[2 * blockIdx.x + 1] = (double)bad;
    }
}

// a9, part 2: the first violation over all blocks and its counter-example.
__global__ __launch_bounds__(kBlock) void k_check_final(CheckArgs C, int nb) {
    __shared__ double s_min[kBlock / 64];
    __shared__ double s_bad[kBlock / 64];
    const double total = (double)((C.steps + 1) * C.o);
    double best = total, bad = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        best = fmin(best, C.part[2 * b]);
        bad = fmax(bad, C.part[2 * b + 1]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        best = fmin(best, __shfl_xor(best, off, 64));
        bad = fmax(bad, __shfl_xor(bad, off, 64));
    }
    if ((threadIdx.x & 63) == 0) { s_min[threadIdx.x >> 6] = best; s_bad[threadIdx.x >> 6] = bad; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 1; w < kBlock / 64; ++w) {
        best = fmin(best, s_min[w]);
        bad = fmax(bad, s_bad[w]);
    }
    double* out = C.verdict;
    out[5] = bad > 0.0 ? 4.0 : 0.0;    // KRY_ENUMERIC
    if (best >= total) {
        out[0] = -1.0; out[1] = -1.0; out[2] = 0.0; out[3] = 0.0; out[4] = 0.0;
        for (int r = 0; r < C.nruns; ++r) out[6 + r] = C.zc[r];
        return;
    }
    const int64_t e = (int64_t)best;
    const int64_t s = e / C.o;
    const int q = (int)(e % C.o);
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

size_t expm_lds_bytes() { return (size_t)6 * kSlot * sizeof(double); }

hipError_t expm_prepare() {
    return hipFuncSetAttribute((const void*)k_expm_chain, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)expm_lds_bytes());
}

hipError_t launch_expm_chain(const ExpmArgs& E, int32_t nruns, hipStream_t s) {
    if (nruns <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_expm_chain, dim3(nruns), dim3(kExpmThreads), expm_lds_bytes(), s, E);
    return hipGetLastError();
}

hipError_t launch_assemble(const AssembleArgs& A, hipStream_t s) {
    const int64_t total = (A.steps + 1) * A.nruns;
    const int64_t blocks = (total + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

int check_blocks(int64_t steps, int32_t o) { return (int)(((steps + 1) * o + kBlock - 1) / kBlock); }

hipError_t launch_check(const CheckArgs& C, hipStream_t s) {
    const int nb = check_blocks(C.steps, C.o);
    hipLaunchKernelGGL(k_check_blocks, dim3(nb), dim3(kBlock), 0, s, C);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_check_final, dim3(1), dim3(kBlock), 0, s, C, nb);
    return hipGetLastError();
}

}  // namespace kry
