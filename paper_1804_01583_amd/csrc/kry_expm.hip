// Small dense stage on gfx950: e^{H t} e_1 for every time step (paper
// Section 4.2, Eq. approx-formula), the basis matrix of Section 3.2 and the
// per-step box check that stands in for the LP of Section 2.1.
//
// Per run, one workgroup keeps H in LDS and computes
//   Phi = e^{H dt}   by the degree-18 Taylor polynomial of H dt / 2^s with
//                    |H dt / 2^s|_1 <= 1 (Paterson-Stockmeyer), then s squarings
//                    (the same approximant as the dense stage for larger k),
//   Psi = Phi^B      by squaring (B a power of two near sqrt(steps + 1)),
// then two short chains, Z_r = P Phi^r (r < B) and a_b = Psi^b e_1, so that
//   y_s = beta0 * Z_{s mod B} a_{s div B},   s = 0..steps,
// is assembled for all steps in parallel by k_assemble.  The chains are
// at most B and (steps+1)/B long, instead of one recurrence over all steps.
// The augmented run uses the bordered matrix H~ = [[0, 0], [|b| e_1, T]] and
// P~ = [0, C Q] with scale 1; generator and center runs use T itself.
//
// Transposed route (Section 4.1): a run of A^T from the output row c_q is
// projected on the rows of E^T.  Its generator and center values come from
// T itself; the forcing column's value is the b row's projection of
// beta0 times the integral of e^{T s} e_1, which is the bordered exponential
// again with the whole of T (size k + 1).  Each such exponential is a job;
// k_assemble scatters the jobs' rows to their (output row, column) places.
#include "kry_internal.h"
#include "kry_ldsmm.h"

#include <cmath>

namespace kry {

namespace {

__device__ __forceinline__ const double* run_scal(const ExpmArgs& E, int r) {
    return E.scal + (int64_t)r * E.L.stride;
}

using namespace ldsmm;

// One workgroup per run: Phi, Psi and the two chains.
__global__ __launch_bounds__(kExpmThreads) void k_expm_chain(ExpmArgs E) {
    extern __shared__ double lds[];
    double* S0 = lds;
    double* S1 = lds + 1 * kSlot;
    double* S2 = lds + 2 * kSlot;
    double* S3 = lds + 3 * kSlot;
    double* S4 = lds + 4 * kSlot;
    double* S5 = lds + 5 * kSlot;
    __shared__ double s_red[kExpmThreads / 64];

    // one job per workgroup; a job exponentiates the matrix of one Krylov run
    const int job = blockIdx.x;
    const int run = E.job_run ? E.job_run[job] : job;
    const double* sc = run_scal(E, run);
    const int k = E.L.k, o = E.L.o;
    const int keff = min((int)sc[E.L.misc + MISC_KEFF], (int)sc[E.L.misc + MISC_KSTOP]);
    const int role = E.role[job];
    const bool bordered = role >= 2;
    int m = keff;                            // size of H
    if (role == 2) m = (keff > k - 1 ? k - 1 : keff) + 1;
    if (role == 3) m = keff + 1;
    if (keff <= 0) m = 0;                    // zero start vector: the run contributes nothing
    if (threadIdx.x == 0) {
        E.msize[job] = m;
        // a non-finite start norm or coefficient makes the run's columns NaN
        // (the assembly scales even an empty run), so the box check reports it
        E.scale[job] = sc[E.L.misc + MISC_NONFINITE] != 0.0 ? __builtin_nan("") :
                       (bordered ? 1.0 : sc[E.L.beta + 0]);
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

    // scaling: |X / 2^sq|_1 <= 1
    const double nrm = norm1_slot0(lds, mm, s_red);
    int sq = 0;
    // a non-finite H (flagged by the iteration) gets no squarings
    while (isfinite(nrm) && nrm > ldexp(1.0, sq) && sq < 1100) ++sq;
    const double shrink = ldexp(1.0, -sq);
    for (int idx = tid; idx < mm * mm; idx += blockDim.x) {
        const int i = idx / mm, c = idx % mm;
        S0[i * kLd + c] *= shrink;
    }
    __syncthreads();
    taylor18(lds, mm, 1.0);                                                    // T(X) in slot 4
    auto none = [](int, int) { return 0.0; };

    // LDS matrices below are addressed as lds + slot * kSlot with an integer
    // slot, never through stored pointers, so the accesses stay ds_* (LDS)
    // instructions instead of generic flat ones.
    // undo the scaling: Phi = T(X)^(2^sq), ping-pong between slots 4 and 5
    int phi = 4;
    for (int i = 0; i < sq; ++i) {
        mm_mfma(lds, phi, phi, 9 - phi, mm, none);
        phi = 9 - phi;
    }
    // Psi = Phi^B, ping-pong between slots 1 and 2
    int psi = phi;
    for (int e = 1, nxt = 1; e < E.B; e <<= 1) {
        mm_mfma(lds, psi, psi, nxt, mm, none);
        psi = nxt;
        nxt = 3 - nxt;
    }
    const double* Phi = lds + phi * kSlot;
    const double* Psi = lds + psi * kSlot;

    // chains: Z_{r+1} = Z_r Phi (r + 1 < B), a_{b+1} = Psi a_b (b + 1 < nanch).
    // Thread t < o mm owns Z entry (q, c) = (t / mm, t % mm) and keeps column c
    // of Phi in registers; thread o mm + i (i < mm) owns anchor entry i and
    // keeps row i of Psi.  Slot 0 holds the ping-pong vectors: Z at
    // [cur * kMaxO * kLd], a at [2 * kMaxO * kLd + cur * kLd].
    // When the threads suffice, the Z chain runs in two halves at once: the
    // first B/2 steps by Phi, and Z_{B/2 + r} = Z_r Phi^{B/2} by a second set
    // of o mm threads that keep a column of Phi^{B/2} (the last square before
    // Psi), so the chains take max(B/2, nanch - 1) steps instead of B - 1.
    constexpr int kZ = kMaxO * kLd;
    double* Zg = E.Z + (int64_t)job * E.B * kMaxO * kMaxK;
    double* Ag = E.anch + (int64_t)job * E.nanch * kMaxK;
    const int nz = o * mm;
    const int half = (E.B >= 2 && (2 * o + 1) * mm <= (int)blockDim.x) ? E.B / 2 : 0;
    const int nz2 = half > 0 ? nz : 0;
    const int zlen = half > 0 ? half : E.B;           // steps of the first chain
    const double* Phh = lds + (half > 0 && E.B > 2 ? 3 - psi : phi) * kSlot;   // Phi^{B/2} when half > 0
    const bool zthr = tid < nz;
    const bool z2thr = tid >= nz && tid < nz + nz2;
    const bool athr = tid >= nz + nz2 && tid < nz + nz2 + mm;
    const int zt = zthr ? tid : (z2thr ? tid - nz : 0);
    const int zq = zt / mm, zc_ = zt % mm, ai = athr ? tid - nz - nz2 : 0;
    double reg[kMaxK];
#pragma unroll
    for (int l = 0; l < kMaxK; ++l) {
        double v = 0.0;
        if (l < mm) {
            if (zthr) v = Phi[l * kLd + zc_];
            else if (z2thr) v = Phh[l * kLd + zc_];
            else if (athr) v = Psi[ai * kLd + l];
        }
        reg[l] = v;
    }
    // entries mm..kMaxK-1 of both ping-pong buffers stay zero, so the dot
    // products below run over kMaxK entries without a branch
    for (int idx = tid; idx < 2 * (kMaxO + 1) * kLd; idx += blockDim.x) {
        const int row = idx / kLd, col = idx % kLd;
        const int off = row < 2 * kMaxO ? row * kLd + col : 2 * kZ + (row - 2 * kMaxO) * kLd + col;
        if (col >= mm) lds[off] = 0.0;
    }
    // step 0: Z_0 = P (bordered: column 0 is the augmented variable), a_0 = e_1
    if (zthr) {
        double pv = 0.0;
        if (zc_ < m) {
            const int col = bordered ? zc_ - 1 : zc_;
            pv = (col >= 0) ? sc[E.L.proj + zq * (k + 1) + col] : 0.0;
        }
        lds[zq * kLd + zc_] = pv;
        Zg[(int64_t)zq * kMaxK + zc_] = pv;
    } else if (athr) {
        const double v = ai == 0 ? 1.0 : 0.0;
        lds[2 * kZ + ai] = v;
        Ag[ai] = v;
    }
    __syncthreads();
    const int iters = max(max(zlen - 1, half), E.nanch - 1);
    for (int r = 0; r < iters; ++r) {
        const int cur = r & 1, nxt = cur ^ 1;
        // step r + 1 from step r; two accumulators halve the dependent chain
        if (z2thr && r < half) {
            // Z_{half + r} = Z_r Phi^{half}; Z_r stays in buffer cur (the first
            // chain has written it and stops before overwriting it)
            const double* zr = lds + cur * kZ + zq * kLd;
            double a0 = 0.0, a1 = 0.0;
#pragma unroll
            for (int l = 0; l < kMaxK; l += 2) {
                a0 = fma(zr[l], reg[l], a0);
                a1 = fma(zr[l + 1], reg[l + 1], a1);
            }
            Zg[((int64_t)(half + r) * kMaxO + zq) * kMaxK + zc_] = a0 + a1;
        } else if (zthr && r + 1 < zlen) {
            const double* zr = lds + cur * kZ + zq * kLd;
            double a0 = 0.0, a1 = 0.0;
#pragma unroll
            for (int l = 0; l < kMaxK; l += 2) {
                a0 = fma(zr[l], reg[l], a0);
                a1 = fma(zr[l + 1], reg[l + 1], a1);
            }
            const double v = a0 + a1;
            lds[nxt * kZ + zq * kLd + zc_] = v;
            Zg[((int64_t)(r + 1) * kMaxO + zq) * kMaxK + zc_] = v;
        } else if (athr && r + 1 < E.nanch) {
            const double* ar = lds + 2 * kZ + cur * kLd;
            double a0 = 0.0, a1 = 0.0;
#pragma unroll
            for (int l = 0; l < kMaxK; l += 2) {
                a0 = fma(reg[l], ar[l], a0);
                a1 = fma(reg[l + 1], ar[l + 1], a1);
            }
            const double v = a0 + a1;
            lds[2 * kZ + nxt * kLd + ai] = v;
            Ag[(int64_t)(r + 1) * kMaxK + ai] = v;
        }
        lds_barrier();
    }
}

// basis[s][q][run] = scale * Z_{s mod B}[q] . a_{s div B}; one thread per (s, job).
// With an output map, row q of job j goes to basis[s][job_run[j]][out_col[j][q]]
// of an (o_out x ncols) basis, or nowhere when out_col is negative.
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
        // eight entries at a time, every load of a chunk issued before the
        // first product (a loop of single loads waits for each in turn);
        // entries i < m + 7 <= kMaxK stay inside the row, and those past m,
        // never written, are replaced by zero
        constexpr int kC = 8;
        static_assert(kMaxK % kC == 0, "chunks must tile a row");
        for (int i0 = 0; i0 < m; i0 += kC) {
            double av[kC], zv[kMaxO][kC];
#pragma unroll
            for (int t = 0; t < kC; ++t) av[t] = a[i0 + t];
#pragma unroll
            for (int q = 0; q < kMaxO; ++q)
                if (q < A.o) {
#pragma unroll
                    for (int t = 0; t < kC; ++t) zv[q][t] = z[q * kMaxK + i0 + t];
                }
#pragma unroll
            for (int t = 0; t < kC; ++t) {
                const bool in = i0 + t < m;
#pragma unroll
                for (int q = 0; q < kMaxO; ++q)
                    if (q < A.o && in) y[q] = fma(zv[q][t], av[t], y[q]);
            }
        }
    }
    const double sc = A.scale[run];
#pragma unroll
    for (int q = 0; q < kMaxO; ++q) y[q] *= sc;
    if (A.out_col) {
        const int64_t row = s * A.o_out + A.job_run[run];
#pragma unroll
        for (int q = 0; q < kMaxO; ++q) {
            const int c = q < A.o ? A.out_col[run * kMaxO + q] : -1;
            if (c >= 0) A.basis[row * A.ncols + c] = y[q];
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < kMaxO; ++q)
        if (q < A.o) A.basis[(s * A.o + q) * A.nruns + run] = y[q];
}

// Basis entry of checked column r at step s and checked row q.
__device__ __forceinline__ double check_entry(const CheckArgs& C, int64_t s, int q, int r) {
    if (!C.mapped) return C.basis[(s * C.o + q) * C.nruns + r];
    return C.basis[(s * C.o_all + C.row_of[q]) * C.n_all + C.col_of[r]];
}
__device__ __forceinline__ int check_col(const CheckArgs& C, int r) { return C.mapped ? C.col_of[r] : r; }

// mid = sum_r M_r zc_r and rad = sum_r |M_r| radius_r over the checked columns
__device__ __forceinline__ void check_range(const CheckArgs& C, int64_t s, int q, double& mid, double& rad) {
    for (int r = 0; r < C.nruns; ++r) {
        const double m = check_entry(C, s, q, r);
        const int c = check_col(C, r);
        mid = fma(m, C.zc[c], mid);
        rad = fma(fabs(m), C.radius[c], rad);
    }
}

// The same sums over many columns by a whole wavefront: lane l takes the
// columns l, l + 64, ... in order, then the lanes are added by a fixed
// butterfly; every lane ends with the result.
__device__ __forceinline__ void check_range_wave(const CheckArgs& C, int64_t s, int q, double& mid, double& rad) {
    const int lane = threadIdx.x & 63;
    double m0 = 0.0, r0 = 0.0;
    for (int r = lane; r < C.nruns; r += 64) {
        const double m = check_entry(C, s, q, r);
        const int c = check_col(C, r);
        m0 = fma(m, C.zc[c], m0);
        r0 = fma(fabs(m), C.radius[c], r0);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        m0 += __shfl_xor(m0, off, 64);
        r0 += __shfl_xor(r0, off, 64);
    }
    mid = m0;
    rad = r0;
}

// Plans with more than this many checked columns sum each range with a
// wavefront (check_range_wave), WIDE below; fewer with one thread.
constexpr int kWideCheck = 64;
constexpr int kWideEntries = 16;   // (step, row) entries per wavefront in the wide form

// a9, part 1: each block finds the first violated (step, row) among its
// entries (step-major order) and whether a non-finite range was met.  WIDE:
// each wavefront takes kWideEntries consecutive entries.
template <bool WIDE>
__global__ __launch_bounds__(kBlock) void k_check_blocks(CheckArgs C) {
    __shared__ long long s_min[kBlock / 64];
    __shared__ int s_bad[kBlock / 64];
    const int64_t total = (C.steps + 1) * C.o;
    long long best = total;
    int bad = 0;
    if constexpr (WIDE) {
        const int64_t e0 = ((int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) * kWideEntries;
        for (int i = 0; i < kWideEntries && best == total; ++i) {
            const int64_t e = e0 + i;
            if (e >= total) break;
            const int64_t s = e / C.o;
            const int q = (int)(e % C.o);
            double mid, rad;
            check_range_wave(C, s, q, mid, rad);
            if (!isfinite(mid) || !isfinite(rad)) bad = 1;
            else if ((mid - rad <= C.uhi[q]) && (mid + rad >= C.ulo[q])) best = e;
        }
    } else {
        const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
        if (e < total) {
            const int64_t s = e / C.o;
            const int q = (int)(e % C.o);
            double mid = 0.0, rad = 0.0;
            check_range(C, s, q, mid, rad);
            if (!isfinite(mid) || !isfinite(rad)) bad = 1;
            else if ((mid - rad <= C.uhi[q]) && (mid + rad >= C.ulo[q])) best = e;
        }
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

// a9, part 2: the first violation over all blocks and its counter-example
// (WIDE: the range by wavefront 0, the counter-example's columns by every
// thread).
template <bool WIDE>
__global__ __launch_bounds__(kBlock) void k_check_final(CheckArgs C, int nb) {
    __shared__ double s_min[kBlock / 64];
    __shared__ double s_bad[kBlock / 64];
    __shared__ double s_sol[4];   // lam, dir, mid, rad
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
    for (int w = 0; w < kBlock / 64; ++w) {
        best = fmin(best, s_min[w]);
        bad = fmax(bad, s_bad[w]);
    }
    double* out = C.verdict;
    if (best >= total) {
        if (threadIdx.x == 0) {
            out[5] = bad > 0.0 ? 4.0 : 0.0;    // KRY_ENUMERIC
            out[0] = -1.0; out[1] = -1.0; out[2] = 0.0; out[3] = 0.0; out[4] = 0.0;
        }
        for (int r = threadIdx.x; r < C.nruns; r += kBlock) out[6 + r] = C.zc[check_col(C, r)];
        return;
    }
    const int64_t e = (int64_t)best;
    const int64_t s = e / C.o;
    const int q = (int)(e % C.o);
    if constexpr (WIDE) {
        if (threadIdx.x < 64) {
            double mid, rad;
            check_range_wave(C, s, q, mid, rad);
            if (threadIdx.x == 0) { s_sol[2] = mid; s_sol[3] = rad; }
        }
    } else if (threadIdx.x == 0) {
        double mid = 0.0, rad = 0.0;
        check_range(C, s, q, mid, rad);
        s_sol[2] = mid;
        s_sol[3] = rad;
    }
    __syncthreads();
    const double mid = s_sol[2], rad = s_sol[3];
    double lam = 0.0, dir = 0.0;
    if (mid < C.ulo[q]) { lam = (C.ulo[q] - mid) / rad; dir = 1.0; }
    else if (mid > C.uhi[q]) { lam = (mid - C.uhi[q]) / rad; dir = -1.0; }
    for (int r = threadIdx.x; r < C.nruns; r += kBlock) {
        const double m = check_entry(C, s, q, r);
        const int c = check_col(C, r);
        const double sg = (m > 0.0) ? 1.0 : ((m < 0.0) ? -1.0 : 0.0);
        out[6 + r] = C.zc[c] + dir * lam * sg * C.radius[c];
    }
    if (threadIdx.x == 0) {
        out[5] = bad > 0.0 ? 4.0 : 0.0;    // KRY_ENUMERIC
        out[0] = (double)s;
        out[1] = (double)q;
        out[2] = mid + dir * lam * rad;
        out[3] = mid - rad;
        out[4] = mid + rad;
    }
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

// blocks of the check's first kernel (the wide form's count, the larger)
int check_blocks(int64_t steps, int32_t o) {
    const int64_t per = (int64_t)(kBlock / 64) * kWideEntries;
    return (int)(((steps + 1) * o + per - 1) / per);
}

hipError_t launch_check(const CheckArgs& C, hipStream_t s) {
    const bool wide = C.nruns > kWideCheck;
    const int64_t total = (C.steps + 1) * C.o;
    const int nb = wide ? check_blocks(C.steps, C.o) : (int)((total + kBlock - 1) / kBlock);
    if (wide) hipLaunchKernelGGL(k_check_blocks<true>, dim3(nb), dim3(kBlock), 0, s, C);
    else hipLaunchKernelGGL(k_check_blocks<false>, dim3(nb), dim3(kBlock), 0, s, C);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (wide) hipLaunchKernelGGL(k_check_final<true>, dim3(1), dim3(kBlock), 0, s, C, nb);
    else hipLaunchKernelGGL(k_check_final<false>, dim3(1), dim3(kBlock), 0, s, C, nb);
    return hipGetLastError();
}

}  // namespace kry
