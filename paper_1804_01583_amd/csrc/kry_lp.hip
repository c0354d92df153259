// Per-step safety LP (paper Section 2.1) for a polytopic initial set and a
// conjunction of output halfspaces.
//
// At step s the reachable outputs are y = M_s z + f_s (M_s: the generator
// columns of the basis, f_s: the sum of its fixed columns).  The step is
// unsafe when some z with zlo <= z <= zhi, G z <= h also has U y <= u.  In
// w = z - zlo >= 0 the rows are the bounds w_j <= zhi_j - zlo_j and
//     G w <= h - G zlo,  (U M_s) w <= u - U (M_s zlo + f_s),
// the G and U rows divided by their magnitude max(|a|_max, |b|) taken in z
// (b = h, or u - U f_s), so that a row whose coefficients vanish against
// its right-hand side reads 0 <= sign(b), and a row below 1e-280 in both is
// dropped.  Phase one with a single artificial variable t in the G and U
// rows (a w - t <= b, minimise t) decides feasibility: after t enters at the
// row of the most negative b every right-hand side is non-negative, and the
// simplex with Bland's rule (smallest entering index, ratio ties to the
// smallest basic index) cannot cycle.  The step is unsafe
// when the optimum t* <= tol (the LP tolerance, on the scaled rows); the
// basic w then gives the counter-example, which violates no scaled row by
// more than t*.
//
// One wavefront per step holds the dense tableau in LDS: rows are the
// constraints (lane i owns row i), columns w, t, the slacks and the
// right-hand side, plus the reduced-cost row.
#include "kry_internal.h"

#include <cmath>

namespace kry {

namespace {

constexpr int kLpThreads = 64;
constexpr int kLpCols = kLpMaxD + 1 + kLpMaxRows + 1;   // w, t, slacks, rhs
constexpr int kLpLd = kLpCols + 1;

__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

__global__ __launch_bounds__(kLpThreads) void k_lp_steps(LpArgs L) {
    __shared__ double T[(kLpMaxRows + 1) * kLpLd];
    __shared__ int bas[kLpMaxRows];
    __shared__ double sM[kMaxO * kLpMaxD];
    __shared__ double sf[kMaxO];
    const int lane = threadIdx.x;
    const int64_t s = blockIdx.x;
    const int d = L.d, o = L.o;
    const int m = d + L.mI + L.mU;
    const int C = d + 1 + m + 1;              // columns incl. rhs
    const int tcol = d, rhs = C - 1;
    double* rec = L.rec + s * kLpRec;

    // this step's generator columns and fixed sum
    const double* Bs = L.basis + s * o * L.ncols;
    for (int idx = lane; idx < o * d; idx += kLpThreads) sM[idx] = Bs[(idx / d) * L.ncols + idx % d];
    if (lane < o) {
        double f = 0.0;
        for (int c = d; c < L.ncols; ++c) f += Bs[lane * L.ncols + c];
        sf[lane] = f;
    }
    __syncthreads();

    // constraint rows (lane i builds row i); G and U rows scaled by their magnitude
    bool bad = false;
    if (lane < m) {
        double a[kLpMaxD];
        double b;
        const int i = lane;
        double bz;                           // right-hand side in z
        if (i < d) {
#pragma unroll
            for (int j = 0; j < kLpMaxD; ++j) a[j] = j == i ? 1.0 : 0.0;
            bz = L.zhi[i];
        } else if (i < d + L.mI) {
            const double* g = L.G + (int64_t)(i - d) * d;
            bz = L.h[i - d];
#pragma unroll
            for (int j = 0; j < kLpMaxD; ++j) a[j] = j < d ? g[j] : 0.0;
        } else {
            const double* ur = L.U + (int64_t)(i - d - L.mI) * o;
            bz = L.u[i - d - L.mI];
#pragma unroll
            for (int j = 0; j < kLpMaxD; ++j) a[j] = 0.0;
            for (int q = 0; q < o; ++q) {
                bz -= ur[q] * sf[q];
#pragma unroll
                for (int j = 0; j < kLpMaxD; ++j)
                    if (j < d) a[j] = fma(ur[q], sM[q * d + j], a[j]);
            }
        }
        // in w = z - zlo
        b = bz;
#pragma unroll
        for (int j = 0; j < kLpMaxD; ++j)
            if (j < d) b -= a[j] * L.zlo[j];
        double nrm = fabs(bz);
#pragma unroll
        for (int j = 0; j < kLpMaxD; ++j) nrm = fmax(nrm, fabs(a[j]));
        bad = !std::isfinite(nrm) || !std::isfinite(b);
        const bool bound = i < d;
        const bool drop = !bound && nrm < 1e-280;
        const double sc = bound || drop ? 1.0 : 1.0 / nrm;
        double* row = T + i * kLpLd;
        for (int c = 0; c < C; ++c) row[c] = 0.0;
        if (!drop)
            for (int j = 0; j < d; ++j) row[j] = a[j] * sc;
        row[tcol] = bound ? 0.0 : -1.0;       // the box bounds are not relaxed
        row[d + 1 + i] = 1.0;
        row[rhs] = drop ? 1.0 : (bound ? L.zhi[i] - L.zlo[i] : b * sc);
        bas[i] = d + 1 + i;
    }
    // reduced costs of min t with the slack basis
    for (int c = lane; c < C; c += kLpThreads) T[m * kLpLd + c] = c == tcol ? 1.0 : 0.0;
    const bool any_bad = __any(bad);
    __syncthreads();
    if (any_bad) {
        if (lane == 0) { rec[0] = -1.0; rec[1] = 0.0; }
        return;
    }

    auto pivot = [&](int r, int e) {
        const double piv = T[r * kLpLd + e];
        __syncthreads();
        for (int c = lane; c < C; c += kLpThreads) T[r * kLpLd + c] /= piv;
        __syncthreads();
        for (int row = lane; row <= m; row += kLpThreads) {
            if (row == r) continue;
            double* tr = T + row * kLpLd;
            const double f = tr[e];
            if (f != 0.0) {
                const double* pr = T + r * kLpLd;
                for (int c = 0; c < C; ++c) tr[c] = fma(-f, pr[c], tr[c]);
                tr[e] = 0.0;
            }
        }
        if (lane == 0) bas[r] = e;
        __syncthreads();
    };

    // t enters at the row of the most negative right-hand side
    int r0 = m;
    double bmin = 0.0;
    for (int i = 0; i < m; ++i) {
        const double bi = T[i * kLpLd + rhs];
        if (bi < bmin) { bmin = bi; r0 = i; }
    }
    double tstar = 0.0;
    int status = 1;                          // feasible unless phase one says otherwise
    if (r0 < m) {
        pivot(r0, tcol);
        int it = 0;
        for (;;) {
            // t left the basis: t = 0 is reached
            bool t_basic = false;
            for (int i = 0; i < m; ++i) t_basic = t_basic || bas[i] == tcol;
            if (!t_basic) { tstar = 0.0; break; }
            if (it++ >= L.max_pivots) { status = -1; break; }
            // Bland: the smallest non-basic column with a negative reduced cost
            int cand = 1 << 30;
            for (int c = lane; c < rhs; c += kLpThreads) {
                bool basic = false;
                for (int i = 0; i < m; ++i) basic = basic || bas[i] == c;
                if (!basic && T[m * kLpLd + c] < -1e-12) cand = min(cand, c);
            }
            const int e = wave_min_int(cand);
            if (e >= (1 << 30)) {            // optimal
                for (int i = 0; i < m; ++i)
                    if (bas[i] == tcol) tstar = T[i * kLpLd + rhs];
                break;
            }
            // ratio test; ties go to the smallest basic index
            double best = INFINITY;
            int bkey = 1 << 30, brow = -1;
            if (lane < m) {
                const double a = T[lane * kLpLd + e];
                if (a > 1e-12) { best = T[lane * kLpLd + rhs] / a; bkey = bas[lane]; brow = lane; }
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ob = __shfl_xor(best, off, 64);
                const int ok = __shfl_xor(bkey, off, 64);
                const int orow = __shfl_xor(brow, off, 64);
                if (ob < best || (ob == best && ok < bkey)) { best = ob; bkey = ok; brow = orow; }
            }
            if (brow < 0) { status = -1; break; }   // unbounded: cannot happen with t >= 0
            pivot(brow, e);
        }
        if (status == 1 && tstar > L.tol) status = 0;
    }
    // counter-example: the basic w (non-basic w are 0)
    if (lane == 0) {
        rec[0] = (double)status;
        rec[1] = tstar;
    }
    if (lane < kLpMaxD) {
        double w = 0.0;
        if (lane < d)
            for (int i = 0; i < m; ++i)
                if (bas[i] == lane) w = T[i * kLpLd + rhs];
        rec[2 + lane] = lane < d ? L.zlo[lane] + w : 0.0;
    }
}

// The first unsafe step, whether an undecided step precedes it (status 4,
// KRY_ENUMERIC), and its counter-example z with the outputs y = M z + f.
__global__ __launch_bounds__(256) void k_lp_first(LpArgs L) {
    __shared__ long long s_first[4], s_und[4];
    long long first = L.steps + 1, und = L.steps + 1;
    for (int64_t s = threadIdx.x; s <= L.steps; s += 256) {
        const double f = L.rec[s * kLpRec];
        if (f > 0.5 && s < first) first = s;
        if (f < -0.5 && s < und) und = s;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        first = min(first, (long long)__shfl_xor(first, off, 64));
        und = min(und, (long long)__shfl_xor(und, off, 64));
    }
    if ((threadIdx.x & 63) == 0) { s_first[threadIdx.x >> 6] = first; s_und[threadIdx.x >> 6] = und; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 1; w < 4; ++w) { first = min(first, s_first[w]); und = min(und, s_und[w]); }
    double* v = L.verdict;
    const bool found = first <= L.steps;
    v[0] = found ? (double)first : -1.0;
    v[1] = und <= (found ? first : L.steps) ? 4.0 : 0.0;
    for (int j = 0; j < kLpMaxD; ++j) v[2 + j] = found && j < L.d ? L.rec[first * kLpRec + 2 + j] : 0.0;
    for (int q = 0; q < kMaxO; ++q) {
        double y = 0.0;
        if (found && q < L.o) {
            const double* row = L.basis + (first * L.o + q) * L.ncols;
            for (int c = 0; c < L.ncols; ++c) y += row[c] * (c < L.d ? L.rec[first * kLpRec + 2 + c] : 1.0);
        }
        v[2 + kLpMaxD + q] = y;
    }
}

}  // namespace

hipError_t launch_lp(const LpArgs& L, hipStream_t s) {
    hipLaunchKernelGGL(k_lp_steps, dim3((unsigned)(L.steps + 1)), dim3(kLpThreads), 0, s, L);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lp_first, dim3(1), dim3(256), 0, s, L);
    return hipGetLastError();
}

}  // namespace kry
