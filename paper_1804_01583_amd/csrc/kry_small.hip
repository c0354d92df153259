// Persistent Lanczos for small symmetric systems (paper Algorithm 3, and
// Algorithm 4's three-vector form): one workgroup runs a whole Krylov run,
// start vector, k iterations and the projections C v_j, in a single launch,
// with its three vectors in LDS.  On a system of a few thousand rows every
// streaming launch of the general path is bound by launch latency, not by
// memory (an iteration moves a few tens of KB), so k iterations cost 2k
// launches there and a few microseconds of barriers here.  All runs of the
// plan go in one launch, one workgroup each.
//
// The results land where the general path puts them (alpha_j, beta_j,
// sigma_j, P = C V and the misc entries of each run's scalar array), so the
// small stage, the assembly and the check read them unchanged.  Vectors are
// normalised as they are formed (v_{j+1} = w / beta_j) instead of carried
// unnormalised; breakdown follows the same rule (beta_j at most
// 1024 eps ||A||_inf ends the run with k_eff = j).
#include "kry_device.h"

namespace kry {

namespace {

using namespace dev;

// Sum of v over the workgroup, the same on every thread: a wave butterfly,
// then the waves' sums added in order.  red: kBlock / 64 doubles.
__device__ __forceinline__ double wg_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();                 // earlier readers of red are done
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
    return t;
}

// The first segment of set s that ends after row c0 (segments are sorted and
// disjoint).
__device__ __forceinline__ int32_t seg_first(const SegTable& T, int s, int64_t c0) {
    int32_t lo = T.set_begin[s], hi = T.set_begin[s + 1];
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (T.hi[mid] <= c0) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// sum over rows r in [c0, c1) of weight_s(r) x[r], rows in ascending order
__device__ __forceinline__ double seg_dot(const SegTable& T, int s, int64_t c0, int64_t c1, const double* x) {
    double acc = 0.0;
    const int32_t end = T.set_begin[s + 1];
    for (int32_t g = seg_first(T, s, c0); g < end && T.lo[g] < c1; ++g) {
        const int64_t a = max(T.lo[g], c0), b = min(T.hi[g], c1);
        const double w = T.w[g];
        for (int64_t r = a; r < b; ++r) acc = fma(w, x[r], acc);
    }
    return acc;
}

__device__ __forceinline__ void seg_fill(const SegTable& T, int s, int64_t c0, int64_t c1, double* x) {
    const int32_t end = T.set_begin[s + 1];
    for (int32_t g = seg_first(T, s, c0); g < end && T.lo[g] < c1; ++g) {
        const int64_t a = max(T.lo[g], c0), b = min(T.hi[g], c1);
        for (int64_t r = a; r < b; ++r) x[r] = T.w[g];
    }
}

// (A x)_r for the rows [c0, c1) of this thread, into y (A in CSR order, or
// the 7-point stencil with its neighbours in ascending index order)
__device__ __forceinline__ void small_matvec(const SmallArgs& a, int64_t c0, int64_t c1, const double* x,
                                             double* y) {
    if (a.kind == 0) {
        for (int64_t r = c0; r < c1; ++r) {
            double acc = 0.0;
            for (int64_t e = a.A.rowptr[r]; e < a.A.rowptr[r + 1]; ++e) acc = fma(a.A.vals[e], x[a.A.colidx[e]], acc);
            y[r] = acc;
        }
        return;
    }
    const StencilArgs& S = a.S;
    const int64_t sx = S.ny * S.nz, sy = S.nz;
    for (int64_t r = c0; r < c1; ++r) {
        const int64_t iz = r % S.nz, iy = (r / S.nz) % S.ny, ix = r / sx;
        const bool xl = ix > 0, xh = ix < S.nx - 1;
        const bool yl = iy > 0, yh = iy < S.ny - 1;
        const bool zl = iz > 0, zh = iz < S.nz - 1;
        double acc = 0.0;
        if (xl) acc = fma(S.cx, x[r - sx], acc);
        if (yl) acc = fma(S.cy, x[r - sy], acc);
        if (zl) acc = fma(S.cz, x[r - 1], acc);
        acc = fma(stencil_diag(S, xl, xh, yl, yh, zl, zh), x[r], acc);
        if (zh) acc = fma(S.cz, x[r + 1], acc);
        if (yh) acc = fma(S.cy, x[r + sy], acc);
        if (xh) acc = fma(S.cx, x[r + sx], acc);
        y[r] = acc;
    }
}

// P[:, c] = C v for the o output sets (v in LDS), recorded by thread 0
__device__ __forceinline__ void small_project(const SmallArgs& a, double* sc, int c, int64_t c0, int64_t c1,
                                              const double* v, double* red) {
    for (int q = 0; q < a.o; ++q) {
        const double t = wg_sum(seg_dot(a.T, a.oset0 + q, c0, c1, v), red);
        if (threadIdx.x == 0) sc[a.L.proj + q * (a.L.k + 1) + c] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_small_lanczos(SmallArgs a) {
    __shared__ double s_v[3][kSmallN];
    __shared__ double s_red[kBlock / 64];
    double* vp = s_v[0];
    double* vc = s_v[1];
    double* w = s_v[2];
    const int64_t n = a.n;
    const int k = a.L.k;
    const int64_t rpt = (n + kBlock - 1) / kBlock;
    const int64_t c0 = min(n, (int64_t)threadIdx.x * rpt), c1 = min(n, c0 + rpt);
    double* sc = a.scal + (int64_t)(a.run0 + blockIdx.x) * a.L.stride;
    const double tau = a.tau_scale * *a.anorm;
    // u_1: generator segments, the center or the forcing
    const int src = a.src[blockIdx.x];
    const double* dense = src == -1 ? a.center : (src == -2 ? a.b : nullptr);
    for (int64_t r = c0; r < c1; ++r) {
        vc[r] = dense != nullptr ? dense[r] : 0.0;
        vp[r] = 0.0;
    }
    if (src >= 0) seg_fill(a.T, src, c0, c1, vc);
    double nrm = 0.0;
    for (int64_t r = c0; r < c1; ++r) nrm = fma(vc[r], vc[r], nrm);
    nrm = wg_sum(nrm, s_red);
    Stage st = stage_update_v(k, 0.0, tau, 1, nrm);
    if (threadIdx.x == 0) {
        sc[a.L.beta + 0] = st.beta;
        sc[a.L.sigma + 1] = st.sigma;
        sc[a.L.misc + MISC_KEFF] = (double)st.keff;
        sc[a.L.misc + MISC_NONFINITE] = st.nonfinite ? 1.0 : 0.0;
        sc[a.L.misc + MISC_KSTOP] = (double)k;
        sc[a.L.misc + MISC_STOPPED] = 0.0;
        sc[a.L.misc + MISC_BOUND] = -1.0;
    }
    double sig = st.sigma;
    for (int64_t r = c0; r < c1; ++r) vc[r] *= sig;
    small_project(a, sc, 0, c0, c1, vc, s_red);
    __syncthreads();                                 // vc whole before the product reads it
    double beta_prev = 0.0;
    int j = 1;
    for (; j <= k && sig != 0.0; ++j) {
        // w = A v_j - beta_{j-1} v_{j-1}; alpha_j = v_j . w; w -= alpha_j v_j
        small_matvec(a, c0, c1, vc, w);
        double dot = 0.0;
        for (int64_t r = c0; r < c1; ++r) {
            w[r] = fma(-beta_prev, vp[r], w[r]);
            dot = fma(vc[r], w[r], dot);
        }
        const double alpha = wg_sum(dot, s_red);
        nrm = 0.0;
        for (int64_t r = c0; r < c1; ++r) {
            w[r] = fma(-alpha, vc[r], w[r]);
            nrm = fma(w[r], w[r], nrm);
        }
        nrm = wg_sum(nrm, s_red);
        st = stage_update_v(k, sig, tau, j + 1, nrm);
        if (threadIdx.x == 0) {
            sc[a.L.alpha + j] = alpha;
            sc[a.L.beta + j] = st.beta;
            sc[a.L.sigma + j + 1] = st.sigma;
            if (st.keff >= 0) sc[a.L.misc + MISC_KEFF] = (double)st.keff;
            if (st.nonfinite) sc[a.L.misc + MISC_NONFINITE] = 1.0;
        }
        // v_{j+1} = sigma_{j+1} w; the buffers rotate
        sig = st.sigma;
        for (int64_t r = c0; r < c1; ++r) w[r] *= sig;
        double* t = vp;
        vp = vc;
        vc = w;
        w = t;
        beta_prev = st.beta;
        small_project(a, sc, j, c0, c1, vc, s_red);
        __syncthreads();
    }
    // after a breakdown the later entries are those of zero vectors
    if (threadIdx.x == 0) {
        for (; j <= k; ++j) {
            sc[a.L.alpha + j] = 0.0;
            sc[a.L.beta + j] = 0.0;
            sc[a.L.sigma + j + 1] = 0.0;
            for (int q = 0; q < a.o; ++q) sc[a.L.proj + q * (k + 1) + j] = 0.0;
        }
    }
}

// sum over rows r in [c0, c1) of x[r] y[r] for the stored vector x
__device__ __forceinline__ double row_dot(const double* __restrict__ x, const double* y, int64_t c0, int64_t c1) {
    double acc = 0.0;
    for (int64_t r = c0; r < c1; ++r) acc = fma(x[r], y[r], acc);
    return acc;
}

// Arnoldi (Algorithm 1 with classical Gram-Schmidt applied twice, as the
// general path) for one run per workgroup: w and v_j in LDS, the basis
// v_1..v_{k+1} in this workgroup's slice of a.basis (at these sizes it
// stays in L2).  A pass forms the j dot products from per-thread partials:
// each wave sums a dot by butterfly, the waves' sums land in LDS and every
// thread adds them in wave order, one barrier per pass.
__global__ __launch_bounds__(kBlock) void k_small_arnoldi(SmallArgs a) {
    constexpr int NW = kBlock / 64;
    __shared__ double s_vc[kSmallN];
    __shared__ double s_w[kSmallN];
    __shared__ double s_dot[kSmallArnK][NW];
    __shared__ double s_h[kSmallArnK];
    __shared__ double s_red[NW];
    const int64_t n = a.n;
    const int k = a.L.k;
    const int64_t rpt = (n + kBlock - 1) / kBlock;
    const int64_t c0 = min(n, (int64_t)threadIdx.x * rpt), c1 = min(n, c0 + rpt);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* sc = a.scal + (int64_t)(a.run0 + blockIdx.x) * a.L.stride;
    double* V = a.basis + (int64_t)blockIdx.x * (k + 1) * n;    // v_{i+1} at V + i n
    const double tau = a.tau_scale * *a.anorm;
    const int src = a.src[blockIdx.x];
    const double* dense = src == -1 ? a.center : (src == -2 ? a.b : nullptr);
    for (int64_t r = c0; r < c1; ++r) s_vc[r] = dense != nullptr ? dense[r] : 0.0;
    if (src >= 0) seg_fill(a.T, src, c0, c1, s_vc);
    double nrm = 0.0;
    for (int64_t r = c0; r < c1; ++r) nrm = fma(s_vc[r], s_vc[r], nrm);
    nrm = wg_sum(nrm, s_red);
    Stage st = stage_update_v(k, 0.0, tau, 1, nrm);
    if (threadIdx.x == 0) {
        sc[a.L.beta + 0] = st.beta;
        sc[a.L.sigma + 1] = st.sigma;
        sc[a.L.misc + MISC_KEFF] = (double)st.keff;
        sc[a.L.misc + MISC_NONFINITE] = st.nonfinite ? 1.0 : 0.0;
        sc[a.L.misc + MISC_KSTOP] = (double)k;
        sc[a.L.misc + MISC_STOPPED] = 0.0;
        sc[a.L.misc + MISC_BOUND] = -1.0;
    }
    double sig = st.sigma;
    for (int64_t r = c0; r < c1; ++r) {
        s_vc[r] *= sig;
        V[r] = s_vc[r];
    }
    small_project(a, sc, 0, c0, c1, s_vc, s_red);
    __syncthreads();
    int j = 1;
    for (; j <= k && sig != 0.0; ++j) {
        small_matvec(a, c0, c1, s_vc, s_w);
        // two classical Gram-Schmidt passes against v_1..v_j; this thread's
        // own rows of w only, so no barrier is needed between the passes'
        // subtractions and the next dots
        for (int pass = 0; pass < 2; ++pass) {
            for (int i = 0; i < j; ++i) {
                double d = row_dot(V + (int64_t)i * n, s_w, c0, c1);
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) d += __shfl_xor(d, off, 64);
                if (lane == 0) s_dot[i][wave] = d;
            }
            __syncthreads();
            for (int i = 0; i < j; ++i) {
                double h = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) h += s_dot[i][w];
                for (int64_t r = c0; r < c1; ++r) s_w[r] = fma(-h, V[(int64_t)i * n + r], s_w[r]);
                if (threadIdx.x == 0) s_h[i] = pass == 0 ? h : s_h[i] + h;
            }
            __syncthreads();     // s_dot is rewritten by the next pass
        }
        if (threadIdx.x == 0) {
            bool bad = false;
            for (int i = 0; i < j; ++i) {
                sc[a.L.hess + i * k + (j - 1)] = s_h[i];
                bad = bad || !isfinite(s_h[i]);
            }
            if (bad) sc[a.L.misc + MISC_NONFINITE] = 1.0;
        }
        nrm = 0.0;
        for (int64_t r = c0; r < c1; ++r) nrm = fma(s_w[r], s_w[r], nrm);
        nrm = wg_sum(nrm, s_red);
        st = stage_update_v(k, sig, tau, j + 1, nrm);
        if (threadIdx.x == 0) {
            sc[a.L.beta + j] = st.beta;
            sc[a.L.sigma + j + 1] = st.sigma;
            if (st.keff >= 0) sc[a.L.misc + MISC_KEFF] = (double)st.keff;
            if (st.nonfinite) sc[a.L.misc + MISC_NONFINITE] = 1.0;
        }
        sig = st.sigma;
        for (int64_t r = c0; r < c1; ++r) {
            const double v = s_w[r] * sig;
            s_vc[r] = v;
            V[(int64_t)j * n + r] = v;
        }
        small_project(a, sc, j, c0, c1, s_vc, s_red);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (; j <= k; ++j) {
            for (int i = 0; i < j; ++i) sc[a.L.hess + i * k + (j - 1)] = 0.0;
            sc[a.L.beta + j] = 0.0;
            sc[a.L.sigma + j + 1] = 0.0;
            for (int q = 0; q < a.o; ++q) sc[a.L.proj + q * (k + 1) + j] = 0.0;
        }
    }
}

}  // namespace

hipError_t launch_small_arnoldi(const SmallArgs& a, int32_t nruns, hipStream_t s) {
    if (a.n < 1 || a.n > kSmallN || nruns < 1 || nruns > kSmallRuns || a.o > kMaxO || a.L.k > kSmallArnK ||
        a.basis == nullptr)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_small_arnoldi, dim3(nruns), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_small_lanczos(const SmallArgs& a, int32_t nruns, hipStream_t s) {
    if (a.n < 1 || a.n > kSmallN || nruns < 1 || nruns > kSmallRuns || a.o > kMaxO) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_small_lanczos, dim3(nruns), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace kry
