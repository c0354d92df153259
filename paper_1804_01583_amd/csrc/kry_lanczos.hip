// Streaming kernels of the Lanczos process (paper Algorithms 3 and 4) on gfx950.
//
// One Lanczos iteration j of a batch of P independent runs is two launches:
//   spmv  : w = A v_j - beta_{j-1} v_{j-1}        and the dot alpha_j = v_j . w
//   sweep : w -= alpha_j v_j,  beta_j = |w|,  P[:, j] = C w / beta_j
// Vectors are stored unnormalised (u_j, with v_j = sigma_j u_j and
// sigma_j = 1 / beta_{j-1} kept on the device), so no pass is spent on the
// normalisation of Algorithm 3; the scale is applied where the vector is read.
// Batches store their P vectors interleaved ([n][P]) so a gathered column of
// A reads P contiguous values.
//
// Grid-wide sums are deterministic: each block reduces its rows in a fixed
// order (per-thread row loop, wave butterfly, LDS across waves), writes one
// partial per value, and the last block to arrive sums all partials in block
// order.  The row -> block partition depends on n only, so a run's arithmetic
// does not depend on which batch (or P) it is advanced in.
#include "kry_internal.h"

#include <cmath>

namespace kry {

namespace {

struct OpSum {
    static __device__ __forceinline__ double apply(double a, double b) { return a + b; }
    static constexpr double identity = 0.0;
};
struct OpMax {
    static __device__ __forceinline__ double apply(double a, double b) { return a > b ? a : b; }
    static constexpr double identity = 0.0;   // used on absolute values only
};

template <int NV, class Op>
__device__ __forceinline__ void wave_allreduce(double (&v)[NV]) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = Op::apply(v[i], __shfl_xor(v[i], off, 64));
    }
}

// Reduces v over the block; thread i < NV returns total i.  `lds` holds
// (kBlock / 64) * NV doubles.  Must be reached by every thread.
template <int NV, class Op>
__device__ __forceinline__ double block_reduce(double (&v)[NV], double* lds) {
    wave_allreduce<NV, Op>(v);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) lds[wave * NV + i] = v[i];
    }
    __syncthreads();
    double t = Op::identity;
    if (threadIdx.x < NV) {
        t = lds[threadIdx.x];
#pragma unroll
        for (int w = 1; w < kBlock / 64; ++w) t = Op::apply(t, lds[w * NV + threadIdx.x]);
    }
    __syncthreads();
    return t;
}

// Block partials -> grid totals.  Returns true in the last block to arrive;
// there s_tot[i] holds total i (visible to all threads of that block).  The
// arrival counter is returned to 0 for the next launch.
template <int NV, class Op>
__device__ bool grid_reduce(double (&v)[NV], double* partials, unsigned int* counter,
                            double* s_lds, double* s_tot) {
    __shared__ int s_last;
    const double t = block_reduce<NV, Op>(v, s_lds);
    if (threadIdx.x < NV) {
        __hip_atomic_store(&partials[(int64_t)blockIdx.x * NV + threadIdx.x], t, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev =
            __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!s_last) return false;
    __threadfence();
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = Op::identity;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
            acc[i] = Op::apply(acc[i], __hip_atomic_load(&partials[(int64_t)b * NV + i],
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    const double tot = block_reduce<NV, Op>(acc, s_lds);
    if (threadIdx.x < NV) s_tot[threadIdx.x] = tot;
    if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    return true;
}

// First segment of set `s` with hi > r0, and first with lo >= r1.
__device__ void seg_range(const SegTable& T, int s, int64_t r0, int64_t r1, int32_t* b, int32_t* e) {
    int lo = T.set_begin[s], hi = T.set_begin[s + 1];
    int a = lo, z = hi;
    while (a < z) {
        const int m = (a + z) >> 1;
        if (T.hi[m] > r0) z = m; else a = m + 1;
    }
    int c = a, d = hi;
    while (c < d) {
        const int m = (c + d) >> 1;
        if (T.lo[m] >= r1) d = m; else c = m + 1;
    }
    *b = a;
    *e = c;
}

// Membership of increasing rows in one segment set, amortised O(1) per row.
struct SegCursor {
    int32_t cur, end;
    __device__ __forceinline__ double weight(const SegTable& T, int64_t r) {
        while (cur < end && T.hi[cur] <= r) ++cur;
        return (cur < end && T.lo[cur] <= r) ? T.w[cur] : 0.0;
    }
};

__device__ __forceinline__ double* run_scal(const BatchArgs& B, int p) {
    return B.scal + (int64_t)(B.run0 + p) * B.L.stride;
}

__device__ __forceinline__ int64_t block_row0(const BatchArgs& B) {
    return (int64_t)blockIdx.x * B.rows_per_block;
}

// ---------------------------------------------------------------------------

__global__ void k_fill_zero_u32(unsigned int* p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// max_r sum_e |vals[e]| (row sums in CSR order, one thread per row)
__global__ __launch_bounds__(kBlock) void k_row_abs_max(CsrArgs A, int64_t n, int64_t rows_per_block,
                                                        double* partials, unsigned int* counter,
                                                        double* out) {
    __shared__ double s_lds[(kBlock / 64) * 1];
    __shared__ double s_tot[1];
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    double v[1] = {0.0};
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        double s = 0.0;
        for (int64_t e = A.rowptr[r]; e < A.rowptr[r + 1]; ++e) s += fabs(A.vals[e]);
        v[0] = s > v[0] ? s : v[0];
    }
    if (grid_reduce<1, OpMax>(v, partials, counter, s_lds, s_tot)) {
        if (threadIdx.x == 0) *out = s_tot[0];
    }
}

// a2: start vectors u_1 of the runs, beta0 = |u_1|, sigma_1 = 1/beta0 and
// P[:, 0] = C v_1 (Algorithm 4, first two statements).
template <int P, int O>
__global__ __launch_bounds__(kBlock) void k_start(StartSrc src, SegTable T, int32_t oset0,
                                                  double* __restrict__ u, BatchArgs B) {
    constexpr int NV = P * (1 + O);
    __shared__ double s_lds[(kBlock / 64) * NV];
    __shared__ double s_tot[NV];
    __shared__ int32_t s_b[P + O], s_e[P + O];
    const int64_t r0 = block_row0(B);
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    if (threadIdx.x < P + O) {
        const int i = threadIdx.x;
        const int set = (i < P) ? src.set[i] : oset0 + (i - P);
        if (set >= 0) seg_range(T, set, r0, r1, &s_b[i], &s_e[i]);
        else { s_b[i] = 0; s_e[i] = 0; }
    }
    __syncthreads();
    SegCursor cur[P + O];
#pragma unroll
    for (int i = 0; i < P + O; ++i) { cur[i].cur = s_b[i]; cur[i].end = s_e[i]; }
    const double* dense[P];
#pragma unroll
    for (int p = 0; p < P; ++p) dense[p] = src.dense[p];

    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        double val[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (dense[p] != nullptr) val[p] = dense[p][r];
            else if (src.set[p] >= 0) val[p] = cur[p].weight(T, r);
            else val[p] = 0.0;
            u[r * P + p] = val[p];
            acc[p] = fma(val[p], val[p], acc[p]);
        }
#pragma unroll
        for (int q = 0; q < O; ++q) {
            const double cw = cur[P + q].weight(T, r);
            if (cw != 0.0) {
#pragma unroll
                for (int p = 0; p < P; ++p) acc[P + q * P + p] = fma(cw, val[p], acc[P + q * P + p]);
            }
        }
    }
    if (grid_reduce<NV, OpSum>(acc, B.partials, B.counter, s_lds, s_tot)) {
        if (threadIdx.x < P) {
            const int p = threadIdx.x;
            double* sc = run_scal(B, p);
            const double beta0 = sqrt(s_tot[p]);
            const double sig = beta0 > 0.0 ? 1.0 / beta0 : 0.0;
            sc[B.L.beta + 0] = beta0;
            sc[B.L.sigma + 1] = sig;
            for (int q = 0; q < O; ++q) sc[B.L.proj + q * (B.L.k + 1) + 0] = sig * s_tot[P + q * P + p];
            sc[B.L.misc + MISC_KEFF] = beta0 > 0.0 ? (double)B.L.k : 0.0;
            sc[B.L.misc + MISC_DONE] = beta0 > 0.0 ? 0.0 : 1.0;
            sc[B.L.misc + MISC_NONFINITE] = isfinite(beta0) ? 0.0 : 1.0;
        }
    }
}

// a3 + first half of a4: w = sigma_j A u_j - beta_{j-1} sigma_{j-1} u_{j-1};
// alpha_j = (sigma_j u_j) . w.  LPR lanes cooperate on one row.
template <int P, int LPR>
__global__ __launch_bounds__(kBlock) void k_spmv_csr(CsrArgs A, const double* __restrict__ ucur,
                                                     const double* __restrict__ uprev,
                                                     double* __restrict__ w, BatchArgs B, int j) {
    __shared__ double s_lds[(kBlock / 64) * P];
    __shared__ double s_tot[P];
    double sig[P], cprev[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const double* sc = run_scal(B, p);
        sig[p] = sc[B.L.sigma + j];
        cprev[p] = (j > 1) ? sc[B.L.beta + j - 1] * sc[B.L.sigma + j - 1] : 0.0;
    }
    const int64_t r0 = block_row0(B);
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    constexpr int G = kBlock / LPR;
    const int sub = threadIdx.x % LPR;
    double dot[P];
#pragma unroll
    for (int p = 0; p < P; ++p) dot[p] = 0.0;
    for (int64_t r = r0 + threadIdx.x / LPR; r < r1; r += G) {
        const int64_t e0 = A.rowptr[r], e1 = A.rowptr[r + 1];
        double acc[P];
#pragma unroll
        for (int p = 0; p < P; ++p) acc[p] = 0.0;
        for (int64_t e = e0 + sub; e < e1; e += LPR) {
            const int64_t c = A.colidx[e];
            const double a = A.vals[e];
#pragma unroll
            for (int p = 0; p < P; ++p) acc[p] = fma(a, ucur[c * P + p], acc[p]);
        }
        if (LPR > 1) {
#pragma unroll
            for (int off = LPR / 2; off >= 1; off >>= 1) {
#pragma unroll
                for (int p = 0; p < P; ++p) acc[p] += __shfl_xor(acc[p], off, LPR);
            }
        }
        if (sub == 0) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                double y = sig[p] * acc[p];
                if (j > 1) y = fma(-cprev[p], uprev[r * P + p], y);
                w[r * P + p] = y;
                dot[p] = fma(sig[p] * ucur[r * P + p], y, dot[p]);
            }
        }
    }
    if (grid_reduce<P, OpSum>(dot, B.partials, B.counter, s_lds, s_tot)) {
        if (threadIdx.x < P) {
            double* sc = run_scal(B, threadIdx.x);
            const double a = s_tot[threadIdx.x];
            sc[B.L.alpha + j] = a;
            if (!isfinite(a)) sc[B.L.misc + MISC_NONFINITE] = 1.0;
        }
    }
}

// Matrix-free 7-point stencil version of k_spmv_csr (zero outside the grid),
// neighbours summed in ascending index order like a CSR row.
template <int P>
__global__ __launch_bounds__(kBlock) void k_spmv_stencil(StencilArgs S, const double* __restrict__ ucur,
                                                         const double* __restrict__ uprev,
                                                         double* __restrict__ w, BatchArgs B, int j) {
    __shared__ double s_lds[(kBlock / 64) * P];
    __shared__ double s_tot[P];
    double sig[P], cprev[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const double* sc = run_scal(B, p);
        sig[p] = sc[B.L.sigma + j];
        cprev[p] = (j > 1) ? sc[B.L.beta + j - 1] * sc[B.L.sigma + j - 1] : 0.0;
    }
    const int64_t r0 = block_row0(B);
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    const int64_t sx = S.ny * S.nz, sy = S.nz;
    double dot[P];
#pragma unroll
    for (int p = 0; p < P; ++p) dot[p] = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        const int64_t iz = r % S.nz;
        const int64_t t = r / S.nz;
        const int64_t iy = t % S.ny;
        const int64_t ix = t / S.ny;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            double acc = 0.0;
            if (ix > 0) acc = fma(S.cx, ucur[(r - sx) * P + p], acc);
            if (iy > 0) acc = fma(S.cy, ucur[(r - sy) * P + p], acc);
            if (iz > 0) acc = fma(S.cz, ucur[(r - 1) * P + p], acc);
            acc = fma(S.c0, ucur[r * P + p], acc);
            if (iz < S.nz - 1) acc = fma(S.cz, ucur[(r + 1) * P + p], acc);
            if (iy < S.ny - 1) acc = fma(S.cy, ucur[(r + sy) * P + p], acc);
            if (ix < S.nx - 1) acc = fma(S.cx, ucur[(r + sx) * P + p], acc);
            double y = sig[p] * acc;
            if (j > 1) y = fma(-cprev[p], uprev[r * P + p], y);
            w[r * P + p] = y;
            dot[p] = fma(sig[p] * ucur[r * P + p], y, dot[p]);
        }
    }
    if (grid_reduce<P, OpSum>(dot, B.partials, B.counter, s_lds, s_tot)) {
        if (threadIdx.x < P) {
            double* sc = run_scal(B, threadIdx.x);
            const double a = s_tot[threadIdx.x];
            sc[B.L.alpha + j] = a;
            if (!isfinite(a)) sc[B.L.misc + MISC_NONFINITE] = 1.0;
        }
    }
}

// Second half of a4 + a5 + a6: w -= alpha_j v_j; beta_j = |w|; breakdown test;
// sigma_{j+1} = 1/beta_j; P[:, j] = sigma_{j+1} C w.
template <int P, int O>
__global__ __launch_bounds__(kBlock) void k_sweep(SegTable T, int32_t oset0,
                                                  const double* __restrict__ ucur,
                                                  double* __restrict__ w, BatchArgs B, int j) {
    constexpr int NV = P * (1 + O);
    __shared__ double s_lds[(kBlock / 64) * NV];
    __shared__ double s_tot[NV];
    __shared__ int32_t s_b[O], s_e[O];
    const int64_t r0 = block_row0(B);
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    if (threadIdx.x < O) seg_range(T, oset0 + threadIdx.x, r0, r1, &s_b[threadIdx.x], &s_e[threadIdx.x]);
    double coef[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const double* sc = run_scal(B, p);
        coef[p] = sc[B.L.alpha + j] * sc[B.L.sigma + j];
    }
    __syncthreads();
    SegCursor cur[O];
#pragma unroll
    for (int q = 0; q < O; ++q) { cur[q].cur = s_b[q]; cur[q].end = s_e[q]; }
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        double val[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            val[p] = fma(-coef[p], ucur[r * P + p], w[r * P + p]);
            w[r * P + p] = val[p];
            acc[p] = fma(val[p], val[p], acc[p]);
        }
#pragma unroll
        for (int q = 0; q < O; ++q) {
            const double cw = cur[q].weight(T, r);
            if (cw != 0.0) {
#pragma unroll
                for (int p = 0; p < P; ++p) acc[P + q * P + p] = fma(cw, val[p], acc[P + q * P + p]);
            }
        }
    }
    if (grid_reduce<NV, OpSum>(acc, B.partials, B.counter, s_lds, s_tot)) {
        if (threadIdx.x < P) {
            const int p = threadIdx.x;
            double* sc = run_scal(B, p);
            const bool done = sc[B.L.misc + MISC_DONE] != 0.0;
            const double beta = sqrt(s_tot[p]);
            sc[B.L.beta + j] = beta;
            double sig = 0.0;
            if (!done) {
                if (!isfinite(beta)) {
                    sc[B.L.misc + MISC_NONFINITE] = 1.0;
                    sc[B.L.misc + MISC_DONE] = 1.0;
                    sc[B.L.misc + MISC_KEFF] = (double)j;
                } else if (beta <= B.tau_scale * *B.anorm) {
                    sc[B.L.misc + MISC_DONE] = 1.0;
                    sc[B.L.misc + MISC_KEFF] = (double)j;
                } else {
                    sig = 1.0 / beta;
                }
            }
            sc[B.L.sigma + j + 1] = sig;
            if (j < B.L.k) {
                for (int q = 0; q < O; ++q) sc[B.L.proj + q * (B.L.k + 1) + j] = sig * s_tot[P + q * P + p];
            }
        }
    }
}

template <int P, int O>
hipError_t launch_start_t(const StartSrc& src, const SegTable& T, int32_t oset0, double* u,
                          const BatchArgs& B, hipStream_t s) {
    hipLaunchKernelGGL((k_start<P, O>), dim3(B.nblocks), dim3(kBlock), 0, s, src, T, oset0, u, B);
    return hipGetLastError();
}

template <int P, int O>
hipError_t launch_sweep_t(const SegTable& T, int32_t oset0, const double* ucur, double* w,
                          const BatchArgs& B, int j, hipStream_t s) {
    hipLaunchKernelGGL((k_sweep<P, O>), dim3(B.nblocks), dim3(kBlock), 0, s, T, oset0, ucur, w, B, j);
    return hipGetLastError();
}

template <int P, int LPR>
hipError_t launch_spmv_t(const CsrArgs& A, const double* ucur, const double* uprev, double* w,
                         const BatchArgs& B, int j, hipStream_t s) {
    hipLaunchKernelGGL((k_spmv_csr<P, LPR>), dim3(B.nblocks), dim3(kBlock), 0, s, A, ucur, uprev, w, B, j);
    return hipGetLastError();
}

// Dispatch over O for a fixed P; P * (1 + O) <= kMaxNV limits P = 8 to O <= 4.
#define KRY_DISPATCH_O4(FN, P, O, ...)                \
    switch (O) {                                      \
        case 1: return FN<P, 1>(__VA_ARGS__);         \
        case 2: return FN<P, 2>(__VA_ARGS__);         \
        case 3: return FN<P, 3>(__VA_ARGS__);         \
        case 4: return FN<P, 4>(__VA_ARGS__);         \
        default: return hipErrorInvalidValue;         \
    }
#define KRY_DISPATCH_O8(FN, P, O, ...)                \
    switch (O) {                                      \
        case 1: return FN<P, 1>(__VA_ARGS__);         \
        case 2: return FN<P, 2>(__VA_ARGS__);         \
        case 3: return FN<P, 3>(__VA_ARGS__);         \
        case 4: return FN<P, 4>(__VA_ARGS__);         \
        case 5: return FN<P, 5>(__VA_ARGS__);         \
        case 6: return FN<P, 6>(__VA_ARGS__);         \
        case 7: return FN<P, 7>(__VA_ARGS__);         \
        case 8: return FN<P, 8>(__VA_ARGS__);         \
        default: return hipErrorInvalidValue;         \
    }

}  // namespace

hipError_t launch_fill_zero_u32(unsigned int* p, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_fill_zero_u32, dim3((unsigned)blocks), dim3(kBlock), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_row_abs_max(const CsrArgs& A, int64_t n, double* partials, int32_t nblocks,
                              int64_t rows_per_block, unsigned int* counter, double* out,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_row_abs_max, dim3(nblocks), dim3(kBlock), 0, s, A, n, rows_per_block,
                       partials, counter, out);
    return hipGetLastError();
}

hipError_t launch_start(int P, int O, const StartSrc& src, const SegTable& T, int32_t oset0,
                        double* u, const BatchArgs& B, hipStream_t s) {
    if (P * (1 + O) > kMaxNV) return hipErrorInvalidValue;
    switch (P) {
        case 1: KRY_DISPATCH_O8(launch_start_t, 1, O, src, T, oset0, u, B, s)
        case 2: KRY_DISPATCH_O8(launch_start_t, 2, O, src, T, oset0, u, B, s)
        case 4: KRY_DISPATCH_O8(launch_start_t, 4, O, src, T, oset0, u, B, s)
        case 8: KRY_DISPATCH_O4(launch_start_t, 8, O, src, T, oset0, u, B, s)
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep(int P, int O, const SegTable& T, int32_t oset0, const double* ucur,
                        double* w, const BatchArgs& B, int j, hipStream_t s) {
    if (P * (1 + O) > kMaxNV) return hipErrorInvalidValue;
    switch (P) {
        case 1: KRY_DISPATCH_O8(launch_sweep_t, 1, O, T, oset0, ucur, w, B, j, s)
        case 2: KRY_DISPATCH_O8(launch_sweep_t, 2, O, T, oset0, ucur, w, B, j, s)
        case 4: KRY_DISPATCH_O8(launch_sweep_t, 4, O, T, oset0, ucur, w, B, j, s)
        case 8: KRY_DISPATCH_O4(launch_sweep_t, 8, O, T, oset0, ucur, w, B, j, s)
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_spmv_csr(int P, int lpr, const CsrArgs& A, const double* ucur,
                           const double* uprev, double* w, const BatchArgs& B, int j,
                           hipStream_t s) {
#define KRY_LPR(PP)                                                          \
    switch (lpr) {                                                           \
        case 1: return launch_spmv_t<PP, 1>(A, ucur, uprev, w, B, j, s);     \
        case 2: return launch_spmv_t<PP, 2>(A, ucur, uprev, w, B, j, s);     \
        case 4: return launch_spmv_t<PP, 4>(A, ucur, uprev, w, B, j, s);     \
        case 8: return launch_spmv_t<PP, 8>(A, ucur, uprev, w, B, j, s);     \
        default: return hipErrorInvalidValue;                                \
    }
    switch (P) {
        case 1: KRY_LPR(1)
        case 2: KRY_LPR(2)
        case 4: KRY_LPR(4)
        case 8: KRY_LPR(8)
        default: return hipErrorInvalidValue;
    }
#undef KRY_LPR
}

hipError_t launch_spmv_stencil(int P, const StencilArgs& A, const double* ucur,
                               const double* uprev, double* w, const BatchArgs& B, int j,
                               hipStream_t s) {
    switch (P) {
        case 1: hipLaunchKernelGGL((k_spmv_stencil<1>), dim3(B.nblocks), dim3(kBlock), 0, s, A, ucur, uprev, w, B, j); break;
        case 2: hipLaunchKernelGGL((k_spmv_stencil<2>), dim3(B.nblocks), dim3(kBlock), 0, s, A, ucur, uprev, w, B, j); break;
        case 4: hipLaunchKernelGGL((k_spmv_stencil<4>), dim3(B.nblocks), dim3(kBlock), 0, s, A, ucur, uprev, w, B, j); break;
        case 8: hipLaunchKernelGGL((k_spmv_stencil<8>), dim3(B.nblocks), dim3(kBlock), 0, s, A, ucur, uprev, w, B, j); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace kry
