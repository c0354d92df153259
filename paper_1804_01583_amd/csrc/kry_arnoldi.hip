// Arnoldi orthogonalisation for nonsymmetric A on gfx950 (paper Algorithm 1,
// Section 4.2).  Iteration j projects w = A v_j against every stored basis
// vector.  The paper's loop is modified Gram-Schmidt; here it is classical
// Gram-Schmidt applied twice (CGS2), which orthogonalises to the same
// accuracy and turns each pass into two streaming kernels:
//   k_arn_dots   : partials of u_i . w for all stored u_i (2D grid: row blocks x
//                  chunks of 16 basis vectors)
//   k_arn_reduce : h_i = sigma_i * sum of the partials, added to column j of H;
//                  coefficient h_i sigma_i for the update
//   k_arn_update : w -= sum_i h_i v_i; on the second pass also the partials of
//                  |w|^2 and C w that the next mat-vec turns into beta_j, sigma_{j+1}
// The mat-vec itself is k_spmv_csr / k_spmv_stencil without the three-term part.
//
// The same kernels give Lanczos in FP32-basis mode its one full
// reorthogonalisation pass: after the three-term step (k_spmv + k_sweep) has
// removed beta_{j-1} v_{j-1} and alpha_j v_j, a single classical pass removes
// the rounding-level components left along u_1..u_j, and H keeps the
// tridiagonal entries plus these corrections.  (A single pass over the vector
// before alpha_j v_j is removed is not enough: its error along old vectors
// grows by about |alpha / beta| per step.)  Vectors are E = double or
// E = float; sums are FP64.
#include "kry_device.h"

#include <cmath>

namespace kry {

namespace {

using namespace dev;

template <typename E, int P>
__global__ __launch_bounds__(kBlock) void k_arn_dots(ArnArgs A, BatchArgs B, int j) {
    if (batch_stopped<P>(B)) return;   // the batch met its error target
    constexpr int NV = kArnChunk * P;
    __shared__ double s_lds[(kBlock / 64) * NV];
    const int lb = logical_block(B.nblocks, B.xcd_map);
    const int i0 = blockIdx.y * kArnChunk;
    const int ni = min(kArnChunk, j - i0);
    const int64_t r0 = (int64_t)lb * B.rows_per_block;
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    const E* V = static_cast<const E*>(A.V);
    const E* w = static_cast<const E*>(A.w);
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        // all loads of a row are issued together: slots past the last stored
        // vector re-read vector i0, and their sums are never stored
        double wv[P], uv[kArnChunk][P];
        load_row<E, P>(w, r, wv);
#pragma unroll
        for (int ii = 0; ii < kArnChunk; ++ii)
            load_row<E, P>(V + (int64_t)(ii < ni ? i0 + ii : i0) * A.vstride, r, uv[ii]);
#pragma unroll
        for (int ii = 0; ii < kArnChunk; ++ii) {
#pragma unroll
            for (int p = 0; p < P; ++p) acc[ii * P + p] = fma(uv[ii][p], wv[p], acc[ii * P + p]);
        }
    }
    const double t = block_sum<NV>(acc, s_lds);
    if (threadIdx.x < NV) {
        const int ii = threadIdx.x / P, p = threadIdx.x % P;
        if (ii < ni) A.hpart[((int64_t)(i0 + ii) * kMaxP + p) * B.nblocks + lb] = t;
    }
}

// One block per basis vector i: h = sigma_i * (u_i . w) over all row blocks.
template <int P>
__global__ __launch_bounds__(kBlock) void k_arn_reduce(ArnArgs A, BatchArgs B, int j, int pass) {
    if (batch_stopped<P>(B)) return;   // the batch met its error target
    __shared__ double s_lds[(kBlock / 64) * P];
    const int i = blockIdx.x;
    double acc[P];
#pragma unroll
    for (int p = 0; p < P; ++p) acc[p] = 0.0;
    add_strided_partials<P>(A.hpart + (int64_t)i * kMaxP * B.nblocks, B.nblocks, 0, acc);
    const double t = block_sum<P>(acc, s_lds);
    if (threadIdx.x < P) {
        const int p = threadIdx.x;
        double* sc = run_scal(B, p);
        const double sig = sc[B.L.sigma + i + 1];
        const double h = t * sig;
        double* hij = sc + B.L.hess + i * B.L.k + (j - 1);
        // Lanczos: the three-term step already removed beta_{j-1} v_{j-1} and
        // alpha_j v_j; H keeps them beside this pass's corrections
        double border = 0.0;
        if (A.lanczos && i == j - 2) border = sc[B.L.beta + j - 1];
        if (A.lanczos && i == j - 1) border = sc[B.L.alpha + j];
        if (pass == 1) *hij = h + border;
        else *hij += h;
        if (!isfinite(h)) sc[B.L.misc + MISC_NONFINITE] = 1.0;
        A.hcoef[i * kMaxP + p] = h * sig;
    }
}

template <typename E, int P, int O>
__global__ __launch_bounds__(kBlock) void k_arn_update(SegTable T, int32_t oset0, ArnArgs A, BatchArgs B, int j,
                                                       int last) {
    if (batch_stopped<P>(B)) return;   // the batch met its error target
    constexpr int NV = P * (1 + O);
    __shared__ double s_lds[(kBlock / 64) * NV];
    __shared__ double s_c[kMaxKD * P];
    __shared__ SegStage<O> st;
    const int lb = logical_block(B.nblocks, B.xcd_map);
    const int64_t r0 = (int64_t)lb * B.rows_per_block;
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    for (int idx = threadIdx.x; idx < j * P; idx += kBlock)
        s_c[idx] = A.hcoef[(idx / P) * kMaxP + idx % P];
    int sets[O];
#pragma unroll
    for (int q = 0; q < O; ++q) sets[q] = last ? oset0 + q : -1;
    stage_segments<O>(st, T, sets, lb, B.nblocks);     // contains the barrier for s_c
    SegCursor cur[O];
#pragma unroll
    for (int q = 0; q < O; ++q) cur[q].init(st, q);
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    const E* V = static_cast<const E*>(A.V);
    E* w = static_cast<E*>(A.w);
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        double val[P];
        load_row<E, P>(w, r, val);
        for (int i = 0; i < j; ++i) {
            double uv[P];
            load_row<E, P>(V + (int64_t)i * A.vstride, r, uv);
#pragma unroll
            for (int p = 0; p < P; ++p) val[p] = fma(-s_c[i * P + p], uv[p], val[p]);
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            val[p] = (double)(E)val[p];
            acc[p] = fma(val[p], val[p], acc[p]);
        }
        store_row<E, P>(w, r, val);
        if (last) {
#pragma unroll
            for (int q = 0; q < O; ++q) {
                const double cw = cur[q].weight(st, q, T, r);
                if (cw != 0.0) {
#pragma unroll
                    for (int p = 0; p < P; ++p) acc[P + q * P + p] = fma(cw, val[p], acc[P + q * P + p]);
                }
            }
        }
    }
    if (last) store_partials<NV>(acc, stage_part(B, j), B.nblocks, s_lds, B.xcd_map);
}

template <typename E, int P, int O>
hipError_t launch_update_t(const SegTable& T, int32_t oset0, const ArnArgs& A, const BatchArgs& B, int j,
                           int last, hipStream_t s) {
    hipLaunchKernelGGL((k_arn_update<E, P, O>), dim3(B.nblocks), dim3(kBlock), 0, s, T, oset0, A, B, j, last);
    return hipGetLastError();
}

template <typename E>
hipError_t launch_dots_e(int P, const ArnArgs& A, const BatchArgs& B, int j, hipStream_t s) {
    const dim3 grid(B.nblocks, (j + kArnChunk - 1) / kArnChunk);
    switch (P) {
        case 1: hipLaunchKernelGGL((k_arn_dots<E, 1>), grid, dim3(kBlock), 0, s, A, B, j); break;
        case 2: hipLaunchKernelGGL((k_arn_dots<E, 2>), grid, dim3(kBlock), 0, s, A, B, j); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename E>
hipError_t launch_update_e(int P, int O, const SegTable& T, int32_t oset0, const ArnArgs& A,
                           const BatchArgs& B, int j, int last, hipStream_t s) {
#define KRY_ARN_O(PP)                                                                \
    switch (O) {                                                                     \
        case 1: return launch_update_t<E, PP, 1>(T, oset0, A, B, j, last, s);        \
        case 2: return launch_update_t<E, PP, 2>(T, oset0, A, B, j, last, s);        \
        case 3: return launch_update_t<E, PP, 3>(T, oset0, A, B, j, last, s);        \
        case 4: return launch_update_t<E, PP, 4>(T, oset0, A, B, j, last, s);        \
        case 5: return launch_update_t<E, PP, 5>(T, oset0, A, B, j, last, s);        \
        case 6: return launch_update_t<E, PP, 6>(T, oset0, A, B, j, last, s);        \
        case 7: return launch_update_t<E, PP, 7>(T, oset0, A, B, j, last, s);        \
        case 8: return launch_update_t<E, PP, 8>(T, oset0, A, B, j, last, s);        \
        default: return hipErrorInvalidValue;                                        \
    }
    switch (P) {
        case 1: KRY_ARN_O(1)
        case 2: KRY_ARN_O(2)
        default: return hipErrorInvalidValue;
    }
#undef KRY_ARN_O
}

}  // namespace

hipError_t launch_arn_dots(int P, const ArnArgs& A, const BatchArgs& B, int j, hipStream_t s) {
    return A.f32 ? launch_dots_e<float>(P, A, B, j, s) : launch_dots_e<double>(P, A, B, j, s);
}

hipError_t launch_arn_reduce(int P, const ArnArgs& A, const BatchArgs& B, int j, int pass, hipStream_t s) {
    switch (P) {
        case 1: hipLaunchKernelGGL((k_arn_reduce<1>), dim3(j), dim3(kBlock), 0, s, A, B, j, pass); break;
        case 2: hipLaunchKernelGGL((k_arn_reduce<2>), dim3(j), dim3(kBlock), 0, s, A, B, j, pass); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_arn_update(int P, int O, const SegTable& T, int32_t oset0, const ArnArgs& A,
                             const BatchArgs& B, int j, int last, hipStream_t s) {
    return A.f32 ? launch_update_e<float>(P, O, T, oset0, A, B, j, last, s)
                 : launch_update_e<double>(P, O, T, oset0, A, B, j, last, s);
}

}  // namespace kry
