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
// On large systems the second pass is taken from the Gram matrix G = V^T V
// instead of a second pass over the basis: one k_arn_dots pass gives
// S_i = v_i . w, the new column v_i . v_j of G (one step late, when v_j is
// final) and w . w; k_arn_corr forms H_{:,j} = S - (G - I) S (the second
// classical pass is V^T (w - V S) = S - G S), and one k_arn_update removes
// V H_{:,j}.  Two passes over the basis per step instead of four.  What the
// plain second pass also removes, the rounding of S itself, is left, so a
// run whose w lost most of its norm to the projection (|w''|^2 below
// reorth2 |w|^2) gets a plain second pass: k_arn_guard raises a flag and
// the launches made with a condition run only then.
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

// basis vectors per block of the dot kernel: half with the second
// right-hand side, whose sums double the registers
constexpr int arn_chunk(bool two) { return two ? kArnChunk / 2 : kArnChunk; }

// the batch met its error target, or the launch is conditional and the
// guard is down
template <int P>
__device__ __forceinline__ bool arn_skip(const ArnArgs& A, const BatchArgs& B) {
    return batch_stopped<P>(B) || (A.conditional && *A.guard == 0);
}

// Partials of u_i . w for i < nx (TWO: and of u_i . u_j into hpart2).
template <typename E, int P, bool TWO>
__global__ __launch_bounds__(kBlock) void k_arn_dots(ArnArgs A, BatchArgs B, int j, int nx) {
    if (arn_skip<P>(A, B)) return;
    constexpr int CH = arn_chunk(TWO);
    constexpr int NV = CH * P * (TWO ? 2 : 1);
    __shared__ double s_lds[(kBlock / 64) * NV];
    const int lb = logical_block(B.nblocks, B.xcd_map);
    const int i0 = blockIdx.y * CH;
    const int ni = min(CH, nx - i0);
    const int64_t r0 = (int64_t)lb * B.rows_per_block;
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    const E* V = static_cast<const E*>(A.V);
    const E* w = static_cast<const E*>(A.w);
    const E* uj = V + (int64_t)(j - 1) * A.vstride;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        // all loads of a row are issued together: slots past the last stored
        // vector re-read vector i0, and their sums are never stored
        double wv[P], jv[P], uv[CH][P];
        load_row<E, P>(w, r, wv);
        if constexpr (TWO) load_row<E, P>(uj, r, jv);
#pragma unroll
        for (int ii = 0; ii < CH; ++ii)
            load_row<E, P>(V + (int64_t)(ii < ni ? i0 + ii : i0) * A.vstride, r, uv[ii]);
#pragma unroll
        for (int ii = 0; ii < CH; ++ii) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                acc[ii * P + p] = fma(uv[ii][p], wv[p], acc[ii * P + p]);
                if constexpr (TWO) acc[(CH + ii) * P + p] = fma(uv[ii][p], jv[p], acc[(CH + ii) * P + p]);
            }
        }
    }
    const double t = block_sum<NV>(acc, s_lds);
    if (threadIdx.x < NV) {
        const int q = threadIdx.x / P, p = threadIdx.x % P;
        const int ii = q % CH;
        double* part = q < CH ? A.hpart : A.hpart2;
        if (ii < ni) part[((int64_t)(i0 + ii) * kMaxP + p) * B.nblocks + lb] = t;
    }
}

// One block per basis vector i: h = sigma_i * (u_i . w) over all row blocks.
// pass 3 (the one-pass step; blockIdx.y = 0 / 1): u_i . w into sraw, or
// v_i . v_j into column j of the batch's Gram matrix (row j: the transpose).
template <int P>
__global__ __launch_bounds__(kBlock) void k_arn_reduce(ArnArgs A, BatchArgs B, int j, int pass) {
    if (arn_skip<P>(A, B)) return;
    __shared__ double s_lds[(kBlock / 64) * P];
    const int i = blockIdx.x;
    const bool second = pass == 3 && blockIdx.y == 1;
    double acc[P];
#pragma unroll
    for (int p = 0; p < P; ++p) acc[p] = 0.0;
    add_strided_partials<P>((second ? A.hpart2 : A.hpart) + (int64_t)i * kMaxP * B.nblocks, B.nblocks, 0, acc);
    const double t = block_sum<P>(acc, s_lds);
    if (pass == 3) {
        if (threadIdx.x < P) {
            const int p = threadIdx.x;
            if (!second) {
                A.sraw[i * kMaxP + p] = t;
            } else if (i < j) {
                const double* sc = run_scal(B, p);
                const double g = t * sc[B.L.sigma + i + 1] * sc[B.L.sigma + j];
                const int k = B.L.k;
                double* G = A.gram + (int64_t)p * k * k;
                G[(int64_t)i * k + (j - 1)] = g;
                if (i < j - 1) G[(int64_t)(j - 1) * k + i] = g;
            }
        }
        return;
    }
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

// Column j of H for the one-pass step, one block per run p: with
// S_i = sigma_i (u_i . w) and E = V^T V - I over v_1..v_j,
// h_i = S_i - (E S)_i, formed directly (E's diagonal as G_ii - 1) so the
// small correction keeps its relative accuracy; coefficient h_i sigma_i for
// the update.  Block 0 lowers the guard.
template <int P>
__global__ __launch_bounds__(kBlock) void k_arn_corr(ArnArgs A, BatchArgs B, int j) {
    if (arn_skip<P>(A, B)) return;
    __shared__ double s_s[kMaxKD];
    const int p = blockIdx.x;
    double* sc = run_scal(B, p);
    const int k = B.L.k;
    const double* G = A.gram + (int64_t)p * k * k;
    for (int i = threadIdx.x; i < j; i += kBlock) s_s[i] = A.sraw[i * kMaxP + p] * sc[B.L.sigma + i + 1];
    __syncthreads();
    bool bad = false;
    for (int i = threadIdx.x; i < j; i += kBlock) {
        const double* g = G + (int64_t)i * k;
        double es = 0.0;
        for (int l = 0; l < j; ++l) es = fma(g[l] - (l == i ? 1.0 : 0.0), s_s[l], es);
        const double h = s_s[i] - es;
        sc[B.L.hess + i * k + (j - 1)] = h;
        A.hcoef[i * kMaxP + p] = h * sc[B.L.sigma + i + 1];
        bad = bad || !isfinite(h);
    }
    if (bad) sc[B.L.misc + MISC_NONFINITE] = 1.0;
    if (p == 0 && threadIdx.x == 0) *A.guard = 0;
}

// One block: raises the guard when a run (not yet stopped) kept less than
// sqrt(reorth2) of |w| through the projection (|w''|^2 from the update's
// stage j partials, w . w from the dot pass).
template <int P>
__global__ __launch_bounds__(kBlock) void k_arn_guard(ArnArgs A, BatchArgs B, int j) {
    if (batch_stopped<P>(B)) return;
    __shared__ double s_lds[(kBlock / 64) * P];
    double acc[P];
#pragma unroll
    for (int p = 0; p < P; ++p) acc[p] = 0.0;
    add_strided_partials<P>(stage_part(B, j), B.nblocks, 0, acc);
    const double t = block_sum<P>(acc, s_lds);
    if (threadIdx.x < P) {
        const int p = threadIdx.x;
        const double ww = A.sraw[j * kMaxP + p];
        const bool stopped = B.stop != nullptr && B.stop[p] != 0.0;
        if (!stopped && t < A.reorth2 * ww) *A.guard = 1;
    }
}

template <typename E, int P, int O>
__global__ __launch_bounds__(kBlock) void k_arn_update(SegTable T, int32_t oset0, ArnArgs A, BatchArgs B, int j,
                                                       int last) {
    if (arn_skip<P>(A, B)) return;
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
hipError_t launch_dots_e(int P, const ArnArgs& A, const BatchArgs& B, int j, int nx, bool two, hipStream_t s) {
    const int ch = arn_chunk(two);
    const dim3 grid(B.nblocks, (nx + ch - 1) / ch);
    switch (P * 2 + (two ? 1 : 0)) {
        case 2: hipLaunchKernelGGL((k_arn_dots<E, 1, false>), grid, dim3(kBlock), 0, s, A, B, j, nx); break;
        case 3: hipLaunchKernelGGL((k_arn_dots<E, 1, true>), grid, dim3(kBlock), 0, s, A, B, j, nx); break;
        case 4: hipLaunchKernelGGL((k_arn_dots<E, 2, false>), grid, dim3(kBlock), 0, s, A, B, j, nx); break;
        case 5: hipLaunchKernelGGL((k_arn_dots<E, 2, true>), grid, dim3(kBlock), 0, s, A, B, j, nx); break;
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

hipError_t launch_arn_dots(int P, const ArnArgs& A, const BatchArgs& B, int j, hipStream_t s, int nx, bool two) {
    if (nx <= 0) nx = j;
    if (two && (A.hpart2 == nullptr || nx < j)) return hipErrorInvalidValue;
    return A.f32 ? launch_dots_e<float>(P, A, B, j, nx, two, s) : launch_dots_e<double>(P, A, B, j, nx, two, s);
}

hipError_t launch_arn_reduce(int P, const ArnArgs& A, const BatchArgs& B, int j, int pass, hipStream_t s) {
    // pass 3 sums j + 1 dot products (the last is w . w) and j Gram entries
    const dim3 grid(pass == 3 ? j + 1 : j, pass == 3 ? 2 : 1);
    if (pass == 3 && (A.sraw == nullptr || A.gram == nullptr)) return hipErrorInvalidValue;
    switch (P) {
        case 1: hipLaunchKernelGGL((k_arn_reduce<1>), grid, dim3(kBlock), 0, s, A, B, j, pass); break;
        case 2: hipLaunchKernelGGL((k_arn_reduce<2>), grid, dim3(kBlock), 0, s, A, B, j, pass); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_arn_corr(int P, const ArnArgs& A, const BatchArgs& B, int j, hipStream_t s) {
    if (A.sraw == nullptr || A.gram == nullptr || A.guard == nullptr || j > kMaxKD) return hipErrorInvalidValue;
    switch (P) {
        case 1: hipLaunchKernelGGL((k_arn_corr<1>), dim3(1), dim3(kBlock), 0, s, A, B, j); break;
        case 2: hipLaunchKernelGGL((k_arn_corr<2>), dim3(2), dim3(kBlock), 0, s, A, B, j); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_arn_guard(int P, const ArnArgs& A, const BatchArgs& B, int j, hipStream_t s) {
    if (A.sraw == nullptr || A.guard == nullptr) return hipErrorInvalidValue;
    switch (P) {
        case 1: hipLaunchKernelGGL((k_arn_guard<1>), dim3(1), dim3(kBlock), 0, s, A, B, j); break;
        case 2: hipLaunchKernelGGL((k_arn_guard<2>), dim3(1), dim3(kBlock), 0, s, A, B, j); break;
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
