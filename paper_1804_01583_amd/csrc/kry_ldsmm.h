// Small dense matrices held in LDS by one workgroup: products on the f64
// matrix cores and the degree-18 Taylor polynomial of the exponential.
// Shared by the small dense stage (kry_expm.hip) and the error control of
// Arnoldi runs (kry_errctl.hip).
#pragma once

#include "kry_internal.h"

namespace kry {
namespace ldsmm {

constexpr int kLd = kMaxK + 1;          // padded LDS row length
constexpr int kSlot = kMaxK * kLd;      // one matrix in LDS

// Barrier that orders LDS traffic only: a __syncthreads() would also wait for
// every global store of the wave.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

typedef double v4d __attribute__((ext_vector_type(4)));

// C = A B + extra(i, j) for mm x mm matrices in LDS slots sa, sb, sc (mm
// even, <= kMaxK; sc differs from sa and sb) on the f64 16x16x4 matrix cores:
// the 16 x 16 output tiles are spread over the waves, entries past mm read as
// zero.  Lane layout: A[m][k] in lane m + 16k, B[k][n] in lane n + 16k,
// D[m][n] in lane n + 16 (m % 4), accumulator register m / 4.
template <class FE>
__device__ __forceinline__ void mm_mfma(double* lds, int sa, int sb, int sc, int mm, FE extra) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (int)blockDim.x >> 6;
    const int mt = (mm + 15) >> 4;
    const int lr = lane & 15, lk = lane >> 4;
    for (int tile = wave; tile < mt * mt; tile += nw) {
        const int ti = tile / mt, tj = tile % mt;
        const int arow = ti * 16 + lr, bcol = tj * 16 + lr;
        // every fragment of the tile is loaded before the first product (the
        // loads pipeline); clamped addresses stay inside the slot, values past
        // mm are masked to zero
        const int ar = min(arow, mm - 1), bc = min(bcol, mm - 1);
        constexpr int KS = kMaxK / 4;
        double a[KS], b[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int kq = 4 * s + lk, kc = min(kq, mm - 1);
            a[s] = lds[sa * kSlot + ar * kLd + kc];
            b[s] = lds[sb * kSlot + kc * kLd + bc];
            a[s] = (arow < mm && kq < mm) ? a[s] : 0.0;
            b[s] = (bcol < mm && kq < mm) ? b[s] : 0.0;
        }
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KS; ++s)
            if (4 * s < mm) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc, 0, 0, 0);
        const int n = tj * 16 + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int mrow = ti * 16 + 4 * r + lk;
            if (mrow < mm && n < mm) lds[sc * kSlot + mrow * kLd + n] = acc[r] + extra(mrow, n);
        }
    }
    __syncthreads();
}

// Slot 4 <- f0 I + X + X^2/2! + ... + X^18/18! for X in slot 0 (|X|_1 <= 1:
// the remainder of e^X is below e/19! < 2e-17 relative), by Paterson-
// Stockmeyer in chunks of 4:
//   T(X) = L0 + X4 (L1 + X4 (L2 + X4 (L3 + X4 L4))),
//   L_q = f_{4q} I + f_{4q+1} X + f_{4q+2} X2 + f_{4q+3} X3,  f_i = 1/i! (0 past 18),
// with f_0 = f0: 1 gives e^X, 0 gives e^X - I.  Slots 1..3 hold X2..X4 and
// slot 5 is scratch.
__device__ __forceinline__ void taylor18(double* lds, int mm, double f0) {
    double f[20];
    f[0] = f0;
    double fi = 1.0;
    for (int i = 1; i < 20; ++i) {
        fi = i <= 18 ? fi / i : 0.0;
        f[i] = fi;
    }
    const double* S0 = lds;
    const double* S1 = lds + 1 * kSlot;
    const double* S2 = lds + 2 * kSlot;
    auto none = [](int, int) { return 0.0; };
    mm_mfma(lds, 0, 0, 1, mm, none);                                           // X2
    mm_mfma(lds, 1, 0, 2, mm, none);                                           // X3
    mm_mfma(lds, 1, 1, 3, mm, none);                                           // X4
    auto chunk = [=](int q, int i, int j) {
        const int e = i * kLd + j;
        return (i == j ? f[4 * q] : 0.0) + f[4 * q + 1] * S0[e] + f[4 * q + 2] * S1[e] + f[4 * q + 3] * S2[e];
    };
    for (int idx = threadIdx.x; idx < mm * mm; idx += blockDim.x) {
        const int i = idx / mm, c = idx % mm;
        lds[4 * kSlot + i * kLd + c] = chunk(4, i, c);
    }
    __syncthreads();
    mm_mfma(lds, 4, 3, 5, mm, [=](int i, int j) { return chunk(3, i, j); });
    mm_mfma(lds, 5, 3, 4, mm, [=](int i, int j) { return chunk(2, i, j); });
    mm_mfma(lds, 4, 3, 5, mm, [=](int i, int j) { return chunk(1, i, j); });
    mm_mfma(lds, 5, 3, 4, mm, [=](int i, int j) { return chunk(0, i, j); });   // T(X) in slot 4
}

// max over columns of sum_i |M_ij| for the mm x mm matrix in slot 0, on
// every thread (s_red: blockDim.x / 64 doubles).
__device__ __forceinline__ double norm1_slot0(const double* lds, int mm, double* s_red) {
    const int tid = threadIdx.x;
    double colsum = 0.0;
    if (tid < mm) {
        for (int i = 0; i < mm; ++i) colsum += fabs(lds[i * kLd + tid]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) colsum = fmax(colsum, __shfl_xor(colsum, off, 64));
    if ((tid & 63) == 0) s_red[tid >> 6] = colsum;
    __syncthreads();
    double nrm = 0.0;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) nrm = fmax(nrm, s_red[w]);
    __syncthreads();
    return nrm;
}

}  // namespace ldsmm
}  // namespace kry
