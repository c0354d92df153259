// Device helpers shared by the streaming kernels (kry_lanczos.hip,
// kry_arnoldi.hip): block reductions, the XCD-aware row partition, the
// per-stage scalar logic of the Krylov recurrences and the staging of
// segment sets in LDS.  Internal; included by .hip files only.
#pragma once

#include "kry_internal.h"

#include <cmath>

namespace kry {
namespace dev {


template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV]) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] += __shfl_xor(v[i], off, 64);
    }
}

// Sum of v over the block; thread i < NV returns total i.  `lds` holds
// (NTH / 64) * NV doubles (NTH threads in the block).  Every thread must call it.
template <int NV, int NTH = kBlock>
__device__ __forceinline__ double block_sum(double (&v)[NV], double* lds) {
    wave_sum<NV>(v);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) lds[wave * NV + i] = v[i];
    }
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < NV) {
        t = lds[threadIdx.x];
#pragma unroll
        for (int w = 1; w < NTH / 64; ++w) t += lds[w * NV + threadIdx.x];
    }
    __syncthreads();
    return t;
}

// Workgroups are dispatched to the 8 XCDs round-robin by blockIdx; the
// logical block (row range) of a workgroup is chosen so each XCD works on a
// contiguous eighth of the rows, which keeps the +-m^2 neighbours of a 3D
// stencil row in the same XCD's L2.  nblocks is a multiple of 8.
__device__ __forceinline__ int logical_block(int nblocks, int xcd_map = 1) {
    if (!xcd_map) return (int)blockIdx.x;
    return (int)(blockIdx.x & 7) * (nblocks >> 3) + (int)(blockIdx.x >> 3);
}

// Error control: once every run of the batch has met its error target, the
// iterations the host has already queued do nothing (the host does not wait
// for the flags at each checkpoint).  False when the Krylov dimension is fixed.
template <int P>
__device__ __forceinline__ bool batch_stopped(const BatchArgs& B) {
    if (B.stop == nullptr) return false;
    bool all = true;
#pragma unroll
    for (int p = 0; p < P; ++p) all = all && B.stop[p] != 0.0;
    return all;
}

// Writes the block totals of v as partials part[i * nblocks + block].
template <int NV, int NTH = kBlock>
__device__ __forceinline__ void store_partials(double (&v)[NV], double* part, int nblocks, double* lds,
                                               int xcd_map) {
    const double t = block_sum<NV, NTH>(v, lds);
    if (threadIdx.x < NV) part[(int64_t)threadIdx.x * nblocks + logical_block(nblocks, xcd_map)] = t;
}

// acc[i] += part[(vbeg + i) * nb + b] for b = first, first + kBlock, ..., in
// that order.  The loads of U consecutive b are issued before any is
// waited for: a plain loop waits for each load pair in turn (a wait covers
// every earlier load), serialising the round trips.
template <int NV>
struct PartialLoads {
    static constexpr int U = NV <= 4 ? 4 : (NV <= 8 ? 2 : 1);
};
template <int NV, int NTH = kBlock>
__device__ __forceinline__ void add_strided_partials(const double* part, int nb, int vbeg, double (&acc)[NV],
                                                     int first) {
    constexpr int U = PartialLoads<NV>::U;
    for (int b0 = first; b0 < nb; b0 += U * NTH) {
        double v[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // clamped, unconditional loads (a load under a condition becomes
            // a branch that waits for it); entries past nb are not added
            const int b = min(b0 + u * NTH, nb - 1);
#pragma unroll
            for (int i = 0; i < NV; ++i) v[u][i] = part[(int64_t)(vbeg + i) * nb + b];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (b0 + u * NTH < nb) {
#pragma unroll
                for (int i = 0; i < NV; ++i) acc[i] += v[u][i];
            }
        }
    }
}
template <int NV, int NTH = kBlock>
__device__ __forceinline__ void add_strided_partials(const double* part, int nb, int vbeg, double (&acc)[NV]) {
    add_strided_partials<NV, NTH>(part, nb, vbeg, acc, (int)threadIdx.x);
}

// The same sum split in two, so that other loads can be issued between
// them: issue() requests the first U strided partials into registers, sum()
// adds them and the rest, in the same order as add_strided_partials.
// Requires nb >= 1.
template <int NV>
struct PartialBatch {
    static constexpr int U = PartialLoads<NV>::U;
    double v[U][NV];
    __device__ __forceinline__ void issue(const double* part, int nb, int vbeg) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = min((int)threadIdx.x + u * kBlock, nb - 1);   // nb >= 1; see above
#pragma unroll
            for (int i = 0; i < NV; ++i) v[u][i] = part[(int64_t)(vbeg + i) * nb + b];
        }
    }
    __device__ __forceinline__ void sum(const double* part, int nb, int vbeg, double (&acc)[NV]) const {
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if ((int)threadIdx.x + u * kBlock < nb) {
#pragma unroll
                for (int i = 0; i < NV; ++i) {
                    // opaque to the optimiser: the sum stays where sum() is
                    // called instead of being hoisted (with its wait for the
                    // loads) ahead of the caller's own loads
                    double x = v[u][i];
                    asm volatile("" : "+v"(x));
                    acc[i] += x;
                }
            }
        }
        add_strided_partials<NV>(part, nb, vbeg, acc, (int)threadIdx.x + U * kBlock);
    }
};

// Totals of values vbeg..vbeg+NV-1 of a partial array over nb blocks, in a
// fixed order; result in s_out[0..NV) for every thread.
template <int NV>
__device__ __forceinline__ void sum_partials(const double* part, int nb, int vbeg, double* lds, double* s_out) {
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    add_strided_partials<NV>(part, nb, vbeg, acc);
    const double t = block_sum<NV>(acc, lds);
    if (threadIdx.x < NV) s_out[threadIdx.x] = t;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Krylov vectors are stored as E = double (FP64 mode) or E = float (FP32
// basis mode) with the P runs of a batch interleaved ([n][P]); all arithmetic
// is FP64.  load_row / store_row move the P entries of one row with the
// widest aligned vector access (rows are P * sizeof(E) bytes apart and every
// vector starts 256-byte aligned).
template <typename E, int N>
struct VecOf;
template <> struct VecOf<double, 1> { using type = double; };
template <> struct VecOf<double, 2> { using type = double2; };
template <> struct VecOf<float, 1> { using type = float; };
template <> struct VecOf<float, 2> { using type = float2; };
template <> struct VecOf<float, 4> { using type = float4; };

template <typename E, int P>
constexpr int row_chunk() {
    return sizeof(E) == 8 ? (P >= 2 ? 2 : 1) : (P >= 4 ? 4 : P);
}

template <typename E, int P>
__device__ __forceinline__ void load_row(const E* __restrict__ base, int64_t row, double (&v)[P]) {
    constexpr int W = row_chunk<E, P>();
    using Vec = typename VecOf<E, W>::type;
    const Vec* q = reinterpret_cast<const Vec*>(base + row * P);
#pragma unroll
    for (int h = 0; h < P / W; ++h) {
        const Vec t = q[h];
        if constexpr (W == 1) {
            v[h] = (double)t;
        } else {
            const E* e = reinterpret_cast<const E*>(&t);
#pragma unroll
            for (int i = 0; i < W; ++i) v[h * W + i] = (double)e[i];
        }
    }
}

template <typename E, int P>
__device__ __forceinline__ void store_row(E* __restrict__ base, int64_t row, const double (&v)[P]) {
    constexpr int W = row_chunk<E, P>();
    using Vec = typename VecOf<E, W>::type;
    Vec* q = reinterpret_cast<Vec*>(base + row * P);
#pragma unroll
    for (int h = 0; h < P / W; ++h) {
        if constexpr (W == 1) {
            q[h] = (E)v[h];
        } else {
            Vec t;
            E* e = reinterpret_cast<E*>(&t);
#pragma unroll
            for (int i = 0; i < W; ++i) e[i] = (E)v[h * W + i];
            q[h] = t;
        }
    }
}

__device__ __forceinline__ double* run_scal(const BatchArgs& B, int p) {
    return B.scal + (int64_t)(B.run0 + p) * B.L.stride;
}

// Stage j-1 -> sigma_j.  nrm2 = |u_j|^2 (u_j is the start vector for j = 1,
// the swept vector of iteration j-1 otherwise).  A step whose norm is at most
// 1024 eps ||A||_inf ends the run (invariant Krylov space); sigma stays 0 from
// then on, which keeps every later vector exactly zero.
struct Stage {
    double beta, sigma, cprev;
    int keff;          // new k_eff to record, or -1 to leave it
    bool nonfinite;
};

__device__ __forceinline__ Stage stage_update_v(int k, double sig_prev, double tau, int j, double nrm2) {
    Stage st;
    st.beta = sqrt(nrm2);
    st.keff = -1;
    st.nonfinite = false;
    st.cprev = 0.0;
    if (j == 1) {
        const bool ok = st.beta > 0.0 && isfinite(st.beta);
        st.sigma = ok ? 1.0 / st.beta : 0.0;
        st.keff = ok ? k : 0;
        st.nonfinite = !isfinite(st.beta);
        return st;
    }
    st.cprev = st.beta * sig_prev;
    if (sig_prev == 0.0) {
        st.sigma = 0.0;
        st.cprev = 0.0;
    } else if (!isfinite(st.beta)) {
        st.sigma = 0.0;
        st.cprev = 0.0;
        st.keff = j - 1;
        st.nonfinite = true;
    } else if (st.beta <= tau) {
        st.sigma = 0.0;
        st.keff = j - 1;
    } else {
        st.sigma = 1.0 / st.beta;
    }
    return st;
}

__device__ __forceinline__ Stage stage_update(const BatchArgs& B, const double* sc, int j, double nrm2) {
    return stage_update_v(B.L.k, j > 1 ? sc[B.L.sigma + j - 1] : 0.0, B.tau_scale * *B.anorm, j, nrm2);
}

// Block 0 of the kernel that consumes stage j-1 records its scalars (the
// projections are summed later, once per batch, by k_finish).
__device__ __forceinline__ void record_stage(const BatchArgs& B, int P, int j, const double* nrm2) {
    if (threadIdx.x < P) {
        const int p = threadIdx.x;
        double* sc = run_scal(B, p);
        const Stage st = stage_update(B, sc, j, nrm2[p]);
        sc[B.L.beta + j - 1] = st.beta;
        sc[B.L.sigma + j] = st.sigma;
        if (st.keff >= 0) sc[B.L.misc + MISC_KEFF] = (double)st.keff;
        if (j == 1) {
            sc[B.L.misc + MISC_NONFINITE] = st.nonfinite ? 1.0 : 0.0;
            sc[B.L.misc + MISC_KSTOP] = (double)B.L.k;
            sc[B.L.misc + MISC_STOPPED] = 0.0;
            sc[B.L.misc + MISC_BOUND] = -1.0;
        }
        else if (st.nonfinite) sc[B.L.misc + MISC_NONFINITE] = 1.0;
    }
}

__device__ __forceinline__ double* stage_part(const BatchArgs& B, int stage) {
    return B.np_part + (int64_t)stage * B.nvp * B.nblocks;
}

// The reduction of stage j-1's norms, done first: thread t sums blocks t,
// t + kBlock, ... (every block reads the same few KB of partials; issuing
// them alongside the row work, instead of before it, measured slower)
template <int P, int NTH = kBlock>
__device__ __forceinline__ void load_stage_norms(const BatchArgs& B, int j, double (&pacc)[P],
                                                 double (&sig_prev)[P], double& anorm) {
    const double* part = stage_part(B, j - 1);
#pragma unroll
    for (int p = 0; p < P; ++p) pacc[p] = 0.0;
    for (int b = threadIdx.x; b < B.nblocks; b += NTH) {
#pragma unroll
        for (int p = 0; p < P; ++p) pacc[p] += part[(int64_t)p * B.nblocks + b];
    }
#pragma unroll
    for (int p = 0; p < P; ++p) sig_prev[p] = (j > 1) ? run_scal(B, p)[B.L.sigma + j - 1] : 0.0;
    anorm = *B.anorm;
}

// Finishes the stage j-1 reduction: sigma_j and cprev = beta_{j-1} sigma_{j-1}
// for every run; block 0 records the stage.  Every thread must call it.
template <int P, int NTH = kBlock>
__device__ __forceinline__ void finish_stage_norms(const BatchArgs& B, int j, double (&pacc)[P],
                                                   const double (&sig_prev)[P], double anorm, double* s_lds,
                                                   double* s_nrm, double (&sig)[P], double (&cprev)[P]) {
    const double t = block_sum<P, NTH>(pacc, s_lds);
    if (threadIdx.x < P) s_nrm[threadIdx.x] = t;
    __syncthreads();
    if (blockIdx.x == 0) record_stage(B, P, j, s_nrm);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const Stage st = stage_update_v(B.L.k, sig_prev[p], B.tau_scale * anorm, j, s_nrm[p]);
        sig[p] = st.sigma;
        cprev[p] = st.cprev;
    }
}

// Diagonal of a stencil row from which neighbours exist: c0, plus for
// insulated faces each missing neighbour's coefficient, plus the exchange
// term on the last x plane.
__device__ __forceinline__ double stencil_diag(const StencilArgs& S, bool xl, bool xh, bool yl, bool yh, bool zl,
                                               bool zh) {
    double d = S.c0;
    if (S.insulated) {
        if (!xl) d += S.cx;
        if (!xh) d += S.cx;
        if (!yl) d += S.cy;
        if (!yh) d += S.cy;
        if (!zl) d += S.cz;
        if (!zh) d += S.cz;
    }
    if (!xh) d += S.ex;
    return d;
}

// The marching stencil's column: row r = ix * sx + col, its y/z neighbour
// offsets (0 where the neighbour is missing) and which neighbours exist.
struct MarchCol {
    int64_t col, sx;
    int64_t dyl, dyh, dzl, dzh;
    bool yl, yh, zl, zh, live, prev;
};

// ---------------------------------------------------------------------------
// Segment sets (generators and output rows) a block needs are staged in LDS.
// The plan precomputes, for every set and logical block, the range of that
// set's segments overlapping the block's rows (SegTable::blk), so a block
// finds them with one load; up to CAP of them (kSegCap unless a kernel asks
// for more) are copied to LDS, a set with more keeps reading global memory.
constexpr int kSegCap = 64;

template <int NS, int CAP = kSegCap>
struct SegStage {
    int64_t lo[NS][CAP];
    int64_t hi[NS][CAP];
    double w[NS][CAP];
    int32_t beg[NS], end[NS];
};

// Two halves, so a kernel can issue other loads between them: thread i < NS
// loads set i's segment range for the block (seg_range), then every thread
// calls stage_segments with it.  sets[i] < 0 stages an empty set.
struct SegRange {
    int32_t b, e;
};
template <int NS>
__device__ __forceinline__ SegRange seg_range(const SegTable& T, const int (&sets)[NS], int lb, int nblocks) {
    SegRange r{0, 0};
    if (threadIdx.x < NS) {
        const int s = sets[threadIdx.x];
        if (s >= 0) {
            r.b = T.blk[((int64_t)s * nblocks + lb) * 2];
            r.e = T.blk[((int64_t)s * nblocks + lb) * 2 + 1];
        }
    }
    return r;
}

template <int NS, int CAP = kSegCap>
__device__ __forceinline__ void stage_segments(SegStage<NS, CAP>& st, const SegTable& T, SegRange r) {
    if (threadIdx.x < NS) {
        st.beg[threadIdx.x] = r.b;
        st.end[threadIdx.x] = r.e;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < NS * CAP; idx += kBlock) {
        const int i = idx / CAP, c = idx % CAP;
        const int g = st.beg[i] + c;
        if (g < st.end[i]) {
            st.lo[i][c] = T.lo[g];
            st.hi[i][c] = T.hi[g];
            st.w[i][c] = T.w[g];
        }
    }
    __syncthreads();
}

// Both halves at once.  Every thread must call it.
template <int NS, int CAP = kSegCap>
__device__ __forceinline__ void stage_segments(SegStage<NS, CAP>& st, const SegTable& T, const int (&sets)[NS],
                                               int lb, int nblocks) {
    stage_segments<NS, CAP>(st, T, seg_range<NS>(T, sets, lb, nblocks));
}

// Weight of increasing rows in one staged set, amortised O(1) per row.
struct SegCursor {
    int32_t cur, cnt, gcur, gend;
    template <int NS, int CAP>
    __device__ __forceinline__ void init(const SegStage<NS, CAP>& st, int i) {
        const int n = st.end[i] - st.beg[i];
        cur = 0;
        cnt = n <= CAP ? n : 0;
        gcur = n <= CAP ? 0 : st.beg[i];
        gend = n <= CAP ? 0 : st.end[i];
    }
    template <int NS, int CAP>
    __device__ __forceinline__ double weight(const SegStage<NS, CAP>& st, int i, const SegTable& T, int64_t r) {
        while (cur < cnt && st.hi[i][cur] <= r) ++cur;
        if (cur < cnt) return st.lo[i][cur] <= r ? st.w[i][cur] : 0.0;
        while (gcur < gend && T.hi[gcur] <= r) ++gcur;
        return (gcur < gend && T.lo[gcur] <= r) ? T.w[gcur] : 0.0;
    }
};


}  // namespace dev
}  // namespace kry
