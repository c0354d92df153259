// Block Arnoldi on gfx950: p <= 16 generator columns simulated as one block
// Krylov space span{G, A G, ..., A^{k-1} G} (the block form of Algorithm 1,
// Section 4.2 written for a block start).  Blocks are 16 columns wide; a
// block of p < 16 real columns carries zero columns that stay zero.
//
// Storage: block i of the basis is an [n][16] row-major array (one 128-byte
// row of FP64, or 64 bytes of FP32, per grid row), blocks kept for the whole
// run.  One block step j:
//   k_bspmm      W = A V_j                               (16 lanes per CSR row)
//   k_bgram      partials of V_i^T W and V_i^T V_j, i = 1..j, and W^T W
//                (MFMA f64 16x16x4, one pass over the basis)
//   k_bgram_red  S_i = V_i^T W; block column j of G = V^T V
//   k_bcorr      H_{:,j} = S + (I - G) S, the classical Gram-Schmidt
//                coefficients with the second (re-orthogonalising) pass
//                taken from the Gram matrix instead of a second pass over the
//                basis; -H_{:,j} kept for the update
//   k_bupdate    W += sum_i V_i (-H_{i,j})               (MFMA f64 16x16x4)
//   k_bgram / k_bchol / k_bupdate: CholQR2 of W = V_{j+1} H_{j+1,j} (Gram
//   matrix, Cholesky in one thread, W R^{-1} in place), twice.  When W lost
//   most of its norm to the projection (|W_c| below 1e-3 of what it was for
//   a column c), the first Cholesky step raises a flag and a plain second
//   Gram-Schmidt pass over the basis runs before the factorisation is redone
//   (kernels launched with a condition return at once while it is down).
//   k_bproj      partials of C V_{j+1}                   (only rows inside C's segments)
// The plain two-pass form (both passes over the basis) stays available.
// All sums are FP64 and in a fixed order; no atomics.
//
// MFMA f64 16x16x4 lane layout (measured on gfx950): A[m][k] is held by lane
// m + 16k, B[k][n] by lane n + 16k, and D[m][n] by lane n + 16 (m % 4) in
// accumulator register m / 4.
#include "kry_device.h"

#include <cmath>

namespace kry {

namespace {

using namespace dev;

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// the run has ended, or the launch carries a condition that is down
__device__ __forceinline__ bool block_done(const BlockArgs& B) {
    return B.state[0] != 0 || (B.cond != nullptr && *B.cond == 0);
}

// ---------------------------------------------------------------------------
// Start block: column c < p of V_1 (unnormalised) is generator c of the block.
template <typename E>
__global__ __launch_bounds__(kBlock) void k_bstart(SegTable T, BlockStart S, E* __restrict__ V, int64_t n) {
    const int c = threadIdx.x & 15;
    const int grp = threadIdx.x >> 4;
    const int64_t stride = (int64_t)gridDim.x * (kBlock / 16);
    // each lane walks its column's segment set with a cursor over rows
    const int s = c < S.p ? S.set[c] : -1;
    int32_t cur = s >= 0 ? T.set_begin[s] : 0;
    const int32_t end = s >= 0 ? T.set_begin[s + 1] : 0;
    for (int64_t r = (int64_t)blockIdx.x * (kBlock / 16) + grp; r < n; r += stride) {
        double v = 0.0;
        if (s >= 0) {
            while (cur < end && T.hi[cur] <= r) ++cur;
            if (cur < end && T.lo[cur] <= r) v = T.w[cur];
        }
        V[r * kBW + c] = (E)v;
    }
}

// W = A V_j: a group of 16 lanes owns a row, lane c its column c.  The
// group reads up to 16 CSR entries of the row at once (one per lane) and
// passes them round by shuffles, so all 16 gathers of V_j rows (each one
// contiguous 16-value row) are in flight together; slots past the row's end
// carry value 0 and column 0.  Rows are software-pipelined along the group's
// walk: while row r's gathers are in flight the group already holds row
// r + 16's entries and row r + 32's row pointers.  Loads for rows past the
// range read in-range pointers and are dropped.
template <typename E>
__device__ __forceinline__ double bspmm_val(const CsrArgs& A, int64_t e) {
    if constexpr (sizeof(E) == 4) return (double)A.vals32[e];
    else return A.vals[e];
}

template <typename E>
__global__ __launch_bounds__(kBlock) void k_bspmm(CsrArgs A, const E* __restrict__ V, E* __restrict__ W, int64_t n,
                                                  int64_t rows_per_block, BlockArgs B) {
    if (block_done(B)) return;
    const int c = threadIdx.x & 15;
    const int grp = threadIdx.x >> 4;
    // a contiguous range of rows per workgroup, ranges in workgroup order
    // (the rows in flight on the whole chip stay within a narrow band) or
    // XCD-contiguous (each XCD walks its own part of the rows); groups take
    // the range's rows in turn.  Each row's sum is the same either way.
    const int64_t r0 = (int64_t)(B.spmm_xcd ? logical_block((int)gridDim.x) : (int)blockIdx.x) * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    const int64_t stride = kBlock / 16;
    const int64_t last = n - 1;
    n = r1;                                        // the walk below ends at the range's end
    int64_t r = r0 + grp;
    // row pointers of r and r + stride, entries of r
    int64_t e0 = A.rowptr[min(r, last)], e1 = A.rowptr[min(r, last) + 1];
    int64_t f0 = A.rowptr[min(r + stride, last)], f1 = A.rowptr[min(r + stride, last) + 1];
    int32_t mycol;
    double myval;
    {
        const int64_t e = e0 + c;
        const bool ok = r < n && e < e1;
        mycol = ok ? A.colidx[e] : 0;
        myval = ok ? bspmm_val<E>(A, e) : 0.0;
    }
    for (; r < n; r += stride) {
        // next row's entries (its pointers are here) and the pointers two rows ahead
        const int64_t rn = r + stride;
        int32_t ncol;
        double nval;
        {
            const int64_t e = f0 + c;
            const bool ok = rn < n && e < f1;
            ncol = ok ? A.colidx[e] : 0;
            nval = ok ? bspmm_val<E>(A, e) : 0.0;
        }
        const int64_t rnn = min(rn + stride, last);
        const int64_t g0 = A.rowptr[rnn], g1 = A.rowptr[rnn + 1];
        double acc = 0.0;
        {
            double x[16], a[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int32_t col = __shfl(mycol, q, 16);
                a[q] = __shfl(myval, q, 16);
                x[q] = (double)V[(int64_t)col * kBW + c];
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) acc = fma(a[q], x[q], acc);
        }
        // rows longer than 16 entries
        for (int64_t eb = e0 + 16; eb < e1; eb += 16) {
            const int64_t e = eb + c;
            const bool ok = e < e1;
            const int32_t col0 = ok ? A.colidx[e] : 0;
            const double v0 = ok ? bspmm_val<E>(A, e) : 0.0;
            double x[16], a[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int32_t col = __shfl(col0, q, 16);
                a[q] = __shfl(v0, q, 16);
                x[q] = (double)V[(int64_t)col * kBW + c];
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) acc = fma(a[q], x[q], acc);
        }
        W[r * kBW + c] = (E)acc;
        e0 = f0;
        e1 = f1;
        f0 = g0;
        f1 = g1;
        mycol = ncol;
        myval = nval;
    }
}

// Partials of X_i^T Y, i < nx, over the rows of row block blockIdx.x.  Wave
// w of the workgroup owns i = w, w + 4, ... (NI of them at most), so a row of
// Y is fetched from memory once per workgroup; each MFMA consumes 4 rows and
// an iteration issues the loads of RS MFMA steps before using them.  Slots
// past nx re-read X_{nx-1} and are never stored; rows past the block's end
// read row r0 and are multiplied by zero.
// TWO: the same partials against a second block Y2 as well (into gpart2).
template <typename E, int NI, bool TWO>
__global__ __launch_bounds__(kBlock) void k_bgram(const E* __restrict__ X0, int64_t xstride, int nx,
                                                  const E* __restrict__ Y, const E* __restrict__ Y2, BlockArgs B) {
    constexpr int RS = NI <= 4 ? 4 : 2;
    if (block_done(B)) return;
    const int l = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * B.rows_per_rb;
    const int64_t r1 = min(B.n, r0 + B.rows_per_rb);
    const int col = l & 15, sub = l >> 4;
    v4d acc[NI], acc2[TWO ? NI : 1];
#pragma unroll
    for (int u = 0; u < NI; ++u) acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < (TWO ? NI : 1); ++u) acc2[u] = v4d{0.0, 0.0, 0.0, 0.0};
    const E* Xu[NI];
#pragma unroll
    for (int u = 0; u < NI; ++u) Xu[u] = X0 + (int64_t)min(wave + 4 * u, nx - 1) * xstride;
    for (int64_t r = r0; r < r1; r += 4 * RS) {
        int64_t rr[RS];
        bool ok[RS];
        double yb[RS], yc[RS], xa[NI][RS];
#pragma unroll
        for (int q = 0; q < RS; ++q) {
            const int64_t row = r + 4 * q + sub;
            ok[q] = row < r1;
            rr[q] = ok[q] ? row : r0;
            yb[q] = (double)Y[rr[q] * kBW + col];
            if constexpr (TWO) yc[q] = (double)Y2[rr[q] * kBW + col];
        }
#pragma unroll
        for (int u = 0; u < NI; ++u) {
#pragma unroll
            for (int q = 0; q < RS; ++q) xa[u][q] = (double)Xu[u][rr[q] * kBW + col];
        }
#pragma unroll
        for (int q = 0; q < RS; ++q) {
            const double b = ok[q] ? yb[q] : 0.0;
#pragma unroll
            for (int u = 0; u < NI; ++u) acc[u] = mfma16(xa[u][q], b, acc[u]);
            if constexpr (TWO) {
                const double c = ok[q] ? yc[q] : 0.0;
#pragma unroll
                for (int u = 0; u < NI; ++u) acc2[u] = mfma16(xa[u][q], c, acc2[u]);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < NI; ++u) {
        const int i = wave + 4 * u;
        if (i >= nx) continue;
        double* out = B.gpart + ((int64_t)i * B.rb + blockIdx.x) * 256;
#pragma unroll
        for (int q = 0; q < 4; ++q) out[(4 * q + sub) * 16 + col] = acc[u][q];   // D[m][col], m = 4q + sub
        if constexpr (TWO) {
            double* out2 = B.gpart2 + ((int64_t)i * B.rb + blockIdx.x) * 256;
#pragma unroll
            for (int q = 0; q < 4; ++q) out2[(4 * q + sub) * 16 + col] = acc2[u][q];
        }
    }
}

// k_bgram for one block X (the CholQR Gram matrix W^T W, and any nx = 1):
// the four waves take every fourth group of row steps of the row block
// instead of one wave holding the only block while the others idle, and
// their sums are added in wave order through LDS.
template <typename E>
__global__ __launch_bounds__(kBlock) void k_bgram1(const E* __restrict__ X, const E* __restrict__ Y, BlockArgs B) {
    constexpr int RS = 4;
    constexpr int NW = kBlock / 64;
    __shared__ v4d s_acc[NW - 1][64];
    if (block_done(B)) return;
    const int l = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * B.rows_per_rb;
    const int64_t r1 = min(B.n, r0 + B.rows_per_rb);
    const int col = l & 15, sub = l >> 4;
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
    for (int64_t r = r0 + (int64_t)wave * 4 * RS; r < r1; r += (int64_t)4 * RS * NW) {
        int64_t rr[RS];
        bool ok[RS];
        double yb[RS], xa[RS];
#pragma unroll
        for (int q = 0; q < RS; ++q) {
            const int64_t row = r + 4 * q + sub;
            ok[q] = row < r1;
            rr[q] = ok[q] ? row : r0;
            yb[q] = (double)Y[rr[q] * kBW + col];
            xa[q] = (double)X[rr[q] * kBW + col];
        }
#pragma unroll
        for (int q = 0; q < RS; ++q) acc = mfma16(xa[q], ok[q] ? yb[q] : 0.0, acc);
    }
    if (wave > 0) s_acc[wave - 1][l] = acc;
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 0; w < NW - 1; ++w) acc += s_acc[w][l];
    double* out = B.gpart + (int64_t)blockIdx.x * 256;
#pragma unroll
    for (int q = 0; q < 4; ++q) out[(4 * q + sub) * 16 + col] = acc[q];   // D[m][col], m = 4q + sub
}

// Sums the row-block partials of block i = blockIdx.x, entries
// 16 blockIdx.y .. 16 blockIdx.y + 15: 16 threads per entry take every 16th
// row block, then their sums are added in order.  mode 0/1: Gram-Schmidt
// pass 1/2, H_{i,j} = / += result and coef_i = -result; mode 2: Gram matrix
// into coef_0; mode 3 (the one-pass step, blockIdx.z = 0 / 1): S_i into
// sbuf, and V_i^T V_j (i < j) into block column j of G and its transpose
// into block row j.
__global__ __launch_bounds__(256) void k_bgram_red(BlockArgs B, int j, int mode) {
    if (block_done(B)) return;
    __shared__ double s_sum[256];
    const int i = blockIdx.x;
    const int t = blockIdx.y * 16 + (threadIdx.x & 15);
    const int chunk = threadIdx.x >> 4;
    const bool second = mode == 3 && blockIdx.z == 1;
    const double* part = (second ? B.gpart2 : B.gpart) + (int64_t)i * B.rb * 256;
    double s = 0.0;
    for (int b = chunk; b < B.rb; b += 16) s += part[(int64_t)b * 256 + t];
    s_sum[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x >= 16) return;
    s = 0.0;
    for (int c = 0; c < 16; ++c) s += s_sum[c * 16 + threadIdx.x];
    if (mode == 2) {
        B.coef[t] = s;
        return;
    }
    const int m = t >> 4, c = t & 15;
    if (mode == 3) {
        if (!second) {
            B.sbuf[(int64_t)i * 256 + t] = s;
        } else if (i < j) {
            // G[i][j-1] (0-based blocks) = V_i^T V_j; the diagonal block is
            // written once, as computed
            const int64_t col = 16 * (j - 1);
            B.G[(int64_t)(16 * i + m) * B.ldh + col + c] = s;
            if (i < j - 1) B.G[(col + c) * B.ldh + 16 * i + m] = s;
        }
        return;
    }
    double* h = B.H + (int64_t)(16 * i + m) * B.ldh + 16 * (j - 1) + c;
    if (mode == 0) *h = s;
    else *h += s;
    B.coef[(int64_t)i * 256 + t] = -s;
}

// Block column j of H for the one-pass step, block i = blockIdx.x < j (entry
// (a, c) per thread): with S_l = V_l^T W and E = V^T V - I over blocks
// 1..j,  H_{i,j} = S_i - (E S)_i.  This is the second classical Gram-Schmidt
// pass, V^T (W - V S) = S - V^T V S, evaluated on the Gram matrix; E S is
// formed directly (E's diagonal as G_aa - 1) so the small correction keeps
// its relative accuracy.  coef_i = -H_{i,j} for the update.  Block 0 also
// lowers the re-orthogonalisation flag of the step.
__global__ __launch_bounds__(256) void k_bcorr(BlockArgs B, int j) {
    if (block_done(B)) return;
    const int i = blockIdx.x, t = threadIdx.x;
    const int a = t >> 4, c = t & 15;
    const int64_t row = 16 * i + a;
    const double* g = B.G + row * B.ldh;
    double es = 0.0;
    for (int l = 0; l < j; ++l) {
        const double* sl = B.sbuf + (int64_t)l * 256;
#pragma unroll 4
        for (int b = 0; b < 16; ++b) {
            const int64_t gc = 16 * l + b;
            const double e = g[gc] - (gc == row ? 1.0 : 0.0);
            es = fma(e, sl[b * 16 + c], es);
        }
    }
    const double h = B.sbuf[(int64_t)i * 256 + t] - es;
    B.H[row * B.ldh + 16 * (j - 1) + c] = h;
    B.coef[(int64_t)i * 256 + t] = -h;
    if (i == 0 && t == 0) B.state[4] = 0;
}

// CholQR step on the Gram matrix G = W^T W in coef_0 (one wave, 16 x 16 in
// LDS): G = R^T R with R upper triangular and a positive diagonal; padded
// columns (c >= p) get R_cc = 1.  coef_0 <- R^{-1} for the in-place W R^{-1}.
// pass 1 also decides breakdown: a diagonal R_cc <= tau ends the run before
// block j + 1 (or, for the start block j = 0, marks it rank deficient).
// pass 2 writes H_{j+1,j} = R2 R1 (start block: R0 = R2 R1).
__global__ __launch_bounds__(64) void k_bchol(BlockArgs B, int j, int pass) {
    if (block_done(B)) return;
    __shared__ double G[16][17], R[16][17], Ri[16][17];
    __shared__ int s_bad;
    const int tid = threadIdx.x;
    for (int e = tid; e < 256; e += 64) {
        G[e / 16][e % 16] = B.coef[e];
        R[e / 16][e % 16] = 0.0;
        Ri[e / 16][e % 16] = 0.0;
    }
    if (tid == 0) s_bad = 0;
    __syncthreads();
    // breakdown: R_cc <= 1024 eps ||A||_inf for a new block; for the start
    // block, R_cc <= 1024 eps max_c |g_c| (dependent generator columns)
    double gmax = 0.0;
    for (int c = 0; c < B.p; ++c) gmax = fmax(gmax, sqrt(fmax(G[c][c], 0.0)));
    const double tau = j == 0 ? B.tau_scale * gmax : B.tau_scale * *B.anorm;
    // one-pass step: a column that kept less than sqrt(reorth2) of its norm
    // through the projection asks for a plain second pass (|W_c|^2 before
    // the projection is W^T W's diagonal in sbuf); the breakdown decision is
    // then left to the factorisation that follows that pass
    bool raise = false;
    if (pass == 1 && j >= 1 && B.cond == nullptr && B.reorth2 > 0.0) {
        for (int c = 0; c < B.p; ++c)
            raise = raise || G[c][c] < B.reorth2 * B.sbuf[(int64_t)j * 256 + c * 17];
    }
    if (raise && tid == 0) B.state[4] = 1;
    for (int c = 0; c < 16; ++c) {
        // every thread forms the pivot (same operations, same value)
        double d = G[c][c];
        for (int q = 0; q < c; ++q) d -= R[q][c] * R[q][c];
        const bool real = c < B.p;
        const double rc = real ? (d > 0.0 ? sqrt(d) : 0.0) : 1.0;
        if (tid == 0 && real) {
            if (!isfinite(d)) s_bad = 2;
            else if (!raise && (!(rc > 0.0) || (pass == 1 && !(rc > tau)))) s_bad = s_bad ? s_bad : 1;
        }
        const double piv = rc > 0.0 ? rc : 1.0;
        if (tid == c) R[c][c] = piv;
        if (real && tid > c && tid < B.p) {
            double v = G[c][tid];
            for (int q = 0; q < c; ++q) v -= R[q][c] * R[q][tid];
            R[c][tid] = v / piv;
        }
        __syncthreads();
    }
    if (s_bad) {
        if (tid == 0) {
            if (s_bad == 2) B.state[2] = 1;
            B.state[0] = 1;
            B.state[1] = j;        // blocks of the run (0: the start block itself is unusable)
        }
        return;
    }
    // R^{-1}: thread c < 16 solves column c by back substitution
    if (tid < 16) {
        const int c = tid;
        Ri[c][c] = 1.0 / R[c][c];
        for (int a = c - 1; a >= 0; --a) {
            double v = 0.0;
            for (int q = a + 1; q <= c; ++q) v += R[a][q] * Ri[q][c];
            Ri[a][c] = -v / R[a][a];
        }
    }
    __syncthreads();
    for (int e = tid; e < 256; e += 64) B.coef[e] = Ri[e / 16][e % 16];
    if (pass == 1) {
        for (int e = tid; e < 256; e += 64) B.rfirst[e] = R[e / 16][e % 16];
        return;
    }
    // R_total = R2 R1 (both upper triangular)
    double* dst = j == 0 ? B.R0 : B.H + (int64_t)(16 * j) * B.ldh + 16 * (j - 1);
    const int64_t ld = j == 0 ? 16 : B.ldh;
    for (int e = tid; e < 256; e += 64) {
        const int a = e / 16, b = e % 16;
        double v = 0.0;
        for (int q = a; q <= b; ++q) v += R[a][q] * B.rfirst[q * 16 + b];
        dst[a * ld + b] = (a < B.p && b < B.p) ? v : 0.0;
    }
    if (tid == 0) B.state[1] = j + 1;
}

// Y = (accumulate ? Y : 0) + sum_{i < nx} X_i M_i, M_i = coef_i (16 x 16).
// One wave per 16-row tile.  Lane l loads its row r0 + l % 16, columns
// 4 (l / 16) .. 4 (l / 16) + 3 (one 32-byte load); MFMA t (t = 0..3) pairs
// slot k = l / 16 with column 4k + t, so the four MFMAs cover all 16
// columns of X_i without moving data between lanes.  In place (X_0 = Y) is
// safe: a wave reads its whole tile before it writes.
template <typename E>
__global__ __launch_bounds__(kBlock) void k_bupdate(const E* __restrict__ X0, int64_t xstride, int nx,
                                                    E* __restrict__ Y, int accumulate, BlockArgs B) {
    if (block_done(B)) return;
    __shared__ double s_m[8 * 256];
    const int l = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t tiles = (B.n + 15) / 16;
    const int64_t tile = (int64_t)blockIdx.x * (kBlock / 64) + wave;
    const bool live = tile < tiles;
    const int64_t r0 = (live ? tile : 0) * 16;
    const int col = l & 15, sub = l >> 4;
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
    if (accumulate && live) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t row = r0 + 4 * q + sub;
            acc[q] = row < B.n ? (double)Y[row * kBW + col] : 0.0;
        }
    }
    const int64_t xrow = r0 + col;
    const bool xok = live && xrow < B.n;
    for (int i0 = 0; i0 < nx; i0 += 8) {
        const int ni = min(8, nx - i0);
        __syncthreads();
        for (int t = threadIdx.x; t < ni * 256; t += kBlock) s_m[t] = B.coef[(int64_t)i0 * 256 + t];
        __syncthreads();
        for (int ii = 0; ii < ni; ++ii) {
            const E* X = X0 + (int64_t)(i0 + ii) * xstride;
            double xv[4];
            const int64_t rr = xok ? xrow : 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double v = (double)X[rr * kBW + 4 * sub + t];
                xv[t] = xok ? v : 0.0;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) acc = mfma16(xv[t], s_m[ii * 256 + (4 * sub + t) * 16 + col], acc);
        }
    }
    if (!live) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t row = r0 + 4 * q + sub;
        if (row < B.n) Y[row * kBW + col] = (E)acc[q];
    }
}

// Partials of C V_j over the rows of each output set only: workgroup
// (q, g) takes rows lo + g * 16 + group, stepping by 16 * gridDim.y, of every
// segment of set q; group of 16 lanes per row, lane = column.
template <typename E>
__global__ __launch_bounds__(kBlock) void k_bproj(SegTable T, int32_t oset0, const E* __restrict__ V,
                                                  double* __restrict__ part, BlockArgs B) {
    if (block_done(B)) return;
    __shared__ double s_acc[kBlock];
    const int q = blockIdx.x, g = blockIdx.y, G = gridDim.y;
    const int c = threadIdx.x & 15, grp = threadIdx.x >> 4;
    const int s = oset0 + q;
    double acc = 0.0;
    for (int32_t seg = T.set_begin[s]; seg < T.set_begin[s + 1]; ++seg) {
        const int64_t lo = T.lo[seg], hi = T.hi[seg];
        const double w = T.w[seg];
        for (int64_t r = lo + (int64_t)g * 16 + grp; r < hi; r += (int64_t)16 * G)
            acc = fma(w, (double)V[r * kBW + c], acc);
    }
    s_acc[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < 16) {
        double t = 0.0;
        for (int k = 0; k < kBlock / 16; ++k) t += s_acc[k * 16 + threadIdx.x];
        part[((int64_t)q * G + g) * 16 + threadIdx.x] = t;
    }
}

// P[:, 16 j + c] = sum of the projection partials (one thread per (q, c)).
__global__ __launch_bounds__(128) void k_bproj_red(const double* __restrict__ part, int o, int G, int j,
                                                   BlockArgs B) {
    if (block_done(B)) return;
    const int t = threadIdx.x;
    if (t >= o * 16) return;
    const int q = t / 16, c = t % 16;
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += part[((int64_t)q * G + g) * 16 + c];
    B.P[(int64_t)q * B.ldp + 16 * j + c] = c < B.p ? s : 0.0;
}

}  // namespace

// ---- launchers -------------------------------------------------------------

hipError_t launch_bstart(bool f32, const SegTable& T, const BlockStart& S, void* V, int64_t n, hipStream_t s) {
    const int64_t want = (n + kBlock / 16 - 1) / (kBlock / 16);
    const int grid = (int)std::min<int64_t>(want, 8192);
    if (f32) hipLaunchKernelGGL(k_bstart<float>, dim3(grid), dim3(kBlock), 0, s, T, S, static_cast<float*>(V), n);
    else hipLaunchKernelGGL(k_bstart<double>, dim3(grid), dim3(kBlock), 0, s, T, S, static_cast<double*>(V), n);
    return hipGetLastError();
}

hipError_t launch_bspmm(bool f32, const CsrArgs& A, const void* V, void* W, const BlockArgs& B, hipStream_t s) {
    // by default 64 rows per workgroup (4 per group of 16 lanes) in
    // workgroup order.  Measured on the 10^7-row convection-diffusion
    // system, FP64: 2098 us per launch at 64 or 256 rows, 2178 us at 1024,
    // 2275 us at 16, and 2341 us with ~4096 workgroups of 2442 rows each
    // mapped XCD-contiguously.  The tuner may choose others.
    const int64_t rpb = B.spmm_rows > 0 ? B.spmm_rows : 64;
    int64_t grid = (B.n + rpb - 1) / rpb;
    if (B.spmm_xcd) grid = (grid + 7) / 8 * 8;      // the XCD map takes a multiple of 8
    if (f32)
        hipLaunchKernelGGL(k_bspmm<float>, dim3((unsigned)grid), dim3(kBlock), 0, s, A,
                           static_cast<const float*>(V), static_cast<float*>(W), B.n, rpb, B);
    else
        hipLaunchKernelGGL(k_bspmm<double>, dim3((unsigned)grid), dim3(kBlock), 0, s, A,
                           static_cast<const double*>(V), static_cast<double*>(W), B.n, rpb, B);
    return hipGetLastError();
}

template <typename E, int NI, bool TWO>
hipError_t launch_bgram_t(const void* X0, int64_t xstride, int nx, const void* Y, const void* Y2,
                          const BlockArgs& B, hipStream_t s) {
    hipLaunchKernelGGL((k_bgram<E, NI, TWO>), dim3(B.rb), dim3(kBlock), 0, s, static_cast<const E*>(X0), xstride,
                       nx, static_cast<const E*>(Y), static_cast<const E*>(Y2), B);
    return hipGetLastError();
}

template <typename E, bool TWO>
hipError_t launch_bgram_e(const void* X0, int64_t xstride, int nx, const void* Y, const void* Y2,
                          const BlockArgs& B, hipStream_t s) {
    switch ((nx + 3) / 4) {
        case 1: return launch_bgram_t<E, 1, TWO>(X0, xstride, nx, Y, Y2, B, s);
        case 2: return launch_bgram_t<E, 2, TWO>(X0, xstride, nx, Y, Y2, B, s);
        case 3: return launch_bgram_t<E, 3, TWO>(X0, xstride, nx, Y, Y2, B, s);
        case 4: return launch_bgram_t<E, 4, TWO>(X0, xstride, nx, Y, Y2, B, s);
        case 5: return launch_bgram_t<E, 5, TWO>(X0, xstride, nx, Y, Y2, B, s);
        case 6: return launch_bgram_t<E, 6, TWO>(X0, xstride, nx, Y, Y2, B, s);
        case 7: return launch_bgram_t<E, 7, TWO>(X0, xstride, nx, Y, Y2, B, s);
        case 8: return launch_bgram_t<E, 8, TWO>(X0, xstride, nx, Y, Y2, B, s);
        case 9: return launch_bgram_t<E, 9, TWO>(X0, xstride, nx, Y, Y2, B, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bgram(bool f32, const void* X0, int64_t xstride, int nx, const void* Y, const BlockArgs& B,
                        hipStream_t s, const void* Y2) {
    if (nx < 1 || nx > kMaxKB + 1) return hipErrorInvalidValue;
    if (Y2 != nullptr) {
        if (B.gpart2 == nullptr) return hipErrorInvalidValue;
        return f32 ? launch_bgram_e<float, true>(X0, xstride, nx, Y, Y2, B, s)
                   : launch_bgram_e<double, true>(X0, xstride, nx, Y, Y2, B, s);
    }
    if (nx == 1) {
        if (f32)
            hipLaunchKernelGGL(k_bgram1<float>, dim3(B.rb), dim3(kBlock), 0, s, static_cast<const float*>(X0),
                               static_cast<const float*>(Y), B);
        else
            hipLaunchKernelGGL(k_bgram1<double>, dim3(B.rb), dim3(kBlock), 0, s, static_cast<const double*>(X0),
                               static_cast<const double*>(Y), B);
        return hipGetLastError();
    }
    return f32 ? launch_bgram_e<float, false>(X0, xstride, nx, Y, Y, B, s)
               : launch_bgram_e<double, false>(X0, xstride, nx, Y, Y, B, s);
}

hipError_t launch_bgram_red(const BlockArgs& B, int nx, int j, int mode, hipStream_t s) {
    if (mode == 3 && (B.sbuf == nullptr || B.G == nullptr)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bgram_red, dim3(nx, 16, mode == 3 ? 2 : 1), dim3(256), 0, s, B, j, mode);
    return hipGetLastError();
}

hipError_t launch_bcorr(const BlockArgs& B, int j, hipStream_t s) {
    if (B.sbuf == nullptr || B.G == nullptr || j < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bcorr, dim3(j), dim3(256), 0, s, B, j);
    return hipGetLastError();
}

hipError_t launch_bchol(const BlockArgs& B, int j, int pass, hipStream_t s) {
    hipLaunchKernelGGL(k_bchol, dim3(1), dim3(64), 0, s, B, j, pass);
    return hipGetLastError();
}

hipError_t launch_bupdate(bool f32, const void* X0, int64_t xstride, int nx, void* Y, int accumulate,
                          const BlockArgs& B, hipStream_t s) {
    const int64_t tiles = (B.n + 15) / 16;
    const int64_t grid = (tiles + kBlock / 64 - 1) / (kBlock / 64);
    if (grid > INT32_MAX) return hipErrorInvalidValue;
    if (f32)
        hipLaunchKernelGGL(k_bupdate<float>, dim3((unsigned)grid), dim3(kBlock), 0, s, static_cast<const float*>(X0),
                           xstride, nx, static_cast<float*>(Y), accumulate, B);
    else
        hipLaunchKernelGGL(k_bupdate<double>, dim3((unsigned)grid), dim3(kBlock), 0, s,
                           static_cast<const double*>(X0), xstride, nx, static_cast<double*>(Y), accumulate, B);
    return hipGetLastError();
}

hipError_t launch_bproj(bool f32, const SegTable& T, int32_t oset0, int o, const void* V, double* part, int G,
                        int j, const BlockArgs& B, hipStream_t s) {
    const dim3 grid(o, G);
    if (f32)
        hipLaunchKernelGGL(k_bproj<float>, grid, dim3(kBlock), 0, s, T, oset0, static_cast<const float*>(V), part, B);
    else
        hipLaunchKernelGGL(k_bproj<double>, grid, dim3(kBlock), 0, s, T, oset0, static_cast<const double*>(V), part,
                           B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bproj_red, dim3(1), dim3(128), 0, s, part, o, G, j, B);
    return hipGetLastError();
}

}  // namespace kry
