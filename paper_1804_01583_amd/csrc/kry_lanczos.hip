// Streaming kernels of the Lanczos process (paper Algorithms 3 and 4) on gfx950.
//
// One Lanczos iteration j of a batch of P independent runs is two launches:
//   spmv  : w = A v_j - beta_{j-1} v_{j-1}        and block partials of v_j . w
//   sweep : w -= alpha_j v_j                       and block partials of |w|^2, C w
// Vectors are stored unnormalised (u_j, with v_j = sigma_j u_j and
// sigma_j = 1 / beta_{j-1}), so no pass is spent on the normalisation of
// Algorithm 3; the scale is applied where the vector is read.  Batches store
// their P vectors interleaved ([n][P]) so a gathered column of A reads P
// contiguous values.  Vectors (and, for CSR, the matrix values) are held as
// E = double, or E = float in FP32-basis mode; arithmetic and every reduction
// stay FP64.
//
// Reductions: a kernel writes one partial per block and value; every block of
// the next kernel sums them in the same fixed order (strided per thread, wave
// butterfly, waves in order), so all blocks hold bit-identical scalars and
// block 0 records them (alpha_j, beta_{j-1}, sigma_j, k_eff).  The partials of
// |u_j|^2 and C u_j are kept per iteration, and k_finish turns them into the
// columns of P = C V once per batch.  The row -> block partition depends on n
// only, so a run's arithmetic does not depend on which batch (or P) advances it.
#include "kry_device.h"

#include <cmath>

namespace kry {

namespace {

using namespace dev;
// ---------------------------------------------------------------------------

// max_r sum_e |vals[e]| (row sums in CSR order, one thread per row): block
// maxima, then one block reduces them.
__global__ __launch_bounds__(kBlock) void k_row_abs_max(CsrArgs A, int64_t n, int64_t rows_per_block,
                                                        double* part) {
    __shared__ double s_m[kBlock / 64];
    const int lb = logical_block((int)gridDim.x);
    const int64_t r0 = (int64_t)lb * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    double v = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        double s = 0.0;
        for (int64_t e = A.rowptr[r]; e < A.rowptr[r + 1]; ++e) s += fabs(A.vals[e]);
        v = s > v ? s : v;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) v = s_m[w] > v ? s_m[w] : v;
        part[lb] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce_max(const double* part, int nb, double* out) {
    __shared__ double s_m[kBlock / 64];
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) v = part[b] > v ? part[b] : v;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) v = s_m[w] > v ? s_m[w] : v;
        *out = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_to_f32(const double* __restrict__ in, float* __restrict__ out,
                                                   int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) out[i] = (float)in[i];
}

// a2: start vectors u_1 of the runs and the partials of |u_1|^2 and C u_1
// (Algorithm 4, first two statements; the scaling happens in the next kernel).
template <typename E, int P, int O>
__global__ __launch_bounds__(kBlock) void k_start(StartSrc src, SegTable T, int32_t oset0,
                                                  E* __restrict__ u, BatchArgs B) {
    if (batch_stopped<P>(B)) return;   // a fallback the one-pass step did not need
    constexpr int NV = P * (1 + O);
    // up to 256 segments per set and block in LDS when there are few sets:
    // a generator over a region of a large grid has a few hundred per block
    // (the 1000^3 heated region about 200), and a set past the capacity is
    // read from global memory row by row
    constexpr int CAP = P + O <= 4 ? 256 : kSegCap;
    __shared__ double s_lds[(kBlock / 64) * NV];
    __shared__ SegStage<P + O, CAP> st;
    const int lb = logical_block(B.nblocks, B.xcd_map);
    const int64_t r0 = (int64_t)lb * B.rows_per_block;
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    int sets[P + O];
#pragma unroll
    for (int i = 0; i < P; ++i) sets[i] = src.set[i];
#pragma unroll
    for (int q = 0; q < O; ++q) sets[P + q] = oset0 + q;
    stage_segments<P + O, CAP>(st, T, sets, lb, B.nblocks);
    SegCursor cur[P + O];
#pragma unroll
    for (int i = 0; i < P + O; ++i) cur[i].init(st, i);
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    // rows r0 + threadIdx.x, + kBlock, ... in chunks of RC per thread; a
    // chunk's dense start entries are all requested before the first is used
    constexpr int RC = 4;
    const int64_t span = (int64_t)kBlock * RC;
    for (int64_t c0 = r0; c0 < r1; c0 += span) {
        double dv[RC][P];
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            const int64_t r = c0 + (int64_t)i * kBlock + threadIdx.x;
            const int64_t rl = r < r1 ? r : r0;
#pragma unroll
            for (int p = 0; p < P; ++p) dv[i][p] = src.dense[p] != nullptr ? src.dense[p][rl] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            const int64_t r = c0 + (int64_t)i * kBlock + threadIdx.x;
            if (r >= r1) continue;
            double val[P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (src.dense[p] != nullptr) val[p] = dv[i][p];
                else if (src.set[p] >= 0) val[p] = cur[p].weight(st, p, T, r);
                else val[p] = 0.0;
                val[p] = (double)(E)val[p];          // the norm and projection of the stored vector
                acc[p] = fma(val[p], val[p], acc[p]);
            }
            store_row<E, P>(u, r, val);
#pragma unroll
            for (int q = 0; q < O; ++q) {
                const double cw = cur[P + q].weight(st, P + q, T, r);
                if (cw != 0.0) {
#pragma unroll
                    for (int p = 0; p < P; ++p) acc[P + q * P + p] = fma(cw, val[p], acc[P + q * P + p]);
                }
            }
        }
    }
    store_partials<NV>(acc, stage_part(B, 0), B.nblocks, s_lds, B.xcd_map);
}

// a3 + first half of a4: w = sigma_j A u_j - beta_{j-1} sigma_{j-1} u_{j-1}
// (Lanczos), or w = sigma_j A u_j when uprev is null (Arnoldi); partials of
// (sigma_j u_j) . w.  LPR lanes cooperate on one row.  Rows are
// taken in chunks of RC per lane group; the first chunk's gathers are issued
// before the stage reduction they do not depend on.
template <typename E, int P, int LPR>
__device__ __forceinline__ double csr_val(const CsrArgs& A, int64_t e) {
    if constexpr (sizeof(E) == 4) return (double)A.vals32[e];
    else return A.vals[e];
}

template <typename E, int P, int LPR>
__global__ __launch_bounds__(kBlock) void k_spmv_csr(CsrArgs A, const E* __restrict__ ucur,
                                                     const E* __restrict__ uprev,
                                                     E* __restrict__ w, BatchArgs B, int j) {
    if (batch_stopped<P>(B)) return;   // the batch met its error target
    constexpr int G = kBlock / LPR;
    constexpr int RC = 2;
    constexpr int U = P >= 8 ? 2 : (P >= 4 ? 4 : 8);
    __shared__ double s_lds[(kBlock / 64) * P];
    __shared__ double s_nrm[P];
    const int lb = logical_block(B.nblocks, B.xcd_map);
    const int64_t r0 = (int64_t)lb * B.rows_per_block;
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    const int sub = threadIdx.x % LPR;
    const int slot = threadIdx.x / LPR;
    double pacc[P], sig_prev[P], anorm;
    load_stage_norms<P>(B, j, pacc, sig_prev, anorm);
    double sig[P], cprev[P], dot[P];
#pragma unroll
    for (int p = 0; p < P; ++p) { sig[p] = 0.0; cprev[p] = 0.0; dot[p] = 0.0; }
    const int64_t span = (int64_t)G * RC;
    const int nch = (int)((B.rows_per_block + span - 1) / span);
    for (int ch = 0; ch < nch; ++ch) {
        int64_t rr[RC], e0[RC], e1[RC];
        double acc[RC][P];
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            rr[i] = r0 + (int64_t)ch * span + (int64_t)i * G + slot;
            const bool live = rr[i] < r1;
            e0[i] = live ? A.rowptr[rr[i]] : 0;
            e1[i] = live ? A.rowptr[rr[i] + 1] : 0;
#pragma unroll
            for (int p = 0; p < P; ++p) acc[i][p] = 0.0;
        }
        // first U entries per lane of every row of the chunk, predicated; a
        // masked slot reads entry 0 of the vector and adds nothing
        {
            int32_t c[RC][U];
            double a[RC][U];
#pragma unroll
            for (int i = 0; i < RC; ++i) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t ee = e0[i] + sub + (int64_t)u * LPR;
                    const bool ok = ee < e1[i];
                    c[i][u] = ok ? A.colidx[ee] : 0;
                    a[i][u] = ok ? csr_val<E, P, LPR>(A, ee) : 0.0;
                }
            }
#pragma unroll
            for (int i = 0; i < RC; ++i) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    // element-wise gathers keep the live registers (and so the
                    // occupancy) lower than one wide load per row; a masked
                    // slot adds 0 * u[0] unconditionally (a non-finite u is
                    // flagged through its norm anyway), so no gather waits
                    // behind a branch of its own
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const double x = (double)ucur[(int64_t)c[i][u] * P + p];
                        acc[i][p] = fma(a[i][u], x, acc[i][p]);
                    }
                }
            }
        }
        // longer rows
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            for (int64_t e = e0[i] + sub + (int64_t)U * LPR; e < e1[i]; e += LPR) {
                const int64_t c = A.colidx[e];
                const double a = csr_val<E, P, LPR>(A, e);
                double x[P];
                load_row<E, P>(ucur, c, x);
#pragma unroll
                for (int p = 0; p < P; ++p) acc[i][p] = fma(a, x[p], acc[i][p]);
            }
        }
        if (LPR > 1) {
#pragma unroll
            for (int off = LPR / 2; off >= 1; off >>= 1) {
#pragma unroll
                for (int i = 0; i < RC; ++i) {
#pragma unroll
                    for (int p = 0; p < P; ++p) acc[i][p] += __shfl_xor(acc[i][p], off, LPR);
                }
            }
        }
        if (ch == 0) finish_stage_norms<P>(B, j, pacc, sig_prev, anorm, s_lds, s_nrm, sig, cprev);
        if (sub == 0) {
#pragma unroll
            for (int i = 0; i < RC; ++i) {
                if (rr[i] < r1) {
                    const int64_t r = rr[i];
                    double own[P], pv[P], y[P];
                    load_row<E, P>(ucur, r, own);
                    if (j > 1 && uprev != nullptr) load_row<E, P>(uprev, r, pv);
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        y[p] = sig[p] * acc[i][p];
                        if (j > 1 && uprev != nullptr) y[p] = fma(-cprev[p], pv[p], y[p]);
                        y[p] = (double)(E)y[p];
                        dot[p] = fma(sig[p] * own[p], y[p], dot[p]);
                    }
                    store_row<E, P>(w, r, y);
                }
            }
        }
    }
    if (nch == 0) finish_stage_norms<P>(B, j, pacc, sig_prev, anorm, s_lds, s_nrm, sig, cprev);
    store_partials<P>(dot, B.ap_part, B.ap_nblocks, s_lds, B.xcd_map);
}

// Matrix-free 7-point stencil version of k_spmv_csr (zero outside the grid),
// neighbours summed in ascending index order like a CSR row.  Each thread
// decodes its first row's grid coordinates once and advances them as it
// strides by kBlock rows, so no division runs per row.
template <typename E, int P>
__global__ __launch_bounds__(kBlock) void k_spmv_stencil(StencilArgs S, const E* __restrict__ ucur,
                                                         const E* __restrict__ uprev,
                                                         E* __restrict__ w, BatchArgs B, int j) {
    if (batch_stopped<P>(B)) return;   // the batch met its error target
    __shared__ double s_lds[(kBlock / 64) * P];
    __shared__ double s_nrm[P];
    const int lb = logical_block(B.nblocks, B.xcd_map);
    const int64_t r0 = (int64_t)lb * B.rows_per_block;
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    double pacc[P], sig_prev[P], anorm;
    load_stage_norms<P>(B, j, pacc, sig_prev, anorm);
    int64_t r = r0 + threadIdx.x;
    int64_t iz = r % S.nz;
    int64_t iy = (r / S.nz) % S.ny;
    int64_t ix = r / (S.nz * S.ny);
    double sig[P], cprev[P];
    finish_stage_norms<P>(B, j, pacc, sig_prev, anorm, s_lds, s_nrm, sig, cprev);
    const int64_t sx = S.ny * S.nz, sy = S.nz;
    const bool prev = j > 1 && uprev != nullptr;
    double dot[P];
#pragma unroll
    for (int p = 0; p < P; ++p) dot[p] = 0.0;
    for (; r < r1; r += kBlock) {
        const bool xl = ix > 0, xh = ix < S.nx - 1;
        const bool yl = iy > 0, yh = iy < S.ny - 1;
        const bool zl = iz > 0, zh = iz < S.nz - 1;
        double vxl[P], vyl[P], vzl[P], own[P], vzh[P], vyh[P], vxh[P], pv[P], y[P];
        load_row<E, P>(ucur, xl ? r - sx : r, vxl);
        load_row<E, P>(ucur, yl ? r - sy : r, vyl);
        load_row<E, P>(ucur, zl ? r - 1 : r, vzl);
        load_row<E, P>(ucur, r, own);
        load_row<E, P>(ucur, zh ? r + 1 : r, vzh);
        load_row<E, P>(ucur, yh ? r + sy : r, vyh);
        load_row<E, P>(ucur, xh ? r + sx : r, vxh);
        load_row<E, P>(prev ? uprev : ucur, r, pv);
        const double diag = stencil_diag(S, xl, xh, yl, yh, zl, zh);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            double acc = 0.0;
            if (xl) acc = fma(S.cx, vxl[p], acc);
            if (yl) acc = fma(S.cy, vyl[p], acc);
            if (zl) acc = fma(S.cz, vzl[p], acc);
            acc = fma(diag, own[p], acc);
            if (zh) acc = fma(S.cz, vzh[p], acc);
            if (yh) acc = fma(S.cy, vyh[p], acc);
            if (xh) acc = fma(S.cx, vxh[p], acc);
            y[p] = sig[p] * acc;
            if (prev) y[p] = fma(-cprev[p], pv[p], y[p]);
            y[p] = (double)(E)y[p];
            dot[p] = fma(sig[p] * own[p], y[p], dot[p]);
        }
        store_row<E, P>(w, r, y);
        iz += kBlock;
        while (iz >= S.nz) {
            iz -= S.nz;
            if (++iy == S.ny) { iy = 0; ++ix; }
        }
    }
    store_partials<P>(dot, B.ap_part, B.ap_nblocks, s_lds, B.xcd_map);
}

// One x step of the marching stencil: row r = ix * sx + col with u at x-1,
// x, x+1 in xm, x0, xp; loads the x+2 plane into nx2 (a clamped in-bounds
// address past the end: that value is never used, since the x + 1 term is
// skipped at the last plane).
// store_row with non-temporal stores, element by element
template <typename E, int P>
__device__ __forceinline__ void store_row_nt(E* __restrict__ base, int64_t row, const double (&v)[P]) {
#pragma unroll
    for (int p = 0; p < P; ++p) __builtin_nontemporal_store((E)v[p], base + row * P + p);
}

template <typename E, int P, bool NT = false>
__device__ __forceinline__ void march_step(const StencilArgs& S, const MarchCol& M, int64_t ix,
                                           const E* __restrict__ ucur, const E* __restrict__ up,
                                           E* __restrict__ w, const double (&sig)[P],
                                           const double (&cprev)[P], const double (&xm)[P],
                                           const double (&x0)[P], const double (&xp)[P], double (&nx2)[P],
                                           double (&dot)[P]) {
    const int64_t r = ix * M.sx + M.col;
    double vyl[P], vzl[P], vzh[P], vyh[P], vpr[P];
    load_row<E, P>(ucur, r + M.dyl, vyl);
    load_row<E, P>(ucur, r + M.dzl, vzl);
    load_row<E, P>(ucur, r + M.dzh, vzh);
    load_row<E, P>(ucur, r + M.dyh, vyh);
    load_row<E, P>(up, r, vpr);
    load_row<E, P>(ucur, ix + 2 < S.nx ? r + 2 * M.sx : r, nx2);
    double y[P];
    const double diag = stencil_diag(S, ix > 0, ix < S.nx - 1, M.yl, M.yh, M.zl, M.zh);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        double acc = 0.0;
        if (ix > 0) acc = fma(S.cx, xm[p], acc);
        if (M.yl) acc = fma(S.cy, vyl[p], acc);
        if (M.zl) acc = fma(S.cz, vzl[p], acc);
        acc = fma(diag, x0[p], acc);
        if (M.zh) acc = fma(S.cz, vzh[p], acc);
        if (M.yh) acc = fma(S.cy, vyh[p], acc);
        if (ix < S.nx - 1) acc = fma(S.cx, xp[p], acc);
        y[p] = sig[p] * acc;
        if (M.prev) y[p] = fma(-cprev[p], vpr[p], y[p]);
        y[p] = (double)(E)y[p];
        dot[p] = fma(sig[p] * x0[p], y[p], dot[p]);
    }
    if (M.live) {
        if constexpr (NT) store_row_nt<E, P>(w, r, y);
        else store_row<E, P>(w, r, y);
    }
}

// Matrix-free 7-point stencil, marching form: one thread per (y, z) grid
// column walks along x and keeps u at x-1, x, x+1 in registers (the x+2 plane
// is loaded one step ahead), so each element of u is read from HBM once; the
// y and z neighbours are the same plane's entries of neighbouring threads and
// come from cache.  Column blocks are mapped XCD-contiguously so the y +- 1
// columns share an L2.  Every load is unconditional (boundary neighbours read
// a clamped in-bounds address and are then dropped) and the four plane
// registers rotate by unrolling, so the x+2 load stays in flight across the
// step.  Same summation order per row as k_spmv_stencil.  The dot partials
// are indexed by column block (ap_nblocks of them).
template <typename E, int P, bool NT = false>
__global__ __launch_bounds__(kBlock) void k_spmv_stencil_march(StencilArgs S, const E* __restrict__ ucur,
                                                               const E* __restrict__ uprev,
                                                               E* __restrict__ w, BatchArgs B, int j) {
    if (batch_stopped<P>(B)) return;   // the batch met its error target
    __shared__ double s_lds[(kBlock / 64) * P];
    __shared__ double s_nrm[P];
    const int cb = logical_block(B.ap_nblocks, B.xcd_map);
    const int64_t ncol = S.ny * S.nz;
    const int64_t col0 = (int64_t)cb * kBlock + threadIdx.x;
    MarchCol M;
    M.live = col0 < ncol;
    M.col = M.live ? col0 : ncol - 1;          // dead lanes shadow a live column and store nothing
    M.sx = ncol;
    double pacc[P], sig_prev[P], anorm;
    load_stage_norms<P>(B, j, pacc, sig_prev, anorm);
    const int64_t iy = M.col / S.nz;
    const int64_t iz = M.col % S.nz;
    double a[P], b[P], c[P], d[P];
    load_row<E, P>(ucur, M.col, b);
    load_row<E, P>(ucur, S.nx > 1 ? M.col + M.sx : M.col, c);
#pragma unroll
    for (int p = 0; p < P; ++p) a[p] = 0.0;
    double sig[P], cprev[P];
    finish_stage_norms<P>(B, j, pacc, sig_prev, anorm, s_lds, s_nrm, sig, cprev);
    M.prev = j > 1 && uprev != nullptr;
    const E* __restrict__ up = M.prev ? uprev : ucur;
    M.yl = iy > 0;
    M.yh = iy < S.ny - 1;
    M.zl = iz > 0;
    M.zh = iz < S.nz - 1;
    M.dyl = M.yl ? -S.nz : 0;
    M.dyh = M.yh ? S.nz : 0;
    M.dzl = M.zl ? -1 : 0;
    M.dzh = M.zh ? 1 : 0;
    double dot[P];
#pragma unroll
    for (int p = 0; p < P; ++p) dot[p] = 0.0;
    for (int64_t ix = 0; ix < S.nx; ix += 4) {
        march_step<E, P, NT>(S, M, ix, ucur, up, w, sig, cprev, a, b, c, d, dot);
        if (ix + 1 >= S.nx) break;
        march_step<E, P, NT>(S, M, ix + 1, ucur, up, w, sig, cprev, b, c, d, a, dot);
        if (ix + 2 >= S.nx) break;
        march_step<E, P, NT>(S, M, ix + 2, ucur, up, w, sig, cprev, c, d, a, b, dot);
        if (ix + 3 >= S.nx) break;
        march_step<E, P, NT>(S, M, ix + 3, ucur, up, w, sig, cprev, d, a, b, c, dot);
    }
    if (!M.live) {
#pragma unroll
        for (int p = 0; p < P; ++p) dot[p] = 0.0;
    }
    store_partials<P>(dot, B.ap_part, B.ap_nblocks, s_lds, B.xcd_map);
}

// Second half of a4 + the partials of a5 and a6: alpha_j = sum of the dot
// partials; w -= alpha_j sigma_j u_j; partials of |w|^2 and C w.  The first
// chunk of rows is loaded before the alpha reduction completes.
constexpr int64_t kSweepLongBlock = 65536;   // rows per block from which the sweep takes long chunks

template <typename E, int P, int O, bool LONG, bool NT = false>
__global__ __launch_bounds__(kBlock) void k_sweep(SegTable T, int32_t oset0,
                                                  const E* __restrict__ ucur,
                                                  E* __restrict__ w, BatchArgs B, int j) {
    if (batch_stopped<P>(B)) return;   // the batch met its error target
    constexpr int NV = P * (1 + O);
    // rows per thread and chunk, measured on MI355X: blocks of up to a few
    // thousand rows keep two chunks in flight (one row per thread and chunk,
    // two for two runs); blocks of very many rows (LONG, chosen at launch)
    // stream best in chunks of four rows per thread, one chunk at a time
    constexpr int RC = LONG ? 4 : (P == 2 ? 2 : 1);
    __shared__ double s_lds[(kBlock / 64) * NV];
    __shared__ double s_alpha[P];
    __shared__ SegStage<O> st;
    const int lb = logical_block(B.nblocks, B.xcd_map);
    const int64_t r0 = (int64_t)lb * B.rows_per_block;
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    const int64_t span = (int64_t)kBlock * RC;
    const int nch = max((int)((B.rows_per_block + span - 1) / span), 1);
    // rows of chunk ch in one of two register buffers (the next chunk's loads
    // are in flight while a chunk is processed); dead rows read row 0 and drop it
    double uv[RC][P], wv[RC][P], uv2[RC][P], wv2[RC][P];
    int64_t rr[RC], rr2[RC];
    auto load_into = [&](int ch, double (&u_)[RC][P], double (&w_)[RC][P], int64_t (&r_)[RC]) {
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            r_[i] = r0 + (int64_t)ch * span + (int64_t)i * kBlock + threadIdx.x;
            const int64_t rl = r_[i] < r1 ? r_[i] : 0;
            load_row<E, P>(ucur, rl, u_[i]);
            load_row<E, P>(w, rl, w_[i]);
        }
    };
    auto load_chunk = [&](int ch) { load_into(ch, uv, wv, rr); };
    // Loads are issued in the order they are waited for (a wait covers every
    // load issued before it): the alpha partials, sigma_j and the output
    // sets' segment ranges, then the first chunk's rows, which stay in
    // flight through the alpha reduction and any segment staging.
    PartialBatch<P> pb;
    pb.issue(B.ap_part, B.ap_nblocks, 0);
    double sigj[P];
#pragma unroll
    for (int p = 0; p < P; ++p) sigj[p] = run_scal(B, p)[B.L.sigma + j];
    // every thread reads the output sets' segment ranges for this block
    // (uniform addresses); most blocks meet no output segment and then skip
    // the staging, its barriers and the per-row weights
    SegRange own{0, 0};
    bool any = false;
#pragma unroll
    for (int q = 0; q < O; ++q) {
        const int32_t* rq = T.blk + ((int64_t)(oset0 + q) * B.nblocks + lb) * 2;
        const SegRange r{rq[0], rq[1]};
        any = any || r.e > r.b;
        if ((int)threadIdx.x == q) own = r;
    }
    load_chunk(0);
    SegCursor cur[O];
    if (any) {
        stage_segments<O>(st, T, own);
#pragma unroll
        for (int q = 0; q < O; ++q) cur[q].init(st, q);
    }
    double acc[NV], coef[P];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    {
        double pacc[P];
        pb.sum(B.ap_part, B.ap_nblocks, 0, pacc);
        const double t = block_sum<P>(pacc, s_lds);
        if (threadIdx.x < P) s_alpha[threadIdx.x] = t;
        __syncthreads();
#pragma unroll
        for (int p = 0; p < P; ++p) coef[p] = s_alpha[p] * sigj[p];
        if (blockIdx.x == 0 && threadIdx.x < P) {
            double* sc = run_scal(B, threadIdx.x);
            sc[B.L.alpha + j] = s_alpha[threadIdx.x];
            if (!isfinite(s_alpha[threadIdx.x])) sc[B.L.misc + MISC_NONFINITE] = 1.0;
        }
    }
    auto process = [&](const double (&u_)[RC][P], const double (&w_)[RC][P], const int64_t (&r_)[RC]) {
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            if (r_[i] < r1) {
                const int64_t r = r_[i];
                double val[P];
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    val[p] = (double)(E)fma(-coef[p], u_[i][p], w_[i][p]);
                    acc[p] = fma(val[p], val[p], acc[p]);
                }
                if constexpr (NT) store_row_nt<E, P>(w, r, val);
                else store_row<E, P>(w, r, val);
                if (any) {
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
        }
    };
    if constexpr (LONG) {
        for (int ch = 0; ch < nch; ++ch) {
            if (ch > 0) load_chunk(ch);
            process(uv, wv, rr);
        }
    } else {
        for (int ch = 0; ch < nch; ch += 2) {
            if (ch + 1 < nch) load_into(ch + 1, uv2, wv2, rr2);
            process(uv, wv, rr);
            if (ch + 1 < nch) {
                if (ch + 2 < nch) load_into(ch + 2, uv, wv, rr);
                process(uv2, wv2, rr2);
            }
        }
    }
    store_partials<NV>(acc, stage_part(B, j), B.nblocks, s_lds, B.xcd_map);
}

// After the last sweep, one block per stage c = 0..kdone: P[:, c] = sigma_{c+1} C u_{c+1}
// from the stored partials of that stage; block kdone also records the final
// stage (beta_kdone, sigma_{kdone+1}, and k_eff when the run breaks down there).
// Values are summed by groups of threads, each group in a fixed order.
template <int P>
__global__ __launch_bounds__(kBlock) void k_finish(BatchArgs B, int o, int kdone) {
    __shared__ double s_part[kBlock];
    __shared__ double s_tot[P * (1 + kMaxO)];
    const int c = blockIdx.x;
    if (B.stop != nullptr) {
        // error control: the batch iterated up to the largest Krylov dimension
        // its runs settled on (k when one of them never met its target)
        int kd = 0;
#pragma unroll
        for (int p = 0; p < P; ++p) kd = max(kd, (int)run_scal(B, p)[B.L.misc + MISC_KSTOP]);
        kdone = min(kd, kdone);
    }
    if (c > kdone) return;
    const int nv = P * (1 + o);
    const int grp = kBlock / nv;
    const int v = threadIdx.x / grp, g = threadIdx.x % grp;
    const double* part = stage_part(B, c);
    double acc = 0.0;
    if (v < nv) {
        // four loads in flight per step, summed in b order
        const double* pv = part + (int64_t)v * B.nblocks;
        for (int b0 = g; b0 < B.nblocks; b0 += 4 * grp) {
            double x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = b0 + u * grp < B.nblocks ? pv[b0 + u * grp] : 0.0;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (b0 + u * grp < B.nblocks) acc += x[u];
        }
    }
    s_part[threadIdx.x] = acc;
    __syncthreads();
    if (v < nv && g == 0) {
        double t = 0.0;
        for (int i = 0; i < grp; ++i) t += s_part[v * grp + i];
        s_tot[v] = t;
    }
    __syncthreads();
    if (c == kdone) record_stage(B, P, c + 1, s_tot);
    __syncthreads();
    if (threadIdx.x < P * o) {
        const int q = threadIdx.x / P, p = threadIdx.x % P;
        double* sc = run_scal(B, p);
        double sig;
        if (c == kdone) sig = stage_update(B, sc, c + 1, s_tot[p]).sigma;
        else sig = sc[B.L.sigma + c + 1];
        sc[B.L.proj + q * (B.L.k + 1) + c] = sig * s_tot[P + q * P + p];
    }
}

template <typename E, int P, int O>
hipError_t launch_start_t(const StartSrc& src, const SegTable& T, int32_t oset0, void* u,
                          const BatchArgs& B, hipStream_t s) {
    hipLaunchKernelGGL((k_start<E, P, O>), dim3(B.nblocks), dim3(kBlock), 0, s, src, T, oset0, static_cast<E*>(u),
                       B);
    return hipGetLastError();
}

template <typename E, int P, int O>
hipError_t launch_sweep_t(const SegTable& T, int32_t oset0, const void* ucur, void* w,
                          const BatchArgs& B, int j, hipStream_t s) {
    // blocks of very many rows (grids far past the caches) store the swept
    // vector non-temporally: the 10^9-state sweep took 9.8 ms instead of 10.2
    if (B.rows_per_block >= kSweepLongBlock)
        hipLaunchKernelGGL((k_sweep<E, P, O, true, true>), dim3(B.nblocks), dim3(kBlock), 0, s, T, oset0,
                           static_cast<const E*>(ucur), static_cast<E*>(w), B, j);
    else
        hipLaunchKernelGGL((k_sweep<E, P, O, false>), dim3(B.nblocks), dim3(kBlock), 0, s, T, oset0,
                           static_cast<const E*>(ucur), static_cast<E*>(w), B, j);
    return hipGetLastError();
}

template <typename E, int P, int LPR>
hipError_t launch_spmv_t(const CsrArgs& A, const void* ucur, const void* uprev, void* w,
                         const BatchArgs& B, int j, hipStream_t s) {
    hipLaunchKernelGGL((k_spmv_csr<E, P, LPR>), dim3(B.nblocks), dim3(kBlock), 0, s, A,
                       static_cast<const E*>(ucur), static_cast<const E*>(uprev), static_cast<E*>(w), B, j);
    return hipGetLastError();
}

// Dispatch over O for fixed E and P; P * (1 + O) <= kMaxNV limits P = 4 to
// O <= 5 and P = 8 to O <= 2.
#define KRY_DISPATCH_O2(FN, E, P, O, ...)             \
    switch (O) {                                      \
        case 1: return FN<E, P, 1>(__VA_ARGS__);      \
        case 2: return FN<E, P, 2>(__VA_ARGS__);      \
        default: return hipErrorInvalidValue;         \
    }
#define KRY_DISPATCH_O5(FN, E, P, O, ...)             \
    switch (O) {                                      \
        case 1: return FN<E, P, 1>(__VA_ARGS__);      \
        case 2: return FN<E, P, 2>(__VA_ARGS__);      \
        case 3: return FN<E, P, 3>(__VA_ARGS__);      \
        case 4: return FN<E, P, 4>(__VA_ARGS__);      \
        case 5: return FN<E, P, 5>(__VA_ARGS__);      \
        default: return hipErrorInvalidValue;         \
    }
#define KRY_DISPATCH_O8(FN, E, P, O, ...)             \
    switch (O) {                                      \
        case 1: return FN<E, P, 1>(__VA_ARGS__);      \
        case 2: return FN<E, P, 2>(__VA_ARGS__);      \
        case 3: return FN<E, P, 3>(__VA_ARGS__);      \
        case 4: return FN<E, P, 4>(__VA_ARGS__);      \
        case 5: return FN<E, P, 5>(__VA_ARGS__);      \
        case 6: return FN<E, P, 6>(__VA_ARGS__);      \
        case 7: return FN<E, P, 7>(__VA_ARGS__);      \
        case 8: return FN<E, P, 8>(__VA_ARGS__);      \
        default: return hipErrorInvalidValue;         \
    }
#define KRY_DISPATCH_PO(FN, E, P, O, ...)                                  \
    switch (P) {                                                           \
        case 1: KRY_DISPATCH_O8(FN, E, 1, O, __VA_ARGS__)                  \
        case 2: KRY_DISPATCH_O8(FN, E, 2, O, __VA_ARGS__)                  \
        case 4: KRY_DISPATCH_O5(FN, E, 4, O, __VA_ARGS__)                  \
        case 8: KRY_DISPATCH_O2(FN, E, 8, O, __VA_ARGS__)                  \
        default: return hipErrorInvalidValue;                              \
    }

template <typename E>
hipError_t launch_start_e(int P, int O, const StartSrc& src, const SegTable& T, int32_t oset0, void* u,
                          const BatchArgs& B, hipStream_t s) {
    KRY_DISPATCH_PO(launch_start_t, E, P, O, src, T, oset0, u, B, s)
}

template <typename E>
hipError_t launch_sweep_e(int P, int O, const SegTable& T, int32_t oset0, const void* ucur, void* w,
                          const BatchArgs& B, int j, hipStream_t s) {
    KRY_DISPATCH_PO(launch_sweep_t, E, P, O, T, oset0, ucur, w, B, j, s)
}

template <typename E>
hipError_t launch_spmv_csr_e(int P, int lpr, const CsrArgs& A, const void* ucur, const void* uprev, void* w,
                             const BatchArgs& B, int j, hipStream_t s) {
#define KRY_LPR(PP)                                                                \
    switch (lpr) {                                                                 \
        case 1: return launch_spmv_t<E, PP, 1>(A, ucur, uprev, w, B, j, s);        \
        case 2: return launch_spmv_t<E, PP, 2>(A, ucur, uprev, w, B, j, s);        \
        case 4: return launch_spmv_t<E, PP, 4>(A, ucur, uprev, w, B, j, s);        \
        case 8: return launch_spmv_t<E, PP, 8>(A, ucur, uprev, w, B, j, s);        \
        default: return hipErrorInvalidValue;                                      \
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

template <typename E, int P>
hipError_t launch_stencil_pe(bool march, const StencilArgs& A, const void* ucur, const void* uprev, void* w,
                             const BatchArgs& B, int j, hipStream_t s) {
    const E* uc = static_cast<const E*>(ucur);
    const E* up = static_cast<const E*>(uprev);
    E* ww = static_cast<E*>(w);
    // the marching form (large grids) stores w non-temporally: 10.6 ms
    // instead of 11.6 per launch on the 10^9-state grid with two runs
    if (march)
        hipLaunchKernelGGL((k_spmv_stencil_march<E, P, true>), dim3(B.ap_nblocks), dim3(kBlock), 0, s, A, uc, up, ww,
                           B, j);
    else
        hipLaunchKernelGGL((k_spmv_stencil<E, P>), dim3(B.nblocks), dim3(kBlock), 0, s, A, uc, up, ww, B, j);
    return hipGetLastError();
}

template <typename E>
hipError_t launch_stencil_e(int P, bool march, const StencilArgs& A, const void* ucur, const void* uprev,
                            void* w, const BatchArgs& B, int j, hipStream_t s) {
    switch (P) {
        case 1: return launch_stencil_pe<E, 1>(march, A, ucur, uprev, w, B, j, s);
        case 2: return launch_stencil_pe<E, 2>(march, A, ucur, uprev, w, B, j, s);
        case 4: return launch_stencil_pe<E, 4>(march, A, ucur, uprev, w, B, j, s);
        case 8: return launch_stencil_pe<E, 8>(march, A, ucur, uprev, w, B, j, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_row_abs_max(const CsrArgs& A, int64_t n, double* partials, int32_t nblocks,
                              int64_t rows_per_block, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_row_abs_max, dim3(nblocks), dim3(kBlock), 0, s, A, n, rows_per_block, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(kBlock), 0, s, partials, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_to_f32(const double* in, float* out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + kBlock - 1) / kBlock;
    const int grid = (int)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(k_to_f32, dim3(grid), dim3(kBlock), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_start(int P, int O, bool f32, const StartSrc& src, const SegTable& T, int32_t oset0,
                        void* u, const BatchArgs& B, hipStream_t s) {
    if (P * (1 + O) > kMaxNV) return hipErrorInvalidValue;
    return f32 ? launch_start_e<float>(P, O, src, T, oset0, u, B, s)
               : launch_start_e<double>(P, O, src, T, oset0, u, B, s);
}

hipError_t launch_sweep(int P, int O, bool f32, const SegTable& T, int32_t oset0, const void* ucur,
                        void* w, const BatchArgs& B, int j, hipStream_t s) {
    if (P * (1 + O) > kMaxNV) return hipErrorInvalidValue;
    return f32 ? launch_sweep_e<float>(P, O, T, oset0, ucur, w, B, j, s)
               : launch_sweep_e<double>(P, O, T, oset0, ucur, w, B, j, s);
}

hipError_t launch_finish(int P, int O, const BatchArgs& B, int kdone, hipStream_t s) {
    const dim3 grid(kdone + 1);
    switch (P) {
        case 1: hipLaunchKernelGGL((k_finish<1>), grid, dim3(kBlock), 0, s, B, O, kdone); break;
        case 2: hipLaunchKernelGGL((k_finish<2>), grid, dim3(kBlock), 0, s, B, O, kdone); break;
        case 4: hipLaunchKernelGGL((k_finish<4>), grid, dim3(kBlock), 0, s, B, O, kdone); break;
        case 8: hipLaunchKernelGGL((k_finish<8>), grid, dim3(kBlock), 0, s, B, O, kdone); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_spmv_csr(int P, int lpr, bool f32, const CsrArgs& A, const void* ucur,
                           const void* uprev, void* w, const BatchArgs& B, int j, hipStream_t s) {
    return f32 ? launch_spmv_csr_e<float>(P, lpr, A, ucur, uprev, w, B, j, s)
               : launch_spmv_csr_e<double>(P, lpr, A, ucur, uprev, w, B, j, s);
}

hipError_t launch_spmv_stencil(int P, bool march, bool f32, const StencilArgs& A, const void* ucur,
                               const void* uprev, void* w, const BatchArgs& B, int j, hipStream_t s) {
    return f32 ? launch_stencil_e<float>(P, march, A, ucur, uprev, w, B, j, s)
               : launch_stencil_e<double>(P, march, A, ucur, uprev, w, B, j, s);
}

}  // namespace kry
