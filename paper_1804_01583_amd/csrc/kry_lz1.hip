// The Lanczos iteration in one pass over the vectors (FP64 three-vector
// Lanczos of Algorithms 3 and 4) on gfx950.
//
// The two-launch step of kry_lanczos.hip streams six vector passes per
// iteration: the mat-vec reads u_j and u_{j-1} and writes w, the sweep reads
// u_j and w and writes w - alpha_j v_j.  Here an iteration is one launch over
// a pair buffer that holds, per row, the P entries of u_{j-1} and the P
// entries of r_j = A v_{j-1} - beta_{j-2} v_{j-2} (the mat-vec result before
// its alpha term):
//   u_j     = r_j - alpha_{j-1} sigma_{j-1} u_{j-1}     formed on the fly,
//                                                     at the row and at every
//                                                     neighbour it gathers
//   r_{j+1} = sigma_j A u_j - beta_{j-1} sigma_{j-1} u_{j-1}
// and it writes the pair (u_j, r_{j+1}): two vectors read and two written,
// four passes.  alpha_{j-1} is the sum of the previous launch's partials of
// sigma_{j-1} u_{j-1} . r_j, and |u_j|^2 follows without a pass over u_j:
//   |u_j|^2 = |r_j|^2 - alpha^2 (2 - sigma_{j-1}^2 |u_{j-1}|^2)
// (the square of r_j - alpha sigma u_{j-1} expanded with the partials of
// |r_j|^2 and |u_{j-1}|^2).  The expansion loses accuracy when the new
// direction is small against r_j (|u_j|^2 well below |r_j|^2: a Krylov space
// close to invariant, a breakdown); such a step clears the run's flag and
// the batch is computed again with the two-launch step (whose kernels take
// the flags as their stop flags, so a fallback recorded into a graph runs
// only when needed).  The vectors follow the two-launch step's formulas, so
// both produce the same vectors up to rounding (the sliced-ELL kernel sums
// A r_j and A u_{j-1} separately, so that its gathers need no coefficient).
//
// The partials of |u_j|^2 and C u_j that the finishing kernel turns into P =
// C V are formed by the launch that forms u_j (stage j - 1).  The marching
// stencil walks (y, z) columns, which do not follow the row partition of the
// output segment tables, so there a small kernel sums C u_j over the output
// segments only.  After the last iteration a tail kernel forms u_{k+1} for
// its norm and projection, as the last sweep of the two-launch step does.
#include "kry_device.h"

#include <hip/hip_ext.h>

#include <cmath>

namespace kry {

namespace {

using namespace dev;

// A double that every lane of the wave holds, moved to scalar registers.
__device__ __forceinline__ double wave_uniform(double v) {
    const uint64_t b = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// |u_j|^2 expanded below this fraction of |r_j|^2 is not trusted
constexpr double kLz1Guard = 1e-4;

// The pair (u_{j-1}, r_j) of a row.  The first step reads the start kernel's
// plain vectors ([n][P]: r_1 = the start, u_0 = 0) instead.
template <int P>
__device__ __forceinline__ void load_pair(bool first, const double* __restrict__ X, int64_t row, double (&u)[P],
                                          double (&r)[P]) {
    if (first) {
        load_row<double, P>(X, row, r);
#pragma unroll
        for (int p = 0; p < P; ++p) u[p] = 0.0;
        return;
    }
    double t[2 * P];
    load_row<double, 2 * P>(X, row, t);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        u[p] = t[p];
        r[p] = t[P + p];
    }
}

template <int P>
__device__ __forceinline__ void store_pair(double* __restrict__ X, int64_t row, const double (&u)[P],
                                           const double (&r)[P]) {
    double t[2 * P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        t[p] = u[p];
        t[P + p] = r[p];
    }
    store_row<double, 2 * P>(X, row, t);
}

// u_j from the pair (u_{j-1}, r_j): the same expression everywhere it is
// formed, so the gathered neighbours and the stored vector agree bit for bit
template <int P>
__device__ __forceinline__ void form(const double (&coef)[P], const double (&u)[P], const double (&r)[P],
                                     double (&x)[P]) {
#pragma unroll
    for (int p = 0; p < P; ++p) x[p] = fma(-coef[p], u[p], r[p]);
}

// The scalars iteration j starts from, identical in every block (partials
// summed in a fixed order).  j = 1: |u_1|^2 from the start kernel's stage-0
// partials, coef = 0.  j >= 2: D = alpha_{j-1}, R = |r_j|^2, N = |u_{j-1}|^2
// from the previous launch; coef = alpha_{j-1} sigma_{j-1} and |u_j|^2 by the
// expansion.  With `record`, block 0 records alpha_{j-1}, the stage
// (beta_{j-1}, sigma_j, k_eff) and the cancellation flag; the tail kernel
// records alpha_k only (its stage is recorded from the exact norm).
template <int P, int NTH = kBlock>
__device__ __forceinline__ void lz1_prologue(const BatchArgs& B, const Lz1Args& Z, int j, bool record, double* s_lds,
                                             double* s_tot, double* s_nrm, double (&coef)[P], double (&sig)[P],
                                             double (&cprev)[P]) {
    if (j == 1) {
        double pacc[P], sig_prev[P], anorm;
        load_stage_norms<P, NTH>(B, 1, pacc, sig_prev, anorm);
        finish_stage_norms<P, NTH>(B, 1, pacc, sig_prev, anorm, s_lds, s_nrm, sig, cprev);
#pragma unroll
        for (int p = 0; p < P; ++p) coef[p] = 0.0;
        return;
    }
    double acc[3 * P];
#pragma unroll
    for (int i = 0; i < 3 * P; ++i) acc[i] = 0.0;
    add_strided_partials<3 * P, NTH>(Z.ap_in, Z.nb_in, 0, acc);
    const double t = block_sum<3 * P, NTH>(acc, s_lds);
    if (threadIdx.x < 3 * P) s_tot[threadIdx.x] = t;
    __syncthreads();
    const double tau = B.tau_scale * *B.anorm;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const double D = s_tot[p], R = s_tot[P + p], N = s_tot[2 * P + p];
        const double sp = run_scal(B, p)[B.L.sigma + j - 1];
        double b2 = R - D * D * (2.0 - sp * sp * N);
        if (b2 < 0.0) b2 = 0.0;
        coef[p] = D * sp;
        const Stage st = stage_update_v(B.L.k, sp, tau, j, b2);
        sig[p] = st.sigma;
        cprev[p] = st.cprev;
    }
    if (blockIdx.x == 0 && threadIdx.x < P) {
        const int p = threadIdx.x;
        const double D = s_tot[p], R = s_tot[P + p], N = s_tot[2 * P + p];
        double* sc = run_scal(B, p);
        const double sp = sc[B.L.sigma + j - 1];
        sc[B.L.alpha + j - 1] = D;
        if (!isfinite(D)) sc[B.L.misc + MISC_NONFINITE] = 1.0;
        if (record) {
            double b2 = R - D * D * (2.0 - sp * sp * N);
            if (b2 < 0.0) b2 = 0.0;
            const Stage st = stage_update_v(B.L.k, sp, tau, j, b2);
            sc[B.L.beta + j - 1] = st.beta;
            sc[B.L.sigma + j] = st.sigma;
            if (st.keff >= 0) sc[B.L.misc + MISC_KEFF] = (double)st.keff;
            if (st.nonfinite) sc[B.L.misc + MISC_NONFINITE] = 1.0;
            // a live run whose new direction cancelled (a step of at most tau
            // is a breakdown whatever the rounding: |u_j| <= |r_j| <= tau)
            if (sp != 0.0 && R > tau * tau && isfinite(b2) && b2 < kLz1Guard * R) Z.flag[p] = 0.0;
        }
    }
}

// Output segments of this block (row partition) staged in LDS, as in the
// sweep: `any` is false for the (many) blocks that meet no output row.
template <int O>
__device__ __forceinline__ bool stage_outputs(SegStage<O>& st, const SegTable& T, int32_t oset0, int lb,
                                              int nblocks, SegCursor (&cur)[O]) {
    SegRange own{0, 0};
    bool any = false;
#pragma unroll
    for (int q = 0; q < O; ++q) {
        const int32_t* rq = T.blk + ((int64_t)(oset0 + q) * nblocks + lb) * 2;
        const SegRange r{rq[0], rq[1]};
        any = any || r.e > r.b;
        if ((int)threadIdx.x == q) own = r;
    }
    if (any) {
        stage_segments<O>(st, T, own);
#pragma unroll
        for (int q = 0; q < O; ++q) cur[q].init(st, q);
    }
    return any;
}

// One row of a row-partitioned launch: forms u_j, finishes r_{j+1} from the
// gathered sum, stores the pair and adds the row to the partials
// (pa: sigma_j u_j . r_{j+1}, |r_{j+1}|^2, |u_j|^2; ps: |u_j|^2, C u_j).
template <int P, int O>
__device__ __forceinline__ void lz1_row(bool first, int64_t r, const double* __restrict__ xin,
                                        double* __restrict__ xout,
                                        const double (&acc)[P], const double (&coef)[P], const double (&sig)[P],
                                        const double (&cprev)[P], bool any, SegStage<O>& st, SegCursor (&cur)[O],
                                        const SegTable& T, double (&pa)[3 * P], double (&ps)[P * (1 + O)]) {
    double up[P], rj[P], uj[P], y[P];
    load_pair<P>(first, xin, r, up, rj);
    form<P>(coef, up, rj, uj);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        ps[p] = fma(uj[p], uj[p], ps[p]);
        y[p] = fma(-cprev[p], up[p], sig[p] * acc[p]);
        pa[p] = fma(sig[p] * uj[p], y[p], pa[p]);
        pa[P + p] = fma(y[p], y[p], pa[P + p]);
        pa[2 * P + p] = fma(uj[p], uj[p], pa[2 * P + p]);
    }
    store_pair<P>(xout, r, uj, y);
    if (any) {
#pragma unroll
        for (int q = 0; q < O; ++q) {
            const double cw = cur[q].weight(st, q, T, r);
            if (cw != 0.0) {
#pragma unroll
                for (int p = 0; p < P; ++p) ps[P + q * P + p] = fma(cw, uj[p], ps[P + q * P + p]);
            }
        }
    }
}

// Block partials of a row-partitioned launch: the next iteration's
// (ap_out) and stage j - 1's (|u_j|^2, C u_j); at j = 1 the start kernel has
// written stage 0 and it is read by this launch, so it is left alone.
template <int P, int O>
__device__ __forceinline__ void lz1_store(const BatchArgs& B, const Lz1Args& Z, int j, double (&pa)[3 * P],
                                          double (&ps)[P * (1 + O)], double* s_lds) {
    store_partials<3 * P>(pa, Z.ap_out, B.nblocks, s_lds, B.xcd_map);
    if (j > 1) store_partials<P * (1 + O)>(ps, stage_part(B, j - 1), B.nblocks, s_lds, B.xcd_map);
}

constexpr int lz1_lds(int P, int O) { return (3 * P > P * (1 + O) ? 3 * P : P * (1 + O)) * (kBlock / 64); }

// Sliced-ELL mat-vec step (CSR systems), the layout and gather scheme of
// k_spmv_sell with the neighbours formed from pairs.
template <int P, int O, bool D, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_lz1_sell(SellArgs A, const double* __restrict__ xin,
                                                     double* __restrict__ xout, SegTable T, int32_t oset0,
                                                     BatchArgs B, Lz1Args Z, int j) {
    constexpr int RC = 2;
    constexpr int KU = 8;
    __shared__ double s_lds[lz1_lds(P, O)];
    __shared__ double s_tot[3 * P];
    __shared__ double s_nrm[P];
    __shared__ SegStage<O> st;
    constexpr bool first = FIRST;
    const int lb = logical_block(B.nblocks, B.xcd_map);
    const int64_t r0 = (int64_t)lb * B.rows_per_block;
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    const int lane = threadIdx.x & 63;
    const int64_t span = (int64_t)kBlock * RC;
    const int nch = (int)((B.rows_per_block + span - 1) / span);
    int64_t off_nx[RC], srow_nx[RC];
    int32_t wd_nx[RC];
    auto slice_info = [&](int ch) {
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            const int64_t r = r0 + (int64_t)ch * span + (int64_t)i * kBlock + threadIdx.x;
            const int64_t rs = r < r1 ? r : (r0 < B.n ? r0 : 0);
            const int64_t s = rs / kSlice;
            off_nx[i] = A.off[s] + lane;
            wd_nx[i] = A.width[s];
            srow_nx[i] = s * kSlice + lane;
        }
    };
    const int64_t nlast = A.n - 1;
    slice_info(0);
    SegCursor cur[O];
    const bool any = stage_outputs<O>(st, T, oset0, lb, B.nblocks, cur);
    double coef[P], sig[P], cprev[P];
    double pa[3 * P], ps[P * (1 + O)];
#pragma unroll
    for (int i = 0; i < 3 * P; ++i) pa[i] = 0.0;
#pragma unroll
    for (int i = 0; i < P * (1 + O); ++i) ps[i] = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
        int64_t rr[RC], off[RC], srow[RC];
        int32_t wd[RC];
        // the gathered sums of r_j and of u_{j-1}: A u_j = A r_j - coef A u_{j-1}
        // needs coef only at the row, so the first chunk's gathers are in
        // flight while the previous launch's partials are summed
        double acc[RC][P], accu[RC][P];
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            rr[i] = r0 + (int64_t)ch * span + (int64_t)i * kBlock + threadIdx.x;
            off[i] = off_nx[i];
            wd[i] = wd_nx[i];
            srow[i] = srow_nx[i];
#pragma unroll
            for (int p = 0; p < P; ++p) { acc[i][p] = 0.0; accu[i][p] = 0.0; }
        }
        if (ch + 1 < nch) slice_info(ch + 1);
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            for (int kb = 0; kb < wd[i]; kb += KU) {
                int32_t c[KU];
                double a[KU];
#pragma unroll
                for (int u = 0; u < KU; ++u) {
                    const int k = kb + u < wd[i] ? kb + u : wd[i] - 1;
                    const int64_t idx = off[i] + (int64_t)k * kSlice;
                    if constexpr (D) {
                        const int64_t cc = srow[i] + (int64_t)A.dcol[idx];
                        c[u] = (int32_t)min(max(cc, (int64_t)0), nlast);
                    } else {
                        c[u] = A.col[idx];
                    }
                    a[u] = kb + u < wd[i] ? A.val[idx] : 0.0;
                }
                // unconditional gathers (a slot past the width adds 0 times
                // an entry the row already reads)
#pragma unroll
                for (int u = 0; u < KU; ++u) {
                    double gu[P], gr[P];
                    load_pair<P>(first, xin, c[u], gu, gr);
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        acc[i][p] = fma(a[u], gr[p], acc[i][p]);
                        accu[i][p] = fma(a[u], gu[p], accu[i][p]);
                    }
                }
            }
        }
        if (ch == 0) lz1_prologue<P>(B, Z, j, true, s_lds, s_tot, s_nrm, coef, sig, cprev);
#pragma unroll
        for (int i = 0; i < RC; ++i) {
#pragma unroll
            for (int p = 0; p < P; ++p) acc[i][p] = fma(-coef[p], accu[i][p], acc[i][p]);
            if (rr[i] < r1)
                lz1_row<P, O>(first, rr[i], xin, xout, acc[i], coef, sig, cprev, any, st, cur, T, pa, ps);
        }
    }
    if (nch == 0) lz1_prologue<P>(B, Z, j, true, s_lds, s_tot, s_nrm, coef, sig, cprev);
    lz1_store<P, O>(B, Z, j, pa, ps, s_lds);
}

// After the last step: alpha_k, beta_k, sigma_{k+1} and k_eff from the last
// launch's partials by the same expansion as every other step (one block,
// j = k + 1), and stage k's partials written for the finishing kernel:
// |u_{k+1}|^2 in block 0, zero elsewhere (C u_{k+1} is no column of
// P = C V_k), so it records the same beta_k.  u_{k+1} itself is never formed.
template <int P>
__global__ __launch_bounds__(kBlock) void k_lz1_close(BatchArgs B, Lz1Args Z, int j) {
    __shared__ double s_lds[(kBlock / 64) * 3 * P];
    __shared__ double s_tot[3 * P];
    __shared__ double s_nrm[P];
    double coef[P], sig[P], cprev[P];
    lz1_prologue<P>(B, Z, j, true, s_lds, s_tot, s_nrm, coef, sig, cprev);
    double* part = stage_part(B, j - 1);
    const int64_t total = (int64_t)B.nvp * B.nblocks;
    for (int64_t i = threadIdx.x; i < total; i += kBlock) {
        const int v = (int)(i / B.nblocks);
        double val = 0.0;
        if (i % B.nblocks == 0 && v < P) {
            const double D = s_tot[v], R = s_tot[P + v], N = s_tot[2 * P + v];
            const double sp = run_scal(B, v)[B.L.sigma + j - 1];
            val = R - D * D * (2.0 - sp * sp * N);
            if (val < 0.0) val = 0.0;
        }
        part[i] = val;
    }
}

// Row-partitioned 7-point stencil step (grids too small for the marching
// kernel), neighbours summed in the order of k_spmv_stencil.
template <int P, int O, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_lz1_stencil(StencilArgs S, const double* __restrict__ xin,
                                                        double* __restrict__ xout, SegTable T, int32_t oset0,
                                                        BatchArgs B, Lz1Args Z, int j) {
    constexpr bool first = FIRST;
    __shared__ double s_lds[lz1_lds(P, O)];
    __shared__ double s_tot[3 * P];
    __shared__ double s_nrm[P];
    __shared__ SegStage<O> st;
    const int lb = logical_block(B.nblocks, B.xcd_map);
    const int64_t r0 = (int64_t)lb * B.rows_per_block;
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    SegCursor cur[O];
    const bool any = stage_outputs<O>(st, T, oset0, lb, B.nblocks, cur);
    double coef[P], sig[P], cprev[P];
    lz1_prologue<P>(B, Z, j, true, s_lds, s_tot, s_nrm, coef, sig, cprev);
    double pa[3 * P], ps[P * (1 + O)];
#pragma unroll
    for (int i = 0; i < 3 * P; ++i) pa[i] = 0.0;
#pragma unroll
    for (int i = 0; i < P * (1 + O); ++i) ps[i] = 0.0;
    int64_t r = r0 + threadIdx.x;
    int64_t iz = r % S.nz;
    int64_t iy = (r / S.nz) % S.ny;
    int64_t ix = r / (S.nz * S.ny);
    const int64_t sx = S.ny * S.nz, sy = S.nz;
    for (; r < r1; r += kBlock) {
        const bool xl = ix > 0, xh = ix < S.nx - 1;
        const bool yl = iy > 0, yh = iy < S.ny - 1;
        const bool zl = iz > 0, zh = iz < S.nz - 1;
        double nu[6][P], nr[6][P];
        load_pair<P>(first, xin, xl ? r - sx : r, nu[0], nr[0]);
        load_pair<P>(first, xin, yl ? r - sy : r, nu[1], nr[1]);
        load_pair<P>(first, xin, zl ? r - 1 : r, nu[2], nr[2]);
        load_pair<P>(first, xin, zh ? r + 1 : r, nu[3], nr[3]);
        load_pair<P>(first, xin, yh ? r + sy : r, nu[4], nr[4]);
        load_pair<P>(first, xin, xh ? r + sx : r, nu[5], nr[5]);
        double own_u[P], own_r[P], own[P];
        load_pair<P>(first, xin, r, own_u, own_r);
        form<P>(coef, own_u, own_r, own);
        const double diag = stencil_diag(S, xl, xh, yl, yh, zl, zh);
        double acc[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            double v[6];
#pragma unroll
            for (int t = 0; t < 6; ++t) v[t] = fma(-coef[p], nu[t][p], nr[t][p]);
            double a = 0.0;
            if (xl) a = fma(S.cx, v[0], a);
            if (yl) a = fma(S.cy, v[1], a);
            if (zl) a = fma(S.cz, v[2], a);
            a = fma(diag, own[p], a);
            if (zh) a = fma(S.cz, v[3], a);
            if (yh) a = fma(S.cy, v[4], a);
            if (xh) a = fma(S.cx, v[5], a);
            acc[p] = a;
        }
        lz1_row<P, O>(first, r, xin, xout, acc, coef, sig, cprev, any, st, cur, T, pa, ps);
        iz += kBlock;
        while (iz >= S.nz) {
            iz -= S.nz;
            if (++iy == S.ny) { iy = 0; ++ix; }
        }
    }
    lz1_store<P, O>(B, Z, j, pa, ps, s_lds);
}

// Marching one-pass stencil on (y, z) tiles.  A workgroup owns a tile of
// TY grid rows in y by kMarchOwn columns in z and walks it along x: wave w
// holds row y0 + w, lanes 1..60 its owned columns, lanes 0 and 61 the columns
// just outside (loaded, never stored; lanes 62 and 63 idle).  60 owned
// columns of pairs are whole 128-byte lines for one to eight runs, so no
// line is written by two tiles.  Each lane's pair is 2P doubles, which one
// store instruction cannot cover: written straight from the lanes, every
// instruction would fill only part of each line (on the 1000^3 system 6.6 %
// more than the pair buffer reached HBM that way).  The owned pairs are
// therefore staged in LDS and stored as consecutive 16-byte pieces, so each
// instruction writes whole contiguous lines (the buffer is then written
// once).  Per x step every wave forms its
// plane-x values, the z neighbours come from the adjacent lanes (wave
// shuffles), the y neighbours from the adjacent waves through LDS (one
// barrier per step, double-buffered), and only the tile's first and last wave
// load the row beyond the tile from memory.  The pairs of planes x - 1, x,
// x + 1 stay in registers (x + 2 loaded one step ahead, four planes rotated
// by unrolling); the outer rows of plane x + 1 are loaded during step x.  Each
// element of the pair buffer is then read from memory about once per
// iteration (rows beyond a tile twice).  Tiles are numbered y first, so the
// workgroups an XCD runs at once hold neighbouring rows of the same columns
// (2.3 % faster on the 1000^3 system than z first).
constexpr int kMarchOwn = 60;                          // z columns a wavefront owns


struct Lz1Col {
    int64_t col, sx, dout;     // dout: offset of this wave's outer row (y - 1 for wave 0, y + 1 for the last)
    int64_t base;              // the wave's first owned column at plane 0
    int nchunk;                // 16-byte pieces of the wave's owned columns (0 past the grid)
    bool own, yl, yh, zl, zh, outer;
};

// One x step.  fm: the formed value of plane x - 1 (on return, that of plane
// x); (u0, r0), (up, rp): pairs of planes x, x + 1 of this lane's column;
// (un, rn) receives plane x + 2; (ou, orr): the outer
// row's pair at plane x (first and last wave), (nou, nor) receives it at
// plane x + 1.  lds: [2][TY][64][P] formed plane values.
template <int P, bool NT, int TY, bool FIRST>
__device__ __forceinline__ void lz1_march_step(const StencilArgs& S, const Lz1Col& M, int64_t ix,
                                               const double* __restrict__ xin, double* __restrict__ xout,
                                               const double (&coef)[P], const double (&sig)[P],
                                               const double (&cprev)[P], double (&fm)[P], const double (&u0)[P],
                                               const double (&r0)[P], const double (&up)[P],
                                               const double (&rp)[P], double (&un)[P], double (&rn)[P],
                                               const double (&ou)[P], const double (&orr)[P], double (&nou)[P],
                                               double (&nor)[P], double* lds, double (&pa)[3 * P],
                                               double* stage) {
    const int64_t r = ix * M.sx + M.col;
    load_pair<P>(FIRST, xin, ix + 2 < S.nx ? r + 2 * M.sx : r, un, rn);
    if (M.outer) load_pair<P>(FIRST, xin, (ix + 1 < S.nx ? r + M.sx : r) + M.dout, nou, nor);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double x0[P];
#pragma unroll
    for (int p = 0; p < P; ++p) x0[p] = fma(-coef[p], u0[p], r0[p]);
    double* buf = lds + (ix & 1) * (TY * 64 * P);
#pragma unroll
    for (int p = 0; p < P; ++p) buf[(wave * 64 + lane) * P + p] = x0[p];
    __syncthreads();
    const double diag = stencil_diag(S, ix > 0, ix < S.nx - 1, M.yl, M.yh, M.zl, M.zh);
    double y[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const double xm = fm[p];
        const double xp = fma(-coef[p], up[p], rp[p]);
        const double vout = fma(-coef[p], ou[p], orr[p]);
        // y - 1: the wave above, or (wave 0) the outer row; y + 1 likewise
        const double vyl = wave > 0 ? buf[((wave - 1) * 64 + lane) * P + p] : vout;
        const double vyh = wave < TY - 1 ? buf[((wave + 1) * 64 + lane) * P + p] : vout;
        const double vzl = __shfl_up(x0[p], 1, 64);
        const double vzh = __shfl_down(x0[p], 1, 64);
        double acc = 0.0;
        if (ix > 0) acc = fma(S.cx, xm, acc);
        if (M.yl) acc = fma(S.cy, vyl, acc);
        if (M.zl) acc = fma(S.cz, vzl, acc);
        acc = fma(diag, x0[p], acc);
        if (M.zh) acc = fma(S.cz, vzh, acc);
        if (M.yh) acc = fma(S.cy, vyh, acc);
        if (ix < S.nx - 1) acc = fma(S.cx, xp, acc);
        y[p] = fma(-cprev[p], u0[p], sig[p] * acc);
        if (M.own) {
            pa[p] = fma(sig[p] * x0[p], y[p], pa[p]);
            pa[P + p] = fma(y[p], y[p], pa[P + p]);
            pa[2 * P + p] = fma(x0[p], x0[p], pa[2 * P + p]);
        }
    }
    {
        // the wave's owned pairs go through LDS so that every store
        // instruction writes whole contiguous lines
        double* st = stage + wave * 64 * 2 * P;
        if (M.own) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                st[(lane - 1) * 2 * P + p] = x0[p];
                st[(lane - 1) * 2 * P + P + p] = y[p];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
        typedef double v2d __attribute__((ext_vector_type(2)));
        v2d* q = reinterpret_cast<v2d*>(xout + (ix * M.sx + M.base) * 2 * P);
        constexpr int NQ = (kMarchOwn * P + 63) / 64;
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const int c = i * 64 + lane;
            if (c < M.nchunk) {
                const v2d v = *reinterpret_cast<const v2d*>(st + 2 * c);
                // non-temporal: the output stream bypasses the L2 that the
                // rows other tiles read again need (13.8 ms against 15.2 ms
                // with plain stores on the 1000^3 system, before staging)
                if constexpr (NT) __builtin_nontemporal_store(v, q + c);
                else q[c] = v;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    }
#pragma unroll
    for (int p = 0; p < P; ++p) fm[p] = x0[p];   // plane x - 1 of the next step
}

template <int P, bool NT, int TY, bool FIRST>
__global__ __launch_bounds__(TY * 64) void k_lz1_march(StencilArgs S, const double* __restrict__ xin,
                                                       double* __restrict__ xout, BatchArgs B, Lz1Args Z, int nb,
                                                       int j) {
    constexpr int NTH = TY * 64;
    __shared__ double s_lds[TY * 3 * P];
    __shared__ double s_tot[3 * P];
    __shared__ double s_nrm[P];
    __shared__ double s_plane[2 * TY * 64 * P];
    __shared__ double s_stage[TY * 64 * 2 * P];
    const int cb = logical_block(nb, B.xcd_map);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tiles_y = (int)((S.ny + TY - 1) / TY);
    const int64_t ty = cb % tiles_y, tz = cb / tiles_y;
    const int64_t iy = ty * TY + wave;
    const int64_t iz = tz * kMarchOwn + lane - 1;
    const int64_t ncol = S.ny * S.nz;
    Lz1Col M;
    M.own = lane >= 1 && lane <= kMarchOwn && iy < S.ny && iz < S.nz;
    // lanes and waves outside the grid read an in-range column and never store
    const int64_t cy = iy < S.ny ? iy : S.ny - 1;
    const int64_t cz = iz < 0 ? 0 : (iz < S.nz ? iz : S.nz - 1);
    M.col = cy * S.nz + cz;
    M.sx = ncol;
    M.yl = iy > 0;
    M.yh = iy < S.ny - 1;
    M.zl = iz > 0;
    M.zh = iz < S.nz - 1;
    M.outer = (wave == 0 && M.yl) || (wave == TY - 1 && M.yh);
    M.dout = wave == 0 ? -S.nz : S.nz;
    M.base = cy * S.nz + tz * kMarchOwn;
    M.nchunk = iy < S.ny ? (int)min((int64_t)kMarchOwn, S.nz - tz * kMarchOwn) * P : 0;
    double fm[P], ua[P], ra[P], ub[P], rb[P], uc[P], rc[P];
    double oa_u[P], oa_r[P], ob_u[P], ob_r[P];
#pragma unroll
    for (int p = 0; p < P; ++p) { oa_u[p] = 0.0; oa_r[p] = 0.0; ob_u[p] = 0.0; ob_r[p] = 0.0; fm[p] = 0.0; }
    load_pair<P>(FIRST, xin, M.col, ua, ra);
    load_pair<P>(FIRST, xin, S.nx > 1 ? M.col + M.sx : M.col, ub, rb);
    if (M.outer) load_pair<P>(FIRST, xin, M.col + M.dout, oa_u, oa_r);
    double coef[P], sig[P], cprev[P];
    lz1_prologue<P, NTH>(B, Z, j, true, s_lds, s_tot, s_nrm, coef, sig, cprev);
    // the same for every thread: keep them in scalar registers
#pragma unroll
    for (int p = 0; p < P; ++p) {
        coef[p] = wave_uniform(coef[p]);
        sig[p] = wave_uniform(sig[p]);
        cprev[p] = wave_uniform(cprev[p]);
    }
    double pa[3 * P];
#pragma unroll
    for (int i = 0; i < 3 * P; ++i) pa[i] = 0.0;
    // three pair slots rotate by unrolling: planes x, x + 1 and the x + 2 load
    for (int64_t ix = 0; ix < S.nx; ix += 3) {
        lz1_march_step<P, NT, TY, FIRST>(S, M, ix, xin, xout, coef, sig, cprev, fm, ua, ra, ub, rb, uc, rc, oa_u,
                                  oa_r, ob_u, ob_r, s_plane, pa, s_stage);
        if (ix + 1 >= S.nx) break;
        lz1_march_step<P, NT, TY, FIRST>(S, M, ix + 1, xin, xout, coef, sig, cprev, fm, ub, rb, uc, rc, ua, ra,
                                  ob_u, ob_r, oa_u, oa_r, s_plane, pa, s_stage);
        if (ix + 2 >= S.nx) break;
        lz1_march_step<P, NT, TY, FIRST>(S, M, ix + 2, xin, xout, coef, sig, cprev, fm, uc, rc, ua, ra, ub, rb,
                                  oa_u, oa_r, ob_u, ob_r, s_plane, pa, s_stage);
        // (the outer-row slots alternate with odd period: swap them for the next round)
        if (ix + 3 >= S.nx) break;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const double tu = oa_u[p], tr = oa_r[p];
            oa_u[p] = ob_u[p]; oa_r[p] = ob_r[p];
            ob_u[p] = tu; ob_r[p] = tr;
        }
    }
    store_partials<3 * P, NTH>(pa, Z.ap_out, nb, s_lds, B.xcd_map);
}

// C u_j over the output segments only (the marching step's stage j - 1
// partials; its |u_j|^2 slots are written as 0, the norm travels in the
// step's own partials).  Row partition of the segment tables: each block
// takes its segments of every output row up to kBlock at a time, clipped to
// its rows, lays their lengths out as a prefix sum in LDS and spreads the
// rows over its threads, several loads in flight per thread.
template <int P, int O>
__global__ __launch_bounds__(kBlock) void k_lz1_proj(const double* __restrict__ x, SegTable T, int32_t oset0,
                                                     BatchArgs B, int j) {
    constexpr int NV = P * (1 + O);
    constexpr int U = 8;
    __shared__ double s_lds[(kBlock / 64) * NV];
    __shared__ int64_t s_lo[kBlock];
    __shared__ int64_t s_pre[kBlock + 1];
    __shared__ double s_w[kBlock];
    const int lb = logical_block(B.nblocks, B.xcd_map);
    const int64_t r0 = (int64_t)lb * B.rows_per_block;
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
#pragma unroll
    for (int q = 0; q < O; ++q) {
        const int32_t* rq = T.blk + ((int64_t)(oset0 + q) * B.nblocks + lb) * 2;
        const int32_t gb = rq[0], ge = rq[1];
        for (int32_t g0 = gb; g0 < ge; g0 += kBlock) {
            const int32_t g = g0 + (int32_t)threadIdx.x;
            int64_t lo = 0, len = 0;
            double w = 0.0;
            if (g < ge) {
                lo = max(T.lo[g], r0);
                const int64_t hi = min(T.hi[g], r1);
                len = hi > lo ? hi - lo : 0;
                w = T.w[g];
            }
            s_lo[threadIdx.x] = lo;
            s_w[threadIdx.x] = w;
            s_pre[threadIdx.x + 1] = len;
            __syncthreads();
            if (threadIdx.x == 0) {
                s_pre[0] = 0;
                for (int t = 1; t <= kBlock; ++t) s_pre[t] += s_pre[t - 1];
            }
            __syncthreads();
            const int64_t total = s_pre[kBlock];
            for (int64_t v0 = 0; v0 < total; v0 += (int64_t)kBlock * U) {
                int64_t row[U];
                double wt[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t v = v0 + (int64_t)u * kBlock + threadIdx.x;
                    // the segment holding virtual row v: the last s with s_pre[s] <= v
                    int s = 0;
#pragma unroll
                    for (int step = kBlock / 2; step >= 1; step >>= 1)
                        if (s + step < kBlock && s_pre[s + step] <= v) s += step;
                    const bool ok = v < total;
                    row[u] = ok ? s_lo[s] + (v - s_pre[s]) : r0;
                    wt[u] = ok ? s_w[s] : 0.0;
                }
                double xv[U][2 * P];
#pragma unroll
                for (int u = 0; u < U; ++u) load_row<double, 2 * P>(x, row[u], xv[u]);
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int p = 0; p < P; ++p) acc[P + q * P + p] = fma(wt[u], xv[u][p], acc[P + q * P + p]);
                }
            }
            __syncthreads();
        }
    }
    store_partials<NV>(acc, stage_part(B, j - 1), B.nblocks, s_lds, B.xcd_map);
}

// ---- launches ---------------------------------------------------------------

template <typename K, typename... Args>
void go(K kernel, dim3 g, hipStream_t s, Args... args) {
    const ExtEvents ev = *ext_events();
    if (ev.start != nullptr) {
        hipExtLaunchKernelGGL(kernel, g, dim3(kBlock), 0, s, ev.start, ev.stop, 0, args...);
        ext_events()->start = nullptr;   // consumed
    } else {
        hipLaunchKernelGGL(kernel, g, dim3(kBlock), 0, s, args...);
    }
}

template <int P, int O>
hipError_t launch_sell_po(const SellArgs& A, const double* xin, double* xout, const SegTable& T, int32_t oset0,
                          const BatchArgs& B, const Lz1Args& Z, int j, hipStream_t s) {
    // the first step reads plain start vectors: an instantiation of its own
    if (j == 1) {
        if (A.dcol) go(k_lz1_sell<P, O, true, true>, dim3(B.nblocks), s, A, xin, xout, T, oset0, B, Z, j);
        else go(k_lz1_sell<P, O, false, true>, dim3(B.nblocks), s, A, xin, xout, T, oset0, B, Z, j);
    } else {
        if (A.dcol) go(k_lz1_sell<P, O, true, false>, dim3(B.nblocks), s, A, xin, xout, T, oset0, B, Z, j);
        else go(k_lz1_sell<P, O, false, false>, dim3(B.nblocks), s, A, xin, xout, T, oset0, B, Z, j);
    }
    return hipGetLastError();
}

template <int P, int O>
hipError_t launch_stencil_po(const StencilArgs& S, const double* xin, double* xout, const SegTable& T,
                             int32_t oset0, const BatchArgs& B, const Lz1Args& Z, int j, hipStream_t s) {
    if (j == 1) go(k_lz1_stencil<P, O, true>, dim3(B.nblocks), s, S, xin, xout, T, oset0, B, Z, j);
    else go(k_lz1_stencil<P, O, false>, dim3(B.nblocks), s, S, xin, xout, T, oset0, B, Z, j);
    return hipGetLastError();
}

template <int P, int O>
hipError_t launch_proj_po(const double* x, const SegTable& T, int32_t oset0, const BatchArgs& B, int j,
                          hipStream_t s) {
    go(k_lz1_proj<P, O>, dim3(B.nblocks), s, x, T, oset0, B, j);
    return hipGetLastError();
}

// P * (1 + O) <= kMaxNV: P = 4 with O <= 5, P = 8 with O <= 2
#define KRY_LZ1_O(FN, PP, ...)                                 \
    switch (O) {                                               \
        case 1: return FN<PP, 1>(__VA_ARGS__);                 \
        case 2: return FN<PP, 2>(__VA_ARGS__);                 \
        case 3: if (PP <= 4) return FN<PP, (PP <= 4 ? 3 : 1)>(__VA_ARGS__); break;   \
        case 4: if (PP <= 4) return FN<PP, (PP <= 4 ? 4 : 1)>(__VA_ARGS__); break;   \
        case 5: if (PP <= 4) return FN<PP, (PP <= 4 ? 5 : 1)>(__VA_ARGS__); break;   \
        case 6: if (PP <= 2) return FN<PP, (PP <= 2 ? 6 : 1)>(__VA_ARGS__); break;   \
        case 7: if (PP <= 2) return FN<PP, (PP <= 2 ? 7 : 1)>(__VA_ARGS__); break;   \
        case 8: if (PP <= 2) return FN<PP, (PP <= 2 ? 8 : 1)>(__VA_ARGS__); break;   \
        default: break;                                        \
    }                                                          \
    return hipErrorInvalidValue;
#define KRY_LZ1_PO(FN, ...)                                    \
    switch (P) {                                               \
        case 1: { KRY_LZ1_O(FN, 1, __VA_ARGS__) }              \
        case 2: { KRY_LZ1_O(FN, 2, __VA_ARGS__) }              \
        case 4: { KRY_LZ1_O(FN, 4, __VA_ARGS__) }              \
        case 8: { KRY_LZ1_O(FN, 8, __VA_ARGS__) }              \
        default: return hipErrorInvalidValue;                  \
    }

template <int P, int O>
hipError_t launch_sell_step_po(const SellArgs& A, const double* xin, double* xout, const SegTable& T, int32_t oset0,
                               const BatchArgs& B, const Lz1Args& Z, int j, hipStream_t s) {
    return launch_sell_po<P, O>(A, xin, xout, T, oset0, B, Z, j, s);
}

}  // namespace

hipError_t launch_lz1_sell(int P, int O, const SellArgs& A, const double* xin, double* xout, const SegTable& T,
                           int32_t oset0, const BatchArgs& B, const Lz1Args& Z, int j, hipStream_t s) {
    KRY_LZ1_PO(launch_sell_step_po, A, xin, xout, T, oset0, B, Z, j, s)
}

hipError_t launch_lz1_stencil(int P, int O, const StencilArgs& S, const double* xin, double* xout,
                              const SegTable& T, int32_t oset0, const BatchArgs& B, const Lz1Args& Z, int j,
                              hipStream_t s) {
    KRY_LZ1_PO(launch_stencil_po, S, xin, xout, T, oset0, B, Z, j, s)
}

static int64_t lz1_tiles_z(int64_t nz) { return (nz + kMarchOwn - 1) / kMarchOwn; }

// y rows per tile of the marching kernel (one wavefront each): 16 for up to
// two runs per launch, 4 for more (their registers leave no room for more
// wavefronts).  The rows beyond a tile are read twice, so the reads exceed
// the pair buffer by 2/TY.  Measured on the 1000^3 system with two runs:
// 14.8 ms per launch with 8 rows, 14.4 ms with 16 (13.6 ms with 16 rows and
// 60 owned columns, against 14.2 ms with 8).
static int lz1_tile_y(int P) { return P <= 2 ? 16 : 4; }

int32_t lz1_march_blocks(int64_t ny, int64_t nz, int P) {
    const int ty = lz1_tile_y(P);
    const int64_t nb = (ny + ty - 1) / ty * lz1_tiles_z(nz);
    return (int32_t)((nb + 7) / 8 * 8);
}

template <int P, bool NT, int TY, bool FIRST>
void launch_march_f(const StencilArgs& S, const double* xin, double* xout, const BatchArgs& B, const Lz1Args& Z,
                    int nb, int j, hipStream_t s) {
    const ExtEvents ev = *ext_events();
    if (ev.start != nullptr) {
        hipExtLaunchKernelGGL(k_lz1_march<P, NT, TY, FIRST>, dim3(nb), dim3(TY * 64), 0, s, ev.start, ev.stop, 0, S,
                              xin, xout, B, Z, nb, j);
        ext_events()->start = nullptr;   // consumed
    } else {
        hipLaunchKernelGGL((k_lz1_march<P, NT, TY, FIRST>), dim3(nb), dim3(TY * 64), 0, s, S, xin, xout, B, Z, nb,
                           j);
    }
}

// the first step reads plain start vectors: its own instantiation keeps the
// pair path's registers as they are
template <int P, bool NT, int TY>
void launch_march_t(const StencilArgs& S, const double* xin, double* xout, const BatchArgs& B, const Lz1Args& Z,
                    int nb, int j, hipStream_t s) {
    if (j == 1) launch_march_f<P, NT, TY, true>(S, xin, xout, B, Z, nb, j, s);
    else launch_march_f<P, NT, TY, false>(S, xin, xout, B, Z, nb, j, s);
}

hipError_t launch_lz1_march(int P, const StencilArgs& S, const double* xin, double* xout, const BatchArgs& B,
                            const Lz1Args& Z, int j, hipStream_t s, int nt) {
    const int nb = lz1_march_blocks(S.ny, S.nz, P);
    switch (P * 2 + (nt ? 1 : 0)) {
        case 3: launch_march_t<1, true, 16>(S, xin, xout, B, Z, nb, j, s); break;
        case 2: launch_march_t<1, false, 16>(S, xin, xout, B, Z, nb, j, s); break;
        case 5: launch_march_t<2, true, 16>(S, xin, xout, B, Z, nb, j, s); break;
        case 4: launch_march_t<2, false, 16>(S, xin, xout, B, Z, nb, j, s); break;
        case 9: launch_march_t<4, true, 4>(S, xin, xout, B, Z, nb, j, s); break;
        case 8: launch_march_t<4, false, 4>(S, xin, xout, B, Z, nb, j, s); break;
        case 17: launch_march_t<8, true, 4>(S, xin, xout, B, Z, nb, j, s); break;
        case 16: launch_march_t<8, false, 4>(S, xin, xout, B, Z, nb, j, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lz1_proj(int P, int O, const double* x, const SegTable& T, int32_t oset0, const BatchArgs& B,
                           int j, hipStream_t s) {
    KRY_LZ1_PO(launch_proj_po, x, T, oset0, B, j, s)
}

// (through go(): a timed launch records the events it is handed)
hipError_t launch_lz1_close(int P, const BatchArgs& B, const Lz1Args& Z, int j, hipStream_t s) {
    switch (P) {
        case 1: go(k_lz1_close<1>, dim3(1), s, B, Z, j); break;
        case 2: go(k_lz1_close<2>, dim3(1), s, B, Z, j); break;
        case 4: go(k_lz1_close<4>, dim3(1), s, B, Z, j); break;
        case 8: go(k_lz1_close<8>, dim3(1), s, B, Z, j); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace kry
