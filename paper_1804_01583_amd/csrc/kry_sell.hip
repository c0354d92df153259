// Sliced-ELL copy of a CSR matrix and the mat-vec that reads it (gfx950).
//
// Rows are grouped in slices of 64 (one wavefront).  Slice s stores its
// entries column-major: entry k of row 64 s + l sits at off[s] + 64 k + l,
// k < width[s] = the slice's longest row; shorter rows are padded with
// value 0 at their own row index.  A wavefront then reads entry k of its 64
// rows with one contiguous load (the CSR layout spreads the same load over
// 64 rows' worth of entries), needs no row-pointer loads, and issues the
// loads of 8 entries per row at once.  Each row's sum runs over its entries
// in CSR order, as in k_spmv_csr; padding adds exact zeros for finite
// vectors.
//
// The conversion runs once per plan (or once per system when prepared):
// slice widths, an exclusive scan of the slice sizes (tiles of kScanTile
// slices, then the tile totals), and a fill.  When every column lies within
// 32767 of its row (banded and stencil matrices), the fill stores column -
// row as 16 bits instead of the 32-bit column, which saves 2 of the 12
// bytes an FP64 entry streams per mat-vec.
#include "kry_device.h"

#include <hip/hip_ext.h>

#include <cmath>

namespace kry {

namespace {

using namespace dev;

constexpr int kScanTile = 4096;   // slices per scan workgroup (256 threads x 16)

// One thread per row, one wavefront per slice: the slice width is the
// wavefront's largest row, and the slice is wide when any of its rows has a
// column farther than 32767 from the row.
__global__ __launch_bounds__(256) void k_sell_width(const int64_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ colidx, int64_t n, int64_t ns,
                                                    int32_t* __restrict__ width,
                                                    unsigned long long* __restrict__ nwide) {
    const int64_t rows = ns * kSlice;
    for (int64_t b0 = (int64_t)blockIdx.x * 256; b0 < rows; b0 += (int64_t)gridDim.x * 256) {
        const int64_t r = b0 + threadIdx.x;    // rows is a multiple of 64, so a wavefront is all in or all out
        if (r >= rows) continue;
        int64_t w = 0;
        bool wide = false;
        if (r < n) {
            const int64_t e0 = rowptr[r], e1 = rowptr[r + 1];
            w = e1 - e0;
            for (int64_t e = e0; e < e1; ++e) {
                const int64_t d = (int64_t)colidx[e] - r;
                wide = wide || d < -32768 || d > 32767;
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) w = max(w, (int64_t)__shfl_xor(w, off, 64));
        const bool any_wide = __any(wide);
        if ((threadIdx.x & 63) == 0) {
            width[r / kSlice] = (int32_t)w;
            if (any_wide) atomicAdd(nwide, 1ull);
        }
    }
}

// exclusive scan of 64 * width within tiles; tile totals to `tiles`
__global__ __launch_bounds__(256) void k_sell_scan_tiles(const int32_t* __restrict__ width, int64_t ns,
                                                         int64_t* __restrict__ off, int64_t* __restrict__ tiles) {
    __shared__ int64_t s_sum[256];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * (kScanTile / 256);
    int64_t local = 0;
    for (int i = 0; i < kScanTile / 256; ++i) {
        const int64_t s = base + i;
        if (s < ns) local += (int64_t)kSlice * width[s];
    }
    s_sum[threadIdx.x] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int t = 0; t < 256; ++t) {
            const int64_t v = s_sum[t];
            s_sum[t] = run;
            run += v;
        }
        tiles[blockIdx.x] = run;
    }
    __syncthreads();
    int64_t run = s_sum[threadIdx.x];
    for (int i = 0; i < kScanTile / 256; ++i) {
        const int64_t s = base + i;
        if (s < ns) {
            off[s] = run;
            run += (int64_t)kSlice * width[s];
        }
    }
}

// adds the exclusive prefix of the tile totals (one thread walks them) and
// writes off[ns] = total
__global__ __launch_bounds__(256) void k_sell_scan_add(int64_t* __restrict__ off, int64_t ns,
                                                       const int64_t* __restrict__ tiles, int64_t ntiles) {
    __shared__ int64_t s_pre;
    const int64_t tile = blockIdx.x;
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int64_t t = 0; t < tile; ++t) run += tiles[t];
        s_pre = run;
        if (tile == ntiles - 1) off[ns] = run + tiles[tile];
    }
    __syncthreads();
    const int64_t pre = s_pre;
    for (int64_t i = threadIdx.x; i < kScanTile; i += 256) {
        const int64_t s = tile * kScanTile + i;
        if (s < ns) off[s] += pre;
    }
}

template <typename V, typename IT>
__global__ __launch_bounds__(256) void k_sell_fill(CsrArgs A, int64_t n, int64_t ns, const int64_t* __restrict__ off,
                                                   const int32_t* __restrict__ width, IT* __restrict__ col,
                                                   V* __restrict__ val) {
    const int64_t rows = ns * kSlice;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < rows; r += (int64_t)gridDim.x * 256) {
        const int64_t s = r / kSlice, l = r % kSlice;
        const int32_t w = width[s];
        const int64_t base = off[s] + l;
        int64_t e0 = 0, len = 0;
        if (r < n) {
            e0 = A.rowptr[r];
            len = A.rowptr[r + 1] - e0;
        }
        for (int32_t k = 0; k < w; ++k) {
            const bool real = k < len;
            if constexpr (sizeof(IT) == 2)   // column - row; padding points at the row itself
                col[base + (int64_t)k * kSlice] = real ? (IT)((int64_t)A.colidx[e0 + k] - r) : (IT)0;
            else
                col[base + (int64_t)k * kSlice] = real ? A.colidx[e0 + k] : (int32_t)(r < n ? r : 0);
            val[base + (int64_t)k * kSlice] = real ? (V)A.vals[e0 + k] : (V)0;
        }
    }
}

// a3 + first half of a4 on the sliced-ELL copy: w = sigma_j A u_j -
// beta_{j-1} sigma_{j-1} u_{j-1} (or without the second term), partials of
// (sigma_j u_j) . w.  Rows in chunks of RC per thread; entries of a row in
// groups of KU whose loads are issued together (slots past the slice width
// re-read the last entry and add nothing).
template <typename E, int P, bool D>
__global__ __launch_bounds__(kBlock) void k_spmv_sell(SellArgs A, const E* __restrict__ ucur,
                                                      const E* __restrict__ uprev, E* __restrict__ w, BatchArgs B,
                                                      int j) {
    if (batch_stopped<P>(B)) return;   // the batch met its error target
    constexpr int RC = 2;
    constexpr int KU = 8;
    __shared__ double s_lds[(kBlock / 64) * P];
    __shared__ double s_nrm[P];
    const int lb = logical_block(B.nblocks, B.xcd_map);
    const int64_t r0 = (int64_t)lb * B.rows_per_block;
    const int64_t r1 = min(B.n, r0 + B.rows_per_block);
    const int lane = threadIdx.x & 63;
    const int64_t span = (int64_t)kBlock * RC;
    const int nch = (int)((B.rows_per_block + span - 1) / span);
    // slice offset and width of a chunk's rows; a wavefront's 64 rows are one
    // slice, rows past the block (or n) read slice 0 and are not stored.
    // Each chunk's are requested one chunk ahead (the first ones before the
    // norm partials), so no chunk starts with a round trip of its own.
    // (delta mode) the row whose entries a thread reads is 64 s + lane
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
    double pacc[P], sig_prev[P], anorm;
    load_stage_norms<P>(B, j, pacc, sig_prev, anorm);
    double sig[P], cprev[P], dot[P];
#pragma unroll
    for (int p = 0; p < P; ++p) { sig[p] = 0.0; cprev[p] = 0.0; dot[p] = 0.0; }
    const bool prev = j > 1 && uprev != nullptr;
    for (int ch = 0; ch < nch; ++ch) {
        int64_t rr[RC], off[RC], srow[RC];
        int32_t wd[RC];
        double acc[RC][P];
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            rr[i] = r0 + (int64_t)ch * span + (int64_t)i * kBlock + threadIdx.x;
            off[i] = off_nx[i];
            wd[i] = wd_nx[i];
            srow[i] = srow_nx[i];
#pragma unroll
            for (int p = 0; p < P; ++p) acc[i][p] = 0.0;
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
                        // rows past n in the last slice hold delta 0: clamp to a real row
                        const int64_t cc = srow[i] + (int64_t)A.dcol[idx];
                        c[u] = (int32_t)min(max(cc, (int64_t)0), nlast);
                    } else {
                        c[u] = A.col[idx];
                    }
                    const double v = sizeof(E) == 4 ? (double)A.val32[idx] : A.val[idx];
                    a[u] = kb + u < wd[i] ? v : 0.0;
                }
                // unconditional: a slot past the width adds 0 * (an entry the
                // row already reads); a conditional use lets the compiler move
                // each gather behind a branch of its own and wait for it there
#pragma unroll
                for (int u = 0; u < KU; ++u) {
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const double x = (double)ucur[(int64_t)c[u] * P + p];
                        acc[i][p] = fma(a[u], x, acc[i][p]);
                    }
                }
            }
        }
        if (ch == 0) finish_stage_norms<P>(B, j, pacc, sig_prev, anorm, s_lds, s_nrm, sig, cprev);
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            if (rr[i] < r1) {
                const int64_t r = rr[i];
                double own[P], pv[P], y[P];
                load_row<E, P>(ucur, r, own);
                if (prev) load_row<E, P>(uprev, r, pv);
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    y[p] = sig[p] * acc[i][p];
                    if (prev) y[p] = fma(-cprev[p], pv[p], y[p]);
                    y[p] = (double)(E)y[p];
                    dot[p] = fma(sig[p] * own[p], y[p], dot[p]);
                }
                store_row<E, P>(w, r, y);
            }
        }
    }
    if (nch == 0) finish_stage_norms<P>(B, j, pacc, sig_prev, anorm, s_lds, s_nrm, sig, cprev);
    store_partials<P>(dot, B.ap_part, B.ap_nblocks, s_lds, B.xcd_map);
}

int grid_for(int64_t count) { return (int)std::min<int64_t>((count + 255) / 256, 4096); }

}  // namespace

int64_t sell_slices(int64_t n) { return (n + kSlice - 1) / kSlice; }
int64_t sell_scan_tiles(int64_t n) { return (sell_slices(n) + kScanTile - 1) / kScanTile; }

hipError_t launch_sell_layout(const CsrArgs& A, int64_t n, int32_t* width, int64_t* off, int64_t* tiles,
                              hipStream_t s) {
    const int64_t ns = sell_slices(n), nt = sell_scan_tiles(n);
    // the count of wide slices sits after the nt tile totals
    hipError_t e = launch_fill(reinterpret_cast<double*>(tiles + nt), 1, 0.0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sell_width, dim3(grid_for(ns * kSlice)), dim3(256), 0, s, A.rowptr, A.colidx, n, ns, width,
                       reinterpret_cast<unsigned long long*>(tiles + nt));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sell_scan_tiles, dim3((unsigned)nt), dim3(256), 0, s, width, ns, off, tiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sell_scan_add, dim3((unsigned)nt), dim3(256), 0, s, off, ns, tiles, nt);
    return hipGetLastError();
}

hipError_t launch_sell_fill(bool f32, bool narrow, const CsrArgs& A, int64_t n, const int64_t* off,
                            const int32_t* width, void* col, void* val, hipStream_t s) {
    const int64_t ns = sell_slices(n);
    const dim3 g(grid_for(ns * kSlice)), b(256);
    int16_t* c16 = static_cast<int16_t*>(col);
    int32_t* c32 = static_cast<int32_t*>(col);
    float* v32 = static_cast<float*>(val);
    double* v64 = static_cast<double*>(val);
    if (f32 && narrow) hipLaunchKernelGGL((k_sell_fill<float, int16_t>), g, b, 0, s, A, n, ns, off, width, c16, v32);
    else if (f32) hipLaunchKernelGGL((k_sell_fill<float, int32_t>), g, b, 0, s, A, n, ns, off, width, c32, v32);
    else if (narrow) hipLaunchKernelGGL((k_sell_fill<double, int16_t>), g, b, 0, s, A, n, ns, off, width, c16, v64);
    else hipLaunchKernelGGL((k_sell_fill<double, int32_t>), g, b, 0, s, A, n, ns, off, width, c32, v64);
    return hipGetLastError();
}

template <typename E, bool D>
hipError_t launch_spmv_sell_ed(int P, const SellArgs& A, const void* ucur, const void* uprev, void* w,
                               const BatchArgs& B, int j, hipStream_t s) {
    const E* uc = static_cast<const E*>(ucur);
    const E* up = static_cast<const E*>(uprev);
    E* ww = static_cast<E*>(w);
    const dim3 g(B.nblocks), b(kBlock);
    const ExtEvents ev = *ext_events();
    auto go = [&](auto kernel) {
        if (ev.start != nullptr) {
            hipExtLaunchKernelGGL(kernel, g, b, 0, s, ev.start, ev.stop, 0, A, uc, up, ww, B, j);
            ext_events()->start = nullptr;   // consumed
        } else {
            hipLaunchKernelGGL(kernel, g, b, 0, s, A, uc, up, ww, B, j);
        }
    };
    switch (P) {
        case 1: go(k_spmv_sell<E, 1, D>); break;
        case 2: go(k_spmv_sell<E, 2, D>); break;
        case 4: go(k_spmv_sell<E, 4, D>); break;
        case 8: go(k_spmv_sell<E, 8, D>); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename E>
hipError_t launch_spmv_sell_e(int P, const SellArgs& A, const void* ucur, const void* uprev, void* w,
                              const BatchArgs& B, int j, hipStream_t s) {
    return A.dcol ? launch_spmv_sell_ed<E, true>(P, A, ucur, uprev, w, B, j, s)
                  : launch_spmv_sell_ed<E, false>(P, A, ucur, uprev, w, B, j, s);
}

hipError_t launch_spmv_sell(int P, bool f32, const SellArgs& A, const void* ucur, const void* uprev, void* w,
                            const BatchArgs& B, int j, hipStream_t s) {
    return f32 ? launch_spmv_sell_e<float>(P, A, ucur, uprev, w, B, j, s)
               : launch_spmv_sell_e<double>(P, A, ucur, uprev, w, B, j, s);
}

}  // namespace kry
