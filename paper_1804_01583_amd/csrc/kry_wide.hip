// The transposed route with many initial-space rows (paper Section 4.1: one
// simulation of A^T per output row instead of one per column of E, which
// pays when E has far more columns than C has rows).  The Krylov runs are the
// usual ones; what changes is the projection on the rows of E^T and the
// small stage, which no longer fit the fused per-block projection (at most 8
// rows) and the per-run LDS chains.
//
// Projection: after each Krylov vector u_{j+1} is formed, every segment of
// the initial-space rows is summed by one wavefront (k_wseg, into the
// step's slice of the segment sums); after the batch's last step one launch
// adds the segments of each row in their order for every step (k_wset):
// Pw[run][c][j] = E_c^T u_{j+1}, unscaled (v_{j+1} = sigma_{j+1} u_{j+1}).
//
// Small stage, per run (as the oracle states it): the matrix
//     M = H                          (no forcing), or
//     M = [[H, 0], [p_b^T, 0]]       (forcing: p_b = b's row of E^T V, size m + 1)
// is exponentiated once, Phi = e^{M dt} (Taylor polynomial and squarings in
// LDS), and x_s = e^{M s dt} x0 with x0 = (beta0 e_1; 0) is formed for every
// step from anchors: s = b B + r, x_s = Phi^r a_b, a_b = Phi^{B b} x0
// (k_wide_stage writes Phi^r, r < B, and the anchors).  k_wide_vals then
// forms basis[s][q][c] = sum_j sigma_{j+1} Pw[q][c][j] x_s[j] for the
// generator and center rows, and x_s[m] for the forcing column.
#include "kry_device.h"
#include "kry_ldsmm.h"

#include <cmath>

namespace kry {

namespace {

using namespace dev;
using ldsmm::kLd;
using ldsmm::kSlot;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// segsum[(g - g0) P + p] = w_g sum_{r in [lo_g, hi_g)} x[r][p] for the ng
// segments g0.. of the wide rows (x: the batch's [n][P] vectors).
template <typename E, int P>
__global__ __launch_bounds__(kBlock) void k_wseg(const E* __restrict__ x, SegTable T, int32_t g0, int32_t ng,
                                                 double* __restrict__ segsum) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t gi = wave; gi < ng; gi += nwaves) {
        const int64_t g = g0 + gi;
        const int64_t lo = T.lo[g], hi = T.hi[g];
        double acc[P];
#pragma unroll
        for (int p = 0; p < P; ++p) acc[p] = 0.0;
        for (int64_t r = lo + lane; r < hi; r += 64) {
            double v[P];
            load_row<E, P>(x, r, v);
#pragma unroll
            for (int p = 0; p < P; ++p) acc[p] += v[p];
        }
        const double wg = T.w[g];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const double t = wave_sum(acc[p]);
            if (lane == 0) segsum[gi * P + p] = wg * t;
        }
    }
}

// Pw[(run0 + p) ncw + c][j] = the segments of row c added in order, for
// every step j < kdone of the batch at once (segsum: [kdone][ng][P]); one
// thread per (row, step, run), nreal runs of the batch real.
template <int P>
__global__ __launch_bounds__(kBlock) void k_wset(SegTable T, int32_t set0, int32_t nsets, int32_t g0, int32_t ng,
                                                 const double* __restrict__ segsum, double* __restrict__ Pw,
                                                 int32_t run0, int32_t nreal, int32_t ncw, int32_t ldk, int32_t kdone) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)nsets * kdone * P) return;
    const int p = (int)(t % P);
    const int j = (int)((t / P) % kdone);
    const int c = (int)(t / ((int64_t)P * kdone));
    if (p >= nreal) return;
    const int32_t s = set0 + c;
    const double* sj = segsum + (int64_t)j * ng * P;
    double acc = 0.0;
    for (int32_t g = T.set_begin[s]; g < T.set_begin[s + 1]; ++g) acc += sj[(int64_t)(g - g0) * P + p];
    Pw[((int64_t)(run0 + p) * ncw + c) * ldk + j] = acc;
}

__device__ __forceinline__ const double* run_sc(const WideArgs& W, int run) {
    return W.scal + (int64_t)run * W.L.stride;
}

// Size of run's matrix M (0: the run contributes nothing) and whether the
// run's data are finite.
__device__ __forceinline__ int wide_size(const WideArgs& W, const double* sc, int* m_out) {
    int m = (int)sc[W.L.misc + MISC_KEFF];
    if (m > W.L.k) m = W.L.k;
    if (m < 0) m = 0;
    *m_out = m;
    return m == 0 ? 0 : m + (W.forcing ? 1 : 0);
}

// One workgroup per run: Phi = e^{M dt}, its powers Phi^r (r < B) to
// W.pow[run][r], anchors a_b = (Phi^B)^b x0 (b < nanch) to W.anch[run][b].
__global__ __launch_bounds__(kExpmThreads) void k_wide_stage(WideArgs W) {
    extern __shared__ double lds[];
    __shared__ double s_red[kExpmThreads / 64];
    __shared__ double s_vec[2][kMaxK + 1];
    const int run = blockIdx.x;
    const double* sc = run_sc(W, run);
    int m;
    const int ms = wide_size(W, sc, &m);
    if (ms == 0) return;
    const int mm = ms + (ms & 1);
    const int k = W.L.k;
    const int tid = threadIdx.x;
    const double* pw = W.Pw + (int64_t)run * W.ncw * W.ldk;
    // X = M dt, zero padded to mm
    for (int idx = tid; idx < mm * mm; idx += blockDim.x) {
        const int a = idx / mm, b = idx % mm;
        double h = 0.0;
        if (a < m && b < m) {
            if (W.hess) {
                if (a <= b) h = sc[W.L.hess + a * k + b];
                else if (a == b + 1) h = sc[W.L.beta + b + 1];
            } else {
                if (a == b) h = sc[W.L.alpha + a + 1];
                else if (b == a + 1) h = sc[W.L.beta + a + 1];
                else if (a == b + 1) h = sc[W.L.beta + b + 1];
            }
        } else if (W.forcing && a == m && b < m) {
            h = sc[W.L.sigma + b + 1] * pw[(int64_t)W.bcol * W.ldk + b];   // p_b^T
        }
        lds[a * kLd + b] = h * W.dt;
    }
    __syncthreads();
    const double nrm = ldsmm::norm1_slot0(lds, mm, s_red);
    int sq = 0;
    while (isfinite(nrm) && nrm > ldexp(1.0, sq) && sq < 1100) ++sq;
    const double shrink = ldexp(1.0, -sq);
    for (int idx = tid; idx < mm * mm; idx += blockDim.x) {
        const int a = idx / mm, b = idx % mm;
        lds[a * kLd + b] *= shrink;
    }
    __syncthreads();
    ldsmm::taylor18(lds, mm, 1.0);
    auto none = [](int, int) { return 0.0; };
    int phi = 4;
    for (int i = 0; i < sq; ++i) {
        ldsmm::mm_mfma(lds, phi, phi, 9 - phi, mm, none);
        phi = 9 - phi;
    }
    // powers Phi^r, r < B: r = 0 is I, r = 1 is Phi, then Phi^{r-1} Phi,
    // ping-ponging between slots 1 and 2; cur ends as Phi^B
    double* pw_out = W.pow + (int64_t)run * W.B * kMaxK1 * kMaxK1;
    for (int idx = tid; idx < ms * ms; idx += blockDim.x) {
        const int a = idx / ms, b = idx % ms;
        pw_out[a * kMaxK1 + b] = a == b ? 1.0 : 0.0;
    }
    int cur = phi;
    for (int r = 1; r < W.B; ++r) {
        double* dst = pw_out + (int64_t)r * kMaxK1 * kMaxK1;
        for (int idx = tid; idx < ms * ms; idx += blockDim.x) {
            const int a = idx / ms, b = idx % ms;
            dst[a * kMaxK1 + b] = lds[cur * kSlot + a * kLd + b];
        }
        const int nxt = cur == 1 ? 2 : 1;
        ldsmm::mm_mfma(lds, cur, phi, nxt, mm, none);
        cur = nxt;
    }
    if (W.B == 1) cur = phi;   // Phi^B = Phi
    // anchors: a_0 = x0, a_{b+1} = Phi^B a_b
    const double beta0 = sc[W.L.beta + 0];
    double* an = W.anch + (int64_t)run * W.nanch * kMaxK1;
    if (tid < ms) {
        const double v = tid == 0 ? beta0 : 0.0;
        s_vec[0][tid] = v;
        an[tid] = v;
    }
    __syncthreads();
    for (int b = 1; b < W.nanch; ++b) {
        const int src = (b - 1) & 1, dst = b & 1;
        if (tid < ms) {
            double acc = 0.0;
            for (int l = 0; l < ms; ++l) acc = fma(lds[cur * kSlot + tid * kLd + l], s_vec[src][l], acc);
            s_vec[dst][tid] = acc;
            an[(int64_t)b * kMaxK1 + tid] = acc;
        }
        __syncthreads();
    }
}

// basis[s][q][c] for every step s (blockIdx.x) and run q (blockIdx.y):
// x_s = Phi^r a_b in LDS, then one thread per basis column.
__global__ __launch_bounds__(kBlock) void k_wide_vals(WideArgs W) {
    __shared__ double s_x[kMaxK1];
    __shared__ double s_sig[kMaxK1];
    const int64_t s = blockIdx.x;
    const int run = blockIdx.y;
    const double* sc = run_sc(W, run);
    int m;
    const int ms = wide_size(W, sc, &m);
    const bool bad = sc[W.L.misc + MISC_NONFINITE] != 0.0;
    const int tid = threadIdx.x;
    if (ms > 0) {
        const int r = (int)(s % W.B), b = (int)(s / W.B);
        const double* Pr = W.pow + ((int64_t)run * W.B + r) * kMaxK1 * kMaxK1;
        const double* ab = W.anch + ((int64_t)run * W.nanch + b) * kMaxK1;
        if (tid < ms) {
            double acc = 0.0;
            for (int l = 0; l < ms; ++l) acc = fma(Pr[tid * kMaxK1 + l], ab[l], acc);
            s_x[tid] = acc;
        }
        if (tid < m) s_sig[tid] = sc[W.L.sigma + tid + 1];
    }
    __syncthreads();
    const double* pw = W.Pw + (int64_t)run * W.ncw * W.ldk;
    double* out = W.basis + (s * W.o_out + run) * W.ncols;
    for (int c = tid; c < W.ncols; c += kBlock) {
        double v = 0.0;
        if (ms > 0) {
            if (W.forcing && c == W.bcol) {
                v = s_x[m];
            } else {
                for (int j = 0; j < m; ++j) v = fma(s_sig[j] * pw[(int64_t)c * W.ldk + j], s_x[j], v);
            }
        }
        out[c] = bad ? __builtin_nan("") : v;
    }
}

}  // namespace

size_t wide_stage_lds_bytes() { return (size_t)6 * kSlot * sizeof(double); }

hipError_t wide_prepare() {
    return hipFuncSetAttribute((const void*)k_wide_stage, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)wide_stage_lds_bytes());
}

template <typename E>
static hipError_t launch_wseg_e(int P, const void* x, const SegTable& T, int32_t g0, int32_t ng, double* segsum,
                                hipStream_t s) {
    const int wb = (int)std::min<int64_t>(4096, ((int64_t)ng + kBlock / 64 - 1) / (kBlock / 64));
    const E* xe = static_cast<const E*>(x);
    switch (P) {
        case 1: hipLaunchKernelGGL((k_wseg<E, 1>), dim3(wb), dim3(kBlock), 0, s, xe, T, g0, ng, segsum); break;
        case 2: hipLaunchKernelGGL((k_wseg<E, 2>), dim3(wb), dim3(kBlock), 0, s, xe, T, g0, ng, segsum); break;
        case 4: hipLaunchKernelGGL((k_wseg<E, 4>), dim3(wb), dim3(kBlock), 0, s, xe, T, g0, ng, segsum); break;
        case 8: hipLaunchKernelGGL((k_wseg<E, 8>), dim3(wb), dim3(kBlock), 0, s, xe, T, g0, ng, segsum); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_wide_proj(int P, bool f32, const void* x, const SegTable& T, int32_t g0, int32_t ng,
                            double* segsum, int32_t j, hipStream_t s) {
    if (ng <= 0) return hipSuccess;
    double* sj = segsum + (int64_t)j * ng * P;
    return f32 ? launch_wseg_e<float>(P, x, T, g0, ng, sj, s) : launch_wseg_e<double>(P, x, T, g0, ng, sj, s);
}

hipError_t launch_wide_sets(int P, const SegTable& T, int32_t set0, int32_t nsets, int32_t g0, int32_t ng,
                            const double* segsum, double* Pw, int32_t run0, int32_t nreal, int32_t ncw, int32_t ldk,
                            int32_t kdone, hipStream_t s) {
    if (nsets <= 0 || kdone <= 0) return hipSuccess;
    const int64_t total = (int64_t)nsets * kdone * P;
    const unsigned sb = (unsigned)((total + kBlock - 1) / kBlock);
    switch (P) {
        case 1: hipLaunchKernelGGL((k_wset<1>), dim3(sb), dim3(kBlock), 0, s, T, set0, nsets, g0, ng, segsum, Pw, run0, nreal, ncw, ldk, kdone); break;
        case 2: hipLaunchKernelGGL((k_wset<2>), dim3(sb), dim3(kBlock), 0, s, T, set0, nsets, g0, ng, segsum, Pw, run0, nreal, ncw, ldk, kdone); break;
        case 4: hipLaunchKernelGGL((k_wset<4>), dim3(sb), dim3(kBlock), 0, s, T, set0, nsets, g0, ng, segsum, Pw, run0, nreal, ncw, ldk, kdone); break;
        case 8: hipLaunchKernelGGL((k_wset<8>), dim3(sb), dim3(kBlock), 0, s, T, set0, nsets, g0, ng, segsum, Pw, run0, nreal, ncw, ldk, kdone); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_wide_stage(const WideArgs& W, int32_t nruns, int64_t steps, hipStream_t s) {
    if (nruns <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wide_stage, dim3(nruns), dim3(kExpmThreads), wide_stage_lds_bytes(), s, W);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wide_vals, dim3((unsigned)(steps + 1), nruns), dim3(kBlock), 0, s, W);
    return hipGetLastError();
}

}  // namespace kry
