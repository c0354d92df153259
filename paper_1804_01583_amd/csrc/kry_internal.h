// Internal declarations shared by the host API (kry_api.cpp) and the gfx950
// kernels (kry_lanczos.hip, kry_expm.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kry {

constexpr int kBlock = 256;      // threads per block of the streaming kernels
constexpr int kMaxO = 8;         // output rows
constexpr int kMaxK = 64;        // Krylov dimension (eigen-solve held in LDS)
constexpr int kMaxP = 8;         // runs advanced per mat-vec launch
constexpr int kMaxNV = 40;       // values reduced per block: P * (1 + O)

// All segment sets of a plan (generators and output rows) concatenated:
// set s owns segments [set_begin[s], set_begin[s+1]), sorted and disjoint.
struct SegTable {
    const int64_t* lo;
    const int64_t* hi;
    const double* w;
    const int32_t* set_begin;
};

// Per-run scalars live in one FP64 array; run r starts at r * stride.
// Index conventions are 1-based in the iteration number j like the paper's
// algorithms:  alpha[j] = H_{j,j};  beta[0] = |start|, beta[j] = H_{j+1,j};
// sigma[j] = 1 / beta[j-1] scales the stored vector u_j to v_j = sigma[j] u_j;
// proj[q * (k + 1) + c] = (C v_{c+1})_q;  misc: k_eff, done, non-finite.
struct ScalLayout {
    int32_t k;
    int32_t o;
    int64_t stride;
    int32_t alpha;
    int32_t beta;
    int32_t sigma;
    int32_t proj;
    int32_t misc;
};
enum { MISC_KEFF = 0, MISC_DONE = 1, MISC_NONFINITE = 2, MISC_COUNT = 4 };

// One batch of runs that a mat-vec launch advances together.
struct BatchArgs {
    int64_t n;
    int64_t rows_per_block;
    int32_t nblocks;
    int32_t run0;            // first run of the batch
    double* scal;            // per-run scalar base
    ScalLayout L;
    double* partials;        // [nblocks][NV] block partial sums
    unsigned int* counter;   // arrival counter of the grid reduction (left at 0)
    const double* anorm;     // ||A||_inf on the device
    double tau_scale;        // breakdown when beta_j <= tau_scale * ||A||_inf
};

struct CsrArgs {
    const int64_t* rowptr;
    const int32_t* colidx;
    const double* vals;
};

struct StencilArgs {
    int64_t nx, ny, nz;
    double c0, cx, cy, cz;
};

// Start-vector sources of the runs in a batch.
struct StartSrc {
    const double* dense[kMaxP];  // dense n-vector (center, forcing) or null
    int32_t set[kMaxP];          // segment set of a generator, or -1
};

// Inputs of the small eigen-solve / exponential stage, one entry per run.
struct ExpmArgs {
    double* scal;
    ScalLayout L;
    const int32_t* role;     // 0 generator, 1 center, 2 augmented
    double* theta;           // [nruns][k] eigenvalues of H
    double* coef;            // [nruns][o][k] beta0 * (P Q)[q,i] * Q[0,i]
    int32_t* msize;          // [nruns] size of the tridiagonal used
};

struct AssembleArgs {
    const double* theta;
    const double* coef;
    const int32_t* msize;
    const int32_t* role;
    int32_t nruns, o, k;
    int64_t steps;
    double dt;
    double* basis;           // [(steps+1)][o][nruns]
};

struct CheckArgs {
    const double* basis;
    const double* zc;        // per run: box center (1 for fixed runs)
    const double* radius;    // per run: box radius (0 for fixed runs)
    int32_t nruns, o;
    int64_t steps;
    double ulo[kMaxO], uhi[kMaxO];
    double* verdict;         // [first_step, row, y, lo, hi, status, z[nruns]]
};

// ---- launchers (kry_lanczos.hip, kry_expm.hip) ----------------------------
hipError_t launch_fill_zero_u32(unsigned int* p, int64_t count, hipStream_t s);
hipError_t launch_row_abs_max(const CsrArgs& A, int64_t n, double* partials, int32_t nblocks,
                              int64_t rows_per_block, unsigned int* counter, double* out,
                              hipStream_t s);
hipError_t launch_start(int P, int O, const StartSrc& src, const SegTable& T, int32_t oset0,
                        double* u, const BatchArgs& B, hipStream_t s);
hipError_t launch_spmv_csr(int P, int lpr, const CsrArgs& A, const double* ucur,
                           const double* uprev, double* w, const BatchArgs& B, int j,
                           hipStream_t s);
hipError_t launch_spmv_stencil(int P, const StencilArgs& A, const double* ucur,
                               const double* uprev, double* w, const BatchArgs& B, int j,
                               hipStream_t s);
hipError_t launch_sweep(int P, int O, const SegTable& T, int32_t oset0, const double* ucur,
                        double* w, const BatchArgs& B, int j, hipStream_t s);
hipError_t launch_eig_coeffs(const ExpmArgs& E, int32_t nruns, hipStream_t s);
hipError_t launch_assemble(const AssembleArgs& A, hipStream_t s);
hipError_t launch_check(const CheckArgs& C, hipStream_t s);

}  // namespace kry
