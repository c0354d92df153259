// Internal declarations shared by the host API (kry_api.cpp) and the gfx950
// kernels (kry_lanczos.hip, kry_expm.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include <cstdint>

namespace kry {

constexpr int kBlock = 256;      // threads per block of the streaming kernels
constexpr int kMaxO = 8;         // output rows
constexpr int kMaxK = 56;        // Krylov dimension of the one-workgroup LDS exponential
constexpr int kMaxKD = 512;      // Krylov dimension with the dense stage (k > kMaxK)
constexpr int kMaxKP = 8192;     // Krylov dimension of three-vector (plain) Lanczos
constexpr int kMaxKE = 2048;     // Krylov dimension the error control's eigen-solve holds in LDS
constexpr int kExpmThreads = 576;
constexpr int kMaxP = 8;         // runs advanced per mat-vec launch
constexpr int kMaxNV = 24;       // values reduced per block: P * (1 + O)

// All segment sets of a plan (generators and output rows) concatenated:
// set s owns segments [set_begin[s], set_begin[s+1]), sorted and disjoint.
struct SegTable {
    const int64_t* lo;
    const int64_t* hi;
    const double* w;
    const int32_t* set_begin;
    const int32_t* blk;      // [nsets][nblocks][2]: segments of set s overlapping logical block b
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
    int32_t hess;    // Arnoldi: H[i][c] at hess + i * k + c, i <= k, c < k
};
// misc: k_eff (breakdown), done, non-finite, k_stop (error control; k when
// off), the last error bound, stopped (error target met)
enum { MISC_KEFF = 0, MISC_DONE = 1, MISC_NONFINITE = 2, MISC_KSTOP = 3, MISC_BOUND = 4, MISC_STOPPED = 5,
       MISC_COUNT = 6 };

// One batch of runs that a mat-vec launch advances together.
//
// Grid-wide sums never cross blocks inside a kernel: each block writes one
// partial per value, and every block of the next kernel sums those partials
// itself, in the same fixed order, so all blocks hold bit-identical totals.
// Only kernel boundaries order memory between blocks (no device-scope
// fences, which on a multi-XCD part write back and invalidate L2).
struct BatchArgs {
    int64_t n;
    int64_t rows_per_block;
    int32_t nblocks;
    int32_t xcd_map;         // 1: contiguous row ranges per XCD (see logical_block)
    int32_t run0;            // first run of the batch
    double* scal;            // per-run scalar base
    ScalLayout L;
    double* np_part;         // [k+1 stages][nvp][nblocks]: |u_j|^2 per run, then (C u_j)_q per run
    int32_t nvp;             // values per stage in np_part (>= P * (1 + o))
    double* ap_part;         // [kMaxP][ap_nblocks]:  v_j . w per run
    int32_t ap_nblocks;      // blocks of the mat-vec launch (its own partition for the marching stencil)
    const double* anorm;     // ||A||_inf on the device
    double tau_scale;        // breakdown when beta_j <= tau_scale * ||A||_inf
    const double* stop;      // error control: [P] nonzero once run p met its target; null: fixed k
};

struct CsrArgs {
    const int64_t* rowptr;
    const int32_t* colidx;
    const double* vals;
    const float* vals32;     // FP32 copy of vals, read by the FP32-basis kernels
};

// Sliced-ELL copy of a CSR matrix (kry_sell.hip): slices of kSlice rows,
// entries column-major within a slice, padded to the slice's longest row.
constexpr int kSlice = 64;
struct SellArgs {
    const int64_t* off;      // [slices + 1] first entry of each slice
    const int32_t* width;    // [slices] entries per row in the slice
    const int32_t* col;      // column indices, or (col null)
    const double* val;       // FP64 values, or
    const float* val32;      // FP32 values (FP32-basis mode)
    const int16_t* dcol;     // column - row of every entry, when all of them fit 16 bits
    int64_t n;               // rows (delta mode clamps reconstructed columns to n - 1)
};
int64_t sell_slices(int64_t n);
// scan tiles of the layout, plus one more int64 after them: the number of
// slices with a column farther than 32767 from its row
int64_t sell_scan_tiles(int64_t n);
struct CsrArgs;
hipError_t launch_sell_layout(const CsrArgs& A, int64_t n, int32_t* width, int64_t* off, int64_t* tiles,
                              hipStream_t s);
// narrow: store column - row as int16 (col then points to int16 storage)
hipError_t launch_sell_fill(bool f32, bool narrow, const CsrArgs& A, int64_t n, const int64_t* off,
                            const int32_t* width, void* col, void* val, hipStream_t s);

struct StencilArgs {
    int64_t nx, ny, nz;
    double c0, cx, cy, cz;
    int32_t insulated;       // 1: faces without flux (missing neighbours leave the diagonal)
    double ex;               // added to the diagonal on the face ix = nx - 1
};

// Start-vector sources of the runs in a batch.
struct StartSrc {
    const double* dense[kMaxP];  // dense n-vector (center, forcing) or null
    int32_t set[kMaxP];          // segment set of a generator, or -1
};

// Inputs of the small exponential stage, one workgroup per run.
struct ExpmArgs {
    const double* scal;
    ScalLayout L;
    const int32_t* role;     // per job: 0 generator or center, 2 augmented (k - 1 steps of T),
                             // 3 transposed forcing column (bordered with the whole of T)
    const int32_t* job_run;  // per job: the Krylov run it exponentiates (null: job j is run j)
    double dt;
    int32_t hess_mode;       // 0: tridiagonal from alpha/beta (Lanczos); 1: Hessenberg (Arnoldi)
    int32_t B;               // anchor spacing (power of two)
    int32_t nanch;           // anchors per run: ceil((steps + 1) / B)
    double* Z;               // [njobs][B][kMaxO][kMaxK]  P Phi^r
    double* anch;            // [njobs][nanch][kMaxK]     Psi^b e_1
    int32_t* msize;          // [njobs] size of H used (0: the job contributes 0)
    double* scale;           // [njobs] beta0, or 1 for a bordered job
};

struct AssembleArgs {
    const double* Z;
    const double* anch;
    const int32_t* msize;
    const double* scale;
    int32_t nruns, o, B, nanch;   // nruns: jobs
    int64_t steps;
    double* basis;           // [(steps+1)][o][nruns], or [(steps+1)][o_out][ncols] with an output map
    const int32_t* job_run;  // output map (null: none): job -> output row of the basis
    const int32_t* out_col;  // [njobs][kMaxO]: projection row -> basis column, -1 to drop
    int32_t o_out, ncols;
};

// Transposed route with more initial-space rows than the fused projection
// holds (kry_wide.hip).
constexpr int kMaxK1 = kMaxK + 1;   // row stride of the wide stage's stored matrices
constexpr int kMaxWide = 4096;      // initial-space rows of a wide transposed plan
struct WideArgs {
    const double* scal;
    ScalLayout L;
    const double* Pw;        // [nruns][ncw][ldk]: E_c^T u_{j+1} (unscaled)
    int32_t ncw, ldk;        // rows of E^T (= basis columns) and the stride of Pw
    int32_t bcol;            // the forcing's column (forcing != 0)
    int32_t forcing;         // the last row is b: bordered matrix of size m + 1
    int32_t hess;            // H from the Hessenberg store (Arnoldi) or alpha/beta
    double dt;
    int32_t B, nanch;        // anchor spacing and count, as for the small stage
    double* pow;             // [nruns][B][kMaxK1][kMaxK1]: Phi^r
    double* anch;            // [nruns][nanch][kMaxK1]:     Phi^{B b} x0
    double* basis;           // [(steps+1)][o_out][ncols]
    int32_t o_out, ncols;
};
hipError_t wide_prepare();
// Step j of a batch of P runs (vectors x, [n][P]): segments g0 .. g0 + ng - 1
// of the wide rows summed into segsum[j] ([k][ng][P]).  After the batch:
// Pw[run0 + p][c][j] for every row c < nsets and step j < kdone, the row's
// segments added in order.
hipError_t launch_wide_proj(int P, bool f32, const void* x, const SegTable& T, int32_t g0, int32_t ng,
                            double* segsum, int32_t j, hipStream_t s);
hipError_t launch_wide_sets(int P, const SegTable& T, int32_t set0, int32_t nsets, int32_t g0, int32_t ng,
                            const double* segsum, double* Pw, int32_t run0, int32_t nreal, int32_t ncw, int32_t ldk,
                            int32_t kdone, hipStream_t s);
hipError_t launch_wide_stage(const WideArgs& W, int32_t nruns, int64_t steps, hipStream_t s);

constexpr int kMaxCheckCols = 64;   // columns of a check over part of the basis
struct CheckArgs {
    const double* basis;
    const double* zc;        // per basis column: box center (1 for fixed runs)
    const double* radius;    // per basis column: box radius (0 for fixed runs)
    int32_t nruns, o;        // columns and output rows checked
    int64_t steps;
    double ulo[kMaxO], uhi[kMaxO];
    double* part;            // [2 * check_blocks] first hit and non-finite flag per block
    double* verdict;         // [first_step, row, y, lo, hi, status, z[nruns]]
    // part of the basis: checked row q is basis row row_of[q] and checked
    // column r basis column col_of[r] of a [steps+1][o_all][n_all] basis
    int32_t mapped;          // 0: the whole basis (o_all = o, n_all = nruns, identity maps)
    int32_t o_all, n_all;
    int32_t row_of[kMaxO];
    int32_t col_of[kMaxCheckCols];
};

// Classical Gram-Schmidt against the stored basis: CGS2 for Arnoldi, and the
// one full reorthogonalisation pass of Lanczos in FP32-basis mode.  The
// basis is stored unnormalised, column-major per run batch: u_i at
// V + (i - 1) * vstride ([n][P] interleaved, elements of type E), v_i = sigma_i u_i.
struct ArnArgs {
    const void* V;           // u_1 .. u_j (j = iteration), each [n][P]
    int64_t vstride;         // elements from u_i to u_{i+1} (n * the plan's largest batch)
    void* w;                 // vector being orthogonalised ([n][P]), u_{j+1} once swept
    double* hpart;           // [k][kMaxP][nblocks] partials of u_i . w
    double* hcoef;           // [k][kMaxP] coefficients of the current pass (h_i * sigma_i)
    int32_t f32;             // 1: E = float, else double
    int32_t lanczos;         // 1: w is a Lanczos three-term result; H_{j-1,j} and H_{j,j} add beta_{j-1}, alpha_j
    // the step with the second pass from the Gram matrix (Arnoldi):
    double* hpart2;          // [k + 1][kMaxP][nblocks] partials of u_i . u_j
    double* sraw;            // [k + 1][kMaxP] u_i . w (last: w . w)
    double* gram;            // [kMaxP][k][k] V^T V of the batch's runs (v_i = sigma_i u_i)
    int32_t* guard;          // 1: a run's w kept too little of its norm; a plain second pass follows
    int32_t conditional;     // 1: the launch returns at once unless *guard
    double reorth2;          // the guard: |w''|^2 < reorth2 |w|^2
};
constexpr int kArnChunk = 16;    // basis vectors per block of the dot kernel

// ---- error control (kry_errctl.hip) ----------------------------------------
struct ErrArgs {
    const int32_t* role;     // per run of the plan: 2 = augmented (integrated bound)
    double tau;              // time horizon steps * dt
    double lam_plus;         // max(0, upper bound of lambda_max((A + A^T)/2))
    double eps;              // error target
    double gl_x[8], gl_w[8]; // 8-point Gauss-Legendre nodes and weights on [-1, 1]
    double* flags;           // [kMaxP] 1 when the run has stopped
    int hess;                // T's diagonal from the Hessenberg store (stored-basis Lanczos)
};
hipError_t launch_record_stage(int P, const BatchArgs& B, int j, hipStream_t s);
// Lanczos error control at large k (kry_errbig.hip): per run of the batch,
// theta [ld] and w [ld] (eigenvalues of T_j and q_{1,i} q_{j,i}), work
// [ld][chunk] (pivots of the eigenvalues in flight); j <= ld.
constexpr int kBigFrom = 128;       // checkpoints past this k take the parallel eigen-solve
struct BigErrArgs {
    double* theta;
    double* w;
    double* work;
    int32_t ld, chunk;
};
hipError_t big_prepare();
hipError_t launch_lemma1_big(int P, const BatchArgs& B, const ErrArgs& X, int j, const BigErrArgs& G, hipStream_t s);
hipError_t launch_lemma1(int P, const BatchArgs& B, const ErrArgs& X, int j, hipStream_t s);
hipError_t launch_row_gersh(const CsrArgs& A, int64_t n, double* partials, int32_t nblocks, int64_t rows_per_block,
                            double* out, hipStream_t s);
// Arnoldi runs (Hessenberg H): partials holds lemma1_hess_partials() doubles
hipError_t errctl_prepare();
int lemma1_hess_partials();
hipError_t launch_lemma1_hess(int P, const BatchArgs& B, const ErrArgs& X, int j, double* partials, hipStream_t s);
// largest |a| (block maxima in partials, nblocks of them)
hipError_t launch_abs_max(const double* vals, int64_t nnz, double* partials, int32_t nblocks, double* out,
                          hipStream_t s);
// Gershgorin bound of the symmetric part of a general CSR matrix; colfix
// holds n integers of scratch, *overflow is set when a column sum overflows
hipError_t launch_gersh_general(const CsrArgs& A, int64_t n, double u, unsigned long long* colfix, int* overflow,
                                double* partials, int32_t nblocks, int64_t rows_per_block, double* out,
                                hipStream_t s);

// ---- block Arnoldi (kry_block.hip) ------------------------------------------
constexpr int kBW = 16;          // block width: p <= 16 real columns, the rest zero
constexpr int kMaxKB = 32;       // block steps (Krylov dimension 16 k <= 512)

struct BlockStart {
    int32_t set[kBW];            // segment set of generator column c (c < p)
    int32_t p;
};

// ---- launch choices that leave results unchanged (kry_tune.cpp) ------------
struct TuneChoice {
    int32_t a = 0, b = 0;    // kernel-specific: bspmm (rows per workgroup, XCD map); lz1_march (non-temporal, -)
    double us = 0.0;         // the measured time per launch
};
bool tune_lookup(const std::string& kernel, int64_t n, int32_t runs, TuneChoice* out);
void tune_store(const std::string& kernel, int64_t n, int32_t runs, const TuneChoice& c);
void tune_clear();
std::string tune_device_tag();

struct BlockArgs {
    int64_t n;
    int32_t p;                   // real columns of this block run
    int32_t rb;                  // row blocks of the Gram kernel
    int64_t rows_per_rb;         // rows per row block
    double* gpart;               // [kMaxKB + 1][rb][256] partials of 16 x 16 products
    double* gpart2;              // the same for the second right-hand side of the one-pass Gram
    double* coef;                // [kMaxKB + 1][256] reduced blocks / update coefficients
    double* sbuf;                // [kMaxKB + 1][256] S_i = V_i^T W of the one-pass step (last: W^T W)
    double* G;                   // V^T V of the stored blocks, row-major, ldh columns
    const int32_t* cond;         // launches with a condition return while *cond == 0 (null: none)
    double reorth2;              // one-pass step: a plain second pass when |W''_c|^2 < reorth2 |W_c|^2
    double* H;                   // block Hessenberg, row-major, ldh columns
    int32_t ldh;
    double* P;                   // C V, o rows of ldp
    int32_t ldp;
    double* R0;                  // 16 x 16: G = V_1 R0
    double* rfirst;              // 16 x 16: R of the first CholQR pass
    int32_t* state;              // [0] done, [1] blocks formed, [2] non-finite, [4] second pass wanted
    const double* anorm;         // ||A||_inf on the device
    double tau_scale;            // breakdown when R_cc <= tau_scale * ||A||_inf
    int32_t spmm_rows;           // rows per workgroup of the block mat-vec (0: the default)
    int32_t spmm_xcd;            // 1: row ranges XCD-contiguous, 0: in workgroup order
};

hipError_t launch_bstart(bool f32, const SegTable& T, const BlockStart& S, void* V, int64_t n, hipStream_t s);
hipError_t launch_bspmm(bool f32, const CsrArgs& A, const void* V, void* W, const BlockArgs& B, hipStream_t s);
// Y2 non-null: the partials against Y2 as well (gpart2)
hipError_t launch_bgram(bool f32, const void* X0, int64_t xstride, int nx, const void* Y, const BlockArgs& B,
                        hipStream_t s, const void* Y2 = nullptr);
// mode 0 / 1: Gram-Schmidt pass 1 / 2 of block column j; mode 2: Gram matrix;
// mode 3: S and block column j of V^T V for the one-pass step
hipError_t launch_bgram_red(const BlockArgs& B, int nx, int j, int mode, hipStream_t s);
hipError_t launch_bcorr(const BlockArgs& B, int j, hipStream_t s);
hipError_t launch_bchol(const BlockArgs& B, int j, int pass, hipStream_t s);
hipError_t launch_bupdate(bool f32, const void* X0, int64_t xstride, int nx, void* Y, int accumulate,
                          const BlockArgs& B, hipStream_t s);
hipError_t launch_bproj(bool f32, const SegTable& T, int32_t oset0, int o, const void* V, double* part, int G,
                        int j, const BlockArgs& B, hipStream_t s);

// ---- dense stage for large Krylov dimensions (kry_dense.hip) --------------
struct DenseJob {
    const double* H;             // m x m (row-major, ldh)
    int32_t ldh;
    int32_t m;
    double dt;
    const double* P;             // o x m (ldp)
    int32_t ldp;
    int32_t o;
    const double* S0;            // m x w start coefficients (lds0)
    int32_t lds0;
    int32_t w;
    int32_t B, nanch;            // steps s = b B + r
    int64_t steps;
    double* basis;               // [(steps+1)][o][nruns]
    int32_t nruns, run0;
    int32_t nonfinite;           // the run met a non-finite value: its columns become NaN
};
size_t dense_workspace_doubles(int m, int o, int w, int B, int nanch);
// Enqueues the whole stage; waits once for |H|_1 (the number of squarings).
hipError_t dense_expm_steps(const DenseJob& J, double* ws, double* host_norm, hipStream_t s);
// H (m x m), P (o x m) and S0 = scale e_1 (m) of one single-vector run for
// the dense stage, laid out as the LDS exponential assembles them.
hipError_t launch_build_dense(const ExpmArgs& E, int run, int m, double* H, double* P, double* S0, hipStream_t s);
hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s);

// ---- launchers (kry_lanczos.hip, kry_expm.hip) ----------------------------
hipError_t launch_row_abs_max(const CsrArgs& A, int64_t n, double* partials, int32_t nblocks,
                              int64_t rows_per_block, double* out, hipStream_t s);
// Columns 0..kdone of P = C V and the record of stage kdone.
hipError_t launch_finish(int P, int O, const BatchArgs& B, int kdone, hipStream_t s);
hipError_t launch_to_f32(const double* in, float* out, int64_t n, hipStream_t s);
// f32 selects E = float storage of the Krylov vectors (and vals32 for CSR).
hipError_t launch_start(int P, int O, bool f32, const StartSrc& src, const SegTable& T, int32_t oset0,
                        void* u, const BatchArgs& B, hipStream_t s);
hipError_t launch_spmv_sell(int P, bool f32, const SellArgs& A, const void* ucur, const void* uprev, void* w,
                            const BatchArgs& B, int j, hipStream_t s);
// Kernel timing: when the pair is set, the next sliced-ELL mat-vec launch
// passes it to hipExtLaunchKernelGGL, which stamps the kernel's own start
// and end (instead of events recorded around the launch).
struct ExtEvents {
    hipEvent_t start, stop;
};
ExtEvents* ext_events();   // this thread's pending pair (null members: none)
hipError_t launch_spmv_csr(int P, int lpr, bool f32, const CsrArgs& A, const void* ucur,
                           const void* uprev, void* w, const BatchArgs& B, int j, hipStream_t s);
// march: the column-marching kernel (grid ap_nblocks), else the row kernel.
hipError_t launch_spmv_stencil(int P, bool march, bool f32, const StencilArgs& A, const void* ucur,
                               const void* uprev, void* w, const BatchArgs& B, int j, hipStream_t s);
hipError_t launch_sweep(int P, int O, bool f32, const SegTable& T, int32_t oset0, const void* ucur,
                        void* w, const BatchArgs& B, int j, hipStream_t s);
// ---- one-pass Lanczos step (kry_lz1.hip) -----------------------------------
// Iteration j reads the pair buffer xin = (u_{j-1}, r_j) ([n][2P]; at j = 1
// the start kernel's plain [n][P] vectors, u_0 = 0) and writes
// xout = (u_j, r_{j+1}).  Partials ping-pong between two arrays: ap_in holds
// the previous launch's sigma_{j-1} u_{j-1} . r_j, |r_j|^2 and |u_{j-1}|^2
// per run ([3P][nb_in]); this launch writes its own to ap_out.
struct Lz1Args {
    const double* ap_in;
    double* ap_out;
    int32_t nb_in;           // blocks of the launch that wrote ap_in
    double* flag;            // [P] 1 while a run's |u_j|^2 expansions hold, 0 once one cancelled
};
hipError_t launch_lz1_sell(int P, int O, const SellArgs& A, const double* xin, double* xout, const SegTable& T,
                           int32_t oset0, const BatchArgs& B, const Lz1Args& Z, int j, hipStream_t s);
hipError_t launch_lz1_stencil(int P, int O, const StencilArgs& S, const double* xin, double* xout,
                              const SegTable& T, int32_t oset0, const BatchArgs& B, const Lz1Args& Z, int j,
                              hipStream_t s);
// grid lz1_march_blocks(ny, nz, P) ((y, z) tiles, also the count of its
// partials; the most for P = 8); C u_j then comes from launch_lz1_proj
int32_t lz1_march_blocks(int64_t ny, int64_t nz, int P);
// nt: pair stores non-temporal (1) or plain (0); the values are the same
hipError_t launch_lz1_march(int P, const StencilArgs& S, const double* xin, double* xout, const BatchArgs& B,
                            const Lz1Args& Z, int j, hipStream_t s, int nt = 1);
hipError_t launch_lz1_proj(int P, int O, const double* x, const SegTable& T, int32_t oset0, const BatchArgs& B,
                           int j, hipStream_t s);
// after iteration k (j = k + 1): alpha_k and stage k (beta_k) from the last
// launch's partials, one workgroup
hipError_t launch_lz1_close(int P, const BatchArgs& B, const Lz1Args& Z, int j, hipStream_t s);

hipError_t expm_prepare();
hipError_t launch_expm_chain(const ExpmArgs& E, int32_t nruns, hipStream_t s);
int check_blocks(int64_t steps, int32_t o);
hipError_t launch_assemble(const AssembleArgs& A, hipStream_t s);
hipError_t launch_check(const CheckArgs& C, hipStream_t s);
// nx vectors u_1..u_nx against w; two: against u_j as well (hpart2)
hipError_t launch_arn_dots(int P, const ArnArgs& A, const BatchArgs& B, int j, hipStream_t s, int nx = 0,
                           bool two = false);
// pass 1 / 2: H_{:,j} = / += the pass's coefficients; pass 3: u_i . w into
// sraw and column j of V^T V into gram (i <= j, the one-pass step)
hipError_t launch_arn_reduce(int P, const ArnArgs& A, const BatchArgs& B, int j, int pass, hipStream_t s);
// H_{:,j} = S - (V^T V - I) S from sraw and gram; coefficients for the update
hipError_t launch_arn_corr(int P, const ArnArgs& A, const BatchArgs& B, int j, hipStream_t s);
// raises *guard when a run's |w''|^2 (stage j partials) < reorth2 (w . w)
hipError_t launch_arn_guard(int P, const ArnArgs& A, const BatchArgs& B, int j, hipStream_t s);
hipError_t launch_arn_update(int P, int O, const SegTable& T, int32_t oset0, const ArnArgs& A,
                             const BatchArgs& B, int j, int last, hipStream_t s);

// ---- persistent Lanczos for small systems (kry_small.hip) --------------------
constexpr int kSmallN = 2048;     // rows: three vectors in LDS
constexpr int kSmallRuns = 64;    // runs (workgroups) per launch
constexpr int kSmallArnK = 64;    // Krylov dimension of the small Arnoldi kernel
struct SmallArgs {
    int32_t kind;                // 0: CSR, 1: 7-point stencil
    CsrArgs A;
    StencilArgs S;
    int64_t n;
    int32_t o;                   // output sets oset0 .. oset0 + o - 1
    SegTable T;
    int32_t oset0;
    double* scal;                // per-run scalars; run r at r * L.stride
    ScalLayout L;
    const double* anorm;         // ||A||_inf on the device
    double tau_scale;            // breakdown when beta_j <= tau_scale * ||A||_inf
    const double* center;
    const double* b;
    int32_t run0;                // run of workgroup 0
    int32_t src[kSmallRuns];     // start of each run: segment set (>= 0), -1 center, -2 forcing
    double* basis;               // Arnoldi: [kSmallRuns][k + 1][n] basis of the launch's runs
};
hipError_t launch_small_lanczos(const SmallArgs& a, int32_t nruns, hipStream_t s);
hipError_t launch_small_arnoldi(const SmallArgs& a, int32_t nruns, hipStream_t s);

// ---- per-step safety LP (kry_lp.hip) -----------------------------------------
constexpr int kLpMaxD = 16;      // generator coefficients (LP variables)
constexpr int kLpMaxRows = 64;   // box rows + G rows + U rows
constexpr int kLpRec = 2 + kLpMaxD;   // per step: flag, t*, z
struct LpArgs {
    const double* basis;     // [(steps+1)][o][ncols], generator columns first
    int32_t o, ncols, d;     // d = generators (the first d columns)
    int32_t mI, mU;
    int64_t steps;
    const double* zlo;       // [d] box lower ends zc - r
    const double* zhi;       // [d] box upper ends zc + r
    const double* G;         // [mI][d]
    const double* h;         // [mI]
    const double* U;         // [mU][o]
    const double* u;         // [mU]
    double tol;              // feasible when the phase-one optimum t* <= tol
    int32_t max_pivots;
    double* rec;             // [(steps+1)][kLpRec]: flag (1 feasible, 0 not, -1 undecided), t*, z
    double* verdict;         // [2 + kLpMaxD + kMaxO]: first step, status, z, y
};
hipError_t launch_lp(const LpArgs& L, hipStream_t s);

}  // namespace kry
