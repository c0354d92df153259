/*
 * kry.h -- C ABI of the MI355X (gfx950) projected Krylov simulation library.
 *
 * Method: Bak, Tran, Johnson, "Numerical Verification of Affine Systems with
 * up to a Billion Dimensions" (arXiv 1804.01583).  For a system x' = A x + b,
 * an initial box set x0 = sum_j z_j g_j (+ center), z_j in [zc_j - r_j,
 * zc_j + r_j], output rows y = C x and time points t = s*dt, s = 0..S, the
 * library computes the basis matrix C e^{A s dt} E of Sections 3.1-3.2
 * (output and initial-space projection) one column of E at a time
 * (Section 4.1), each column by the Krylov approximation
 *     e^{A t} v ~ |v| V_k e^{H_k t} e_1            (Section 4.2, Eq. approx-formula)
 * with Lanczos (Algorithm 3) for symmetric A, projecting P = C V_k on the
 * fly so the basis V_k is never stored (Algorithm 4).  The affine term b is
 * removed by augmenting the state with a constant variable (Section 2.1).
 * It then checks every time step for an intersection of the reachable output
 * range with the unsafe set (the per-step LP of Section 2.1, specialised to a
 * box initial set) and returns the first violation with a counter-example.
 *
 * Beside that path: the same basis one output row at a time by the
 * transposed dynamics (Section 4.1, kry_plan_create_transposed); the per-step
 * LP itself for a polytopic initial set and a conjunction of output
 * halfspaces (kry_check_lp_safety); the Krylov dimension chosen by the
 * a-posteriori bound of Lemma 1 (kry_plan_set_error_target); block Arnoldi
 * over up to 16 generators; an FP32-stored basis; a sliced-ELL copy of a CSR
 * matrix shared by plans (kry_matrix_create); and a projection recorded once
 * as a HIP graph and replayed (kry_plan_set_graph).
 *
 * Conventions for every entry point:
 *  - Device pointers are caller-owned and borrowed until kry_plan_destroy.
 *    Host pointers are read during the call only.
 *  - All GPU work is enqueued on the caller's hipStream_t given to kry_plan
 *    (or kry_plan_create).
 *  - Every call returns a kry_status; no C++ exception crosses this ABI.  On
 *    a non-OK status, kry_last_error() returns a thread-local message.
 *  - Dimensions are 64-bit; vectors of n > 2^31 entries are supported.
 *  - Environment switches, read when a plan projects, choose between forms
 *    that compute the same quantities (results agree to rounding):
 *    KRY_SMALL=0 keeps systems of at most 2048 rows off the one-launch
 *    persistent kernels; KRY_BLOCK_GS=0 / KRY_ARN_GS=0 make both classical
 *    Gram-Schmidt passes of block / single-vector Arnoldi over the basis
 *    instead of taking the second from the Gram matrix (KRY_ARN_GS=1 forces
 *    that form below its default of 2^16 rows); KRY_BLOCK_REORTH2 /
 *    KRY_ARN_REORTH2 set the squared norm ratio under which the Gram-matrix
 *    form adds a plain second pass (default 1e-6); KRY_ONEPASS=0/1 turns the
 *    one-pass Lanczos step off / on for CSR matrices.
 */
#ifndef KRY_H
#define KRY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KRY_OK = 0,
    KRY_EINVAL = 1,    /* invalid argument: shapes, ranges, NULL pointers, non-finite scalars */
    KRY_ENOMEM = 2,    /* device allocation failed or workspace too small */
    KRY_EDEVICE = 3,   /* a HIP runtime call failed */
    KRY_ENUMERIC = 4,  /* non-finite value met in the Krylov recurrence */
    KRY_ENOTSUP = 5    /* combination of options the library does not offer */
} kry_status;

typedef enum { KRY_FP64 = 0, KRY_FP32_BASIS = 1 } kry_precision;

/* KRY_AUTO picks Lanczos when the system is declared symmetric. */
typedef enum {
    KRY_AUTO = 0,
    KRY_LANCZOS = 1,
    KRY_ARNOLDI = 2,
    KRY_BLOCK_ARNOLDI = 3,
    KRY_LANCZOS_PLAIN = 4
} kry_method;

typedef enum { KRY_CSR = 0, KRY_STENCIL7 = 1 } kry_kind;

/* A sparse vector as nseg disjoint half-open index ranges [lo, hi), sorted
 * ascending, each with one value w.  Host arrays. */
typedef struct kry_segs {
    int64_t nseg;
    const int64_t* lo;
    const int64_t* hi;
    const double* w;
} kry_segs;

/* The system matrix A and the forcing b (Section 2, x' = A x + b).
 * KRY_CSR: rowptr[n+1] (int64), colidx[nnz] (int32, < n), vals[nnz] (FP64),
 *   all device memory, rows in order; duplicate columns are summed.
 * KRY_STENCIL7: matrix-free 7-point stencil on an nx*ny*nz grid ordered
 *   index = (ix*ny + iy)*nz + iz; (A v)_i = c0 v_i + cx (v_{i-+x}) + cy (...) +
 *   cz (...), neighbours outside the grid are zero (Dirichlet).
 * b: device n-vector or NULL.  When non-NULL the state is augmented with a
 *   constant variable a = 1 (Section 2.1) and one extra simulation runs.
 * b_segs: the forcing as index ranges (host), used when b is NULL; for large
 *   systems whose forcing is a few regions.
 * symmetric: the caller promises A == A^T (needed by Lanczos, Section 4.3).
 * anorm: max absolute row sum of A, or 0 to let kry_plan compute it; it only
 *   scales the breakdown test (a Krylov step whose new norm is at most
 *   1024 * eps * anorm ends the run: the space is invariant, Section 4.2).
 * stencil_bc (KRY_STENCIL7): KRY_BC_DIRICHLET (0; zero outside the grid) or
 *   KRY_BC_INSULATED (1; no flux through the faces: a face cell's missing
 *   neighbour is dropped together with its share of the diagonal, i.e. the
 *   diagonal becomes c0 + cx per missing x neighbour + cy ... + cz ...).
 * stencil_exchange (KRY_STENCIL7): added to the diagonal of the cells of the
 *   face ix = nx - 1 (heat exchange through x = 1 with a zero ambient, the
 *   3D heat benchmark of Section 5.3); 0 for none.
 * prepared: NULL, or a kry_matrix made by kry_matrix_create from this same
 *   CSR system (same three arrays) for the plan's precision.  Plans then read
 *   its sliced-ELL copy and its anorm instead of building their own, and
 *   kry_footprint leaves the copy out. */
typedef struct kry_matrix kry_matrix;
typedef struct kry_system {
    int64_t n;
    int32_t kind;
    int32_t symmetric;
    const int64_t* rowptr;
    const int32_t* colidx;
    const double* vals;
    int64_t nnz;
    int64_t nx, ny, nz;
    double c0, cx, cy, cz;
    const double* b;
    double anorm;
    const kry_segs* b_segs;
    const kry_matrix* prepared;
    int32_t stencil_bc;
    double stencil_exchange;
} kry_system;

enum { KRY_BC_DIRICHLET = 0, KRY_BC_INSULATED = 1 };

/* One column g_j of E with its box coefficient z_j in [zc - radius, zc + radius]
 * (Section 3.2, initial space I_z given as a box). */
typedef struct kry_gen {
    kry_segs seg;
    double zc;
    double radius;
} kry_gen;

/* Output row r is unsafe at a step when y_r can take a value in [lo, hi]
 * (closed; +-INFINITY allowed).  The unsafe set is the union over rows. */
typedef struct kry_interval {
    double lo, hi;
} kry_interval;

typedef struct kry_verdict {
    int64_t first_step;  /* first violated step s (time s*dt), or -1 when safe */
    int32_t row;         /* violated output row at that step, -1 when safe */
    int32_t status;      /* KRY_OK, or KRY_ENUMERIC if a non-finite basis entry was met */
    double y;            /* output value of the counter-example */
    double lo, hi;       /* reachable output range of that row at that step */
} kry_verdict;

/* The plan object.  Its type is kry_plan_t (struct kry_plan): the name
 * kry_plan itself is the entry point that creates one. */
typedef struct kry_plan kry_plan_t;

/* Names of the boundary's sketch for the same structures: an output row is a
 * segment set, an unsafe interval a kry_interval. */
typedef kry_segs kry_row;
typedef kry_interval kry_unsafe;

/* kry_plan_create -- validate the problem, split E into simulation runs and
 * prepare the device state for them (Sections 2.1, 3.2, 4.1).
 * Runs, in this order: one per generator [g_j; 0], one for the fixed center
 * [x_c; 0] when center != NULL (device n-vector), one for the augmented
 * variable [0; 1] when sys->b or sys->b_segs is given.
 *  C, o: o >= 1 output rows (host segment sets, Section 3.1); o <= 8.
 *  k: Krylov dimension per run, 1 <= k <= 512 (8192 for KRY_LANCZOS_PLAIN);
 *     past k = 56 the small exponential runs as a dense stage.  The augmented run uses k-1
 *     Lanczos steps on A from b bordered by one row and column, which spans
 *     the same k-dimensional Krylov space of the augmented matrix.  For
 *     KRY_BLOCK_ARNOLDI, k counts block steps (1 <= k <= 32; dimension p k).
 *  dt, steps: time points s*dt for s = 0..steps (steps + 1 rows of output).
 *  precision: KRY_FP64, or KRY_FP32_BASIS: Krylov vectors (and CSR values)
 *     stored in FP32, every sum, coefficient and the small exponential in
 *     FP64, the whole basis kept and each new vector reorthogonalised against
 *     it (Lanczos: one classical pass after the three-term step; Arnoldi and
 *     block Arnoldi: two passes).  Breakdown then uses eps of FP32.
 *  method: KRY_AUTO (Lanczos when symmetric, else Arnoldi), KRY_LANCZOS
 *     (Algorithm 3; needs symmetric; past k = 56 it keeps its basis and
 *     reorthogonalises each new vector once), KRY_LANCZOS_PLAIN (the
 *     three-vector projected Lanczos of Algorithm 4 at any k: three
 *     n-vectors per run, no reorthogonalisation, FP64 only; the same as
 *     KRY_LANCZOS for k <= 56), KRY_ARNOLDI (Algorithm 1, classical
 *     Gram-Schmidt twice), or KRY_BLOCK_ARNOLDI: the generators in blocks of
 *     p <= 16 columns, each block one block Krylov space
 *     span{G, AG, ..., A^{k-1} G} with C e^{At} G ~ C V e^{Ht} E_1 R_0
 *     (CSR systems, generator runs only: KRY_ENOTSUP with a center or a
 *     forcing; KRY_ENUMERIC when a block's generators are dependent).
 *  block_p: runs advanced together per sparse mat-vec launch (1, 2, 4 or 8;
 *     0 = automatic); results do not depend on it.  For KRY_BLOCK_ARNOLDI
 *     the block width p (1..16; 0 = min(ngen, 16)).
 *  workspace: device buffer of workspace_bytes >= kry_plan_workspace(...), or NULL
 *     to let the plan allocate (and free) its own.  A smaller one gives
 *     KRY_ENOMEM (the message names the bytes needed), one not 256-byte
 *     aligned KRY_EINVAL, both before any device work.
 *  hip_stream: hipStream_t to enqueue on (NULL = default stream).
 * The plan borrows sys->rowptr/colidx/vals/b and center until destroyed. */
kry_status kry_plan_create(const kry_system* sys, const kry_gen* gens, int32_t ngen,
                           const double* center, const kry_segs* C, int32_t o, int32_t k,
                           double dt, int64_t steps, int32_t precision, int32_t method,
                           int32_t block_p, void* workspace, size_t workspace_bytes,
                           void* hip_stream, kry_plan_t** out);

/* kry_plan -- the plan of kry_plan_create with a workspace the plan
 * allocates and frees itself (Sections 2.1, 3.2, 4.1): every argument as
 * there.  C holds o output rows; center is a device n-vector or NULL. */
kry_status kry_plan(const kry_system* sys, const kry_gen* gens, int32_t ngen, const double* center,
                    const kry_row* C, int32_t o, int32_t k, double dt, int64_t steps, int32_t precision,
                    int32_t method, int32_t block_p, void* hip_stream, kry_plan_t** out);

/* kry_plan_create_transposed -- the same basis C e^{At} E by simulations of
 * the transposed dynamics (Section 4.1): C e^{At} E = (E^T e^{A^T t} C^T)^T,
 * so one run per output row instead of one per column of E, each projected
 * on the rows of E^T as it goes (Algorithm 4 with E^T in place of C,
 * Section 4.3).  Worth it when o is smaller than the number of columns.
 *  sys_t: the system whose matrix is A^T (for a symmetric A, the system
 *     itself).  Its forcing, when given, is the original system's b and
 *     must come as b_segs (it is a projection row); a dense b gives
 *     KRY_ENOTSUP.
 *  gens, ngen, center: the initial space (center: host segment set or
 *     NULL, a fixed coefficient-1 column).  Generators + center + forcing
 *     make ncols <= 4096 basis columns.  Up to 8 are projected inside the
 *     Krylov sweep and exponentiated per run in LDS; past 8 each Krylov
 *     vector is projected on the rows of E^T by segment sums (one
 *     wavefront per index range), and the small stage forms
 *     e^{M s dt} x0 once per step and run (M = H, bordered by b's
 *     projection row with forcing) and multiplies it by the projections.
 *  C, o: 1 <= o <= 8 output rows, the runs' start vectors.
 *  k: 1..56 Krylov steps per run, 1..55 with forcing.  With forcing each
 *     run is the Galerkin projection of the transposed augmented matrix
 *     [[A^T, 0], [b^T, 0]] on the run's Krylov basis plus the augmented
 *     coordinate, a matrix of size k + 1.
 *  method: KRY_AUTO, KRY_LANCZOS (symmetric sys_t) or KRY_ARNOLDI; others
 *     give KRY_ENOTSUP.  dt, steps, precision, hip_stream: as for
 *     kry_plan_create.
 *  workspace: device buffer of workspace_bytes >= kry_footprint_transposed(...)
 *     (256-byte aligned), or NULL to let the plan allocate its own.  A
 *     smaller one gives KRY_ENOMEM (the message names the bytes needed), a
 *     misaligned one KRY_EINVAL, both before any device work.
 * kry_project_expm and kry_check_box_safety then behave as for a forward
 * plan with columns in the order generators, center, forcing; kry_plan_runs
 * and kry_plan_krylov describe the o transposed runs (P has one row per
 * initial-space row).  Error control (kry_plan_set_error_target) is not
 * offered on this route (KRY_ENOTSUP). */
kry_status kry_plan_create_transposed(const kry_system* sys_t, const kry_gen* gens, int32_t ngen,
                                      const kry_segs* center, const kry_segs* C, int32_t o, int32_t k,
                                      double dt, int64_t steps, int32_t precision, int32_t method,
                                      void* workspace, size_t workspace_bytes, void* hip_stream,
                                      kry_plan_t** out);

/* kry_footprint_transposed -- device workspace bytes of a transposed plan:
 * ngen generators, has_center (0/1) a center row, o output rows (the runs),
 * the forcing when sys_t->b_segs is given; nseg_total = segments of the
 * generators, the center, the output rows and b_segs together (an upper
 * bound serves: the wide route sizes its segment sums by it).  Host only. */
kry_status kry_footprint_transposed(const kry_system* sys_t, int32_t ngen, int32_t has_center, int32_t o,
                                    int32_t k, int64_t steps, int64_t nseg_total, int32_t precision,
                                    int32_t method, size_t* bytes);

/* kry_project_expm -- run the Krylov process of every run (Algorithms 3-4),
 * then form the basis matrix for all steps:
 *   basis[s][r][run] = beta0_run * (P_run e^{H_run s dt} e_1)[r]
 * (Eq. approx-formula projected by C).  basis_out: host or device pointer to
 * (steps+1) * o * ncols doubles (ncols = generators + center + forcing: the
 * runs of a forward plan), or NULL to keep the basis on the device for
 * kry_check_box_safety only.  With a host pointer the call waits for the
 * stream; otherwise it returns once the work is enqueued.  FP64 Lanczos
 * plans, and FP64 Arnoldi plans with k <= 64, of at most 2048 rows and
 * without an error target run every run's whole Krylov process in one
 * launch (results equal the general path's to rounding); set KRY_SMALL=0 in
 * the environment to keep the general path. */
kry_status kry_project_expm(kry_plan_t* plan, double* basis_out);

/* kry_check_box_safety -- per step s and output row r, the reachable output
 * range over the box is [mid - rad, mid + rad] with
 *   mid = sum_gen basis*zc + sum_fixed basis,  rad = sum_gen |basis|*radius,
 * exact for a box initial set (the LP of Section 2.1 reduces to it).  Row r is
 * violated when the range meets unsafe[r].  Reports the first (step, row) in
 * step-major order and a counter-example z (z_out: host array of ngen doubles,
 * may be NULL): the box point z_j = zc_j + d*lam*sign(basis_j)*r_j whose output
 * is the nearest end of unsafe[r] (lam = 0 when mid is already inside).
 * Needs kry_project_expm first.  Waits for the stream. */
kry_status kry_check_box_safety(kry_plan_t* plan, const kry_interval* unsafe, kry_verdict* out,
                                double* z_out);

/* kry_check_box_subset -- kry_check_box_safety over part of a plan's basis,
 * for one plan that carries several verification problems on the same
 * system (Section 4.1: each column of E is its own simulation, so columns
 * of different problems can share the Krylov launches): the reachable
 * range of Section 2.1's per-step check over the box of the generator
 * columns among cols (the other columns enter with coefficient 1), on output
 * rows rows[i] with unsafe set unsafe[i], at steps 0..steps.
 *  cols: ncols distinct basis columns of the plan, 1 <= ncols <= 64.
 *  rows: nrows output rows of the plan (1 <= nrows <= the plan's o).
 *  steps: 0 <= steps <= the plan's steps.
 *  out->row is an index into rows; z_out: the counter-example's
 *     coefficients of the generator columns among cols, in their order.
 * KRY_EINVAL for bad indices or sizes.  Needs kry_project_expm first.
 * Waits for the stream. */
kry_status kry_check_box_subset(kry_plan_t* plan, const int32_t* cols, int32_t ncols, const int32_t* rows,
                                int32_t nrows, int64_t steps, const kry_interval* unsafe, kry_verdict* out,
                                double* z_out);

/* kry_verify_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): kry_plan_create + kry_project_expm + kry_check_box_safety in
 * one call, every argument as there, with the plan's workspace in the
 * library's fixed per-device scratch array of KRY_NOALLOC_SCRATCH_BYTES
 * (128 MiB, held by each device the library runs on until the process ends)
 * instead of a caller buffer or an allocation.  The call makes no device or
 * pinned-host allocation and frees nothing on the device (its host-side
 * bookkeeping uses the C++ heap).
 *  basis_out: host or device pointer to (steps+1) * o * nruns doubles, or
 *     NULL (the basis then stays in the scratch array until the next call).
 *  unsafe, verdict, z_out: as for kry_check_box_safety.
 * Sizes whose workspace (kry_plan_workspace) exceeds the scratch array give
 * KRY_ENOMEM naming the bytes needed, before any device work; a CSR system
 * is best passed prepared (kry_matrix_create) so the sliced-ELL copy does
 * not take scratch space.  No error target, graph mode or LP check.
 * Waits for hip_stream before returning.  Every call on one device shares
 * that device's array and leaves its contents behind (each call initialises
 * what it reads): calls that overlap on one device (other host threads,
 * other streams) race and must be serialised by the caller. */
#define KRY_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
kry_status kry_verify_noalloc(const kry_system* sys, const kry_gen* gens, int32_t ngen, const double* center,
                              const kry_segs* C, int32_t o, int32_t k, double dt, int64_t steps, int32_t precision,
                              int32_t method, int32_t block_p, const kry_interval* unsafe, double* basis_out,
                              kry_verdict* verdict, double* z_out, void* hip_stream);

/* kry_plan_set_graph -- graph mode (on != 0): the next kry_project_expm
 * records everything it enqueues (the Krylov batches, the small stage and
 * the assembly) as one HIP graph and launches it; later calls launch the
 * recorded graph again, with one host call instead of one per kernel.  The
 * graph reads the plan's inputs through the same device pointers, so new
 * values written there (forcing, center, matrix values) are picked up;
 * the plan's sizes and segment sets are fixed.  For Lanczos and Arnoldi
 * plans with k <= 56 and no error target, on a stream other than the
 * default one (KRY_EINVAL), and not while kernel timing is on (the capture
 * returns KRY_ENOTSUP).  on = 0 returns to per-kernel launches and frees
 * the graph. */
kry_status kry_plan_set_graph(kry_plan_t* plan, int32_t on);

/* kry_check_lp_safety -- the per-step LP of Section 2.1 for a polytopic
 * initial set and a conjunction of output halfspaces, on the basis of
 * kry_project_expm.  With M_s the generator columns of the basis at step s
 * and f_s the sum of its fixed columns (center, forcing), step s is unsafe
 * when some z with
 *     zc_j - r_j <= z_j <= zc_j + r_j (the generators' box),  G z <= h,
 *     U (M_s z + f_s) <= u
 * exists.  Each step is decided by phase one of the simplex method (one
 * artificial variable, Bland's rule) on rows scaled to a largest
 * coefficient of 1: unsafe when the smallest uniform violation is <= 1e-6
 * (the LP tolerance of Section 4.2; the decision errs towards unsafe by at
 * most that much).
 *  G: host, mI x ngen row-major; h: mI.  U: host, mU x o row-major; u: mU.
 *     ngen <= 16 and ngen + mI + mU <= 64; all entries finite.
 *  first_step: the first unsafe step, -1 when every step is safe.
 *  status: 0, or KRY_ENUMERIC when a step up to first_step (every step when
 *     safe) was left undecided (iteration cap, non-finite basis).
 *  z_out (ngen), y_out (o): the counter-example of Section 2.2 at
 *     first_step and its outputs (may be NULL).
 *  step_flags: host array of steps + 1 ints (1 unsafe, 0 safe, -1
 *     undecided) or NULL.
 * The plan keeps a device buffer for the LP from the first call on.
 * Needs kry_project_expm first.  Waits for the stream. */
kry_status kry_check_lp_safety(kry_plan_t* plan, const double* G, const double* h, int32_t mI, const double* U,
                               const double* u, int32_t mU, int64_t* first_step, int32_t* status, double* z_out,
                               double* y_out, int32_t* step_flags);

/* kry_plan_workspace -- device workspace bytes a plan with these sizes needs
 * (the Krylov vectors, per-block partial sums, H, P and the basis; Section 3.5
 * gives the method's own memory model, this adds the GPU's staging): the
 * exact size kry_plan_create asks of a caller's workspace.
 * nruns = generators + (center given) + (b given); nseg_total = segments of
 * all generators and output rows together.  Host only. */
kry_status kry_plan_workspace(const kry_system* sys, int32_t nruns, int32_t o, int32_t k, int64_t steps,
                              int64_t nseg_total, int32_t precision, int32_t method, int32_t block_p,
                              size_t* bytes);

/* kry_footprint -- the HBM a plan made by kry_plan with these sizes holds
 * for its Krylov state (Section 3.5's memory model: n-vectors per run, or
 * the stored basis; here also the per-block partial sums, a sliced-ELL copy
 * of a CSR matrix that is not prepared, H and P), for method KRY_AUTO, one
 * segment per generator and output row, and no time steps: a plan holds
 * another 8 o runs bytes per time step for the basis and its check (plus the
 * small stage's tables); kry_plan_workspace gives the exact total.  The
 * runs are ngen generators plus the forcing when sys->b or sys->b_segs is
 * given (count a center as one more generator).  block_p as for kry_plan.
 * For admission of work by memory (the serving loop).  Host only;
 * KRY_EINVAL for bad sizes. */
kry_status kry_footprint(const kry_system* sys, int32_t ngen, int32_t o, int32_t k, int32_t precision,
                         int32_t block_p, size_t* bytes);

/* kry_plan_runs -- number of runs of a plan and their roles
 * (roles_out: nruns ints, 0 = generator, 1 = center, 2 = augmented; may be NULL). */
kry_status kry_plan_runs(const kry_plan_t* plan, int32_t* nruns, int32_t* roles_out);

/* kry_plan_block -- after kry_project_expm of a KRY_BLOCK_ARNOLDI plan, the
 * number of block runs (nblocks; generators b*p .. b*p + p - 1 form block b)
 * and, for block >= 0, that run's data on the host: k_eff (block steps used,
 * fewer than k after a breakdown), p (its columns), H ((p k_eff) x (p k_eff)
 * row-major block Hessenberg, H = V^T A V), R0 (p x p upper triangular with a
 * positive diagonal, G = V_1 R0 for the block's generators G) and
 * P = C V (o x p k_eff).  Any output pointer may be NULL. */
kry_status kry_plan_block(const kry_plan_t* plan, int32_t block, int32_t* nblocks, int32_t* k_eff, int32_t* p,
                          double* H, double* R0, double* P);
/* kry_plan_krylov -- after kry_project_expm, copy one run's Krylov data to the
 * host: k_eff (Krylov dimension used; smaller than k after a breakdown),
 * beta0 = |start|, the run's Hessenberg matrix H (k_eff x k_eff row-major,
 * bordered for the augmented run), h_next = h_{k+1,k}, and P = C V
 * (o x k_eff row-major).  Any output pointer may be NULL.  Waits for the stream. */
kry_status kry_plan_krylov(kry_plan_t* plan, int32_t run, int32_t* k_eff, double* beta0, double* H,
                           double* h_next, double* P);

/* kry_plan_set_error_target -- choose each run's Krylov dimension a
 * posteriori (paper Section 4.2, Lemma 1; the checks of Algorithms 2 and 4).
 * With eps > 0, kry_project_expm evaluates after iteration j = 4, then
 * j <- ceil(1.1 j) (1.1 j rounded to double, as the algorithms print it), the
 * bound of the normalised process (the algorithms start from v / |v|, so eps
 * is an error relative to |v|)
 *     h_{j+1,j} e^{max(lambda,0) tau} int_0^tau w(t) |(e^{t H_j})_{j,1}| dt
 * (tau = steps * dt; lambda an upper bound of the largest eigenvalue of
 * (A + A^T)/2 computed here by Gershgorin, on the device for a CSR system:
 * max over rows of a_rr plus half the absolute off-diagonal sums of row r
 * and column r, which is Gershgorin's bound of A for a symmetric A; w = 1,
 * or tau - t for the augmented run, whose bordered matrix integrates the
 * approximation of e^{As} b / |b|) and ends a run at the first checkpoint
 * where the bound is below eps; a batch stops iterating once all its runs
 * have ended.  k stays the cap (the augmented run: k - 1 Krylov steps).  The
 * integral uses a fixed composite 8-point Gauss-Legendre rule on
 * [0, tau 2^-40] and on [tau 2^-(i+1), tau 2^-i], i < 40, each cut into 8
 * equal parts.  eps = 0 turns the control off (the default: every run uses
 * k).  Lanczos plans (symmetric A, H_j tridiagonal: Algorithm 4), k <= 8192
 * (past k = 128 the eigen-solve of T_j runs in parallel on device memory
 * this call allocates: runs per batch x k x 514 doubles), and Arnoldi plans
 * (Algorithm 2, H_j upper Hessenberg), k <= 56; other
 * methods, the transposed route and graph mode give KRY_ENOTSUP, and so does
 * a CSR matrix with a column of more than 2^24 entries (Arnoldi).  Waits for
 * the plan's stream for a CSR system. */
kry_status kry_plan_set_error_target(kry_plan_t* plan, double eps);
/* kry_plan_error -- after kry_project_expm, run `run`'s Krylov dimension
 * (k_used: Lanczos steps used, the least of the breakdown dimension, the
 * error-control stop and k, or k - 1 for the augmented run) and
 * its last evaluated bound (-1 when none was evaluated, 0 after a breakdown,
 * which makes the projection exact).  Either pointer may be NULL; waits for
 * the plan's stream.  KRY_ENOTSUP for block plans. */
kry_status kry_plan_error(kry_plan_t* plan, int32_t run, int32_t* k_used, double* bound);

/* kry_plan_autotune -- time the launch choices of this plan's hot kernel
 * that leave every result bit for bit unchanged, on the plan's own data, and
 * keep the fastest for this device, kernel, n and runs per launch (a process
 * table; with the environment variable KRY_TUNE_CACHE naming a file, read from
 * it on first use and written back after each tuning).  Later plans of the
 * same shape use the choice.  Tuned: block plans' block mat-vec (rows per
 * workgroup 32..512, workgroups in row order or XCD-contiguous, timed on the
 * run's first block) and the one-pass marching stencil step (non-temporal or
 * plain pair stores, timed over whole projections).  Other plans tune
 * nothing.  The plan is projected first if it was not; afterwards its basis
 * and verdicts are valid (the choices change no value).  reps: timed calls
 * per candidate, 1..1000 (two rounds, the better kept).  *tuned (may be NULL):
 * kernels tuned.  KRY_ENOTSUP in graph mode.  Waits for the stream. */
kry_status kry_plan_autotune(kry_plan_t* plan, int32_t reps, int32_t* tuned);
/* kry_tune_choice -- the stored choice for kernel ("bspmm", "bspmm32" (FP32
 * basis) with runs = 16; "lz1_march" with runs = runs per launch) and n on the
 * current device: *found = 1 and (a, b, us) = (rows per workgroup, XCD map,
 * microseconds) or (non-temporal, 0, microseconds), else *found = 0. */
kry_status kry_tune_choice(const char* kernel, int64_t n, int32_t runs, int32_t* found, int32_t* a, int32_t* b,
                           double* us);
/* kry_tune_clear -- forget every stored choice of this process; the next
 * lookup reads the KRY_TUNE_CACHE file again (left as it is) when one is set. */
void kry_tune_clear(void);

void kry_plan_destroy(kry_plan_t* plan);

/* kry_matrix_create -- device-side preparation of a KRY_CSR system that any
 * number of plans can share (every simulation of Section 4.1, one per
 * column of E, and every later query uses the same A): a sliced-ELL copy of
 * A (slices of 64 rows,
 * entries column-major within a slice and padded to the slice's longest row;
 * FP64 values, or FP32 values for precision KRY_FP32_BASIS) and
 * anorm = max absolute row sum, both computed on the device.  sys->vals,
 * colidx and rowptr must not change while the matrix is in use.  The library
 * allocates the matrix's device memory (kry_matrix_bytes reports it); the
 * call waits for `hip_stream` (NULL: the default stream).  KRY_EINVAL for a
 * stencil system, nnz = 0 or bad arguments; KRY_ENOMEM when allocation fails. */
kry_status kry_matrix_create(const kry_system* sys, int32_t precision, void* hip_stream, kry_matrix** out);
kry_status kry_matrix_bytes(const kry_matrix* mat, size_t* bytes);
/* Frees the matrix; destroy the plans that use it first. */
void kry_matrix_destroy(kry_matrix* mat);

/* Thread-local text of the last error on this thread. */
const char* kry_last_error(void);

/* Kernel timing with HIP events on the plan's stream: when enabled, each
 * launch of the library's kernels is bracketed by events and its duration
 * added to a per-kernel total.  kry_profile_read returns, for kernel name
 * `name` (see kry_profile_names), the number of launches and the summed
 * milliseconds since the last reset; it waits for outstanding events. */
kry_status kry_profile_enable(int32_t on);
kry_status kry_profile_reset(void);
kry_status kry_profile_read(const char* name, int64_t* launches, double* total_ms);
const char* kry_profile_names(void);   /* comma-separated kernel names */

#ifdef __cplusplus
}
#endif

#endif /* KRY_H */
