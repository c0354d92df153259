// Host side of the C ABI declared in include/kry.h: validation, the split of
// the initial space into simulation runs (paper Sections 2.1, 3.2, 4.1),
// workspace layout, batching of runs per mat-vec launch, and the launch
// sequence of the Lanczos process (Algorithms 3-4) and of the small stage.
#include "kry.h"
#include "kry_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace kry;

namespace kry {
ExtEvents* ext_events() {
    thread_local ExtEvents pending{nullptr, nullptr};
    return &pending;
}
}  // namespace kry

namespace {

thread_local std::string g_err;

kry_status fail(kry_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

// Last resort of guarded(): record a fixed message without allocating.
kry_status fail_quiet(kry_status st, const char* msg) noexcept {
    try {
        g_err = msg;
    } catch (...) {
    }
    return st;
}

// No C++ exception crosses the C ABI: every entry point runs its body
// through guarded(), which turns a failed host allocation into KRY_ENOMEM
// and any other exception into KRY_EDEVICE, with the message kept for
// kry_last_error().
template <class F>
kry_status guarded(const char* what, F&& body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc&) {
        return fail_quiet(KRY_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        try {
            return fail(KRY_EDEVICE, std::string(what) + ": " + e.what());
        } catch (...) {
            return fail_quiet(KRY_EDEVICE, "unexpected exception");
        }
    } catch (...) {
        return fail_quiet(KRY_EDEVICE, "unexpected exception");
    }
}

template <class F>
void guarded_void(F&& body) noexcept {
    try {
        body();
    } catch (...) {
    }
}

// hipMalloc that leaves no error behind: a failed allocation also sets the
// thread's last HIP error, which the next launch's hipGetLastError() would
// report as that launch's own failure.
hipError_t device_alloc(void** p, size_t bytes) {
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
    }
    return e;
}

#define KRY_HIP(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(KRY_EDEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// Kernel timing with events (opt-in)
// ---------------------------------------------------------------------------
struct Profiler {
    std::mutex mu;
    bool on = false;
    struct Pending { std::string name; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<int64_t, double>> totals;

    hipEvent_t get() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void drain() {
        for (auto& p : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                auto& t = totals[p.name];
                t.first += 1;
                t.second += ms;
            } else {
                (void)hipGetLastError();   // a timing failure must not surface in a later call
            }
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
};
Profiler& prof() {
    static Profiler* p = new Profiler();
    return *p;
}

const char* kKernelNames =
    "row_abs_max,start,spmv_csr,spmv_sell,spmv_stencil,sweep,arn_dots,arn_reduce,arn_update,finish,expm_chain,"
    "assemble,check,bfill,bstart,bspmm,bgram,bgram_red,bchol,bupdate,bproj,dense_expm,sell_build,errctl,lp,"
    "lz1_sell,lz1_stencil,lz1_march,lz1_proj,lz1_close,wide_proj,wide_sets,wide_stage,bcorr,arn_corr,arn_guard,"
    "small_lanczos,small_arnoldi";

// Runs `launch` bracketed by events when profiling is on.  The sliced-ELL
// mat-vec and the one-pass step's kernels take the events into their own
// launch (hipExtLaunchKernelGGL), so they time the kernel itself rather than
// the gap around it.
template <class F>
hipError_t timed(const char* name, hipStream_t s, F&& launch) {
    Profiler& P = prof();
    if (!P.on) return launch();
    hipEvent_t a, b;
    {
        std::lock_guard<std::mutex> g(P.mu);
        a = P.get();
        b = P.get();
    }
    if (!a || !b) return launch();
    hipError_t e;
    if (std::strcmp(name, "spmv_sell") == 0 || std::strncmp(name, "lz1_", 4) == 0) {
        // the launcher stamps the kernel's own start and end into (a, b) and
        // clears the pending start; a launch that did not leaves them unused
        *ext_events() = ExtEvents{a, b};
        e = launch();
        const bool used = ext_events()->start == nullptr;
        *ext_events() = ExtEvents{nullptr, nullptr};
        if (!used) {
            std::lock_guard<std::mutex> g(P.mu);
            P.pool.push_back(a);
            P.pool.push_back(b);
            return e;
        }
    } else {
        (void)hipEventRecord(a, s);
        e = launch();
        (void)hipEventRecord(b, s);
    }
    std::lock_guard<std::mutex> g(P.mu);
    P.pending.push_back({name, a, b});
    return e;
}

int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v);
}

double env_double(const char* name, double dflt) {
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::strtod(v, nullptr);
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Row partition: depends on n only (never on the batch), so results of a run
// do not depend on how runs are batched.
int64_t rows_per_block_for(int64_t n) {
    const int64_t env = env_int("KRY_ROWS_PER_BLOCK", 0);
    if (env > 0) return align_up((size_t)env, kBlock);
    // blocks per kernel: enough waves to hide gather latency, few enough that
    // every block can re-read all block partials of the previous kernel
    const int64_t target_blocks = env_int("KRY_TARGET_BLOCKS", 1024);
    int64_t rpb = (n + target_blocks - 1) / target_blocks;
    rpb = (int64_t)align_up((size_t)std::max<int64_t>(rpb, kBlock), kBlock);
    return rpb;
}

// Blocks of the row partition, rounded up to a multiple of the 8 XCDs
// (trailing blocks may own no rows).
int32_t nblocks_for(int64_t n, int64_t rpb) {
    const int64_t nb = (n + rpb - 1) / rpb;
    return (int32_t)align_up((size_t)nb, 8);
}

// Column blocks of the marching stencil mat-vec (one thread per (y, z) column
// walking along x), or 0 where the row-partitioned kernel is used: marching
// needs enough columns to fill the chip.  KRY_STENCIL_MARCH=0/1 forces it.
int32_t march_blocks_for(const kry_system& sys) {
    if (sys.kind != KRY_STENCIL7) return 0;
    const int64_t ncol = sys.ny * sys.nz;
    const int mode = env_int("KRY_STENCIL_MARCH", -1);
    const bool use = mode >= 0 ? mode != 0 : (ncol >= (int64_t)kBlock * 1024 && sys.nx >= 64);
    if (!use) return 0;
    return (int32_t)align_up((size_t)((ncol + kBlock - 1) / kBlock), 8);
}

// Tiles of the one-pass marching stencil kernel where the marching form is
// used, else 0.
int32_t lz1_blocks_for(const kry_system& sys) {
    return march_blocks_for(sys) > 0 ? lz1_march_blocks(sys.ny, sys.nz, kMaxP) : 0;
}

constexpr int kProjGroups = 32;   // workgroups per output row in the block projection

// CSR systems of the single-vector methods read a sliced-ELL copy (see
// kry_sell.hip) unless KRY_SELL=0.
int64_t sell_nnz_for(const kry_system& sys, int32_t method) {
    if (sys.kind != KRY_CSR || method == KRY_BLOCK_ARNOLDI || sys.nnz <= 0 || sys.prepared) return 0;
    if (env_int("KRY_SELL", 1) == 0) return 0;
    return sys.nnz;
}

int max_batch_for(int o, int block_p) {
    int p = 8;
    while (p > 1 && p * (1 + o) > kMaxNV) p >>= 1;
    if (block_p > 0) {
        int b = 1;
        while (b * 2 <= block_p && b * 2 <= p) b *= 2;
        p = b;
    }
    return p;
}

struct Layout {
    size_t vec, np_part, ap_part, scal, zmat, anch, msize, scale, basis, cpart, verdict, anorm, meta, total;
    ScalLayout L;
    int64_t rpb;
    int32_t nblocks;
    int pmax;
    int32_t B, nanch;
    int32_t nvp;
    int32_t nvec;
    int32_t march;        // column blocks of the marching stencil kernel (0: row kernel)
    // block Arnoldi
    int32_t bw = 0;       // block width (generators per block run)
    int32_t brb = 0;      // row blocks of the Gram kernel
    int64_t brows = 0;    // rows per Gram row block
    size_t bvec = 0, bgpart = 0, bgpart2 = 0, bsbuf = 0, bG = 0, bcoef = 0, bH = 0, bP = 0, bR0 = 0, brfirst = 0,
           bstate = 0, bppart = 0, bS0 = 0,
           bdense = 0;
    int32_t esize;        // bytes per stored vector element: 8 (FP64) or 4 (FP32 basis)
    bool dense_runs = false;   // k > 56: each run's exponential in the dense stage
    int64_t scap = 0;          // sliced-ELL entry capacity (0: no sliced-ELL copy)
    size_t swidth = 0, soff = 0, stiles = 0, scol = 0, sval = 0;
    size_t eflags = 0;          // error control: stop flags, Gershgorin bound, Arnoldi chain sums, overflow
    size_t dH = 0, dP = 0, dS0 = 0, dws = 0;
    bool stored;          // whole basis kept (Arnoldi, or any method in FP32-basis mode)
    bool lz1 = false;     // FP64 three-vector Lanczos: room for the one-pass step (two pair buffers)
    size_t hpart, hcoef, vals32;
    size_t hpart2 = 0, sraw = 0, gram = 0, guard = 0;   // Arnoldi: the second pass from the Gram matrix
    size_t sbasis = 0;    // small FP64 Arnoldi: the persistent kernel's per-run basis
    size_t oflag = 0;     // one-pass step: per-run cancellation flags of a batch
    size_t ap_stride = 0; // doubles between the two ping-pong partial arrays of the one-pass step
    // transposed route with many initial-space rows: E^T u per step, segment
    // sums, Phi powers and anchors of the wide small stage
    size_t wpw = 0, wseg = 0, wpow = 0, wanch = 0;
};

// lz1_march: tiles of the one-pass marching stencil kernel (0 when it is not used)
Layout make_layout(int64_t n, int32_t nruns, int32_t o, int32_t k, int64_t steps, int32_t block_p,
                   size_t meta_bytes, int32_t method, int32_t march, int32_t precision, int64_t nnz32,
                   int64_t sell_nnz, int32_t lz1_march, int32_t njobs = -1, int32_t ncols = -1, int32_t o_out = -1,
                   int32_t wide_rows = 0, int64_t wide_segs = 0) {
    // the forward route has one job and one basis column per run
    if (njobs < 0) njobs = nruns;
    if (ncols < 0) ncols = nruns;
    if (o_out < 0) o_out = o;
    Layout Y{};
    Y.rpb = rows_per_block_for(n);
    Y.nblocks = nblocks_for(n, Y.rpb);
    Y.march = march;
    Y.esize = precision == KRY_FP32_BASIS ? 4 : 8;
    // Lanczos keeps its basis and reorthogonalises when it stores FP32 vectors
    // or runs past k = 56 (plain three-term Lanczos loses orthogonality there)
    Y.stored = method == KRY_ARNOLDI || precision == KRY_FP32_BASIS || (k > kMaxK && method != KRY_LANCZOS_PLAIN);
    Y.pmax = std::min(max_batch_for(o, block_p), std::max(1, nruns));
    if (Y.stored) Y.pmax = std::min(Y.pmax, 2);     // dot partials: 16 vectors x P per block
    {
        int p = 1;
        while (p * 2 <= Y.pmax) p *= 2;
        Y.pmax = p;
    }
    ScalLayout& L = Y.L;
    L.k = k;
    L.o = o;
    L.alpha = 0;
    L.beta = L.alpha + (k + 2);
    L.sigma = L.beta + (k + 2);
    L.proj = L.sigma + (k + 3);
    L.misc = L.proj + o * (k + 1);
    L.hess = L.misc + MISC_COUNT;
    // the Hessenberg store only where a basis is kept (Arnoldi, reorthogonalised Lanczos)
    L.stride = (int64_t)align_up((size_t)(L.hess + (Y.stored ? (int64_t)(k + 1) * k : 0)), 8);
    // offset 0 is reserved: an offset of 0 marks a region the plan does not have
    size_t off = 256;
    auto take = [&](size_t bytes) { size_t at = off; off = align_up(off + bytes, 256); return at; };
    // Lanczos keeps three vectors per run (Algorithm 4); Arnoldi, and every
    // method in FP32-basis mode (full reorthogonalisation), the whole basis
    if (method == KRY_BLOCK_ARNOLDI) { Y.pmax = 1; Y.stored = false; }
    // FP64 three-vector Lanczos may take the one-pass step, whose two pair
    // buffers (u_{j-1}, r_j) and (u_j, r_{j+1}) need a fourth vector
    Y.lz1 = (method == KRY_LANCZOS || method == KRY_LANCZOS_PLAIN) && !Y.stored && precision == KRY_FP64;
    Y.nvec = method == KRY_BLOCK_ARNOLDI ? 0 : (Y.stored ? k + 1 : (Y.lz1 ? 4 : 3));
    Y.vec = take((size_t)Y.nvec * n * Y.pmax * Y.esize);
    Y.hpart = Y.stored ? take((size_t)(k + 1) * kMaxP * Y.nblocks * sizeof(double)) : 0;
    Y.hcoef = Y.stored ? take((size_t)k * kMaxP * sizeof(double)) : 0;
    if (method == KRY_ARNOLDI && precision == KRY_FP64 && n <= kSmallN && k <= kSmallArnK)
        Y.sbasis = take((size_t)std::min(std::max(nruns, 1), kSmallRuns) * (k + 1) * n * sizeof(double));
    if (method == KRY_ARNOLDI) {
        Y.hpart2 = take((size_t)(k + 1) * kMaxP * Y.nblocks * sizeof(double));
        Y.sraw = take((size_t)(k + 1) * kMaxP * sizeof(double));
        Y.gram = take((size_t)kMaxP * k * k * sizeof(double));
        Y.guard = take(sizeof(int32_t));
    }
    Y.vals32 = nnz32 > 0 ? take((size_t)nnz32 * sizeof(float)) : 0;
    // sliced-ELL copy of a CSR matrix: room for the entries plus a quarter
    // for padding (and one slice's worth); a matrix that needs more keeps CSR
    if (sell_nnz > 0) {
        const int64_t ns = sell_slices(n);
        Y.scap = sell_nnz + sell_nnz / 4 + (int64_t)kSlice * 8;
        Y.swidth = take((size_t)ns * sizeof(int32_t));
        Y.soff = take((size_t)(ns + 1) * sizeof(int64_t));
        Y.stiles = take((size_t)(sell_scan_tiles(n) + 1) * sizeof(int64_t));
        Y.scol = take((size_t)Y.scap * sizeof(int32_t));
        Y.sval = take((size_t)Y.scap * (precision == KRY_FP32_BASIS ? sizeof(float) : sizeof(double)));
    }
    Y.nvp = Y.pmax * (1 + o);
    Y.np_part = take((size_t)(k + 1) * Y.nvp * Y.nblocks * sizeof(double));
    // mat-vec dot partials; the one-pass step keeps two arrays of three
    // values per run (the previous launch's and its own)
    Y.ap_stride = (size_t)std::max(Y.nblocks, lz1_march) * kMaxP * 3;
    Y.ap_part = take((Y.lz1 ? 2 * Y.ap_stride : Y.ap_stride / 3) * sizeof(double));
    Y.oflag = take(kMaxP * sizeof(double));
    Y.scal = take((size_t)nruns * L.stride * sizeof(double));
    // time steps s = b * B + r: B anchors of the Z chain, nanch of the anchor chain
    Y.B = 1;
    while ((int64_t)Y.B * Y.B < steps + 1 && Y.B < 256) Y.B <<= 1;
    Y.nanch = (int32_t)((steps + 1 + Y.B - 1) / Y.B);
    // small exponential in LDS (k <= 56) or the dense stage, one run at a time
    Y.dense_runs = method != KRY_BLOCK_ARNOLDI && k > kMaxK;
    Y.zmat = Y.dense_runs ? 0 : take((size_t)njobs * Y.B * kMaxO * kMaxK * sizeof(double));
    Y.anch = Y.dense_runs ? 0 : take((size_t)njobs * Y.nanch * kMaxK * sizeof(double));
    if (Y.dense_runs) {
        Y.dH = take((size_t)k * k * sizeof(double));
        Y.dP = take((size_t)o * k * sizeof(double));
        Y.dS0 = take((size_t)k * sizeof(double));
        Y.dws = take(dense_workspace_doubles(k, o, 1, Y.B, Y.nanch) * sizeof(double));
    }
    if (wide_rows > 0) {
        Y.wpw = take((size_t)nruns * wide_rows * k * sizeof(double));
        Y.wseg = take((size_t)k * std::max<int64_t>(wide_segs, 1) * kMaxP * sizeof(double));   // per step
        Y.wpow = take((size_t)nruns * Y.B * kMaxK1 * kMaxK1 * sizeof(double));
        Y.wanch = take((size_t)nruns * Y.nanch * kMaxK1 * sizeof(double));
    }
    Y.msize = take((size_t)std::max(njobs, nruns) * sizeof(int32_t));
    Y.scale = take((size_t)std::max(njobs, nruns) * sizeof(double));
    Y.basis = take((size_t)(steps + 1) * o_out * ncols * sizeof(double));
    Y.cpart = take((size_t)2 * check_blocks(steps, o_out) * sizeof(double));
    Y.verdict = take((size_t)(6 + ncols) * sizeof(double));
    Y.anorm = take(sizeof(double));
    // error control: stop flags, the Gershgorin bound, the Arnoldi chains'
    // sums, an overflow flag
    Y.eflags = take((kMaxP + 1 + (size_t)lemma1_hess_partials() + 1) * sizeof(double));
    if (method == KRY_BLOCK_ARNOLDI) {
        Y.bw = block_p;
        Y.brb = (int32_t)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 63) / 64));
        Y.brows = (int64_t)align_up((size_t)((n + Y.brb - 1) / Y.brb), 4);
        const int64_t m = (int64_t)kBW * k;
        Y.bvec = take((size_t)(k + 1) * n * kBW * Y.esize);
        Y.bgpart = take((size_t)(k + 1) * Y.brb * 256 * sizeof(double));
        Y.bgpart2 = take((size_t)(k + 1) * Y.brb * 256 * sizeof(double));
        Y.bsbuf = take((size_t)(k + 1) * 256 * sizeof(double));
        Y.bG = take((size_t)m * m * sizeof(double));
        Y.bcoef = take((size_t)(k + 1) * 256 * sizeof(double));
        Y.bH = take((size_t)(m + kBW) * m * sizeof(double));
        Y.bP = take((size_t)o * (m + kBW) * sizeof(double));
        Y.bR0 = take(256 * sizeof(double));
        Y.brfirst = take(256 * sizeof(double));
        Y.bstate = take(8 * sizeof(int32_t));
        Y.bppart = take((size_t)o * kProjGroups * kBW * sizeof(double));
        Y.bS0 = take((size_t)m * kBW * sizeof(double));
        Y.bdense = take(dense_workspace_doubles((int)m, o, kBW, Y.B, Y.nanch) * sizeof(double));
    }
    Y.meta = take(meta_bytes);
    Y.total = off;
    return Y;
}

kry_status check_segs(const kry_segs& s, int64_t n, const char* what) {
    if (s.nseg < 0) return fail(KRY_EINVAL, std::string(what) + ": negative segment count");
    if (s.nseg > 0 && (!s.lo || !s.hi || !s.w)) return fail(KRY_EINVAL, std::string(what) + ": NULL segment array");
    for (int64_t i = 0; i < s.nseg; ++i) {
        if (s.lo[i] < 0 || s.hi[i] > n || s.hi[i] <= s.lo[i])
            return fail(KRY_EINVAL, std::string(what) + ": segment out of range or empty");
        if (i > 0 && s.lo[i] < s.hi[i - 1])
            return fail(KRY_EINVAL, std::string(what) + ": segments not sorted and disjoint");
        if (!std::isfinite(s.w[i])) return fail(KRY_EINVAL, std::string(what) + ": non-finite segment value");
    }
    return KRY_OK;
}

// Max absolute row sum of a stencil operator: rows differ only by which
// neighbours exist, so enumerate the (up to 27) boundary classes.  Terms
// are added in ascending column order like a CSR row.
// Over the 27 classes of stencil rows (first, interior or last index in each
// dimension): the largest absolute row sum (||A||_inf) and the largest
// diagonal plus off-diagonal absolute row sum (a Gershgorin bound of the
// largest eigenvalue when A is symmetric).  The diagonal follows the face
// conditions: insulated faces return a missing neighbour's coefficient to it,
// and the last x plane adds the exchange term.
void stencil_row_bounds(const kry_system& s, double* inf_norm, double* gersh) {
    double best = 0.0, top = -INFINITY;
    const int64_t dims[3] = {s.nx, s.ny, s.nz};
    const double cf[3] = {s.cx, s.cy, s.cz};
    for (int cx = 0; cx < 3; ++cx)
        for (int cy = 0; cy < 3; ++cy)
            for (int cz = 0; cz < 3; ++cz) {
                // class c: 0 = first index, 1 = interior, 2 = last index
                const int cls[3] = {cx, cy, cz};
                bool exists = true;
                bool lo[3], hi[3];
                for (int d = 0; d < 3; ++d) {
                    const int64_t m = dims[d];
                    if (cls[d] == 1 && m < 3) exists = false;
                    if (cls[d] == 2 && m < 2) exists = false;
                    const int64_t idx = cls[d] == 0 ? 0 : (cls[d] == 1 ? 1 : m - 1);
                    lo[d] = idx > 0;
                    hi[d] = idx < m - 1;
                }
                if (!exists) continue;
                double diag = s.c0, off = 0.0;
                for (int d = 0; d < 3; ++d) {
                    if (lo[d]) off += std::fabs(cf[d]);
                    else if (s.stencil_bc == KRY_BC_INSULATED) diag += cf[d];
                    if (hi[d]) off += std::fabs(cf[d]);
                    else if (s.stencil_bc == KRY_BC_INSULATED) diag += cf[d];
                }
                if (!hi[0]) diag += s.stencil_exchange;
                best = std::max(best, std::fabs(diag) + off);
                top = std::max(top, diag + off);
            }
    if (inf_norm) *inf_norm = best;
    if (gersh) *gersh = top;
}

double stencil_inf_norm(const kry_system& s) {
    double a = 0.0;
    stencil_row_bounds(s, &a, nullptr);
    return a;
}

// Nodes and weights of the 8-point Gauss-Legendre rule on [-1, 1]: roots of
// the Legendre polynomial P_8 by Newton's method from the Chebyshev-like
// guesses cos(pi (i - 1/4) / (8 + 1/2)); w_i = 2 / ((1 - x_i^2) P_8'(x_i)^2).
void gauss_legendre8(double* x, double* w) {
    const int n = 8;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;           // P_0, P_1
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);   // P_8'(z)
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

kry_status prepare_device() {
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
        err = expm_prepare();
        if (err == hipSuccess) err = errctl_prepare();
        if (err == hipSuccess) err = wide_prepare();
        if (err == hipSuccess) err = big_prepare();
    });
    if (err != hipSuccess) return fail(KRY_EDEVICE, std::string("expm LDS setup: ") + hipGetErrorString(err));
    return KRY_OK;
}

}  // namespace

// A CSR system prepared once for many plans: sliced-ELL copy and ||A||_inf.
struct kry_matrix {
    int64_t n = 0, nnz = 0;
    const int64_t* rowptr = nullptr;
    const int32_t* colidx = nullptr;
    const double* vals = nullptr;
    int32_t precision = KRY_FP64;
    char* mem = nullptr;
    size_t bytes = 0;
    kry::SellArgs sell{};
    double* anorm_dev = nullptr;
};

struct kry_plan {
    kry_system sys{};
    int32_t ngen = 0, nruns = 0, o = 0, k = 0;
    double dt = 0.0;
    int64_t steps = 0;
    hipStream_t stream = nullptr;
    std::vector<int32_t> role;
    std::vector<double> zc, radius;
    std::vector<int32_t> gen_set;
    int32_t oset0 = 0;
    int32_t bset = -1;
    const double* center = nullptr;
    Layout Y{};
    char* ws = nullptr;
    bool owns_ws = false;
    std::vector<char> meta_host;
    SegTable T{};
    int32_t* role_dev = nullptr;   // per job of the small stage (per run on the forward route)
    double* zc_dev = nullptr;      // per basis column
    double* rad_dev = nullptr;
    // transposed route (Section 4.1): the Krylov runs start from the output
    // rows and project on the initial-space rows; the basis keeps the
    // forward shape (o_out output rows x ncols columns)
    bool transposed = false;
    // more initial-space rows than the fused projection holds: the rows of
    // E^T are sets wset0 .. wset0 + ncols - 1, their segments wseg0 ..
    // wseg0 + wnseg - 1 (kry_wide.hip)
    bool wide = false;
    int32_t wset0 = 0, wseg0 = 0, wnseg = 0;
    // launch choices forced while the tuner times them (-1: the table's or
    // the default)
    int32_t force_spmm_rows = -1, force_spmm_xcd = -1, force_march_nt = -1;
    int32_t njobs = 0;             // exponentials of the small stage
    int32_t o_out = 0, ncols = 0;  // basis shape
    std::vector<int32_t> col_role; // per basis column: 0 generator, 1 center, 2 forcing
    std::vector<int32_t> job_role, job_run, out_col;
    int32_t* job_run_dev = nullptr;
    int32_t* out_col_dev = nullptr;
    // per-step LP: inputs, per-step records and verdict (allocated on first use)
    char* lp_mem = nullptr;
    // graph mode: the projection recorded once and replayed
    bool graph_on = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<double> lp_host;
    int lpr = 1;
    int32_t method = KRY_LANCZOS;
    bool projected = false;
    std::vector<double> verdict_host;
    // block Arnoldi: per block run, k_eff (blocks), width, H (m x m), R0 (p x p), P (o x m) on the host
    struct BlockInfo {
        int32_t k_eff = 0, p = 0;
        std::vector<double> H, R0, P;
    };
    std::vector<BlockInfo> blocks;
    bool nonfinite = false;

    bool f32 = false;
    bool hess_mode = false;   // H assembled from the Hessenberg store (else alpha/beta tridiagonal)
    bool use_sell = false;    // the mat-vec reads the sliced-ELL copy
    SellArgs sell{};          // that copy: the plan's own or a prepared matrix's
    const double* anorm_dev = nullptr;   // ||A||_inf on the device (the plan's or a prepared matrix's)
    double err_eps = 0.0;     // error target of the a-posteriori k (0: fixed k)
    double* hflags = nullptr; // pinned host copy of a batch's stop flags
    int64_t onepass_batches = 0;   // batches finished by the one-pass step
    int64_t twopass_redone = 0;    // batches the one-pass step handed back (cancellation)
    hipEvent_t flag_ev = nullptr;
    double lam_plus = 0.0;    // max(0, Gershgorin bound of lambda_max of the symmetric part of A)
    // Lanczos error control past kBigFrom: eigenvalues, weights and pivots
    // of the parallel eigen-solve (allocated with the error target)
    char* big_mem = nullptr;
    BigErrArgs big{};

    void* vec(int i) { return ws + Y.vec + (size_t)i * sys.n * Y.pmax * Y.esize; }
    float* vals32() { return reinterpret_cast<float*>(ws + Y.vals32); }
    template <typename T>
    T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
    double* hpart() { return reinterpret_cast<double*>(ws + Y.hpart); }
    double* hcoef() { return reinterpret_cast<double*>(ws + Y.hcoef); }
    double* np_part() { return reinterpret_cast<double*>(ws + Y.np_part); }
    double* ap_part() { return reinterpret_cast<double*>(ws + Y.ap_part); }
    double* scal() { return reinterpret_cast<double*>(ws + Y.scal); }
    double* zmat() { return reinterpret_cast<double*>(ws + Y.zmat); }
    double* anch() { return reinterpret_cast<double*>(ws + Y.anch); }
    int32_t* msize() { return reinterpret_cast<int32_t*>(ws + Y.msize); }
    double* scale() { return reinterpret_cast<double*>(ws + Y.scale); }
    double* cpart() { return reinterpret_cast<double*>(ws + Y.cpart); }
    double* basis() { return reinterpret_cast<double*>(ws + Y.basis); }
    double* verdict() { return reinterpret_cast<double*>(ws + Y.verdict); }
    double* anorm() { return reinterpret_cast<double*>(ws + Y.anorm); }
};

namespace {

// Metadata block uploaded once per plan: segment table, per-run roles and
// box coefficients.
size_t meta_size(int64_t total_segs, int32_t nsets, int32_t nruns, int32_t nblocks, int32_t nmap = 0) {
    // nruns: entries of the role and box tables (runs, or jobs and columns of
    // the transposed route); nmap: jobs of a transposed plan's output map
    size_t b = 0;
    b = align_up(b + (size_t)nsets * nblocks * 2 * 4, 16);   // per-block segment ranges
    b = align_up(b + (size_t)total_segs * 8, 16);   // lo
    b = align_up(b + (size_t)total_segs * 8, 16);   // hi
    b = align_up(b + (size_t)total_segs * 8, 16);   // w
    b = align_up(b + (size_t)(nsets + 1) * 4, 16);  // set_begin
    b = align_up(b + (size_t)nruns * 4, 16);        // role
    b = align_up(b + (size_t)nruns * 8, 16);        // zc
    b = align_up(b + (size_t)nruns * 8, 16);        // radius
    b = align_up(b + (size_t)nmap * 4, 16);         // job -> run
    b = align_up(b + (size_t)nmap * kMaxO * 4, 16); // job row -> basis column
    return b;
}

kry_status validate_system(const kry_system* sys) {
    if (!sys) return fail(KRY_EINVAL, "system is NULL");
    if (sys->n <= 0) return fail(KRY_EINVAL, "n must be positive");
    if (sys->kind == KRY_CSR) {
        if (!sys->rowptr || !sys->colidx || !sys->vals) return fail(KRY_EINVAL, "CSR arrays must be non-NULL");
        if (sys->nnz < 0) return fail(KRY_EINVAL, "nnz must be >= 0");
        if (sys->n >= (int64_t)1 << 31) return fail(KRY_EINVAL, "CSR needs n < 2^31 (int32 column indices)");
    } else if (sys->kind == KRY_STENCIL7) {
        if (sys->nx <= 0 || sys->ny <= 0 || sys->nz <= 0 || sys->nx * sys->ny * sys->nz != sys->n)
            return fail(KRY_EINVAL, "stencil grid must satisfy nx*ny*nz == n");
        if (!std::isfinite(sys->c0) || !std::isfinite(sys->cx) || !std::isfinite(sys->cy) || !std::isfinite(sys->cz) ||
            !std::isfinite(sys->stencil_exchange))
            return fail(KRY_EINVAL, "stencil coefficients must be finite");
        if (sys->stencil_bc != KRY_BC_DIRICHLET && sys->stencil_bc != KRY_BC_INSULATED)
            return fail(KRY_EINVAL, "unknown stencil face condition");
    } else {
        return fail(KRY_EINVAL, "unknown system kind");
    }
    if (!(sys->anorm >= 0.0) || !std::isfinite(sys->anorm)) return fail(KRY_EINVAL, "anorm must be finite and >= 0");
    if (sys->prepared) {
        const kry_matrix* M = sys->prepared;
        if (sys->kind != KRY_CSR || M->n != sys->n || M->nnz != sys->nnz || M->rowptr != sys->rowptr ||
            M->colidx != sys->colidx || M->vals != sys->vals)
            return fail(KRY_EINVAL, "the prepared matrix was made from another system");
    }
    if (sys->b && sys->b_segs) return fail(KRY_EINVAL, "give the forcing as b or as b_segs, not both");
    if (sys->b_segs) {
        const kry_status st = check_segs(*sys->b_segs, sys->n, "forcing");
        if (st != KRY_OK) return st;
    }
    return KRY_OK;
}

}  // namespace

extern "C" {

const char* kry_last_error(void) { return g_err.c_str(); }

kry_status kry_plan_workspace(const kry_system* sys, int32_t nruns, int32_t o, int32_t k, int64_t steps,
                              int64_t nseg_total, int32_t precision, int32_t method, int32_t block_p,
                              size_t* bytes) {
    return guarded("kry_plan_workspace", [&]() -> kry_status {
        kry_status st = validate_system(sys);
        if (st != KRY_OK) return st;
        if (!bytes) return fail(KRY_EINVAL, "bytes is NULL");
        if (method == KRY_AUTO) method = sys->symmetric ? KRY_LANCZOS : KRY_ARNOLDI;
        const int kmax = method == KRY_BLOCK_ARNOLDI ? kMaxKB : (method == KRY_LANCZOS_PLAIN ? kMaxKP : kMaxKD);
        if (nruns < 1 || o < 1 || o > kMaxO || k < 1 || k > kmax || steps < 0 || nseg_total < 0)
            return fail(KRY_EINVAL, "nruns >= 1, 1 <= o <= 8, 1 <= k <= 512 (32 block steps), steps >= 0, "
                                    "nseg_total >= 0 required");
        if (precision != KRY_FP64 && precision != KRY_FP32_BASIS) return fail(KRY_EINVAL, "unknown precision");
        if (method == KRY_BLOCK_ARNOLDI) {
            if (block_p < 0 || block_p > kBW) return fail(KRY_EINVAL, "block Arnoldi: block_p must be <= 16");
            block_p = block_p > 0 ? block_p : std::min<int32_t>(nruns, kBW);
        }
        const int32_t nb = nblocks_for(sys->n, rows_per_block_for(sys->n));
        // one segment set per run (generators, forcing b) and per output row; a
        // center run is counted too although its dense vector has none (an upper bound)
        const int32_t nsets = nruns + o;
        const int64_t nnz32 = (precision == KRY_FP32_BASIS && sys->kind == KRY_CSR) ? sys->nnz : 0;
        const Layout Y = make_layout(sys->n, nruns, o, k, steps, block_p, meta_size(nseg_total, nsets, nruns, nb), method,
                                     march_blocks_for(*sys), precision, nnz32, sell_nnz_for(*sys, method),
                                     lz1_blocks_for(*sys));
        *bytes = Y.total;
        return KRY_OK;
    });
}

kry_status kry_footprint(const kry_system* sys, int32_t ngen, int32_t o, int32_t k, int32_t precision,
                         int32_t block_p, size_t* bytes) {
    return guarded("kry_footprint", [&]() -> kry_status {
        kry_status st = validate_system(sys);
        if (st != KRY_OK) return st;
        if (!bytes) return fail(KRY_EINVAL, "bytes is NULL");
        if (ngen < 0) return fail(KRY_EINVAL, "ngen must be >= 0");
        const int32_t nruns = ngen + ((sys->b || sys->b_segs) ? 1 : 0);
        const int64_t nseg = (int64_t)nruns + o + (sys->b_segs ? sys->b_segs->nseg : 0);
        return kry_plan_workspace(sys, nruns, o, k, 0, nseg, precision, KRY_AUTO, block_p, bytes);
    });
}

kry_status kry_footprint_transposed(const kry_system* sys_t, int32_t ngen, int32_t has_center, int32_t o,
                                    int32_t k, int64_t steps, int64_t nseg_total, int32_t precision,
                                    int32_t method, size_t* bytes) {
    return guarded("kry_footprint_transposed", [&]() -> kry_status {
        kry_status st = validate_system(sys_t);
        if (st != KRY_OK) return st;
        if (!bytes) return fail(KRY_EINVAL, "bytes is NULL");
        if (sys_t->b) return fail(KRY_ENOTSUP, "the transposed route takes the forcing as b_segs (a projection row)");
        if (method == KRY_AUTO) method = sys_t->symmetric ? KRY_LANCZOS : KRY_ARNOLDI;
        if (method != KRY_LANCZOS && method != KRY_ARNOLDI)
            return fail(KRY_ENOTSUP, "the transposed route runs Lanczos or Arnoldi");
        const bool has_b = sys_t->b_segs != nullptr;
        const int32_t nproj = ngen + (has_center ? 1 : 0) + (has_b ? 1 : 0);
        if (ngen < 0 || nproj < 1 || nproj > kMaxWide || o < 1 || o > kMaxO || k < 1 ||
            k > (has_b ? kMaxK - 1 : kMaxK) || steps < 0 || nseg_total < 0)
            return fail(KRY_EINVAL, "transposed route: 1 to 4096 initial-space rows, 1 <= o <= 8, k in [1, 56] "
                                    "([1, 55] with forcing), steps >= 0, nseg_total >= 0 required");
        if (precision != KRY_FP64 && precision != KRY_FP32_BASIS) return fail(KRY_EINVAL, "unknown precision");
        // the shapes kry_plan_create_transposed lays out: o runs projected on
        // nproj rows, one job per run plus one per run for the forcing
        // column; past 8 rows the wide stage instead (no jobs, one more set)
        const bool wide = nproj > kMaxO;
        const int32_t njobs = wide ? 0 : o * (has_b ? 2 : 1);
        const int32_t nsets = ngen + o + (has_b ? 1 : 0) + (has_center ? 1 : 0) + (wide ? 1 : 0);
        const int32_t nb = nblocks_for(sys_t->n, rows_per_block_for(sys_t->n));
        const int64_t nnz32 = (precision == KRY_FP32_BASIS && sys_t->kind == KRY_CSR) ? sys_t->nnz : 0;
        const Layout Y = make_layout(sys_t->n, o, wide ? 1 : nproj, k, steps, 0,
                                     meta_size(nseg_total, nsets, std::max(njobs, nproj), nb, njobs), method,
                                     march_blocks_for(*sys_t), precision, nnz32, sell_nnz_for(*sys_t, method),
                                     lz1_blocks_for(*sys_t), njobs, nproj, o, wide ? nproj : 0,
                                     wide ? nseg_total : 0);
        *bytes = Y.total;
        return KRY_OK;
    });
}

}  // extern "C"

namespace {

// Both routes.  Forward: one run per column of E (generators, the dense
// center, the forcing), projected on the output rows.  Transposed
// (center_t instead of center): one run of the given system, which is A^T,
// per output row, projected on the rows of E^T; the basis is scattered back
// to the forward shape.
kry_status plan_create(const kry_system* sys, const kry_gen* gens, int32_t ngen, const double* center,
                       const kry_segs* center_t, bool transposed, const kry_segs* C, int32_t o, int32_t k,
                       double dt, int64_t steps, int32_t precision, int32_t method, int32_t block_p,
                       void* workspace, size_t workspace_bytes, void* hip_stream, kry_plan_t** out) {
    if (!out) return fail(KRY_EINVAL, "out is NULL");
    *out = nullptr;
    kry_status st = validate_system(sys);
    if (st != KRY_OK) return st;
    if (ngen < 0 || (ngen > 0 && !gens)) return fail(KRY_EINVAL, "bad generator list");
    if (o < 1 || o > kMaxO || !C) return fail(KRY_EINVAL, "need 1 <= o <= 8 output rows");
    // transposed route: the initial-space rows (generators, center, b) are
    // the projection rows, at most 8; the forcing column's exponential has
    // size k + 1 and must fit the small stage
    const bool has_b = sys->b || sys->b_segs;
    const int32_t nproj = ngen + (center_t ? 1 : 0) + (has_b ? 1 : 0);
    if (transposed) {
        if (method == KRY_AUTO) method = sys->symmetric ? KRY_LANCZOS : KRY_ARNOLDI;
        if (method != KRY_LANCZOS && method != KRY_ARNOLDI)
            return fail(KRY_ENOTSUP, "the transposed route runs Lanczos or Arnoldi");
        if (sys->b) return fail(KRY_ENOTSUP, "the transposed route takes the forcing as b_segs (a projection row)");
        if (nproj < 1 || nproj > kMaxWide)
            return fail(KRY_EINVAL, "transposed route: 1 to 4096 initial-space rows (generators, center, forcing)");
        if (k < 1 || k > (has_b ? kMaxK - 1 : kMaxK))
            return fail(KRY_EINVAL, "transposed route: k must be in [1, 56] ([1, 55] with forcing)");
        if (center_t) {
            st = check_segs(*center_t, sys->n, "center");
            if (st != KRY_OK) return st;
        }
    }
    if (method == KRY_BLOCK_ARNOLDI) {
        if (k < 1 || k > kMaxKB) return fail(KRY_EINVAL, "block Arnoldi: k (block steps) must be in [1, 32]");
    } else if (method == KRY_LANCZOS_PLAIN) {
        if (k < 1 || k > kMaxKP) return fail(KRY_EINVAL, "plain Lanczos: k must be in [1, 8192]");
    } else if (k < 1 || k > kMaxKD) {
        return fail(KRY_EINVAL, "k must be in [1, 512]");
    }
    if (steps < 0) return fail(KRY_EINVAL, "steps must be >= 0");
    if (!std::isfinite(dt)) return fail(KRY_EINVAL, "dt must be finite");
    if (precision != KRY_FP64 && precision != KRY_FP32_BASIS) return fail(KRY_EINVAL, "unknown precision");
    if (sys->prepared && sys->prepared->precision != precision)
        return fail(KRY_EINVAL, "the prepared matrix holds values of another precision");
    if (method == KRY_AUTO) method = sys->symmetric ? KRY_LANCZOS : KRY_ARNOLDI;
    if (method != KRY_LANCZOS && method != KRY_ARNOLDI && method != KRY_BLOCK_ARNOLDI && method != KRY_LANCZOS_PLAIN)
        return fail(KRY_EINVAL, "unknown method");
    if ((method == KRY_LANCZOS || method == KRY_LANCZOS_PLAIN) && !sys->symmetric)
        return fail(KRY_EINVAL, "Lanczos needs a symmetric system");
    if (method == KRY_LANCZOS_PLAIN && precision != KRY_FP64)
        return fail(KRY_ENOTSUP, "plain Lanczos runs in FP64 (FP32 storage needs the reorthogonalised basis)");
    if (block_p < 0) return fail(KRY_EINVAL, "block_p must be >= 0");
    if (method == KRY_BLOCK_ARNOLDI) {
        if (sys->kind != KRY_CSR) return fail(KRY_ENOTSUP, "block Arnoldi needs a CSR system");
        if (center || sys->b || sys->b_segs)
            return fail(KRY_ENOTSUP, "block Arnoldi simulates generator columns only (no center, no forcing)");
        if (ngen < 1) return fail(KRY_EINVAL, "block Arnoldi needs at least one generator");
        if (block_p > kBW) return fail(KRY_EINVAL, "block Arnoldi: block_p must be <= 16");
        block_p = block_p > 0 ? block_p : std::min<int32_t>(ngen, kBW);
    }
    const int64_t n = sys->n;
    for (int32_t g = 0; g < ngen; ++g) {
        st = check_segs(gens[g].seg, n, "generator");
        if (st != KRY_OK) return st;
        if (!std::isfinite(gens[g].zc) || !(gens[g].radius >= 0.0) || !std::isfinite(gens[g].radius))
            return fail(KRY_EINVAL, "generator box must have finite center and radius >= 0");
    }
    for (int32_t q = 0; q < o; ++q) {
        st = check_segs(C[q], n, "output row");
        if (st != KRY_OK) return st;
    }

    st = prepare_device();
    if (st != KRY_OK) return st;
    auto* plan = new kry_plan_t();
    // the plan is destroyed on every early return and on an exception
    // (guarded() catches it at the entry point); released on success
    struct PlanGuard {
        kry_plan_t* p;
        ~PlanGuard() {
            if (p) kry_plan_destroy(p);
        }
    } guard{plan};
    plan->sys = *sys;
    plan->ngen = ngen;
    plan->k = k;
    plan->dt = dt;
    plan->steps = steps;
    plan->stream = reinterpret_cast<hipStream_t>(hip_stream);
    plan->center = center;
    plan->transposed = transposed;
    // basis columns: generators, the center, the forcing's augmented variable
    for (int32_t g = 0; g < ngen; ++g) {
        plan->col_role.push_back(0);
        plan->zc.push_back(gens[g].zc);
        plan->radius.push_back(gens[g].radius);
    }
    if (center || center_t) { plan->col_role.push_back(1); plan->zc.push_back(1.0); plan->radius.push_back(0.0); }
    if (has_b) { plan->col_role.push_back(2); plan->zc.push_back(1.0); plan->radius.push_back(0.0); }
    plan->ncols = (int32_t)plan->col_role.size();
    plan->o_out = o;
    if (plan->ncols == 0) {
        return fail(KRY_EINVAL, "nothing to simulate: no generator, center or forcing");
    }
    if (transposed && nproj > kMaxO) {
        // wide: the fused projection gets one empty row; the rows of E^T are
        // projected and exponentiated by the wide kernels
        plan->wide = true;
        plan->o = 1;
        plan->role.assign(o, 0);
        plan->nruns = o;
    } else if (transposed) {
        // one run per output row; projection row r is basis column r.  Job
        // q exponentiates run q's T for the generator and center columns;
        // with forcing, job o + q exponentiates the bordered matrix for the
        // forcing column.
        plan->o = nproj;
        plan->role.assign(o, 0);
        plan->nruns = o;
        for (int32_t q = 0; q < o; ++q) {
            plan->job_role.push_back(0);
            plan->job_run.push_back(q);
            for (int32_t r = 0; r < kMaxO; ++r)
                plan->out_col.push_back(r < nproj && plan->col_role[r] != 2 ? r : -1);
        }
        if (has_b)
            for (int32_t q = 0; q < o; ++q) {
                plan->job_role.push_back(3);
                plan->job_run.push_back(q);
                for (int32_t r = 0; r < kMaxO; ++r) plan->out_col.push_back(r == nproj - 1 ? r : -1);
            }
    } else {
        plan->o = o;
        plan->role = plan->col_role;
        plan->job_role = plan->role;
        plan->nruns = plan->ncols;
    }
    plan->njobs = (int32_t)plan->job_role.size();

    // segment table.  Forward: generator sets 0..ngen-1, output sets
    // ngen..ngen+o-1, then b.  Transposed: the output rows (start sets) come
    // first, then the projection sets: generators, center, b.
    int64_t total_segs = 0;
    for (int32_t g = 0; g < ngen; ++g) total_segs += gens[g].seg.nseg;
    for (int32_t q = 0; q < o; ++q) total_segs += C[q].nseg;
    if (sys->b_segs) total_segs += sys->b_segs->nseg;
    if (center_t) total_segs += center_t->nseg;
    if (total_segs >= ((int64_t)1 << 31)) return fail(KRY_EINVAL, "too many segments");
    const int32_t nsets = ngen + o + (sys->b_segs ? 1 : 0) + (center_t ? 1 : 0) + (plan->wide ? 1 : 0);
    int64_t wide_segs = 0;
    if (plan->wide) {
        for (int32_t g = 0; g < ngen; ++g) wide_segs += gens[g].seg.nseg;
        if (center_t) wide_segs += center_t->nseg;
        if (sys->b_segs) wide_segs += sys->b_segs->nseg;
    }
    const int64_t rpb = rows_per_block_for(n);
    const int32_t nblk = nblocks_for(n, rpb);
    const int32_t ntab = std::max(plan->njobs, plan->ncols);
    const int32_t nmap = transposed ? plan->njobs : 0;
    const size_t mbytes = meta_size(total_segs, nsets, ntab, nblk, nmap);
    const int64_t nnz32 = (precision == KRY_FP32_BASIS && sys->kind == KRY_CSR) ? sys->nnz : 0;
    plan->Y = make_layout(n, plan->nruns, plan->o, k, steps, block_p, mbytes, method, march_blocks_for(*sys),
                          precision, nnz32, sell_nnz_for(*sys, method), lz1_blocks_for(*sys), plan->njobs, plan->ncols,
                          plan->o_out, plan->wide ? plan->ncols : 0, wide_segs);
    plan->method = method == KRY_LANCZOS_PLAIN ? KRY_LANCZOS : method;   // the layout tells plain from reorthogonalised
    plan->f32 = precision == KRY_FP32_BASIS;
    plan->hess_mode = plan->Y.stored;
    const Layout& Y = plan->Y;

    if (workspace) {
        if (workspace_bytes < Y.total) {
            return fail(KRY_ENOMEM, "workspace too small: need " + std::to_string(Y.total) + " bytes");
        }
        if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) {
            return fail(KRY_EINVAL, "workspace must be 256-byte aligned");
        }
        plan->ws = static_cast<char*>(workspace);
    } else {
        void* p = nullptr;
        if (device_alloc(&p, Y.total) != hipSuccess) {
            return fail(KRY_ENOMEM, "hipMalloc of " + std::to_string(Y.total) + " bytes failed");
        }
        plan->ws = static_cast<char*>(p);
        plan->owns_ws = true;
    }

    // pack and upload metadata
    plan->meta_host.assign(mbytes, 0);
    char* base = plan->meta_host.data();
    size_t off = 0;
    auto* blk = reinterpret_cast<int32_t*>(base + off); off = align_up(off + (size_t)nsets * Y.nblocks * 2 * 4, 16);
    auto* lo = reinterpret_cast<int64_t*>(base + off); off = align_up(off + total_segs * 8, 16);
    auto* hi = reinterpret_cast<int64_t*>(base + off); off = align_up(off + total_segs * 8, 16);
    auto* w = reinterpret_cast<double*>(base + off); off = align_up(off + total_segs * 8, 16);
    auto* sb = reinterpret_cast<int32_t*>(base + off); off = align_up(off + (nsets + 1) * 4, 16);
    auto* rl = reinterpret_cast<int32_t*>(base + off); off = align_up(off + ntab * 4, 16);
    auto* zc = reinterpret_cast<double*>(base + off); off = align_up(off + ntab * 8, 16);
    auto* rd = reinterpret_cast<double*>(base + off); off = align_up(off + ntab * 8, 16);
    auto* jr = reinterpret_cast<int32_t*>(base + off); off = align_up(off + nmap * 4, 16);
    auto* oc = reinterpret_cast<int32_t*>(base + off); off = align_up(off + (size_t)nmap * kMaxO * 4, 16);
    int64_t at = 0;
    int32_t set = 0;
    auto add_set = [&](const kry_segs& s) {
        sb[set++] = (int32_t)at;
        for (int64_t i = 0; i < s.nseg; ++i, ++at) { lo[at] = s.lo[i]; hi[at] = s.hi[i]; w[at] = s.w[i]; }
    };
    plan->bset = -1;
    if (transposed) {
        for (int32_t q = 0; q < o; ++q) { plan->gen_set.push_back(set); add_set(C[q]); }
        plan->oset0 = set;
        plan->wset0 = set;
        plan->wseg0 = (int32_t)at;
        for (int32_t g = 0; g < ngen; ++g) add_set(gens[g].seg);
        if (center_t) add_set(*center_t);
        if (sys->b_segs) add_set(*sys->b_segs);
        if (plan->wide) {
            plan->wnseg = (int32_t)(at - plan->wseg0);
            plan->oset0 = set;
            sb[set++] = (int32_t)at;             // the fused projection's empty row
        }
    } else {
        for (int32_t g = 0; g < ngen; ++g) { plan->gen_set.push_back(set); add_set(gens[g].seg); }
        plan->oset0 = set;
        for (int32_t q = 0; q < o; ++q) add_set(C[q]);
        if (sys->b_segs) { plan->bset = set; add_set(*sys->b_segs); }
    }
    sb[set] = (int32_t)at;
    // per logical block b (rows [b*rpb, (b+1)*rpb)), the segments of each set
    // that overlap it: [first with hi > row0, first with lo >= row1)
    for (int32_t s = 0; s < nsets; ++s) {
        int32_t first = sb[s], last = sb[s];
        for (int32_t b = 0; b < Y.nblocks; ++b) {
            const int64_t r0 = (int64_t)b * Y.rpb;
            const int64_t r1 = std::min(n, r0 + Y.rpb);
            while (first < sb[s + 1] && hi[first] <= r0) ++first;
            if (last < first) last = first;
            while (last < sb[s + 1] && lo[last] < r1) ++last;
            blk[((int64_t)s * Y.nblocks + b) * 2] = first;
            blk[((int64_t)s * Y.nblocks + b) * 2 + 1] = r1 > r0 ? last : first;
        }
    }
    for (int32_t j = 0; j < plan->njobs; ++j) rl[j] = plan->job_role[j];
    for (int32_t c = 0; c < plan->ncols; ++c) { zc[c] = plan->zc[c]; rd[c] = plan->radius[c]; }
    for (int32_t j = 0; j < nmap; ++j) {
        jr[j] = plan->job_run[j];
        for (int32_t r = 0; r < kMaxO; ++r) oc[j * kMaxO + r] = plan->out_col[(size_t)j * kMaxO + r];
    }
    char* dmeta = plan->ws + Y.meta;
    plan->T.lo = reinterpret_cast<const int64_t*>(dmeta + ((char*)lo - base));
    plan->T.hi = reinterpret_cast<const int64_t*>(dmeta + ((char*)hi - base));
    plan->T.w = reinterpret_cast<const double*>(dmeta + ((char*)w - base));
    plan->T.set_begin = reinterpret_cast<const int32_t*>(dmeta + ((char*)sb - base));
    plan->T.blk = reinterpret_cast<const int32_t*>(dmeta + ((char*)blk - base));
    plan->role_dev = reinterpret_cast<int32_t*>(dmeta + ((char*)rl - base));
    plan->zc_dev = reinterpret_cast<double*>(dmeta + ((char*)zc - base));
    plan->rad_dev = reinterpret_cast<double*>(dmeta + ((char*)rd - base));
    if (nmap > 0) {
        plan->job_run_dev = reinterpret_cast<int32_t*>(dmeta + ((char*)jr - base));
        plan->out_col_dev = reinterpret_cast<int32_t*>(dmeta + ((char*)oc - base));
    }

    if (hipMemcpyAsync(dmeta, base, mbytes, hipMemcpyHostToDevice, plan->stream) != hipSuccess)
        return fail(KRY_EDEVICE, "metadata upload failed");

    // ||A||_inf scales the breakdown test
    plan->anorm_dev = plan->anorm();
    if (sys->prepared) {
        plan->anorm_dev = sys->prepared->anorm_dev;
    } else if (sys->anorm > 0.0 || sys->kind == KRY_STENCIL7) {
        const double a = sys->anorm > 0.0 ? sys->anorm : stencil_inf_norm(*sys);
        plan->verdict_host.assign(1, a);
        if (hipMemcpyAsync(plan->anorm(), plan->verdict_host.data(), sizeof(double), hipMemcpyHostToDevice,
                           plan->stream) != hipSuccess)
            return fail(KRY_EDEVICE, "anorm upload failed");
        if (hipStreamSynchronize(plan->stream) != hipSuccess)
            return fail(KRY_EDEVICE, "stream sync failed");
    } else {
        CsrArgs A{sys->rowptr, sys->colidx, sys->vals};
        hipError_t e = timed("row_abs_max", plan->stream, [&] {
            return launch_row_abs_max(A, n, plan->np_part(), Y.nblocks, Y.rpb, plan->anorm(), plan->stream);
        });
        if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("row_abs_max: ") + hipGetErrorString(e));
    }
    // FP32-basis mode reads an FP32 copy of the CSR values
    if (Y.scap > 0) {
        CsrArgs A{sys->rowptr, sys->colidx, sys->vals, nullptr};
        hipError_t e = timed("sell_build", plan->stream, [&] {
            return launch_sell_layout(A, n, plan->at<int32_t>(Y.swidth), plan->at<int64_t>(Y.soff),
                                      plan->at<int64_t>(Y.stiles), plan->stream);
        });
        if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("sell layout: ") + hipGetErrorString(e));
        int64_t total = 0, nwide = 0;
        if (hipMemcpyAsync(&total, plan->at<int64_t>(Y.soff) + sell_slices(n), sizeof(total), hipMemcpyDeviceToHost,
                           plan->stream) != hipSuccess ||
            hipMemcpyAsync(&nwide, plan->at<int64_t>(Y.stiles) + sell_scan_tiles(n), sizeof(nwide),
                           hipMemcpyDeviceToHost, plan->stream) != hipSuccess ||
            hipStreamSynchronize(plan->stream) != hipSuccess)
            return fail(KRY_EDEVICE, "sell layout readback failed");
        if (total <= Y.scap) {
            const bool narrow = nwide == 0 && env_int("KRY_SELL_NARROW", 1) != 0;
            e = timed("sell_build", plan->stream, [&] {
                return launch_sell_fill(plan->f32, narrow, A, n, plan->at<int64_t>(Y.soff), plan->at<int32_t>(Y.swidth),
                                        plan->ws + Y.scol, plan->ws + Y.sval, plan->stream);
            });
            if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("sell fill: ") + hipGetErrorString(e));
            plan->use_sell = true;
            plan->sell = SellArgs{plan->at<int64_t>(Y.soff), plan->at<int32_t>(Y.swidth),
                                  narrow ? nullptr : plan->at<int32_t>(Y.scol),
                                  plan->f32 ? nullptr : plan->at<double>(Y.sval),
                                  plan->f32 ? plan->at<float>(Y.sval) : nullptr,
                                  narrow ? plan->at<int16_t>(Y.scol) : nullptr, n};
        }
    }
    if (sys->prepared && method != KRY_BLOCK_ARNOLDI) {
        plan->use_sell = true;
        plan->sell = sys->prepared->sell;
    }
    if (Y.vals32 && !plan->use_sell) {
        hipError_t e = launch_to_f32(sys->vals, plan->vals32(), sys->nnz, plan->stream);
        if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("to_f32: ") + hipGetErrorString(e));
    }
    const double avg = sys->kind == KRY_CSR ? (double)sys->nnz / (double)n : 7.0;
    int lpr = env_int("KRY_LPR", 0);
    if (lpr != 1 && lpr != 2 && lpr != 4 && lpr != 8) lpr = avg > 24 ? 8 : (avg > 12 ? 4 : 1);
    plan->lpr = lpr;
    plan->sys.b_segs = nullptr;    // copied into the segment table; not kept
    guard.p = nullptr;
    *out = plan;
    return KRY_OK;
}

}  // namespace

extern "C" {

kry_status kry_plan_create(const kry_system* sys, const kry_gen* gens, int32_t ngen,
                           const double* center, const kry_segs* C, int32_t o, int32_t k,
                           double dt, int64_t steps, int32_t precision, int32_t method,
                           int32_t block_p, void* workspace, size_t workspace_bytes,
                           void* hip_stream, kry_plan_t** out) {
    return guarded("kry_plan_create", [&]() -> kry_status {
        return plan_create(sys, gens, ngen, center, nullptr, false, C, o, k, dt, steps, precision, method, block_p,
                           workspace, workspace_bytes, hip_stream, out);
    });
}

kry_status kry_plan(const kry_system* sys, const kry_gen* gens, int32_t ngen, const double* center,
                    const kry_row* C, int32_t o, int32_t k, double dt, int64_t steps, int32_t precision,
                    int32_t method, int32_t block_p, void* hip_stream, kry_plan_t** out) {
    return guarded("kry_plan", [&]() -> kry_status {
        return plan_create(sys, gens, ngen, center, nullptr, false, C, o, k, dt, steps, precision, method, block_p,
                           nullptr, 0, hip_stream, out);
    });
}

kry_status kry_plan_create_transposed(const kry_system* sys_t, const kry_gen* gens, int32_t ngen,
                                      const kry_segs* center, const kry_segs* C, int32_t o, int32_t k,
                                      double dt, int64_t steps, int32_t precision, int32_t method,
                                      void* workspace, size_t workspace_bytes, void* hip_stream,
                                      kry_plan_t** out) {
    return guarded("kry_plan_create_transposed", [&]() -> kry_status {
        if (out) *out = nullptr;
        if (!out) return fail(KRY_EINVAL, "out is NULL");
        return plan_create(sys_t, gens, ngen, nullptr, center, true, C, o, k, dt, steps, precision, method, 0,
                           workspace, workspace_bytes, hip_stream, out);
    });
}

namespace {

// Marks the basis as formed and copies it out (waits when the target is host memory).
kry_status finish_projection(kry_plan_t* plan, double* basis_out) {
    plan->projected = true;
    if (basis_out) {
        hipStream_t s = plan->stream;
        const size_t bytes = (size_t)(plan->steps + 1) * plan->o_out * plan->ncols * sizeof(double);
        hipPointerAttribute_t attr{};
        bool device_ptr = false;
        if (hipPointerGetAttributes(&attr, basis_out) == hipSuccess)
            device_ptr = attr.type == hipMemoryTypeDevice;
        else
            (void)hipGetLastError();
        KRY_HIP(hipMemcpyAsync(basis_out, plan->basis(), bytes, hipMemcpyDefault, s));
        if (!device_ptr) KRY_HIP(hipStreamSynchronize(s));
    }
    return KRY_OK;
}

// Block Arnoldi for the generator columns, bw at a time (the block form of
// Algorithm 1 with CGS2 and CholQR2), then the dense stage for each block run.
// By default the second Gram-Schmidt pass is taken from the Gram matrix of
// the stored blocks (one pass over the basis for the coefficients, one for
// the update); KRY_BLOCK_GS=0 runs both passes over the basis.
kry_status project_block(kry_plan_t* plan) {
    const Layout& Y = plan->Y;
    const int64_t n = plan->sys.n;
    hipStream_t s = plan->stream;
    const bool f32 = plan->f32;
    const int k = plan->k, o = plan->o;
    const int64_t m_max = (int64_t)kBW * k;
    const int64_t vstride = n * kBW;     // elements from one stored block to the next
    auto V = [&](int i) -> void* { return plan->ws + Y.bvec + (size_t)i * vstride * Y.esize; };
    BlockArgs B{};
    B.n = n;
    B.rb = Y.brb;
    B.rows_per_rb = Y.brows;
    const bool gs1 = env_int("KRY_BLOCK_GS", 1) != 0;
    B.gpart = plan->at<double>(Y.bgpart);
    B.gpart2 = plan->at<double>(Y.bgpart2);
    B.sbuf = plan->at<double>(Y.bsbuf);
    B.G = plan->at<double>(Y.bG);
    // a column that keeps less than 1e-3 of its norm through the projection
    // gets the plain second pass (KRY_BLOCK_REORTH2 sets the squared ratio)
    B.reorth2 = gs1 ? env_double("KRY_BLOCK_REORTH2", 1e-6) : 0.0;
    B.coef = plan->at<double>(Y.bcoef);
    B.H = plan->at<double>(Y.bH);
    B.ldh = (int32_t)m_max;
    B.P = plan->at<double>(Y.bP);
    B.ldp = (int32_t)(m_max + kBW);
    B.R0 = plan->at<double>(Y.bR0);
    B.rfirst = plan->at<double>(Y.brfirst);
    B.state = plan->at<int32_t>(Y.bstate);
    B.anorm = plan->anorm_dev;
    B.tau_scale = 1024.0 * (f32 ? 1.1920928955078125e-07 : 2.220446049250313e-16);
    {
        TuneChoice c{};
        if (plan->force_spmm_rows >= 0) {
            B.spmm_rows = plan->force_spmm_rows;
            B.spmm_xcd = plan->force_spmm_xcd;
        } else if (tune_lookup(f32 ? "bspmm32" : "bspmm", n, kBW, &c)) {
            B.spmm_rows = c.a;
            B.spmm_xcd = c.b;
        }
    }
    CsrArgs A{plan->sys.rowptr, plan->sys.colidx, plan->sys.vals, f32 ? plan->vals32() : nullptr};
    plan->blocks.clear();
    hipError_t e = hipSuccess;
#define KRY_STEP(name, call)                                                                       \
    do {                                                                                           \
        e = timed(name, s, [&] { return call; });                                                  \
        if (e != hipSuccess) return fail(KRY_EDEVICE, std::string(name) + ": " + hipGetErrorString(e)); \
    } while (0)
    for (int32_t b0 = 0; b0 < plan->ngen; b0 += Y.bw) {
        const int p = std::min<int32_t>(Y.bw, plan->ngen - b0);
        B.p = p;
        BlockStart S{};
        for (int c = 0; c < kBW; ++c) S.set[c] = c < p ? plan->gen_set[b0 + c] : -1;
        S.p = p;
        KRY_STEP("bfill", launch_fill_i32(B.state, 8, 0, s));
        KRY_STEP("bfill", launch_fill(B.H, (m_max + kBW) * m_max, 0.0, s));
        KRY_STEP("bfill", launch_fill(B.P, (int64_t)o * (m_max + kBW), 0.0, s));
        KRY_STEP("bfill", launch_fill(plan->at<double>(Y.bS0), m_max * kBW, 0.0, s));
        KRY_STEP("bstart", launch_bstart(f32, plan->T, S, V(0), n, s));
        // CholQR2 of the start block: G = V_1 R0
        for (int pass = 1; pass <= 2; ++pass) {
            KRY_STEP("bgram", launch_bgram(f32, V(0), vstride, 1, V(0), B, s));
            KRY_STEP("bgram_red", launch_bgram_red(B, 1, 0, 2, s));
            KRY_STEP("bchol", launch_bchol(B, 0, pass, s));
            KRY_STEP("bupdate", launch_bupdate(f32, V(0), vstride, 1, V(0), 0, B, s));
        }
        KRY_STEP("bproj", launch_bproj(f32, plan->T, plan->oset0, o, V(0), plan->at<double>(Y.bppart), kProjGroups, 0,
                                       B, s));
        BlockArgs Bc = B;                   // launches that run only when a second pass is wanted
        Bc.cond = B.state + 4;
        for (int j = 1; j <= k; ++j) {
            void* W = V(j);
            KRY_STEP("bspmm", launch_bspmm(f32, A, V(j - 1), W, B, s));
            if (gs1) {
                // V_i^T W, V_i^T V_j (i <= j) and W^T W in one pass (W is
                // stored right after V_j); H_{:,j} from them; the last step
                // only needs the coefficients
                KRY_STEP("bgram", launch_bgram(f32, V(0), vstride, j + 1, W, B, s, V(j - 1)));
                KRY_STEP("bgram_red", launch_bgram_red(B, j + 1, j, 3, s));
                KRY_STEP("bcorr", launch_bcorr(B, j, s));
                if (j == k) break;
                KRY_STEP("bupdate", launch_bupdate(f32, V(0), vstride, j, W, 1, B, s));
            } else {
                // CGS2 against V_1..V_j; the last step only needs the coefficients
                for (int pass = 1; pass <= 2; ++pass) {
                    KRY_STEP("bgram", launch_bgram(f32, V(0), vstride, j, W, B, s));
                    KRY_STEP("bgram_red", launch_bgram_red(B, j, j, pass - 1, s));
                    if (j < k || pass == 1) KRY_STEP("bupdate", launch_bupdate(f32, V(0), vstride, j, W, 1, B, s));
                }
                if (j == k) break;
            }
            // CholQR2: W = V_{j+1} H_{j+1,j}
            for (int pass = 1; pass <= 2; ++pass) {
                KRY_STEP("bgram", launch_bgram(f32, W, vstride, 1, W, B, s));
                KRY_STEP("bgram_red", launch_bgram_red(B, 1, j, 2, s));
                KRY_STEP("bchol", launch_bchol(B, j, pass, s));
                if (pass == 1 && gs1) {
                    // W kept too little of its norm: a plain second pass over
                    // the basis, then the first factorisation again
                    KRY_STEP("bgram", launch_bgram(f32, V(0), vstride, j, W, Bc, s));
                    KRY_STEP("bgram_red", launch_bgram_red(Bc, j, j, 1, s));
                    KRY_STEP("bupdate", launch_bupdate(f32, V(0), vstride, j, W, 1, Bc, s));
                    KRY_STEP("bgram", launch_bgram(f32, W, vstride, 1, W, Bc, s));
                    KRY_STEP("bgram_red", launch_bgram_red(Bc, 1, j, 2, s));
                    KRY_STEP("bchol", launch_bchol(Bc, j, 1, s));
                }
                KRY_STEP("bupdate", launch_bupdate(f32, W, vstride, 1, W, 0, B, s));
            }
            KRY_STEP("bproj", launch_bproj(f32, plan->T, plan->oset0, o, W, plan->at<double>(Y.bppart), kProjGroups,
                                           j, B, s));
        }
        int32_t st[4];
        KRY_HIP(hipMemcpyAsync(st, B.state, sizeof(st), hipMemcpyDeviceToHost, s));
        KRY_HIP(hipStreamSynchronize(s));
        if (st[2]) plan->nonfinite = true;
        const int keff = std::min(st[1], k);
        if (keff <= 0) return fail(KRY_ENUMERIC, "block Arnoldi: the generators of a block are linearly dependent");
        const int m = kBW * keff;
        // S0 = E_1 R0 (first 16 rows)
        KRY_HIP(hipMemcpyAsync(plan->at<double>(Y.bS0), B.R0, 256 * sizeof(double), hipMemcpyDeviceToDevice, s));
        DenseJob J{};
        J.H = B.H;
        J.ldh = B.ldh;
        J.m = m;
        J.dt = plan->dt;
        J.P = B.P;
        J.ldp = B.ldp;
        J.o = o;
        J.S0 = plan->at<double>(Y.bS0);
        J.lds0 = kBW;
        J.w = p;
        J.B = Y.B;
        J.nanch = Y.nanch;
        J.steps = plan->steps;
        J.basis = plan->basis();
        J.nruns = plan->nruns;
        J.run0 = b0;
        double hn = 0.0;
        e = timed("dense_expm", s, [&] { return dense_expm_steps(J, plan->at<double>(Y.bdense), &hn, s); });
        if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("dense stage: ") + hipGetErrorString(e));
        // keep H, R0 and P of this block run for kry_plan_block
        kry_plan_t::BlockInfo bi;
        bi.k_eff = keff;
        bi.p = p;
        std::vector<double> Hfull((size_t)m * m_max), Pfull((size_t)o * B.ldp), R0(256);
        KRY_HIP(hipMemcpyAsync(Hfull.data(), B.H, Hfull.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        KRY_HIP(hipMemcpyAsync(Pfull.data(), B.P, Pfull.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        KRY_HIP(hipMemcpyAsync(R0.data(), B.R0, 256 * sizeof(double), hipMemcpyDeviceToHost, s));
        KRY_HIP(hipStreamSynchronize(s));
        // drop the zero columns of a block narrower than 16
        const int mp = p * keff;
        bi.H.assign((size_t)mp * mp, 0.0);
        bi.P.assign((size_t)o * mp, 0.0);
        bi.R0.assign((size_t)p * p, 0.0);
        for (int a = 0; a < mp; ++a) {
            const int ra = (a / p) * kBW + a % p;
            for (int c = 0; c < mp; ++c) bi.H[(size_t)a * mp + c] = Hfull[(size_t)ra * m_max + (c / p) * kBW + c % p];
        }
        for (int q = 0; q < o; ++q)
            for (int c = 0; c < mp; ++c) bi.P[(size_t)q * mp + c] = Pfull[(size_t)q * B.ldp + (c / p) * kBW + c % p];
        for (int a = 0; a < p; ++a)
            for (int c = 0; c < p; ++c) bi.R0[(size_t)a * p + c] = R0[(size_t)a * kBW + c];
        plan->blocks.push_back(std::move(bi));
    }
#undef KRY_STEP
    return KRY_OK;
}

}  // namespace

}  // extern "C"

namespace {

// Everything kry_project_expm enqueues for the single-vector methods: the
// Krylov batches, the small stage and the assembly (and, with finish, the
// copy of the basis).
// The Krylov process of one batch by the one-pass step (kry_lz1.hip): the
// start vectors in pair layout, k launches (plus, for the marching stencil,
// the output projection of each new vector), then the tail that forms
// u_{k+1}.  Unless `capture`, it waits for the batch and reports in
// `flagged` whether a run's norm expansion cancelled.
kry_status onepass_batch(kry_plan_t* plan, const BatchArgs& B, int P, const StartSrc& src, bool capture,
                         bool* flagged) {
    const Layout& Y = plan->Y;
    hipStream_t s = plan->stream;
    double* X[2] = {static_cast<double*>(plan->vec(0)), static_cast<double*>(plan->vec(2))};
    double* ap[2] = {plan->ap_part(), plan->ap_part() + Y.ap_stride};
    const bool csr = plan->sys.kind == KRY_CSR;
    const bool march = !csr && Y.march > 0;
    const int32_t nb_step = march ? lz1_march_blocks(plan->sys.ny, plan->sys.nz, P) : Y.nblocks;
    if ((size_t)nb_step * kMaxP * 3 > Y.ap_stride) return fail(KRY_EDEVICE, "one-pass step: partial array too small");
    double* flag = plan->at<double>(Y.oflag);
    hipError_t e = launch_fill(flag, kMaxP, 1.0, s);
    if (e == hipSuccess)
        e = timed("start", s, [&] {
            return launch_start(P, plan->o, false, src, plan->T, plan->oset0, X[0], B, s);
        });
    if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("start: ") + hipGetErrorString(e));
    StencilArgs S{};
    if (!csr)
        S = StencilArgs{plan->sys.nx, plan->sys.ny, plan->sys.nz, plan->sys.c0, plan->sys.cx, plan->sys.cy,
                        plan->sys.cz, plan->sys.stencil_bc == KRY_BC_INSULATED ? 1 : 0, plan->sys.stencil_exchange};
    Lz1Args Z{};
    Z.flag = flag;
    Z.nb_in = nb_step;
    const int k = plan->k;
    int nt = 1;   // non-temporal pair stores, unless the tuner found plain ones faster here
    if (march) {
        TuneChoice c{};
        if (plan->force_march_nt >= 0) nt = plan->force_march_nt;
        else if (tune_lookup("lz1_march", plan->sys.n, P, &c)) nt = c.a;
    }
    for (int j = 1; j <= k; ++j) {
        const double* xin = X[(j - 1) & 1];
        double* xout = X[j & 1];
        Z.ap_in = ap[(j - 1) & 1];
        Z.ap_out = ap[j & 1];
        if (csr) {
            e = timed("lz1_sell", s, [&] {
                return launch_lz1_sell(P, plan->o, plan->sell, xin, xout, plan->T, plan->oset0, B, Z, j, s);
            });
        } else if (march) {
            e = timed("lz1_march", s, [&] { return launch_lz1_march(P, S, xin, xout, B, Z, j, s, nt); });
            if (e == hipSuccess && j > 1)
                e = timed("lz1_proj", s, [&] {
                    return launch_lz1_proj(P, plan->o, xout, plan->T, plan->oset0, B, j, s);
                });
        } else {
            e = timed("lz1_stencil", s, [&] {
                return launch_lz1_stencil(P, plan->o, S, xin, xout, plan->T, plan->oset0, B, Z, j, s);
            });
        }
        if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("one-pass step: ") + hipGetErrorString(e));
    }
    Z.ap_in = ap[k & 1];
    Z.ap_out = nullptr;
    e = timed("lz1_close", s, [&] { return launch_lz1_close(P, B, Z, k + 1, s); });
    if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("one-pass close: ") + hipGetErrorString(e));
    *flagged = false;
    if (capture) return KRY_OK;
    double fl[kMaxP];
    KRY_HIP(hipMemcpyAsync(fl, flag, P * sizeof(double), hipMemcpyDeviceToHost, s));
    KRY_HIP(hipStreamSynchronize(s));
    for (int p = 0; p < P; ++p) *flagged = *flagged || fl[p] == 0.0;
    return KRY_OK;
}

// capture: the launches are being recorded into a graph; the one-pass
// step's fallback is then recorded too and decided on the device (its
// kernels return at once while every run's flag holds).
kry_status enqueue_projection(kry_plan_t* plan, double* basis_out, bool finish, bool capture = false) {
    const Layout& Y = plan->Y;
    const int64_t n = plan->sys.n;
    hipStream_t s = plan->stream;
    // breakdown when beta_j <= 1024 eps ||A||_inf, eps of the precision the
    // vectors are stored in (FP32 rounding noise must not pass for a new direction)
    const double tau_scale = 1024.0 * (plan->f32 ? 1.1920928955078125e-07 : 2.220446049250313e-16);
    int32_t r0 = 0;
    // FP64 three-vector Lanczos or Arnoldi (k <= 64) of a small system: every
    // run in one launch of a persistent kernel (KRY_SMALL=0 keeps the general
    // path)
    const bool small_lz = (plan->method == KRY_LANCZOS || plan->method == KRY_LANCZOS_PLAIN) && !Y.stored;
    const bool small_arn = plan->method == KRY_ARNOLDI && Y.sbasis != 0;
    const bool small = (small_lz || small_arn) && !plan->f32 && plan->err_eps <= 0.0 && !plan->wide &&
                       n <= kSmallN && plan->o <= kMaxO &&
                       (plan->sys.kind == KRY_CSR || plan->sys.kind == KRY_STENCIL7) &&
                       env_int("KRY_SMALL", 1) != 0;
    if (small) {
        SmallArgs a{};
        a.kind = plan->sys.kind == KRY_CSR ? 0 : 1;
        a.A = CsrArgs{plan->sys.rowptr, plan->sys.colidx, plan->sys.vals, nullptr};
        if (a.kind == 1)
            a.S = StencilArgs{plan->sys.nx, plan->sys.ny, plan->sys.nz, plan->sys.c0, plan->sys.cx, plan->sys.cy,
                              plan->sys.cz, plan->sys.stencil_bc == KRY_BC_INSULATED ? 1 : 0,
                              plan->sys.stencil_exchange};
        a.n = n;
        a.o = plan->o;
        a.T = plan->T;
        a.oset0 = plan->oset0;
        a.scal = plan->scal();
        a.L = Y.L;
        a.anorm = plan->anorm_dev;
        a.tau_scale = tau_scale;
        a.center = plan->center;
        a.b = plan->sys.b;
        a.basis = small_arn ? plan->at<double>(Y.sbasis) : nullptr;
        for (r0 = 0; r0 < plan->nruns; r0 += kSmallRuns) {
            const int32_t nr = std::min<int32_t>(kSmallRuns, plan->nruns - r0);
            a.run0 = r0;
            for (int32_t i = 0; i < nr; ++i) {
                const int r = r0 + i;
                // generator segments, the center, the forcing (dense, or as segments)
                a.src[i] = plan->role[r] == 0   ? plan->gen_set[r]
                           : plan->role[r] == 1 ? -1
                           : plan->sys.b        ? -2
                                                : plan->bset;
            }
            const hipError_t e = small_arn
                                     ? timed("small_arnoldi", s, [&] { return launch_small_arnoldi(a, nr, s); })
                                     : timed("small_lanczos", s, [&] { return launch_small_lanczos(a, nr, s); });
            if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("small Krylov: ") + hipGetErrorString(e));
        }
    }
    while (r0 < plan->nruns) {
        int P = Y.pmax;
        while (P > 1 && r0 + P > plan->nruns) P >>= 1;
        BatchArgs B{};
        B.n = n;
        B.rows_per_block = Y.rpb;
        B.nblocks = Y.nblocks;
        B.xcd_map = env_int("KRY_XCD_MAP", 1) != 0 ? 1 : 0;
        B.run0 = r0;
        B.scal = plan->scal();
        B.L = Y.L;
        B.np_part = plan->np_part();
        B.nvp = Y.nvp;
        B.ap_part = plan->ap_part();
        B.ap_nblocks = Y.march > 0 ? Y.march : Y.nblocks;
        B.anorm = plan->anorm_dev;
        B.tau_scale = tau_scale;
        StartSrc src{};
        for (int p = 0; p < kMaxP; ++p) { src.dense[p] = nullptr; src.set[p] = -1; }
        for (int p = 0; p < P; ++p) {
            const int r = r0 + p;
            if (plan->role[r] == 0) src.set[p] = plan->gen_set[r];
            else if (plan->role[r] == 1) src.dense[p] = plan->center;
            else if (plan->sys.b) src.dense[p] = plan->sys.b;
            else src.set[p] = plan->bset;
        }
        const bool f32 = plan->f32;
        const bool lanczos = plan->method == KRY_LANCZOS;
        // Arnoldi takes its second Gram-Schmidt pass from the Gram matrix on
        // systems of 2^16 rows or more (below, a step is bound by launches,
        // which this form has more of); KRY_ARN_GS=1 / 0 forces it on / off.
        // A run whose w keeps less than 1e-3 of its norm through the
        // projection gets the plain second pass (KRY_ARN_REORTH2: the squared
        // ratio).
        const int arn_gs = env_int("KRY_ARN_GS", -1);
        const bool arn_gram = plan->method == KRY_ARNOLDI && Y.gram != 0 &&
                              (arn_gs == 1 || (arn_gs != 0 && plan->sys.n >= 65536));
        const double arn_reorth2 = env_double("KRY_ARN_REORTH2", 1e-6);
        // FP64 three-vector Lanczos on a stencil takes the one-pass step; a
        // batch in which a run's norm expansion cancelled is computed again
        // two-pass.  On a CSR matrix the step gathers two vectors per entry
        // instead of one, which measured slower than the two launches on the
        // 100^3 system (whose working set sits in the MALL), so it is used
        // there only on request (KRY_ONEPASS=1; 0 turns it off everywhere).
        const int op_mode = env_int("KRY_ONEPASS", -1);
        const bool onepass = Y.lz1 && lanczos && plan->err_eps <= 0.0 && op_mode != 0 && !plan->wide &&
                             (plan->sys.kind == KRY_STENCIL7 || (plan->use_sell && op_mode == 1));
        const BatchArgs B_fin = B;           // the finishing kernel never reads stop flags here
        if (onepass) {
            bool flagged = false;
            const kry_status st = onepass_batch(plan, B, P, src, capture, &flagged);
            if (st != KRY_OK) return st;
            if (!capture && !flagged) {
                hipError_t ef = timed("finish", s, [&] { return launch_finish(P, plan->o, B, plan->k, s); });
                if (ef != hipSuccess) return fail(KRY_EDEVICE, std::string("finish: ") + hipGetErrorString(ef));
                plan->onepass_batches += 1;
                r0 += P;
                continue;
            }
            if (capture) B.stop = plan->at<double>(Y.oflag);   // the fallback runs only where a flag was cleared
            else plan->twopass_redone += 1;
        }
        hipError_t e = timed("start", s, [&] {
            return launch_start(P, plan->o, f32, src, plan->T, plan->oset0, plan->vec(0), B, s);
        });
        if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("start: ") + hipGetErrorString(e));
        // wide transposed plan: E^T u_{j+1} once u_{j+1} is formed (j = 0: the start)
        auto wide_proj = [&](const void* x, int j) {
            return timed("wide_proj", s, [&] {
                return launch_wide_proj(P, f32, x, plan->T, plan->wseg0, plan->wnseg, plan->at<double>(Y.wseg), j, s);
            });
        };
        if (plan->wide) {
            e = wide_proj(plan->vec(0), 0);
            if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("wide projection: ") + hipGetErrorString(e));
        }
        int next_check = 4;
        bool poll_pending = false;
        ErrArgs X{};
        if (plan->err_eps > 0.0) {
            X.role = plan->role_dev;
            X.tau = (double)plan->steps * plan->dt;
            X.lam_plus = plan->lam_plus;
            X.eps = plan->err_eps;
            gauss_legendre8(X.gl_x, X.gl_w);
            X.flags = plan->at<double>(Y.eflags);
            X.hess = plan->hess_mode ? 1 : 0;
            B.stop = X.flags;
            e = launch_fill(X.flags, kMaxP, 0.0, s);
            if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("error control: ") + hipGetErrorString(e));
        }
        for (int j = 1; j <= plan->k; ++j) {
            // FP64 Lanczos rotates three vectors (Algorithm 4); otherwise u_1..u_{k+1} are kept
            void* ucur = Y.stored ? plan->vec(j - 1) : plan->vec((j - 1) % 3);
            void* uprev = !lanczos ? nullptr : (Y.stored ? (j >= 2 ? plan->vec(j - 2) : nullptr)
                                                         : plan->vec((j + 1) % 3));   // (j - 2) mod 3
            void* w = Y.stored ? plan->vec(j) : plan->vec(j % 3);
            if (plan->sys.kind == KRY_CSR) {
                if (plan->use_sell) {
                    const SellArgs& A = plan->sell;
                    e = timed("spmv_sell", s, [&] { return launch_spmv_sell(P, f32, A, ucur, uprev, w, B, j, s); });
                } else {
                    CsrArgs A{plan->sys.rowptr, plan->sys.colidx, plan->sys.vals, f32 ? plan->vals32() : nullptr};
                    e = timed("spmv_csr", s, [&] {
                        return launch_spmv_csr(P, plan->lpr, f32, A, ucur, uprev, w, B, j, s);
                    });
                }
            } else {
                StencilArgs A{plan->sys.nx, plan->sys.ny, plan->sys.nz, plan->sys.c0, plan->sys.cx,
                              plan->sys.cy, plan->sys.cz, plan->sys.stencil_bc == KRY_BC_INSULATED ? 1 : 0,
                              plan->sys.stencil_exchange};
                e = timed("spmv_stencil", s, [&] {
                    return launch_spmv_stencil(P, Y.march > 0, f32, A, ucur, uprev, w, B, j, s);
                });
            }
            if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("spmv: ") + hipGetErrorString(e));
            if (lanczos) {
                e = timed("sweep", s, [&] {
                    return launch_sweep(P, plan->o, f32, plan->T, plan->oset0, ucur, w, B, j, s);
                });
                if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("sweep: ") + hipGetErrorString(e));
            }
            if (!lanczos && arn_gram) {
                // Arnoldi with the second pass from the Gram matrix: u_i . w,
                // u_i . u_j (i <= j) and w . w in one pass (w is stored right
                // after u_j), H_{:,j} = S - (V^T V - I) S, one update; a plain
                // second pass follows only for a run whose w kept too little
                // of its norm (the guard)
                ArnArgs Ar{plan->vec(0), n * Y.pmax, w, plan->hpart(), plan->hcoef(), f32 ? 1 : 0, 0};
                Ar.hpart2 = plan->at<double>(Y.hpart2);
                Ar.sraw = plan->at<double>(Y.sraw);
                Ar.gram = plan->at<double>(Y.gram);
                Ar.guard = plan->at<int32_t>(Y.guard);
                Ar.reorth2 = arn_reorth2;
                e = timed("arn_dots", s, [&] { return launch_arn_dots(P, Ar, B, j, s, j + 1, true); });
                if (e == hipSuccess) e = timed("arn_reduce", s, [&] { return launch_arn_reduce(P, Ar, B, j, 3, s); });
                if (e == hipSuccess) e = timed("arn_corr", s, [&] { return launch_arn_corr(P, Ar, B, j, s); });
                if (e == hipSuccess)
                    e = timed("arn_update", s, [&] {
                        return launch_arn_update(P, plan->o, plan->T, plan->oset0, Ar, B, j, 1, s);
                    });
                if (e == hipSuccess) e = timed("arn_guard", s, [&] { return launch_arn_guard(P, Ar, B, j, s); });
                ArnArgs Ac = Ar;
                Ac.conditional = 1;
                if (e == hipSuccess) e = timed("arn_dots", s, [&] { return launch_arn_dots(P, Ac, B, j, s); });
                if (e == hipSuccess) e = timed("arn_reduce", s, [&] { return launch_arn_reduce(P, Ac, B, j, 2, s); });
                if (e == hipSuccess)
                    e = timed("arn_update", s, [&] {
                        return launch_arn_update(P, plan->o, plan->T, plan->oset0, Ac, B, j, 1, s);
                    });
                if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("arnoldi: ") + hipGetErrorString(e));
            } else if (Y.stored || !lanczos) {
                // Arnoldi: CGS2 against u_1..u_j (Algorithm 1's projection loop, classical
                // form, twice).  Lanczos with a stored basis: one classical pass over the
                // three-term result removes what rounding left along u_1..u_j.
                ArnArgs Ar{plan->vec(0), n * Y.pmax, w, plan->hpart(), plan->hcoef(), f32 ? 1 : 0, lanczos ? 1 : 0};
                const int passes = lanczos ? 1 : 2;
                for (int pass = 1; pass <= passes; ++pass) {
                    e = timed("arn_dots", s, [&] { return launch_arn_dots(P, Ar, B, j, s); });
                    if (e == hipSuccess)
                        e = timed("arn_reduce", s, [&] { return launch_arn_reduce(P, Ar, B, j, pass, s); });
                    if (e == hipSuccess)
                        e = timed("arn_update", s, [&] {
                            return launch_arn_update(P, plan->o, plan->T, plan->oset0, Ar, B, j,
                                                     pass == passes ? 1 : 0, s);
                        });
                    if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("arnoldi: ") + hipGetErrorString(e));
                }
            }
            if (plan->wide && j < plan->k) {
                e = wide_proj(w, j);
                if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("wide projection: ") + hipGetErrorString(e));
            }
            // Algorithms 2 and 4: check the error bound at k = 4, then ceil(1.1 k)
            // with 1.1 k a double product, as printed (170 is followed by 188).
            // Once every run of the batch met the target, the kernels of the
            // iterations already queued return at once (B.stop); the host
            // stops queueing when a non-blocking look at the flags of an
            // earlier checkpoint finds them all set.
            if (plan->err_eps > 0.0 && j == next_check) {
                next_check = (int)std::ceil(1.1 * (double)next_check);
                e = timed("errctl", s, [&] { return launch_record_stage(P, B, j, s); });
                const bool big = lanczos && plan->big_mem &&
                                 (j > kBigFrom || env_int("KRY_ERRCTL_BIG", 0) == 1);
                if (e == hipSuccess) e = timed("errctl", s, [&] {
                    if (big) return launch_lemma1_big(P, B, X, j, plan->big, s);
                    return lanczos ? launch_lemma1(P, B, X, j, s)
                                   : launch_lemma1_hess(P, B, X, j, X.flags + kMaxP + 1, s);
                });
                if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("error control: ") + hipGetErrorString(e));
                if (poll_pending && hipEventQuery(plan->flag_ev) == hipSuccess) {
                    poll_pending = false;
                    bool all = true;
                    for (int p = 0; p < P; ++p) all = all && plan->hflags[p] != 0.0;
                    if (all) break;
                }
                if (!poll_pending) {
                    KRY_HIP(hipMemcpyAsync(plan->hflags, X.flags, P * sizeof(double), hipMemcpyDeviceToHost, s));
                    KRY_HIP(hipEventRecord(plan->flag_ev, s));
                    poll_pending = true;
                }
            }
        }
        // with error control the finishing kernel takes the batch's Krylov
        // dimension from the device (the largest stop of its runs)
        e = timed("finish", s, [&] { return launch_finish(P, plan->o, onepass ? B_fin : B, plan->k, s); });
        if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("finish: ") + hipGetErrorString(e));
        if (plan->wide) {
            e = timed("wide_sets", s, [&] {
                return launch_wide_sets(P, plan->T, plan->wset0, plan->ncols, plan->wseg0, plan->wnseg,
                                        plan->at<double>(Y.wseg), plan->at<double>(Y.wpw), r0, P, plan->ncols, plan->k,
                                        plan->k, s);
            });
            if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("wide projection: ") + hipGetErrorString(e));
        }
        r0 += P;
    }
    if (plan->wide) {
        WideArgs W{};
        W.scal = plan->scal();
        W.L = Y.L;
        W.Pw = plan->at<double>(Y.wpw);
        W.ncw = plan->ncols;
        W.ldk = plan->k;
        W.forcing = plan->col_role.back() == 2 ? 1 : 0;
        W.bcol = plan->ncols - 1;
        W.hess = plan->hess_mode ? 1 : 0;
        W.dt = plan->dt;
        W.B = Y.B;
        W.nanch = Y.nanch;
        W.pow = plan->at<double>(Y.wpow);
        W.anch = plan->at<double>(Y.wanch);
        W.basis = plan->basis();
        W.o_out = plan->o_out;
        W.ncols = plan->ncols;
        hipError_t e = timed("wide_stage", s, [&] { return launch_wide_stage(W, plan->nruns, plan->steps, s); });
        if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("wide stage: ") + hipGetErrorString(e));
        return finish ? finish_projection(plan, basis_out) : KRY_OK;
    }
    ExpmArgs E{};
    E.scal = plan->scal();
    E.L = Y.L;
    E.role = plan->role_dev;
    E.job_run = plan->job_run_dev;
    E.dt = plan->dt;
    E.hess_mode = plan->hess_mode ? 1 : 0;
    E.B = Y.B;
    E.nanch = Y.nanch;
    if (Y.dense_runs) {
        // sizes of the runs' matrices decide the dense stage's shapes
        std::vector<double> sc((size_t)plan->nruns * Y.L.stride);
        KRY_HIP(hipMemcpyAsync(sc.data(), plan->scal(), sc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        KRY_HIP(hipStreamSynchronize(s));
        for (int32_t run = 0; run < plan->nruns; ++run) {
            const double* msc = sc.data() + (size_t)run * Y.L.stride + Y.L.misc;
            const int keff = std::min((int)msc[MISC_KEFF], (int)msc[MISC_KSTOP]);
            const bool bordered = plan->role[run] == 2;
            int m = bordered ? std::min(keff, plan->k - 1) + 1 : keff;
            if (keff <= 0) m = 0;
            hipError_t e = hipSuccess;
            if (m > 0) e = launch_build_dense(E, run, m, plan->at<double>(Y.dH), plan->at<double>(Y.dP),
                                              plan->at<double>(Y.dS0), s);
            if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("build_dense: ") + hipGetErrorString(e));
            DenseJob J{};
            J.H = plan->at<double>(Y.dH);
            J.ldh = m;
            J.m = m;
            J.dt = plan->dt;
            J.P = plan->at<double>(Y.dP);
            J.ldp = m;
            J.o = plan->o;
            J.S0 = plan->at<double>(Y.dS0);
            J.lds0 = 1;
            J.w = 1;
            J.B = Y.B;
            J.nanch = Y.nanch;
            J.steps = plan->steps;
            J.basis = plan->basis();
            J.nruns = plan->nruns;
            J.run0 = run;
            J.nonfinite = msc[MISC_NONFINITE] != 0.0 ? 1 : 0;
            double hn = 0.0;
            e = timed("dense_expm", s, [&] { return dense_expm_steps(J, plan->at<double>(Y.dws), &hn, s); });
            if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("dense stage: ") + hipGetErrorString(e));
        }
        return finish ? finish_projection(plan, basis_out) : KRY_OK;
    }
    E.Z = plan->zmat();
    E.anch = plan->anch();
    E.msize = plan->msize();
    E.scale = plan->scale();
    hipError_t e = timed("expm_chain", s, [&] { return launch_expm_chain(E, plan->njobs, s); });
    if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("expm_chain: ") + hipGetErrorString(e));
    AssembleArgs A{plan->zmat(), plan->anch(), plan->msize(), plan->scale(), plan->njobs, plan->o,
                   Y.B, Y.nanch, plan->steps, plan->basis(), plan->job_run_dev, plan->out_col_dev,
                   plan->o_out, plan->ncols};
    e = timed("assemble", s, [&] { return launch_assemble(A, s); });
    if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("assemble: ") + hipGetErrorString(e));
    return finish ? finish_projection(plan, basis_out) : KRY_OK;
}

}  // namespace

// The one-call entry point that allocates nothing keeps its plan workspace
// in this fixed array.  Each device holds its own copy for the life of the
// process; host code only ever uses the address that hipGetSymbolAddress
// returns for the current device (the array's name is a host-side stand-in).
static __device__ __align__(256) unsigned char scratch[KRY_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

// The device address of `scratch` on the current device, looked up once per
// device with that device current.
// The box check of the columns and rows C names (sizes and maps set by the
// caller): launch, verdict to the host, counter-example of the generator
// columns among `cols` (plan column indices, in order).
kry_status run_check(kry_plan_t* plan, CheckArgs& C, const int32_t* cols, const kry_interval* unsafe,
                     kry_verdict* out, double* z_out) {
    C.basis = plan->basis();
    C.zc = plan->zc_dev;
    C.radius = plan->rad_dev;
    for (int q = 0; q < C.o; ++q) {
        if (std::isnan(unsafe[q].lo) || std::isnan(unsafe[q].hi)) return fail(KRY_EINVAL, "unsafe interval is NaN");
        C.ulo[q] = unsafe[q].lo;
        C.uhi[q] = unsafe[q].hi;
    }
    C.part = plan->cpart();
    C.verdict = plan->verdict();
    hipError_t e = timed("check", plan->stream, [&] { return launch_check(C, plan->stream); });
    if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("check: ") + hipGetErrorString(e));
    plan->verdict_host.assign(6 + C.nruns, 0.0);
    KRY_HIP(hipMemcpyAsync(plan->verdict_host.data(), plan->verdict(), plan->verdict_host.size() * sizeof(double),
                           hipMemcpyDeviceToHost, plan->stream));
    KRY_HIP(hipStreamSynchronize(plan->stream));
    const double* v = plan->verdict_host.data();
    out->first_step = (int64_t)v[0];
    out->row = (int32_t)v[1];
    out->y = v[2];
    out->lo = v[3];
    out->hi = v[4];
    out->status = (int32_t)v[5];
    if (plan->nonfinite) out->status = KRY_ENUMERIC;
    if (z_out) {
        int32_t g = 0;
        for (int32_t r = 0; r < C.nruns; ++r)
            if (plan->col_role[cols[r]] == 0) z_out[g++] = v[6 + r];
    }
    return KRY_OK;
}

kry_status scratch_address(void** out) {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = -1;
    KRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(KRY_EDEVICE, "device ordinal out of range for the scratch table");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        KRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(KRY_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        addr[dev] = p;
    }
    *out = addr[dev];
    return KRY_OK;
}

}  // namespace

extern "C" {

kry_status kry_project_expm(kry_plan_t* plan, double* basis_out) {
    return guarded("kry_project_expm", [&]() -> kry_status {
        if (!plan) return fail(KRY_EINVAL, "plan is NULL");
        if (plan->method == KRY_BLOCK_ARNOLDI) {
            kry_status st = project_block(plan);
            if (st != KRY_OK) return st;
            return finish_projection(plan, basis_out);
        }
        if (plan->graph_on) {
            // first call: record the whole projection as one graph; then replay it
            if (!plan->graph_exec) {
                if (prof().on) return fail(KRY_ENOTSUP, "kernel timing and graph capture exclude each other");
                KRY_HIP(hipStreamBeginCapture(plan->stream, hipStreamCaptureModeThreadLocal));
                const kry_status st = enqueue_projection(plan, nullptr, false, true);
                hipGraph_t g = nullptr;
                const hipError_t ec = hipStreamEndCapture(plan->stream, &g);
                if (st != KRY_OK || ec != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    if (st != KRY_OK) return st;
                    return fail(KRY_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
                }
                hipGraphExec_t x = nullptr;
                const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
                if (ei != hipSuccess) {
                    (void)hipGraphDestroy(g);
                    return fail(KRY_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
                }
                plan->graph = g;
                plan->graph_exec = x;
            }
            KRY_HIP(hipGraphLaunch(plan->graph_exec, plan->stream));
            return finish_projection(plan, basis_out);
        }
        return enqueue_projection(plan, basis_out, true);
    });
}

kry_status kry_check_box_safety(kry_plan_t* plan, const kry_interval* unsafe, kry_verdict* out, double* z_out) {
    return guarded("kry_check_box_safety", [&]() -> kry_status {
        if (!plan || !unsafe || !out) return fail(KRY_EINVAL, "plan, unsafe and out must be non-NULL");
        if (!plan->projected) return fail(KRY_EINVAL, "kry_project_expm must run first");
        CheckArgs C{};
        C.nruns = plan->ncols;
        C.o = plan->o_out;
        C.steps = plan->steps;
        std::vector<int32_t> cols(plan->ncols);
        for (int32_t c = 0; c < plan->ncols; ++c) cols[c] = c;
        return run_check(plan, C, cols.data(), unsafe, out, z_out);
    });
}

kry_status kry_check_box_subset(kry_plan_t* plan, const int32_t* cols, int32_t ncols, const int32_t* rows,
                                int32_t nrows, int64_t steps, const kry_interval* unsafe, kry_verdict* out,
                                double* z_out) {
    return guarded("kry_check_box_subset", [&]() -> kry_status {
        if (!plan || !cols || !rows || !unsafe || !out)
            return fail(KRY_EINVAL, "plan, cols, rows, unsafe and out must be non-NULL");
        if (!plan->projected) return fail(KRY_EINVAL, "kry_project_expm must run first");
        if (ncols < 1 || ncols > kMaxCheckCols || ncols > plan->ncols)
            return fail(KRY_EINVAL, "ncols must be in [1, min(64, the plan's basis columns)]");
        if (nrows < 1 || nrows > plan->o_out) return fail(KRY_EINVAL, "nrows must be in [1, the plan's output rows]");
        if (steps < 0 || steps > plan->steps) return fail(KRY_EINVAL, "steps must be in [0, the plan's steps]");
        std::vector<char> seen(plan->ncols, 0);
        for (int32_t c = 0; c < ncols; ++c) {
            if (cols[c] < 0 || cols[c] >= plan->ncols || seen[cols[c]])
                return fail(KRY_EINVAL, "cols must be distinct basis columns of the plan");
            seen[cols[c]] = 1;
        }
        for (int32_t q = 0; q < nrows; ++q)
            if (rows[q] < 0 || rows[q] >= plan->o_out) return fail(KRY_EINVAL, "rows must be output rows of the plan");
        CheckArgs C{};
        C.nruns = ncols;
        C.o = nrows;
        C.steps = steps;
        C.mapped = 1;
        C.o_all = plan->o_out;
        C.n_all = plan->ncols;
        for (int32_t q = 0; q < nrows; ++q) C.row_of[q] = rows[q];
        for (int32_t c = 0; c < ncols; ++c) C.col_of[c] = cols[c];
        return run_check(plan, C, cols, unsafe, out, z_out);
    });
}

kry_status kry_verify_noalloc(const kry_system* sys, const kry_gen* gens, int32_t ngen, const double* center,
                              const kry_segs* C, int32_t o, int32_t k, double dt, int64_t steps, int32_t precision,
                              int32_t method, int32_t block_p, const kry_interval* unsafe, double* basis_out,
                              kry_verdict* verdict, double* z_out, void* hip_stream) {
    return guarded("kry_verify_noalloc", [&]() -> kry_status {
        if (!unsafe || !verdict) return fail(KRY_EINVAL, "unsafe and verdict must be non-NULL");
        void* ws = nullptr;
        kry_status st = scratch_address(&ws);
        if (st != KRY_OK) return st;
        // plan_create checks the sizes against the scratch array before any
        // device work (KRY_ENOMEM naming the bytes needed when they exceed it)
        kry_plan_t* plan = nullptr;
        st = plan_create(sys, gens, ngen, center, nullptr, false, C, o, k, dt, steps, precision, method, block_p, ws,
                         (size_t)KRY_NOALLOC_SCRATCH_BYTES, hip_stream, &plan);
        if (st != KRY_OK) return st;
        st = kry_project_expm(plan, basis_out);
        if (st == KRY_OK) st = kry_check_box_safety(plan, unsafe, verdict, z_out);
        // the plan's host state goes; the scratch array keeps its contents
        (void)hipStreamSynchronize(plan->stream);
        delete plan;
        return st;
    });
}

kry_status kry_check_lp_safety(kry_plan_t* plan, const double* G, const double* h, int32_t mI, const double* U,
                               const double* u, int32_t mU, int64_t* first_step, int32_t* status, double* z_out,
                               double* y_out, int32_t* step_flags) {
    return guarded("kry_check_lp_safety", [&]() -> kry_status {
        if (!plan || !first_step || !status) return fail(KRY_EINVAL, "plan, first_step and status must be non-NULL");
        if (!plan->projected) return fail(KRY_EINVAL, "kry_project_expm must run first");
        const int32_t d = plan->ngen, o = plan->o_out;
        if (d > kLpMaxD) return fail(KRY_ENOTSUP, "the per-step LP holds at most 16 generators");
        if (mI < 0 || mU < 0 || d + mI + mU > kLpMaxRows)
            return fail(KRY_EINVAL, "need mI, mU >= 0 and generators + mI + mU <= 64 rows");
        if ((mI > 0 && (!G || !h)) || (mU > 0 && (!U || !u))) return fail(KRY_EINVAL, "G, h, U, u must be non-NULL");
        auto finite = [](const double* a, int64_t cnt) {
            for (int64_t i = 0; i < cnt; ++i)
                if (!std::isfinite(a[i])) return false;
            return true;
        };
        if (!finite(G, (int64_t)mI * d) || !finite(h, mI) || !finite(U, (int64_t)mU * o) || !finite(u, mU))
            return fail(KRY_EINVAL, "LP constraints must be finite");
        hipStream_t s = plan->stream;
        const int64_t nin = 2 * kLpMaxD + (int64_t)kLpMaxRows * kLpMaxD + kLpMaxRows + (int64_t)kLpMaxRows * kMaxO +
                            kLpMaxRows;
        const int64_t nrec = (plan->steps + 1) * kLpRec;
        const int64_t nver = 2 + kLpMaxD + kMaxO;
        if (!plan->lp_mem) {
            void* p = nullptr;
            if (device_alloc(&p, (size_t)(nin + nrec + nver) * sizeof(double)) != hipSuccess)
                return fail(KRY_ENOMEM, "LP buffers: hipMalloc failed");
            plan->lp_mem = static_cast<char*>(p);
        }
        double* dev = reinterpret_cast<double*>(plan->lp_mem);
        // inputs: zlo, zhi, G, h, U, u
        std::vector<double>& H = plan->lp_host;
        H.assign((size_t)nin, 0.0);
        for (int32_t j = 0; j < d; ++j) {
            H[j] = plan->zc[j] - plan->radius[j];
            H[kLpMaxD + j] = plan->zc[j] + plan->radius[j];
        }
        double* hG = H.data() + 2 * kLpMaxD;
        double* hh = hG + (int64_t)kLpMaxRows * kLpMaxD;
        double* hU = hh + kLpMaxRows;
        double* hu = hU + (int64_t)kLpMaxRows * kMaxO;
        if (mI > 0) { std::copy(G, G + (int64_t)mI * d, hG); std::copy(h, h + mI, hh); }
        if (mU > 0) { std::copy(U, U + (int64_t)mU * o, hU); std::copy(u, u + mU, hu); }
        KRY_HIP(hipMemcpyAsync(dev, H.data(), (size_t)nin * sizeof(double), hipMemcpyHostToDevice, s));
        LpArgs L{};
        L.basis = plan->basis();
        L.o = o;
        L.ncols = plan->ncols;
        L.d = d;
        L.mI = mI;
        L.mU = mU;
        L.steps = plan->steps;
        L.zlo = dev;
        L.zhi = dev + kLpMaxD;
        L.G = dev + (hG - H.data());
        L.h = dev + (hh - H.data());
        L.U = dev + (hU - H.data());
        L.u = dev + (hu - H.data());
        L.tol = 1e-6;      // the LP tolerance of Section 4.2, on rows scaled to a largest coefficient of 1
        L.max_pivots = 20 * (d + mI + mU + 2) + 100;
        L.rec = dev + nin;
        L.verdict = dev + nin + nrec;
        hipError_t e = timed("lp", s, [&] { return launch_lp(L, s); });
        if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("lp: ") + hipGetErrorString(e));
        double v[2 + kLpMaxD + kMaxO];
        KRY_HIP(hipMemcpyAsync(v, L.verdict, sizeof(v), hipMemcpyDeviceToHost, s));
        std::vector<double> rec;
        if (step_flags) {
            rec.resize((size_t)nrec);
            KRY_HIP(hipMemcpyAsync(rec.data(), L.rec, (size_t)nrec * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        KRY_HIP(hipStreamSynchronize(s));
        *first_step = (int64_t)v[0];
        *status = (int32_t)v[1];
        if (z_out) std::copy(v + 2, v + 2 + d, z_out);
        if (y_out) std::copy(v + 2 + kLpMaxD, v + 2 + kLpMaxD + o, y_out);
        if (step_flags)
            for (int64_t st = 0; st <= plan->steps; ++st) step_flags[st] = (int32_t)rec[(size_t)st * kLpRec];
        return KRY_OK;
    });
}

kry_status kry_plan_set_graph(kry_plan_t* plan, int32_t on) {
    return guarded("kry_plan_set_graph", [&]() -> kry_status {
        if (!plan) return fail(KRY_EINVAL, "plan is NULL");
        if (on) {
            if (plan->method == KRY_BLOCK_ARNOLDI)
                return fail(KRY_ENOTSUP, "graph mode covers the single-vector methods (block runs read sizes back)");
            if (plan->Y.dense_runs)
                return fail(KRY_ENOTSUP, "graph mode covers k <= 56 (the dense stage reads sizes back)");
            if (plan->err_eps > 0.0)
                return fail(KRY_ENOTSUP, "the error control polls the device between launches: not in graph mode");
            if (plan->stream == nullptr) return fail(KRY_EINVAL, "graph capture needs a stream other than the default one");
        }
        plan->graph_on = on != 0;
        if (!plan->graph_on) {
            if (plan->graph_exec) {
                KRY_HIP(hipStreamSynchronize(plan->stream));
                (void)hipGraphExecDestroy(plan->graph_exec);
                plan->graph_exec = nullptr;
            }
            if (plan->graph) {
                (void)hipGraphDestroy(plan->graph);
                plan->graph = nullptr;
            }
        }
        return KRY_OK;
    });
}

kry_status kry_plan_runs(const kry_plan_t* plan, int32_t* nruns, int32_t* roles_out) {
    return guarded("kry_plan_runs", [&]() -> kry_status {
        if (!plan) return fail(KRY_EINVAL, "plan is NULL");
        if (nruns) *nruns = plan->nruns;
        if (roles_out)
            for (int32_t r = 0; r < plan->nruns; ++r) roles_out[r] = plan->role[r];
        return KRY_OK;
    });
}

kry_status kry_plan_krylov(kry_plan_t* plan, int32_t run, int32_t* k_eff, double* beta0, double* H,
                           double* h_next, double* P) {
    return guarded("kry_plan_krylov", [&]() -> kry_status {
        if (!plan) return fail(KRY_EINVAL, "plan is NULL");
        if (run < 0 || run >= plan->nruns) return fail(KRY_EINVAL, "run out of range");
        if (!plan->projected) return fail(KRY_EINVAL, "kry_project_expm must run first");
        if (plan->method == KRY_BLOCK_ARNOLDI) return fail(KRY_ENOTSUP, "block runs: use kry_plan_block");
        const ScalLayout& L = plan->Y.L;
        std::vector<double> sc(L.stride);
        KRY_HIP(hipMemcpyAsync(sc.data(), plan->scal() + (size_t)run * L.stride, L.stride * sizeof(double),
                               hipMemcpyDeviceToHost, plan->stream));
        KRY_HIP(hipStreamSynchronize(plan->stream));
        const int k = plan->k;
        int m = std::min((int)sc[L.misc + MISC_KEFF], (int)sc[L.misc + MISC_KSTOP]);
        const bool bordered = plan->role[run] == 2;
        // dimension of the (augmented) Krylov space
        int dim = m;
        if (bordered) dim = (m > k - 1 ? k - 1 : m) + 1;
        if (k_eff) *k_eff = dim;
        if (beta0) *beta0 = bordered ? 1.0 : sc[L.beta + 0];
        const int tri = bordered ? dim - 1 : dim;
        if (H) {
            std::fill(H, H + (size_t)dim * dim, 0.0);
            const int sh = bordered ? 1 : 0;
            if (bordered && dim > 1) H[1 * dim + 0] = sc[L.beta + 0];
            for (int i = 0; i < tri; ++i) {
                if (plan->hess_mode) {
                    for (int c = i; c < tri; ++c) H[(i + sh) * dim + (c + sh)] = sc[L.hess + i * k + c];
                    if (i + 1 < tri) H[(i + 1 + sh) * dim + (i + sh)] = sc[L.beta + i + 1];
                    continue;
                }
                H[(i + sh) * dim + (i + sh)] = sc[L.alpha + i + 1];
                if (i + 1 < tri) {
                    H[(i + sh) * dim + (i + 1 + sh)] = sc[L.beta + i + 1];
                    H[(i + 1 + sh) * dim + (i + sh)] = sc[L.beta + i + 1];
                }
            }
        }
        if (h_next) *h_next = tri > 0 ? sc[L.beta + tri] : (bordered ? sc[L.beta + 0] : 0.0);
        if (P && plan->wide) {
            // one row per initial-space row: sigma_{c+1} E^T u_{c+1}
            std::vector<double> pw((size_t)plan->ncols * k);
            KRY_HIP(hipMemcpyAsync(pw.data(), plan->at<double>(plan->Y.wpw) + (size_t)run * plan->ncols * k,
                                   pw.size() * sizeof(double), hipMemcpyDeviceToHost, plan->stream));
            KRY_HIP(hipStreamSynchronize(plan->stream));
            for (int q = 0; q < plan->ncols; ++q)
                for (int c = 0; c < tri; ++c) P[(size_t)q * dim + c] = sc[L.sigma + c + 1] * pw[(size_t)q * k + c];
        } else if (P) {
            for (int q = 0; q < plan->o; ++q) {
                double* row = P + (size_t)q * dim;
                int c0 = 0;
                if (bordered) { if (dim > 0) row[0] = 0.0; c0 = 1; }
                for (int c = 0; c < tri; ++c) row[c0 + c] = sc[L.proj + q * (k + 1) + c];
            }
        }
        return KRY_OK;
    });
}

kry_status kry_plan_set_error_target(kry_plan_t* plan, double eps) {
    return guarded("kry_plan_set_error_target", [&]() -> kry_status {
        if (!plan) return fail(KRY_EINVAL, "plan is NULL");
        if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(KRY_EINVAL, "error target must be finite and >= 0");
        const bool arnoldi = plan->method == KRY_ARNOLDI;
        if (eps > 0.0 && plan->method != KRY_LANCZOS && !arnoldi)
            return fail(KRY_ENOTSUP, "the error-controlled Krylov dimension is built for Lanczos and Arnoldi plans");
        if (eps > 0.0 && plan->transposed)
            return fail(KRY_ENOTSUP, "the error-controlled Krylov dimension is built for the forward route");
        if (eps > 0.0 && plan->graph_on)
            return fail(KRY_ENOTSUP, "the error control polls the device between launches: not in graph mode");
        if (eps > 0.0 && plan->k > kMaxKP) return fail(KRY_ENOTSUP, "the error control holds k <= 8192");
        if (eps > 0.0 && arnoldi && plan->k > kMaxK)
            return fail(KRY_ENOTSUP, "the Arnoldi error control holds k <= 56 (its exponentials sit in LDS)");
        if (eps == 0.0) {
            plan->err_eps = 0.0;
            return KRY_OK;
        }
        if (!plan->hflags) KRY_HIP(hipHostMalloc((void**)&plan->hflags, kMaxP * sizeof(double), hipHostMallocDefault));
        if (!plan->flag_ev) KRY_HIP(hipEventCreateWithFlags(&plan->flag_ev, hipEventDisableTiming));
        if (!arnoldi && !plan->big_mem && (plan->k > kBigFrom || env_int("KRY_ERRCTL_BIG", 0) == 1)) {
            // theta and w per run, and the pivots of up to `chunk` eigenvalues at once
            BigErrArgs G{};
            G.ld = plan->k;
            G.chunk = std::min<int32_t>(plan->k, 512);
            const size_t runs = (size_t)plan->Y.pmax;
            const size_t bytes = runs * G.ld * (2 + (size_t)G.chunk) * sizeof(double);
            void* mem = nullptr;
            if (device_alloc(&mem, bytes) != hipSuccess)
                return fail(KRY_ENOMEM, "error control: no device memory for the eigen-solve (" +
                                            std::to_string(bytes) + " bytes)");
            plan->big_mem = static_cast<char*>(mem);
            G.theta = reinterpret_cast<double*>(plan->big_mem);
            G.w = G.theta + runs * G.ld;
            G.work = G.w + runs * G.ld;
            plan->big = G;
        }
        // lambda_max of the symmetric part of A, bounded by Gershgorin
        double lam;
        const Layout& Y = plan->Y;
        double* out = plan->at<double>(Y.eflags) + kMaxP;
        if (plan->sys.kind == KRY_STENCIL7) {
            stencil_row_bounds(plan->sys, nullptr, &lam);
        } else if (!arnoldi) {
            // Lanczos: A is symmetric, its own rows give the bound
            CsrArgs A{plan->sys.rowptr, plan->sys.colidx, plan->sys.vals, nullptr};
            hipError_t e = launch_row_gersh(A, plan->sys.n, plan->np_part(), Y.nblocks, Y.rpb, out, plan->stream);
            if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("row_gersh: ") + hipGetErrorString(e));
            KRY_HIP(hipMemcpyAsync(&lam, out, sizeof(double), hipMemcpyDeviceToHost, plan->stream));
            KRY_HIP(hipStreamSynchronize(plan->stream));
        } else {
            // general A: rows and columns; the column sums in fixed point with
            // a unit of 2^-40 of the largest |a| (rounded to a power of two)
            CsrArgs A{plan->sys.rowptr, plan->sys.colidx, plan->sys.vals, nullptr};
            const int64_t nnz = plan->sys.nnz;
            double amax = 0.0;
            hipError_t e = launch_abs_max(A.vals, nnz, plan->np_part(), Y.nblocks, out, plan->stream);
            if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("abs_max: ") + hipGetErrorString(e));
            KRY_HIP(hipMemcpyAsync(&amax, out, sizeof(double), hipMemcpyDeviceToHost, plan->stream));
            KRY_HIP(hipStreamSynchronize(plan->stream));
            if (!std::isfinite(amax)) {
                lam = INFINITY;                  // the runs report the non-finite entries themselves
            } else if (amax == 0.0) {
                lam = 0.0;
            } else {
                int ex = 0;
                std::frexp(amax, &ex);           // amax < 2^ex
                const double u = std::ldexp(1.0, ex - 40);
                int* overflow = reinterpret_cast<int*>(out + 1 + lemma1_hess_partials());
                KRY_HIP(hipMemsetAsync(overflow, 0, sizeof(int), plan->stream));
                // the basis store is free here and holds at least 8 n bytes
                auto* colfix = plan->at<unsigned long long>(Y.vec);
                e = launch_gersh_general(A, plan->sys.n, u, colfix, overflow, plan->np_part(), Y.nblocks, Y.rpb, out,
                                         plan->stream);
                if (e != hipSuccess) return fail(KRY_EDEVICE, std::string("gersh_general: ") + hipGetErrorString(e));
                int ovf = 0;
                KRY_HIP(hipMemcpyAsync(&lam, out, sizeof(double), hipMemcpyDeviceToHost, plan->stream));
                KRY_HIP(hipMemcpyAsync(&ovf, overflow, sizeof(int), hipMemcpyDeviceToHost, plan->stream));
                KRY_HIP(hipStreamSynchronize(plan->stream));
                if (ovf) return fail(KRY_ENOTSUP, "a column of A is too dense for the Gershgorin column sums");
            }
        }
        plan->err_eps = eps;
        plan->lam_plus = lam > 0.0 ? lam : 0.0;
        plan->projected = false;
        return KRY_OK;
    });
}

kry_status kry_plan_error(kry_plan_t* plan, int32_t run, int32_t* k_used, double* bound) {
    return guarded("kry_plan_error", [&]() -> kry_status {
        if (!plan) return fail(KRY_EINVAL, "plan is NULL");
        if (run < 0 || run >= plan->nruns) return fail(KRY_EINVAL, "run out of range");
        if (!plan->projected) return fail(KRY_EINVAL, "kry_project_expm must run first");
        if (plan->method == KRY_BLOCK_ARNOLDI) return fail(KRY_ENOTSUP, "block runs carry no error bound");
        const ScalLayout& L = plan->Y.L;
        double misc[MISC_COUNT];
        KRY_HIP(hipMemcpyAsync(misc, plan->scal() + (size_t)run * L.stride + L.misc, sizeof(misc), hipMemcpyDeviceToHost,
                               plan->stream));
        KRY_HIP(hipStreamSynchronize(plan->stream));
        const int keff = (int)misc[MISC_KEFF], kstop = (int)misc[MISC_KSTOP];
        // the augmented run's bordered matrix holds k - 1 Lanczos steps at most
        const int cap = plan->role[run] == 2 ? plan->k - 1 : plan->k;
        if (k_used) *k_used = std::min(std::min(keff, kstop), cap);
        // a breakdown makes the projection exact
        if (bound) *bound = keff < kstop ? 0.0 : misc[MISC_BOUND];
        return KRY_OK;
    });
}

kry_status kry_plan_block(const kry_plan_t* plan, int32_t block, int32_t* nblocks, int32_t* k_eff, int32_t* p,
                          double* H, double* R0, double* P) {
    return guarded("kry_plan_block", [&]() -> kry_status {
        if (!plan) return fail(KRY_EINVAL, "plan is NULL");
        if (plan->method != KRY_BLOCK_ARNOLDI) return fail(KRY_EINVAL, "not a block Arnoldi plan");
        if (!plan->projected) return fail(KRY_EINVAL, "kry_project_expm must run first");
        if (nblocks) *nblocks = (int32_t)plan->blocks.size();
        if (block < 0) return KRY_OK;
        if (block >= (int32_t)plan->blocks.size()) return fail(KRY_EINVAL, "block out of range");
        const auto& b = plan->blocks[block];
        if (k_eff) *k_eff = b.k_eff;
        if (p) *p = b.p;
        if (H) std::copy(b.H.begin(), b.H.end(), H);
        if (R0) std::copy(b.R0.begin(), b.R0.end(), R0);
        if (P) std::copy(b.P.begin(), b.P.end(), P);
        return KRY_OK;
    });
}

kry_status kry_matrix_create(const kry_system* sys, int32_t precision, void* hip_stream, kry_matrix** out) {
    return guarded("kry_matrix_create", [&]() -> kry_status {
        if (!out) return fail(KRY_EINVAL, "out is NULL");
        *out = nullptr;
        kry_status st = validate_system(sys);
        if (st != KRY_OK) return st;
        if (sys->kind != KRY_CSR || sys->nnz <= 0) return fail(KRY_EINVAL, "a prepared matrix needs a CSR system with nnz > 0");
        if (sys->prepared) return fail(KRY_EINVAL, "the system already names a prepared matrix");
        if (precision != KRY_FP64 && precision != KRY_FP32_BASIS) return fail(KRY_EINVAL, "unknown precision");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        const int64_t n = sys->n, ns = sell_slices(n), nt = sell_scan_tiles(n);
        const int64_t rpb = rows_per_block_for(n);
        const int32_t nb = nblocks_for(n, rpb);
        // first allocation: layout arrays, row-sum partials and the norm
        size_t off = 0;
        auto take = [&](size_t b) { const size_t o = off; off = align_up(off + b, 256); return o; };
        const size_t o_width = take((size_t)ns * 4), o_off = take((size_t)(ns + 1) * 8), o_tiles = take((size_t)(nt + 1) * 8);
        const size_t o_part = take((size_t)nb * 8), o_norm = take(8);
        const size_t head = off;
        char* tmp = nullptr;
        if (device_alloc((void**)&tmp, head) != hipSuccess) return fail(KRY_ENOMEM, "prepared matrix: allocation failed");
        auto bail = [&](kry_status code, const std::string& msg) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(tmp);
            return fail(code, msg);
        };
        CsrArgs A{sys->rowptr, sys->colidx, sys->vals, nullptr};
        hipError_t e = launch_sell_layout(A, n, reinterpret_cast<int32_t*>(tmp + o_width), reinterpret_cast<int64_t*>(tmp + o_off),
                                          reinterpret_cast<int64_t*>(tmp + o_tiles), s);
        if (e == hipSuccess)
            e = launch_row_abs_max(A, n, reinterpret_cast<double*>(tmp + o_part), nb, rpb,
                                   reinterpret_cast<double*>(tmp + o_norm), s);
        int64_t total = 0, nwide = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&total, reinterpret_cast<int64_t*>(tmp + o_off) + ns, sizeof(total), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&nwide, reinterpret_cast<int64_t*>(tmp + o_tiles) + nt, sizeof(nwide), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        const bool narrow = nwide == 0 && env_int("KRY_SELL_NARROW", 1) != 0;
        if (e != hipSuccess) return bail(KRY_EDEVICE, std::string("prepared matrix: ") + hipGetErrorString(e));
        // second allocation: the entries, after the layout
        const size_t esz = precision == KRY_FP32_BASIS ? 4 : 8;
        const size_t o_col = take((size_t)total * (narrow ? 2 : 4)), o_val = take((size_t)total * esz);
        kry_matrix* M = new kry_matrix();
        M->bytes = off;
        if (device_alloc((void**)&M->mem, M->bytes) != hipSuccess) {
            delete M;
            return bail(KRY_ENOMEM, "prepared matrix: allocation failed");
        }
        e = hipMemcpyAsync(M->mem, tmp, head, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = launch_sell_fill(precision == KRY_FP32_BASIS, narrow, A, n, reinterpret_cast<int64_t*>(M->mem + o_off),
                                 reinterpret_cast<int32_t*>(M->mem + o_width), M->mem + o_col, M->mem + o_val, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFree(tmp);
        if (e != hipSuccess) {
            (void)hipFree(M->mem);
            delete M;
            return fail(KRY_EDEVICE, std::string("prepared matrix: ") + hipGetErrorString(e));
        }
        M->n = n;
        M->nnz = sys->nnz;
        M->rowptr = sys->rowptr;
        M->colidx = sys->colidx;
        M->vals = sys->vals;
        M->precision = precision;
        M->sell = SellArgs{reinterpret_cast<int64_t*>(M->mem + o_off), reinterpret_cast<int32_t*>(M->mem + o_width),
                           narrow ? nullptr : reinterpret_cast<int32_t*>(M->mem + o_col),
                           precision == KRY_FP32_BASIS ? nullptr : reinterpret_cast<double*>(M->mem + o_val),
                           precision == KRY_FP32_BASIS ? reinterpret_cast<float*>(M->mem + o_val) : nullptr,
                           narrow ? reinterpret_cast<int16_t*>(M->mem + o_col) : nullptr, n};
        M->anorm_dev = reinterpret_cast<double*>(M->mem + o_norm);
        *out = M;
        return KRY_OK;
    });
}

kry_status kry_matrix_bytes(const kry_matrix* mat, size_t* bytes) {
    return guarded("kry_matrix_bytes", [&]() -> kry_status {
        if (!mat || !bytes) return fail(KRY_EINVAL, "NULL argument");
        *bytes = mat->bytes;
        return KRY_OK;
    });
}

void kry_matrix_destroy(kry_matrix* mat) {
    guarded_void([&] {
        if (!mat) return;
        if (mat->mem) (void)hipFree(mat->mem);
        delete mat;
    });
}

kry_status kry_plan_autotune(kry_plan_t* plan, int32_t reps, int32_t* tuned) {
    return guarded("kry_plan_autotune", [&]() -> kry_status {
        if (!plan) return fail(KRY_EINVAL, "plan is NULL");
        if (reps < 1 || reps > 1000) return fail(KRY_EINVAL, "reps must be in [1, 1000]");
        if (plan->graph_on) return fail(KRY_ENOTSUP, "tune before recording the plan as a graph");
        if (tuned) *tuned = 0;
        hipStream_t s = plan->stream;
        const Layout& Y = plan->Y;
        hipEvent_t a = nullptr, b = nullptr;
        KRY_HIP(hipEventCreate(&a));
        KRY_HIP(hipEventCreate(&b));
        struct Ev {
            hipEvent_t a, b;
            ~Ev() {
                if (a) (void)hipEventDestroy(a);
                if (b) (void)hipEventDestroy(b);
            }
        } ev{a, b};
        // microseconds per call of `run`, the better of two rounds of reps calls
        auto time_us = [&](auto&& run, double* us) -> kry_status {
            double best = INFINITY;
            for (int round = 0; round < 2; ++round) {
                KRY_HIP(hipEventRecord(a, s));
                for (int r = 0; r < reps; ++r) {
                    const kry_status st = run();
                    if (st != KRY_OK) return st;
                }
                KRY_HIP(hipEventRecord(b, s));
                KRY_HIP(hipEventSynchronize(b));
                float ms = 0.f;
                KRY_HIP(hipEventElapsedTime(&ms, a, b));
                best = std::min(best, 1000.0 * ms / reps);
            }
            *us = best;
            return KRY_OK;
        };
        if (!plan->projected) {
            const kry_status st = kry_project_expm(plan, nullptr);
            if (st != KRY_OK) return st;
        }
        if (plan->method == KRY_BLOCK_ARNOLDI && plan->k >= 1) {
            // the block mat-vec on the run's first block, written to the last
            // stored block (the projection's result is already in the basis)
            const int64_t n = plan->sys.n;
            const int64_t vstride = n * kBW;
            BlockArgs B{};
            B.n = n;
            B.state = plan->at<int32_t>(Y.bstate) + 3;   // a flag that stays 0: the kernel runs
            KRY_HIP(launch_fill_i32(B.state, 1, 0, s));
            CsrArgs A{plan->sys.rowptr, plan->sys.colidx, plan->sys.vals, plan->f32 ? plan->vals32() : nullptr};
            const void* V0 = plan->ws + Y.bvec;
            void* W = plan->ws + Y.bvec + (size_t)plan->k * vstride * Y.esize;
            TuneChoice best{};
            best.us = INFINITY;
            for (int32_t rows : {32, 64, 128, 256, 512}) {
                for (int32_t xcd : {0, 1}) {
                    B.spmm_rows = rows;
                    B.spmm_xcd = xcd;
                    double us = 0.0;
                    const kry_status st = time_us([&]() -> kry_status {
                        const hipError_t e = launch_bspmm(plan->f32, A, V0, W, B, s);
                        return e == hipSuccess ? KRY_OK : fail(KRY_EDEVICE, std::string("bspmm: ") + hipGetErrorString(e));
                    }, &us);
                    if (st != KRY_OK) return st;
                    if (us < best.us) best = TuneChoice{rows, xcd, us};
                }
            }
            tune_store(plan->f32 ? "bspmm32" : "bspmm", n, kBW, best);
            if (tuned) *tuned += 1;
            return KRY_OK;
        }
        const bool march = plan->sys.kind == KRY_STENCIL7 && Y.march > 0 && Y.lz1 && plan->method == KRY_LANCZOS &&
                           plan->err_eps <= 0.0 && !plan->wide && env_int("KRY_ONEPASS", -1) != 0;
        if (march) {
            // whole projections with plain or non-temporal pair stores (the
            // marching launches are nearly all of it); the results are equal
            int P = Y.pmax;
            while (P > 1 && P > plan->nruns) P >>= 1;
            TuneChoice best{};
            best.us = INFINITY;
            for (int32_t nt : {1, 0}) {
                plan->force_march_nt = nt;
                double us = 0.0;
                kry_status st = enqueue_projection(plan, nullptr, true);
                if (st == KRY_OK) st = time_us([&] { return enqueue_projection(plan, nullptr, true); }, &us);
                plan->force_march_nt = -1;
                if (st != KRY_OK) return st;
                if (us < best.us) best = TuneChoice{nt, 0, us};
            }
            tune_store("lz1_march", plan->sys.n, P, best);
            if (tuned) *tuned += 1;
        }
        return KRY_OK;
    });
}

kry_status kry_tune_choice(const char* kernel, int64_t n, int32_t runs, int32_t* found, int32_t* a, int32_t* b,
                           double* us) {
    return guarded("kry_tune_choice", [&]() -> kry_status {
        if (!kernel || !found) return fail(KRY_EINVAL, "kernel and found must not be NULL");
        TuneChoice c{};
        *found = tune_lookup(kernel, n, runs, &c) ? 1 : 0;
        if (a) *a = c.a;
        if (b) *b = c.b;
        if (us) *us = c.us;
        return KRY_OK;
    });
}

void kry_tune_clear(void) {
    guarded_void([&] { tune_clear(); });
}

void kry_plan_destroy(kry_plan_t* plan) {
    guarded_void([&] {
        if (!plan) return;
        if (plan->flag_ev || (plan->owns_ws && plan->ws)) (void)hipStreamSynchronize(plan->stream);
        if (plan->owns_ws && plan->ws) (void)hipFree(plan->ws);
        if (plan->big_mem) {
            (void)hipStreamSynchronize(plan->stream);
            (void)hipFree(plan->big_mem);
        }
        if (plan->lp_mem) {
            (void)hipStreamSynchronize(plan->stream);
            (void)hipFree(plan->lp_mem);
        }
        if (plan->graph_exec) {
            (void)hipStreamSynchronize(plan->stream);
            (void)hipGraphExecDestroy(plan->graph_exec);
        }
        if (plan->graph) (void)hipGraphDestroy(plan->graph);
        if (plan->flag_ev) (void)hipEventDestroy(plan->flag_ev);
        if (plan->hflags) (void)hipHostFree(plan->hflags);
        delete plan;
    });
}

kry_status kry_profile_enable(int32_t on) {
    return guarded("kry_profile_enable", [&]() -> kry_status {
        Profiler& P = prof();
        std::lock_guard<std::mutex> g(P.mu);
        P.on = on != 0;
        return KRY_OK;
    });
}

kry_status kry_profile_reset(void) {
    return guarded("kry_profile_reset", [&]() -> kry_status {
        Profiler& P = prof();
        std::lock_guard<std::mutex> g(P.mu);
        P.drain();
        P.totals.clear();
        return KRY_OK;
    });
}

kry_status kry_profile_read(const char* name, int64_t* launches, double* total_ms) {
    return guarded("kry_profile_read", [&]() -> kry_status {
        if (!name) return fail(KRY_EINVAL, "name is NULL");
        Profiler& P = prof();
        std::lock_guard<std::mutex> g(P.mu);
        P.drain();
        auto it = P.totals.find(name);
        if (launches) *launches = it == P.totals.end() ? 0 : it->second.first;
        if (total_ms) *total_ms = it == P.totals.end() ? 0.0 : it->second.second;
        return KRY_OK;
    });
}

const char* kry_profile_names(void) { return kKernelNames; }

}  // extern "C"
