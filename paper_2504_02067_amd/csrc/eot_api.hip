// C ABI and host drivers of the truncated-Newton entropic-OT library.
//
// The drivers take the steps of the paper's algorithms in order -- MDOT
// (Alg. 1), TruncatedNewtonProject (Alg. 4), ChiSinkhorn (Alg. 3),
// NewtonSolve (Alg. 2) with diagonally preconditioned CG -- and run every
// O(nm) primitive as a streaming pass on the device (eot_kernels.hip). The
// host only makes the scalar decisions (CG stop, forcing test, Armijo,
// ChiSinkhorn and projection loop tests, schedule updates), reading a few
// FP64 scalars back after the kernels that produce them.
//
// Everything is in the paper's log units inside (u = f / gamma, beta =
// 1 / gamma); the ABI speaks cost units (see include/eot.h).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "eot_internal.h"
#include "eot_tile_table.h"

using namespace eot;

// Workspace of eot_hvp_noalloc: device memory owned by the library for
// callers that cannot allocate. Each GPU the library runs on holds its own
// copy (from the first call on that GPU until the process ends); in host code
// the name is only a stand-in, the device address comes from
// hipGetSymbolAddress (noalloc_scratch below).
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {

static_assert(sizeof(CgScalars) % sizeof(double) == 0, "CgScalars is fetched as doubles");

// Discount cap of NewtonSolve: 1 - 2^-30 (kappa(F_r) <= 2 / (1 - rho) ~ 2e9).
constexpr double kRhoMax = 1.0 - 9.313225746154785e-10;

constexpr size_t kAlign = 256;

struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t off = 0;
    bool dry = true;
    template <typename T>
    T* take(size_t count)
    {
        off = (off + kAlign - 1) / kAlign * kAlign;
        T* p = dry ? nullptr : reinterpret_cast<T*>(base + off);
        off += std::max<size_t>(count, 1) * sizeof(T);
        return p;
    }
};

#define HIPCHK(x)                                          \
    do {                                                   \
        hipError_t e_ = (x);                               \
        if (e_ != hipSuccess) return EOT_ERR_HIP;          \
    } while (0)

#define EOTCHK(x)                                          \
    do {                                                   \
        eot_status s_ = (x);                               \
        if (s_ != EOT_OK) return s_;                       \
    } while (0)

struct Scratch {
    double* row_part = nullptr;  // 2 x tiles_m x waves x n
    double* col_part = nullptr;  // 2 x tiles_n x m
    double* red = nullptr;       // 2 x kMaxRedBlocks
    double* red2 = nullptr;      // 2 x kMaxRedBlocks
    double* scal = nullptr;      // 64 device scalars
    int32_t* flags = nullptr;    // 16 flags
    CgScalars* cg = nullptr;
};

struct NewtonVecs {
    double *rP, *grad, *b, *d, *e1, *dtry, *res, *z, *p, *q, *t, *M, *pcptd_try, *pcptd;  // n
    double *w, *wc, *ptd_try, *ptd;                                                         // m
};

struct SolveVecs {
    double *u, *lr, *s, *rt, *lrt, *du, *u_prev, *ua, *sh, *sh2;   // n
    double *v, *ct, *lct, *inv_ct, *dv, *v_prev, *va, *colsum, *lca; // m
};

struct GradVecs {
    double *u, *sh, *lr, *a, *s, *ra, *g0, *gy0, *gy1, *gy2;                  // n
    double *v, *cP, *bv, *inv_c, *mu, *cb, *tm, *h0, *hy0, *hy1, *hy2;          // m
};

// Buffers of the single-launch CG (launch_cg_persist) for small problems.
struct CgpVecs {
    double* sync = nullptr;       // 8 doubles: the abort word
};

// Single-launch CG: 0 off, 1 on (default); a fixed grid or 0 for the default.
std::atomic<int> g_cgp_mode{1};
std::atomic<int> g_cgp_grid{0};

// Workgroups of the single-launch CG for an n x m problem before the
// co-resident cap: the fixed grid or the smallest one with at most 8 rows and
// 8 columns per workgroup (the kernel's bound), at most kCgpMaxGrid and at
// most min(n, m) (every workgroup owns a row and a column).
int cgp_grid_for(int64_t n, int64_t m)
{
    const int lo = (int)((std::max(n, m) + 7) / 8);
    const int hi = (int)std::min<int64_t>(std::min(n, m), kCgpMaxGrid);
    return std::min(std::max(g_cgp_grid.load(), lo), hi);
}

// Cost kind of the single-launch CG (0 dense FP32, 1 dense FP64, 2 points in
// the plane), or -1 when it does not take the problem: too large, or points in
// R^3, whose version of the kernel gave wrong directions (see the kernel).
int cgp_kind(const eot_cost& c)
{
    if (c.n > kCgpMaxDim || c.m > kCgpMaxDim) return -1;
    if (c.kind == EOT_COST_DENSE_F32) return 0;
    if (c.kind == EOT_COST_DENSE_F64) return 1;
    if (c.kind == EOT_COST_SQEUCLID_POINTS && c.d == 2) return 2;
    return -1;
}

struct HdVecs {
    void *xh = nullptr, *xl = nullptr, *yh = nullptr, *yl = nullptr;   // BF16, n (m) x hd_padded_dim(d)
    float *xx = nullptr, *yy = nullptr;
    int cols = kHdTileCols;                       // columns per tile
    int64_t npad = 0, mpad = 0;                   // rows / columns padded to whole tiles
    float* rt = nullptr;                          // [4][npad] per-row values (mixed pass)
    double* rf = nullptr;                         // [npad] per-row factors
    float* ct = nullptr;                          // [mpad][4] column records
    double* gpart = nullptr;                      // [kHdMaxPart] grid maxima
};

// Pinned host staging for the scalars the host driver reads back (CG scalars,
// reductions, flags). A process-wide pool of small buffers, leased by a call
// that reads back for its lifetime; buffers are reused and never freed (at
// most one per concurrently running call). Every device -> host copy of the
// library goes into such a buffer: a call that cannot lease one fails with
// EOT_ERR_HIP instead of copying into pageable memory (concurrent pageable
// copies from several host threads go through the runtime's shared staging
// path; the batched solver once crashed inside it). A second pool of coherent
// buffers holds the CG progress words the kernels store into (see
// device_pcg); without one the CG loop reads its scalars back in chunks.
constexpr int kPinBytes = 512;
constexpr int kMirrorBytes = 64;

struct HostPool {
    std::mutex mu;
    std::vector<void*>* free = nullptr;         // never destroyed: safe at process exit
    unsigned flags;
    size_t bytes;
};
HostPool g_pin_pool{{}, nullptr, hipHostMallocDefault, kPinBytes};
HostPool g_mirror_pool{{}, nullptr, hipHostMallocCoherent, kMirrorBytes};

struct PinLease {
    HostPool& pool;
    void* p = nullptr;
    explicit PinLease(HostPool& pl) : pool(pl) {}
    // Takes a buffer from the pool (allocating one if the pool is empty); p
    // stays null if that fails.
    void acquire()
    {
        if (p) return;
        std::lock_guard<std::mutex> lk(pool.mu);
        if (!pool.free) pool.free = new std::vector<void*>();
        if (!pool.free->empty()) {
            p = pool.free->back();
            pool.free->pop_back();
        } else if (hipHostMalloc(&p, pool.bytes, pool.flags) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();            // do not leave the failure for a later check
        }
    }
    // After a failed wait a copy into the buffer may still be in flight: the
    // buffer is dropped (never returned to the pool) so no later call reuses it.
    void discard() { p = nullptr; }
    ~PinLease()
    {
        if (!p) return;
        std::lock_guard<std::mutex> lk(pool.mu);
        pool.free->push_back(p);
    }
    PinLease(const PinLease&) = delete;
    PinLease& operator=(const PinLease&) = delete;
};

struct Ctx {
    PinLease pin{g_pin_pool};
    PinLease mirror{g_mirror_pool};
    eot_cost cost{};
    int64_t n = 0, m = 0;
    int tiles_m = 0, tiles_n = 0;
    int rb = kTileRows;           // rows per tile
    int rtiles = 0, ctiles = 0;   // partials per row / column that the merges sum
    int atomic = 0;               // outputs accumulated atomically (huge problems)
    hipStream_t s = nullptr;
    Scratch sc;
    double* tmp_n[4] = {nullptr, nullptr, nullptr, nullptr};
    double* tmp_m[4] = {nullptr, nullptr, nullptr, nullptr};
    NewtonVecs nv{};
    SolveVecs sv{};
    GradVecs gv{};
    HdVecs hd{};
    CgpVecs cgp{};
    int64_t passes = 0;
    int32_t range_retries = 0;
    bool cg_graph = false;        // replay CG chunks from a recorded HIP graph
    bool cgp_ok = true;           // the single-launch CG may be used (not in batch workers)
};

void carve(Arena& ar, Ctx& x, int op)
{
    const int64_t n = x.n, m = x.m;
    if (x.cost.kind == EOT_COST_SQEUCLID_POINTS && x.cost.d > 3) {
        const size_t dp = (size_t)hd_padded_dim(x.cost.d);
        x.hd.xh = ar.take<uint16_t>((size_t)n * dp);
        x.hd.xl = ar.take<uint16_t>((size_t)n * dp);
        x.hd.yh = ar.take<uint16_t>((size_t)m * dp);
        x.hd.yl = ar.take<uint16_t>((size_t)m * dp);
        x.hd.xx = ar.take<float>(n);
        x.hd.yy = ar.take<float>(m);
        x.hd.rt = ar.take<float>((size_t)4 * x.hd.npad);
        x.hd.rf = ar.take<double>((size_t)x.hd.npad);
        x.hd.ct = ar.take<float>((size_t)4 * x.hd.mpad);
        x.hd.gpart = ar.take<double>(kHdMaxPart);
    }
    x.sc.row_part = ar.take<double>((size_t)2 * x.rtiles * n);
    x.sc.col_part = ar.take<double>((size_t)2 * x.ctiles * m);
    x.sc.red = ar.take<double>(2 * kMaxRedBlocks);
    x.sc.red2 = ar.take<double>(2 * kMaxRedBlocks);
    x.sc.scal = ar.take<double>(64);
    x.sc.flags = ar.take<int32_t>(16);
    x.sc.cg = ar.take<CgScalars>(1);
    for (int k = 0; k < 4; ++k) x.tmp_n[k] = ar.take<double>(n);
    for (int k = 0; k < 4; ++k) x.tmp_m[k] = ar.take<double>(m);
    if (op == EOT_OP_GRADIENT || op == EOT_OP_ROUND) {
        GradVecs& v = x.gv;
        double** nvec[] = {&v.u, &v.sh, &v.lr, &v.a, &v.s, &v.ra, &v.g0, &v.gy0, &v.gy1, &v.gy2};
        for (double** p : nvec) *p = ar.take<double>(n);
        double** mvec[] = {&v.v, &v.cP, &v.bv, &v.inv_c, &v.mu, &v.cb, &v.tm, &v.h0, &v.hy0,
                           &v.hy1, &v.hy2};
        for (double** p : mvec) *p = ar.take<double>(m);
    }
    if ((op == EOT_OP_NEWTON_CG || op == EOT_OP_SOLVE || op == EOT_OP_GRADIENT) &&
        cgp_kind(x.cost) >= 0) {
        x.cgp.sync = ar.take<double>(8);
    }
    if (op == EOT_OP_NEWTON_CG || op == EOT_OP_SOLVE || op == EOT_OP_GRADIENT) {
        NewtonVecs& v = x.nv;
        double** nvec[] = {&v.rP, &v.grad, &v.b, &v.d, &v.e1, &v.dtry, &v.res, &v.z,
                           &v.p, &v.q, &v.t, &v.M, &v.pcptd_try, &v.pcptd};
        for (double** p : nvec) *p = ar.take<double>(n);
        double** mvec[] = {&v.w, &v.wc, &v.ptd_try, &v.ptd};
        for (double** p : mvec) *p = ar.take<double>(m);
    }
    if (op == EOT_OP_SOLVE) {
        SolveVecs& v = x.sv;
        double** nvec[] = {&v.u, &v.lr, &v.s, &v.rt, &v.lrt, &v.du, &v.u_prev, &v.ua, &v.sh, &v.sh2};
        for (double** p : nvec) *p = ar.take<double>(n);
        double** mvec[] = {&v.v, &v.ct, &v.lct, &v.inv_ct, &v.dv, &v.v_prev, &v.va, &v.colsum, &v.lca};
        for (double** p : mvec) *p = ar.take<double>(m);
    }
}

eot_status check_cost(const eot_cost* c)
{
    if (!c) return EOT_ERR_INVALID_ARG;
    if (c->n < 1 || c->m < 1) return EOT_ERR_INVALID_ARG;
    if (c->kind == EOT_COST_DENSE_F32 || c->kind == EOT_COST_DENSE_F64) {
        if (!c->C || c->ldc < c->m) return EOT_ERR_INVALID_ARG;
        return EOT_OK;
    }
    if (c->kind == EOT_COST_SQEUCLID_POINTS) {
        if (!c->X || !c->Y || !(c->scale > 0.0) || !std::isfinite(c->scale) || c->d < 1)
            return EOT_ERR_INVALID_ARG;
        const bool low = c->d == 2 || c->d == 3;
        const bool high = c->d >= 16 && c->d <= 64 && c->d % 16 == 0;
        if (!low && !high) return EOT_ERR_UNSUPPORTED;
        return EOT_OK;
    }
    return EOT_ERR_INVALID_ARG;
}

// Tile layout of the passes. Tiles are 2048 columns wide and rb rows high:
// rb = 256 unless that leaves fewer than kMinTiles workgroups (small
// problems), then halved down to 8, so that small problems still spread over
// the chip. Per-tile partial sums are merged in a fixed order
// (bit-reproducible) unless those buffers would exceed 512 MB, in which case
// the pass accumulates into one row and one column vector with FP64 atomics.
// The measured table (eot_tile_table.h) takes precedence where it has an
// entry; eot_set_rows_per_tile overrides both (autotuning and tests).
constexpr int64_t kMinTiles = 512;
std::atomic<int> g_rows_override{0};

int pick_rows_per_tile(int64_t n, int64_t m, int kind)
{
    const int ov = g_rows_override.load();
    if (ov > 0) return ov;
    const int k = (int)std::lround(0.5 * std::log2((double)n * (double)m)) - kTileTableK0;
    if (k >= 0 && k < kTileTableN) {
        const int t = kind == EOT_COST_SQEUCLID_POINTS ? kTileTablePoints[k] : kTileTableDense[k];
        if (t > 0) return t;
    }
    const int64_t tm = tiles_m_of(m);
    int rb = kTileRows;
    while (rb > 8 && tm * tiles_n_of(n, rb) < kMinTiles) rb /= 2;
    return rb;
}

void layout(Ctx& x)
{
    const bool high_d = x.cost.kind == EOT_COST_SQEUCLID_POINTS && x.cost.d > 3;
    int row_parts;
    if (high_d) {                      // matrix-core tiles: one row partial per tile
        x.rb = kHdTileRows;
        x.tiles_n = (int)tiles_n_of(x.n, x.rb);
        // the widest tiles (fewest per-tile set-ups) that still launch >= 2048 workgroups
        int cols = kHdTileColsMax;
        while (cols > kHdTileCols && ((x.m + cols - 1) / cols) * (int64_t)x.tiles_n < 2048) cols /= 2;
        x.hd.cols = cols;
        x.tiles_m = (int)((x.m + cols - 1) / cols);
        x.hd.npad = (int64_t)x.tiles_n * kHdTileRows;
        x.hd.mpad = (int64_t)x.tiles_m * cols;
        row_parts = x.tiles_m;
    } else {
        x.tiles_m = (int)tiles_m_of(x.m);
        x.rb = pick_rows_per_tile(x.n, x.m, x.cost.kind);
        x.tiles_n = (int)tiles_n_of(x.n, x.rb);
        row_parts = row_tiles(x.tiles_m);
    }
    const double part_bytes =
        16.0 * ((double)row_parts * (double)x.n + (double)x.tiles_n * (double)x.m);
    x.atomic = part_bytes > 512.0e6 ? 1 : 0;
    x.rtiles = x.atomic ? 1 : row_parts;
    x.ctiles = x.atomic ? 1 : x.tiles_n;
}

eot_status clear_flags(Ctx& x);

eot_status setup(Ctx& x, const eot_cost* cost, int op, int prec, void* ws, size_t ws_bytes,
                 void* stream)
{
    EOTCHK(check_cost(cost));
    if (prec != EOT_PREC_FP64 && prec != EOT_PREC_MIXED) return EOT_ERR_INVALID_ARG;
    if (prec == EOT_PREC_MIXED && cost->kind == EOT_COST_DENSE_F64) return EOT_ERR_UNSUPPORTED;
    x.cost = *cost;
    x.n = cost->n;
    x.m = cost->m;
    layout(x);
    x.s = static_cast<hipStream_t>(stream);
    Arena dry;
    carve(dry, x, op);
    if (!ws || ws_bytes < dry.off || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0)
        return EOT_ERR_WORKSPACE;
    Arena ar;
    ar.base = static_cast<char*>(ws);
    ar.cap = ws_bytes;
    ar.dry = false;
    carve(ar, x, op);
    if (op == EOT_OP_NEWTON_CG || op == EOT_OP_SOLVE || op == EOT_OP_GRADIENT ||
        op == EOT_OP_ROUND) {                   // host read-backs: pinned buffers
        x.pin.acquire();
        if (!x.pin.p) return EOT_ERR_HIP;
        x.mirror.acquire();
    }
    EOTCHK(clear_flags(x));
    if (x.hd.xh) {
        HIPCHK(launch_hd_prep(x.cost.X, x.n, x.cost.d, x.hd.xh, x.hd.xl, x.hd.xx, x.s));
        HIPCHK(launch_hd_prep(x.cost.Y, x.m, x.cost.d, x.hd.yh, x.hd.yl, x.hd.yy, x.s));
    }
    return EOT_OK;
}

PassArgs make_args(const Ctx& x, const double* u, const double* a, const double* v, double beta)
{
    PassArgs A{};
    A.kind = x.cost.kind;
    A.C = x.cost.C;
    A.n = x.n;
    A.m = x.m;
    A.ldc = x.cost.ldc;
    // 16-byte loads only where a 4-column group never crosses column m: the
    // ldc padding of a row is never read (it may hold anything)
    A.vec_ok = (x.cost.ldc % 4 == 0) && (x.m % 4 == 0) &&
               (reinterpret_cast<uintptr_t>(x.cost.C) % 16 == 0);
    A.u = u;
    A.a = a;
    A.v = v;
    // points: C_ij = |x_i - y_j|^2 / scale; the kernels see |x_i - y_j|^2 and beta / scale
    A.beta = x.cost.kind == EOT_COST_SQEUCLID_POINTS ? beta / x.cost.scale : beta;
    A.X = x.cost.X;
    A.Y = x.cost.Y;
    A.d = x.cost.d;
    A.row_part = x.sc.row_part;
    A.col_part = x.sc.col_part;
    A.tiles_m = x.tiles_m;
    A.tiles_n = x.tiles_n;
    A.atomic = x.atomic;
    A.rb = x.rb;
    A.hd_xh = x.hd.xh;
    A.hd_xl = x.hd.xl;
    A.hd_yh = x.hd.yh;
    A.hd_yl = x.hd.yl;
    A.hd_xx = x.hd.xx;
    A.hd_yy = x.hd.yy;
    A.hd_cols = x.hd.cols;
    A.hd_npad = x.hd.npad;
    A.hd_rt = x.hd.rt;
    A.hd_rf = x.hd.rf;
    A.hd_ct = x.hd.ct;
    A.hd_gpart = x.hd.gpart;
    return A;
}

// Launch one streaming pass; in atomic mode its outputs are cleared first.
hipError_t run_pass(Ctx& x, const PassArgs& A, int prec, int nr, int nc, int mode2)
{
    if (x.atomic) {
        if (nr > 0) {
            hipError_t e = launch_fill(A.row_part, 0.0, (int64_t)nr * x.n, x.s);
            if (e != hipSuccess) return e;
        }
        if (nc > 0) {
            hipError_t e = launch_fill(A.col_part, 0.0, (int64_t)nc * x.m, x.s);
            if (e != hipSuccess) return e;
        }
    }
    return launch_pass(A, prec, nr, nc, mode2, x.s);
}

// Device -> host copy of `bytes` bytes through the call's pinned buffer and a
// wait on the stream. Every return after a queued copy has waited for it (or
// dropped the buffer), so no copy lands in memory the caller no longer owns.
eot_status fetch_bytes(Ctx& x, const void* d, void* h, size_t bytes)
{
    if (!x.pin.p || bytes > (size_t)kPinBytes) return EOT_ERR_HIP;
    HIPCHK(hipMemcpyAsync(x.pin.p, d, bytes, hipMemcpyDeviceToHost, x.s));
    if (hipStreamSynchronize(x.s) != hipSuccess) {
        x.pin.discard();
        return EOT_ERR_HIP;
    }
    std::memcpy(h, x.pin.p, bytes);
    return EOT_OK;
}

eot_status fetch(Ctx& x, const double* d, double* h, int k)
{
    return fetch_bytes(x, d, h, sizeof(double) * (size_t)k);
}

eot_status fetch_flags(Ctx& x, int32_t* h)
{
    return fetch_bytes(x, x.sc.flags, h, sizeof(int32_t) * 2);
}

// The 16 int32 flags are cleared by a fill kernel (8 doubles of +0.0 are the
// same 64 zero bytes), not a memset node, so callers may capture the calls.
eot_status clear_flags(Ctx& x)
{
    HIPCHK(launch_fill(reinterpret_cast<double*>(x.sc.flags), 0.0, 8, x.s));
    return EOT_OK;
}

// Device reduction -> host scalar.
eot_status reduce_host(Ctx& x, int op, const double* a, const double* b, int64_t k, double* out)
{
    int nb = 0;
    HIPCHK(launch_reduce(op, a, b, k, x.sc.red, &nb, x.s));
    if (op == RED_MAXABS2) HIPCHK(launch_finish_max(x.sc.red, nb, x.sc.scal, x.s));
    else HIPCHK(launch_finish_sum(x.sc.red, nb, x.sc.scal, x.s));
    return fetch(x, x.sc.scal, out, 1);
}

// Row shift = exact row maxima (one FP64 pass).
eot_status row_max(Ctx& x, const double* u, const double* v, double beta, double* out)
{
    PassArgs A = make_args(x, u, nullptr, v, beta);
    HIPCHK(launch_rowmax(A, x.sc.row_part, out, x.s));
    x.passes += 1;
    return EOT_OK;
}

// log r(P) (and s_i = sum_j P_ij^2 / c_j when inv_c) at (u, v), shift a.
eot_status row_pass(Ctx& x, int prec, const double* u, const double* a, const double* v,
                    double beta, const double* inv_c, double* log_rP, double* s_out)
{
    PassArgs A = make_args(x, u, a, v, beta);
    A.yw1 = inv_c;
    const int nr = inv_c ? 2 : 1;
    HIPCHK(run_pass(x, A, prec, nr, 0, R2_SQUARE));
    HIPCHK(launch_log_row_from_sums(x.sc.row_part, x.rtiles, x.n, a, log_rP, x.sc.flags, x.s));
    if (inv_c && s_out)
        HIPCHK(launch_merge_rows(x.sc.row_part, x.rtiles, x.n, 2, a, nullptr, s_out, 1, x.s));
    x.passes += 1;
    return EOT_OK;
}

// Column sums sum_i P_ij xw_i (xw nullable = 1) at (u, v), shift a.
eot_status col_pass(Ctx& x, int prec, const double* u, const double* a, const double* v,
                    double beta, const double* xw, double* colsum)
{
    PassArgs A = make_args(x, u, a, v, beta);
    A.xw0 = xw;
    HIPCHK(run_pass(x, A, prec, 0, 1, R2_WEIGHT));
    HIPCHK(launch_merge_cols(x.sc.col_part, x.ctiles, x.m, 1, colsum, nullptr, x.s));
    x.passes += 1;
    return EOT_OK;
}

// Row sums sum_j P_ij yw_j at (u, v), shift a -> out (with exp(a) applied).
eot_status rowsum_pass(Ctx& x, int prec, const double* u, const double* a, const double* v,
                       double beta, const double* yw, double* out)
{
    PassArgs A = make_args(x, u, a, v, beta);
    A.yw0 = yw;
    HIPCHK(run_pass(x, A, prec, 1, 0, R2_WEIGHT));
    HIPCHK(launch_merge_rows(x.sc.row_part, x.rtiles, x.n, 1, a, out, nullptr, 0, x.s));
    x.passes += 1;
    return EOT_OK;
}

// ---------------------------------------------------------------- NewtonSolve
struct NewtonResult {
    double rho = 0.0;
    int32_t cg_iters = 0, levels = 0, miss = 0;
    int64_t passes = 0;
    double forcing_ratio = 0.0;
};

// Grid of the single-launch CG for this problem (cgp_grid_for, at most the
// co-resident capacity), or 0 to use the launches per iteration (also when no
// grid has both at most 8 rows and columns per workgroup and at least one of
// each: min(n, m) < max(n, m) / 8).
eot_status cgp_pick_grid(Ctx& x, int prec, int* grid)
{
    *grid = 0;
    if (!g_cgp_mode.load()) return EOT_OK;
    const int kind = cgp_kind(x.cost);
    const int mixed = prec == EOT_PREC_MIXED ? 1 : 0;
    if (kind < 0 || (kind == 1 && mixed)) return EOT_OK;
    static std::atomic<int> cap[4][2];           // co-resident capacity per kernel, 0 = unknown
    int c = cap[kind][mixed].load();
    if (c == 0) {
        HIPCHK(cg_persist_max_grid(kind, mixed, &c));
        cap[kind][mixed].store(c);
    }
    const int lo = (int)((std::max(x.n, x.m) + 7) / 8);
    const int g = std::min(cgp_grid_for(x.n, x.m), c);
    if (g >= lo) *grid = g;
    return EOT_OK;
}

// Preconditioned CG on F_r(rho) d = V.b (Alg. 2 inner loop) from d = 0, with
// F_r(rho) p = r(P) o p - rho P ((P^T p) / c) and Jacobi preconditioner
// M_i = r(P)_i - rho s_i; r(P) in V.rP, log r(P) in lr (also the row shift).
// Solution in V.dtry (with P^T d in V.ptd_try and P (P^T d / c) in V.pcptd_try).
// The iterations are enqueued without waiting: each kernel of an iteration
// returns at once when the device flag sc.done is set (by the iteration that
// met the stop test, broke down or reached max_cg). The host paces its launches
// by progress words the kernels store into pinned host memory and reads the
// scalars once at the end (without pinned memory: in chunks of 4, 8, 16, 32
// iterations with a read-back after each). exact_sums: the mixed point-cloud
// row-sum pass keeps FP64 sums in every lane (for solves to a tight residual).
eot_status device_pcg(Ctx& x, int prec, const double* u, const double* lr, const double* v,
                      double beta, const double* s, const double* c, double rho, double tol,
                      int max_cg, CgScalars* out, bool exact_sums = false)
{
    NewtonVecs& V = x.nv;
    const int64_t n = x.n, m = x.m;
    int32_t* mirror = static_cast<int32_t*>(x.mirror.p);
    if (mirror) {
        mirror[0] = 0;
        mirror[1] = 0;
    }
    int cgp_grid = 0;
    if (x.cgp.sync && x.cgp_ok && !x.cg_graph) EOTCHK(cgp_pick_grid(x, prec, &cgp_grid));
    if (cgp_grid > 0) {
        // the whole CG solve in one cooperative launch
        CgpArgs A{};
        A.P.kind = x.cost.kind;
        A.P.d = x.cost.d;
        A.P.n = n;
        A.P.m = m;
        A.P.ldc = x.cost.ldc;
        A.P.C = x.cost.C;
        A.P.X = x.cost.X;
        A.P.Y = x.cost.Y;
        A.P.scale = x.cost.scale;
        A.KIND = cgp_kind(x.cost);
        A.mixed = prec == EOT_PREC_MIXED ? 1 : 0;
        A.beta = beta;
        A.u = u;
        A.a = lr;
        A.v = v;
        A.c = c;
        A.rP = V.rP;
        A.s = s;
        A.b = V.b;
        A.rho = rho;
        A.tol = tol;
        A.max_cg = max_cg;
        A.d = V.dtry;
        A.ptd = V.ptd_try;
        A.pcptd = V.pcptd_try;
        A.sc = x.sc.cg;
        A.wc = V.wc;
        A.t = V.t;
        A.abort = reinterpret_cast<int32_t*>(x.cgp.sync);
        HIPCHK(launch_fill(x.cgp.sync, 0.0, 8, x.s));
        HIPCHK(launch_fill(V.wc, 0.0, m, x.s));            // tag 0: nothing published yet
        HIPCHK(launch_fill(V.t, 0.0, n, x.s));
        HIPCHK(launch_cg_persist(A, cgp_grid, x.s));
        CgScalars h{};
        EOTCHK(fetch(x, reinterpret_cast<const double*>(x.sc.cg), reinterpret_cast<double*>(&h),
                     sizeof(CgScalars) / sizeof(double)));
        if (!h.done) return EOT_ERR_HIP;        // a grid wait timed out
        x.passes += 2 * (int64_t)h.iters;
        *out = h;
        return EOT_OK;
    }
    HIPCHK(launch_cg_init(V.b, V.rP, s, rho, V.dtry, V.res, V.z, V.p, V.M, V.ptd_try,
                          V.pcptd_try, n, m, x.sc.red, x.sc.cg, tol, max_cg, mirror, x.s));
    PassArgs pa = make_args(x, u, lr, v, beta);        // pass A: column sums of P p
    pa.xw0 = V.p;
    pa.skip = &x.sc.cg->done;
    PassArgs pb = make_args(x, u, lr, v, beta);        // pass B: row sums of P (w / c)
    pb.yw0 = V.wc;
    pb.skip = &x.sc.cg->done;
    pb.exact_sums = exact_sums ? 1 : 0;
    CgScalars h{};
    const bool small = std::max(n, m) <= kCgSmallMax;
    // one CG iteration; every kernel returns at once once sc.done is set
    auto iteration = [&]() -> hipError_t {
        hipError_t e = run_pass(x, pa, prec, 0, 1, R2_WEIGHT);
        if (e == hipSuccess)
            e = launch_cg_colstep(x.sc.col_part, x.ctiles, m, c, V.w, V.wc, x.sc.cg, x.s);
        if (e == hipSuccess) e = run_pass(x, pb, prec, 1, 0, R2_WEIGHT);
        if (e != hipSuccess) return e;
        if (small)
            return launch_cg_small(x.sc.row_part, x.rtiles, n, m, lr, V.rP, V.p, rho, V.t, V.q,
                                   V.dtry, V.res, V.z, V.M, V.pcptd_try, V.w, V.ptd_try, x.sc.cg,
                                   mirror, x.s);
        int nb_pq = 0, nb = 0;
        e = launch_cg_rowstep(x.sc.row_part, x.rtiles, n, lr, V.rP, V.p, rho, V.t, V.q, x.sc.red2,
                              &nb_pq, x.sc.cg, x.s);
        if (e == hipSuccess)
            e = launch_cg_update(x.sc.red2, nb_pq, V.dtry, V.res, V.z, V.p, V.q, V.M, V.t,
                                 V.pcptd_try, V.w, V.ptd_try, n, m, x.sc.red, &nb, x.sc.cg, x.s);
        if (e == hipSuccess)
            e = launch_cg_direction(x.sc.red, nb, V.z, V.p, n, x.sc.cg, mirror, x.s);
        return e;
    };
    auto read_scalars = [&]() -> eot_status {
        return fetch(x, reinterpret_cast<const double*>(x.sc.cg), reinterpret_cast<double*>(&h),
                     sizeof(CgScalars) / sizeof(double));
    };
    int issued = 0;
    // Graph mode: record kGraphChunk iterations once, replay until the device flag is set.
    bool graphed = false;
    if (x.cg_graph && x.s != nullptr && !pass_timing_on()) {
        constexpr int kGraphChunk = 8;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipError_t e = hipStreamBeginCapture(x.s, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t ee = hipSuccess;
            for (int it = 0; it < kGraphChunk && ee == hipSuccess; ++it) ee = iteration();
            e = hipStreamEndCapture(x.s, &graph);
            if (ee != hipSuccess) e = ee;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        eot_status gs = EOT_OK;
        if (e == hipSuccess) {
            graphed = true;
            for (;;) {
                if (hipGraphLaunch(exec, x.s) != hipSuccess) { gs = EOT_ERR_HIP; break; }
                issued += kGraphChunk;
                gs = read_scalars();
                if (gs != EOT_OK || h.done || issued >= max_cg) break;
            }
        } else {
            (void)hipGetLastError();                  // capture unsupported: direct launches
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        EOTCHK(gs);
    }
    if (!graphed && mirror) {
        // Enqueue while watching the progress words: at most kCgLead iterations
        // in flight, none once the stop test has passed. At the lead limit the
        // host spins on the words (no runtime calls, which would contend with
        // other threads' launches); after kStallUs without progress it asks
        // the stream, and if that has drained it reads the scalars back
        // (authoritative) and goes on from there.
        constexpr int kCgLead = 2;
        constexpr auto kStall = std::chrono::microseconds(200);
        const volatile int32_t* hm = mirror;
        int32_t seen = -1;
        auto t_seen = std::chrono::steady_clock::now();
        while (issued < max_cg && !hm[1]) {
            const int32_t done_it = hm[0];
            if (issued - done_it >= kCgLead) {
                const auto now = std::chrono::steady_clock::now();
                if (done_it != seen) {
                    seen = done_it;
                    t_seen = now;
                    continue;
                }
                if (now - t_seen < kStall) {
                    std::this_thread::yield();
                    continue;
                }
                const hipError_t q = hipStreamQuery(x.s);
                if (q == hipErrorNotReady) {
                    t_seen = now;
                    continue;
                }
                if (q != hipSuccess) return EOT_ERR_HIP;
                EOTCHK(read_scalars());
                if (h.done) break;
            }
            HIPCHK(iteration());
            ++issued;
        }
        EOTCHK(read_scalars());
    } else if (!graphed) {
        int chunk = 4;
        for (;;) {
            for (int it = 0; it < chunk && issued < max_cg; ++it, ++issued) HIPCHK(iteration());
            EOTCHK(read_scalars());
            if (h.done || issued >= max_cg) break;
            chunk = std::min(2 * chunk, 32);
        }
    }
    x.passes += 2 * (int64_t)h.iters;
    *out = h;
    return EOT_OK;
}

// Alg. 2 at (u, v) with c(P) = c: lr = log r(P) (also the row shift), s_i =
// sum_j P_ij^2 / c_j. Writes d_u to du and d_v = -(P^T d_u) / c to dv.
eot_status newton_solve(Ctx& x, int prec, const double* u, const double* v, double beta,
                        const double* lr, const double* s, const double* r, const double* c,
                        double eta, double rho0, int max_cg, int max_levels, double* du,
                        double* dv, NewtonResult* out, double gnorm_known = -1.0)
{
    NewtonVecs& V = x.nv;
    const int64_t n = x.n, m = x.m;
    const int64_t p0 = x.passes;
    HIPCHK(launch_newton_init(lr, r, V.rP, V.grad, V.b, V.d, n, x.s));
    double gnorm = gnorm_known;                 // ||grad||_1, when the caller has it
    if (!(gnorm >= 0.0)) EOTCHK(reduce_host(x, RED_L1, V.grad, nullptr, n, &gnorm));
    // F_r(1) d for the rho = 0 direction: two explicit passes
    EOTCHK(col_pass(x, prec, u, lr, v, beta, V.d, V.ptd));
    HIPCHK(launch_div(V.ptd, c, V.wc, 1.0, m, x.s));
    EOTCHK(rowsum_pass(x, prec, u, lr, v, beta, V.wc, V.pcptd));
    HIPCHK(launch_forcing_resid(V.rP, V.d, V.pcptd, V.grad, V.e1, n, x.s));
    double e1 = 0.0;
    EOTCHK(reduce_host(x, RED_L1, V.e1, nullptr, n, &e1));

    double rho = rho0;
    int32_t lev = 0, cgk = 0, miss = 0;
    for (;;) {
        if (e1 <= eta * gnorm) break;
        if (lev >= max_levels || rho > kRhoMax) { miss = 1; break; }
        if (rho == 0.0) {
            // F_r(0) = D(r(P)): the CG solution is -grad / r(P), the current d.
            cgk += 1;
            rho = 0.75;
            ++lev;
            continue;
        }
        const double tol = 0.25 * eta * gnorm;
        CgScalars h{};
        EOTCHK(device_pcg(x, prec, u, lr, v, beta, s, c, rho, tol, max_cg, &h));
        cgk += h.iters;
        const bool conv = !h.broke && h.res_l1 <= tol;
        if (!conv) { miss = 1; break; }
        std::swap(V.d, V.dtry);
        std::swap(V.ptd, V.ptd_try);
        std::swap(V.pcptd, V.pcptd_try);
        HIPCHK(launch_forcing_resid(V.rP, V.d, V.pcptd, V.grad, V.e1, n, x.s));
        EOTCHK(reduce_host(x, RED_L1, V.e1, nullptr, n, &e1));
        rho = 1.0 - (1.0 - rho) / 4.0;
        ++lev;
    }
    HIPCHK(launch_copy(V.d, du, n, x.s));
    HIPCHK(launch_div(V.ptd, c, dv, -1.0, m, x.s));
    out->rho = rho;
    out->cg_iters = cgk;
    out->levels = lev;
    out->miss = miss;
    out->passes = x.passes - p0;
    out->forcing_ratio = gnorm > 0.0 ? e1 / gnorm : 0.0;
    return EOT_OK;
}

// ---------------------------------------------------------------- projection
struct SolveState {
    const eot_solve_opts* o;
    eot_solve_stats* st;
    eot_solve_trace* tr = nullptr;   // step trace (host, nullable)
    int32_t step = 0;                // MDOT step being projected
    double start_err = 0.0;          // first ||r~ - r(P)||_1 of the step's projection
    int32_t sweeps = 0;              // ChiSinkhorn sweeps of the step
    bool first_projection = true;    // false for the FP64 finish of a mixed step
};

// One Newton step of Alg. 4 into the trace.
void trace_newton(SolveState& ss, double gk, double eta, double rho_in, double rho_out,
                  int32_t cg, int32_t lev, double alpha, double gk1)
{
    eot_solve_trace* tr = ss.tr;
    if (!tr) return;
    const int32_t e = tr->n_newton;
    if (e < tr->cap_newton) {
        if (tr->step_of) tr->step_of[e] = ss.step;
        if (tr->gnorm) tr->gnorm[e] = gk;
        if (tr->eta) tr->eta[e] = eta;
        if (tr->cg_tol) tr->cg_tol[e] = 0.25 * eta * gk;
        if (tr->rho0) tr->rho0[e] = rho_in;
        if (tr->rho_out) tr->rho_out[e] = rho_out;
        if (tr->cg_iters) tr->cg_iters[e] = cg;
        if (tr->levels) tr->levels[e] = lev;
        if (tr->alpha) tr->alpha[e] = alpha;
        if (tr->gnorm_next) tr->gnorm_next[e] = gk1;
    }
    tr->n_newton = e + 1;
}

// Column fix (v <- v + log c~ - log c(P)) followed by the row refresh
// (log r(P), s), with a fallback to FP64 passes from exact row maxima when
// the FP32 range guard fires.
eot_status fix_and_refresh(Ctx& x, int prec, double beta, const double* shift_guess,
                           SolveState& ss)
{
    SolveVecs& S = x.sv;
    EOTCHK(clear_flags(x));
    EOTCHK(col_pass(x, prec, S.u, shift_guess, S.v, beta, nullptr, S.colsum));
    HIPCHK(launch_fix_cols(S.v, S.lct, S.colsum, x.m, x.sc.flags, x.s));
    EOTCHK(row_pass(x, prec, S.u, shift_guess, S.v, beta, S.inv_ct, S.lr, S.s));
    int32_t fl[2] = {0, 0};
    EOTCHK(fetch_flags(x, fl));
    if (fl[0] == 0 && fl[1] == 0) return EOT_OK;
    ss.st->range_retries += 1;
    EOTCHK(clear_flags(x));
    EOTCHK(row_max(x, S.u, S.v, beta, S.sh2));
    EOTCHK(col_pass(x, EOT_PREC_FP64, S.u, S.sh2, S.v, beta, nullptr, S.colsum));
    HIPCHK(launch_fix_cols(S.v, S.lct, S.colsum, x.m, x.sc.flags, x.s));
    EOTCHK(row_max(x, S.u, S.v, beta, S.sh2));
    EOTCHK(row_pass(x, EOT_PREC_FP64, S.u, S.sh2, S.v, beta, S.inv_ct, S.lr, S.s));
    EOTCHK(fetch_flags(x, fl));
    if (fl[0] || fl[1]) return EOT_ERR_NONFINITE;
    return EOT_OK;
}

// Row refresh only (after a Newton step of Alg. 4), same fallback. Also
// returns ||r~ - r(P)||_1 of the refreshed plan (read with the range flags in
// one wait).
eot_status refresh(Ctx& x, int prec, double beta, const double* shift_guess, SolveState& ss,
                   double* gn_out)
{
    SolveVecs& S = x.sv;
    EOTCHK(clear_flags(x));
    EOTCHK(row_pass(x, prec, S.u, shift_guess, S.v, beta, S.inv_ct, S.lr, S.s));
    int32_t fl[2] = {0, 0};
    int nb = 0;
    HIPCHK(launch_reduce(RED_L1_DIFF_EXP, S.rt, S.lr, x.n, x.sc.red, &nb, x.s));
    HIPCHK(launch_finish_sum(x.sc.red, nb, x.sc.scal, x.s));
    if (!x.pin.p) return EOT_ERR_HIP;
    char* pb = static_cast<char*>(x.pin.p);
    const hipError_t e1 = hipMemcpyAsync(pb, x.sc.flags, sizeof(fl), hipMemcpyDeviceToHost, x.s);
    const hipError_t e2 =
        e1 == hipSuccess ? hipMemcpyAsync(pb + 64, x.sc.scal, sizeof(double),
                                          hipMemcpyDeviceToHost, x.s)
                         : e1;
    if (hipStreamSynchronize(x.s) != hipSuccess) {       // wait even when a copy failed
        x.pin.discard();
        return EOT_ERR_HIP;
    }
    if (e2 != hipSuccess) return EOT_ERR_HIP;
    std::memcpy(fl, pb, sizeof(fl));
    std::memcpy(gn_out, pb + 64, sizeof(double));
    if (fl[0] == 0) return EOT_OK;
    ss.st->range_retries += 1;
    EOTCHK(clear_flags(x));
    EOTCHK(row_max(x, S.u, S.v, beta, S.sh2));
    EOTCHK(row_pass(x, EOT_PREC_FP64, S.u, S.sh2, S.v, beta, S.inv_ct, S.lr, S.s));
    EOTCHK(fetch_flags(x, fl));
    if (fl[0]) return EOT_ERR_NONFINITE;
    return reduce_host(x, RED_L1_DIFF_EXP, S.rt, S.lr, x.n, gn_out);
}

// TruncatedNewtonProject (Alg. 4) on the smoothed marginals held in S.rt,
// S.ct (logs S.lrt, S.lct; S.inv_ct = 1 / ct).
// Mixed precision (stall_exit): the FP32 plan entries put a floor under the
// measured row error; when two Newton steps in a row fail to halve it (below
// 1e-3), or the Newton cap is reached, the projection ends with *stalled set
// instead of failing, and the caller continues in FP64.
eot_status tnp(Ctx& x, int prec, double beta, double eps, double* rho0, double* delta_min,
               SolveState& ss, bool stall_exit = false, bool* stalled = nullptr)
{
    SolveVecs& S = x.sv;
    const eot_solve_opts* o = ss.o;
    eot_solve_stats* st = ss.st;
    const int64_t n = x.n, m = x.m;
    int64_t p0 = x.passes;
    // Column fix and row marginals from exact row maxima (the potentials were extrapolated).
    EOTCHK(row_max(x, S.u, S.v, beta, S.sh));
    EOTCHK(fix_and_refresh(x, prec, beta, S.sh, ss));
    st->passes_projection += x.passes - p0;
    double dmin = INFINITY;
    int32_t k = 0;
    eot_status status = EOT_OK;
    double g_prev = INFINITY;
    int slow = 0;
    if (stalled) *stalled = false;
    double gn_known = -1.0;                    // ||r~ - r(P)||_1 from the last row refresh
    for (;;) {
        double gn = gn_known;
        gn_known = -1.0;
        if (!(gn >= 0.0)) EOTCHK(reduce_host(x, RED_L1_DIFF_EXP, S.rt, S.lr, n, &gn));
        if (!std::isfinite(gn)) return EOT_ERR_NONFINITE;
        if (k == 0 && ss.first_projection) ss.start_err = gn;
        if (gn <= eps) break;                                              // tolerance met
        if (stall_exit) {
            slow = (gn <= 1e-3 && gn > 0.5 * g_prev) ? slow + 1 : 0;
            if (slow >= 2 || k >= o->max_newton) { *stalled = true; break; }
        }
        g_prev = gn;
        if (k >= o->max_newton) { status = EOT_ERR_NOT_CONVERGED; break; }
        // ChiSinkhorn (Alg. 3) to eps^(2/5)
        const double eps_chi = std::pow(eps, 0.4);
        int sweeps = 0;
        for (int it = 0;; ++it) {
            double chi2 = 0.0;
            EOTCHK(reduce_host(x, RED_CHI2, S.rt, S.lr, n, &chi2));
            if (!(chi2 > eps_chi)) break;
            if (it >= o->max_sinkhorn) return EOT_ERR_NOT_CONVERGED;
            p0 = x.passes;
            HIPCHK(launch_add_logdiff(S.u, S.lrt, S.lr, n, x.s));           // u += log r - log r(P)
            EOTCHK(fix_and_refresh(x, prec, beta, S.lrt, ss));
            st->passes_sinkhorn += x.passes - p0;
            st->sinkhorn_iters += 1;
            ss.sweeps += 1;
            ++sweeps;
        }
        HIPCHK(launch_newton_init(S.lr, S.rt, x.nv.rP, x.nv.grad, x.nv.b, x.nv.d, n, x.s));
        // ||grad||_1 = ||r(P) - r~||_1 (c(P) = c): the gn above unless ChiSinkhorn moved u
        double gk = gn;
        if (sweeps > 0) EOTCHK(reduce_host(x, RED_L1, x.nv.grad, nullptr, n, &gk));
        const double eta = std::max(gk, 0.8 * eps / gk);                  // forcing term
        NewtonResult nr;                                                   // Alg. 2 and d_v
        const double rho_in = *rho0;
        p0 = x.passes;
        EOTCHK(newton_solve(x, prec, S.u, S.v, beta, S.lr, S.s, S.rt, S.ct, eta, *rho0,
                            o->max_cg, o->max_levels, S.du, S.dv, &nr, gk));
        st->passes_newton += x.passes - p0;
        st->cg_iters += nr.cg_iters;
        st->levels += nr.levels;
        st->forcing_misses += nr.miss;
        st->rho_last = nr.rho;
        *rho0 = o->adaptive_rho0 ? std::max(0.0, 1.0 - 4.0 * (1.0 - nr.rho)) : 0.0;
        // Backtracking line search on the mass, FP64 passes. A trial whose
        // Armijo test fails by less than the FP64 resolution of the mass is
        // taken (armijo_resolution).
        double slope = 0.0;
        EOTCHK(reduce_host(x, RED_DOT, x.nv.grad, S.du, n, &slope));
        slope = -slope;
        double alpha = 1.0, span = -1.0;
        int32_t bt = 0;
        p0 = x.passes;
        for (;;) {
            HIPCHK(launch_shifted(S.u, alpha, S.du, S.ua, n, x.s));
            HIPCHK(launch_shifted(S.v, alpha, S.dv, S.va, m, x.s));
            HIPCHK(launch_shifted(S.lr, alpha, S.du, S.sh, n, x.s));
            EOTCHK(col_pass(x, EOT_PREC_FP64, S.ua, S.sh, S.va, beta, nullptr, S.colsum));
            double mass = 0.0;
            EOTCHK(reduce_host(x, RED_SUM, S.colsum, nullptr, m, &mass));
            if (std::isfinite(mass) && mass - 1.0 <= 0.99 * alpha * slope) break;
            if (std::isfinite(mass)) {
                if (span < 0.0) {
                    double mu = 0.0, mv = 0.0;
                    EOTCHK(reduce_host(x, RED_MAXABS2, S.u, S.du, n, &mu));
                    EOTCHK(reduce_host(x, RED_MAXABS2, S.v, S.dv, m, &mv));
                    span = mu + mv;
                }
                if (mass - 1.0 - 0.99 * alpha * slope <= armijo_resolution(mass, span)) {
                    st->linesearch_unresolved += 1;
                    break;
                }
            }
            if (bt >= o->max_backtrack) { status = EOT_ERR_NOT_CONVERGED; break; }
            alpha *= 0.5;
            ++bt;
        }
        st->passes_linesearch += x.passes - p0;
        st->backtracks += bt;
        if (status != EOT_OK) break;
        // Step: u <- u + alpha d_u ; v <- v + alpha d_v + log c - log c(P(alpha))
        HIPCHK(launch_copy(S.ua, S.u, n, x.s));
        EOTCHK(clear_flags(x));
        HIPCHK(launch_log_ratio_fix(S.v, S.va, S.lct, S.colsum, m, x.sc.flags, x.s));
        // row refresh
        p0 = x.passes;
        double gk1 = 0.0;
        EOTCHK(refresh(x, prec, beta, S.sh, ss, &gk1));
        st->passes_projection += x.passes - p0;
        st->newton_steps += 1;
        gn_known = gk1;
        const double dk = (gk - gk1) / ((1.0 - eta) * gk);
        dmin = std::min(dmin, dk);
        trace_newton(ss, gk, eta, rho_in, nr.rho, nr.cg_iters, nr.levels, alpha, gk1);
        ++k;
    }
    HIPCHK(launch_add_logdiff(S.u, S.lrt, S.lr, n, x.s));                 // closing row fit
    *delta_min = dmin;
    return status;
}

// Sinkhorn as the projection (the baseline the paper compares against): while
// |r~ - r(P)|_1 > eps, a row fit u += log r~ - log r(P), the column fix and
// the row refresh; then the closing row fit. Mixed precision: stall_exit as
// for tnp (no 1% improvement of the best error in 200 sweeps below 1e-3).
eot_status sinkhorn_project(Ctx& x, int prec, double beta, double eps, SolveState& ss,
                            bool stall_exit = false, bool* stalled = nullptr)
{
    SolveVecs& S = x.sv;
    const eot_solve_opts* o = ss.o;
    eot_solve_stats* st = ss.st;
    const int64_t n = x.n;
    int64_t p0 = x.passes;
    EOTCHK(row_max(x, S.u, S.v, beta, S.sh));
    EOTCHK(fix_and_refresh(x, prec, beta, S.sh, ss));
    st->passes_projection += x.passes - p0;
    if (stalled) *stalled = false;
    eot_status status = EOT_OK;
    double best = INFINITY;
    int32_t k = 0, since_best = 0;
    for (;;) {
        double gn = 0.0;
        EOTCHK(reduce_host(x, RED_L1_DIFF_EXP, S.rt, S.lr, n, &gn));
        if (!std::isfinite(gn)) return EOT_ERR_NONFINITE;
        if (gn <= eps) break;
        if (stall_exit) {
            if (gn < 0.99 * best) { best = gn; since_best = 0; }
            else ++since_best;
            if ((gn <= 1e-3 && since_best >= 200) || k >= o->max_sinkhorn) {
                *stalled = true;
                break;
            }
        }
        if (k >= o->max_sinkhorn) { status = EOT_ERR_NOT_CONVERGED; break; }
        p0 = x.passes;
        HIPCHK(launch_add_logdiff(S.u, S.lrt, S.lr, n, x.s));
        EOTCHK(fix_and_refresh(x, prec, beta, S.lrt, ss));
        st->passes_sinkhorn += x.passes - p0;
        st->sinkhorn_iters += 1;
        ++k;
    }
    HIPCHK(launch_add_logdiff(S.u, S.lrt, S.lr, n, x.s));                 // closing row fit
    return status;
}

// FP64 report at the output potentials against the unsmoothed marginals.
eot_status report(Ctx& x, double beta, const double* r, const double* c, eot_solve_stats* st)
{
    SolveVecs& S = x.sv;
    EOTCHK(row_max(x, S.u, S.v, beta, S.sh));
    PassArgs A = make_args(x, S.u, S.sh, S.v, beta);
    HIPCHK(run_pass(x, A, EOT_PREC_FP64, 2, 1, R2_COST));
    x.passes += 1;
    HIPCHK(launch_merge_rows(x.sc.row_part, x.rtiles, x.n, 2, S.sh, x.tmp_n[0], x.tmp_n[1], 0, x.s));
    HIPCHK(launch_merge_cols(x.sc.col_part, x.ctiles, x.m, 1, x.tmp_m[0], nullptr, x.s));
    HIPCHK(launch_log(x.tmp_n[0], x.tmp_n[2], x.n, x.s));
    HIPCHK(launch_log(x.tmp_m[0], x.tmp_m[2], x.m, x.s));
    double er = 0, ec = 0, cost = 0, mass = 0, ur = 0, vc = 0;
    EOTCHK(reduce_host(x, RED_L1_DIFF_EXP, r, x.tmp_n[2], x.n, &er));
    EOTCHK(reduce_host(x, RED_L1_DIFF_EXP, c, x.tmp_m[2], x.m, &ec));
    EOTCHK(reduce_host(x, RED_SUM, x.tmp_n[1], nullptr, x.n, &cost));
    EOTCHK(reduce_host(x, RED_SUM, x.tmp_n[0], nullptr, x.n, &mass));
    EOTCHK(reduce_host(x, RED_DOT, S.u, r, x.n, &ur));
    EOTCHK(reduce_host(x, RED_DOT, S.v, c, x.m, &vc));
    st->err_r = er;
    st->err_c = ec;
    st->cost = x.cost.kind == EOT_COST_SQEUCLID_POINTS ? cost / x.cost.scale : cost;
    st->dual_value = (ur + vc - mass + 1.0) / beta;
    return EOT_OK;
}

eot_status check_marginal(Ctx& x, const double* p, int64_t k)
{
    double bad = 0.0, sum = 0.0;
    EOTCHK(reduce_host(x, RED_BAD, p, nullptr, k, &bad));
    EOTCHK(reduce_host(x, RED_SUM, p, nullptr, k, &sum));
    if (bad != 0.0 || !(std::fabs(sum - 1.0) <= 1e-9)) return EOT_ERR_BAD_MARGINALS;
    return EOT_OK;
}

eot_status solve_impl(Ctx& x, const double* r, const double* c, const eot_solve_opts* o,
                      const eot_solve_state* resume, eot_solve_state* state_out,
                      eot_solve_trace* trace, double* f_out, double* g_out, eot_solve_stats* st)
{
    x.cg_graph = o->cg_graph != 0;
    const auto t_start = std::chrono::steady_clock::now();
    SolveVecs& S = x.sv;
    const int64_t n = x.n, m = x.m;
    const int prec = o->precision;
    EOTCHK(check_marginal(x, r, n));
    EOTCHK(check_marginal(x, c, m));
    double hr = 0.0, hc = 0.0;
    EOTCHK(reduce_host(x, RED_ENTROPY, r, nullptr, n, &hr));
    EOTCHK(reduce_host(x, RED_ENTROPY, c, nullptr, m, &hc));
    // min(H(r), H(c)), floored at tol: a point-mass marginal has entropy 0,
    // which would ask for an exact projection
    const double hmin = std::max(std::min(hr, hc), o->tol);
    const double beta_f = 1.0 / o->gamma_final;
    const double beta_i = 1.0 / o->gamma_init;
    const double w_c = 0.5 - o->w_r;
    double beta_prev = 0.0;
    double beta = std::min(beta_i, beta_f);
    double q = o->q1;
    double rho0 = 0.0;
    SolveState ss{o, st};
    ss.tr = trace;
    if (trace) trace->n_steps = trace->n_newton = 0;
    eot_status status = EOT_OK;
    bool done = false;
    int32_t t = 1;
    bool fresh = true;                                                     // z^(1) still to set
    if (resume) {                                                          // carried state of Alg. 1
        t = resume->t;
        beta = resume->beta;
        beta_prev = resume->beta_prev;
        q = resume->q;
        rho0 = resume->rho0;
        HIPCHK(launch_copy(resume->u, S.u, n, x.s));
        HIPCHK(launch_copy(resume->v, S.v, m, x.s));
        HIPCHK(launch_copy(resume->u_prev, S.u_prev, n, x.s));
        HIPCHK(launch_copy(resume->v_prev, S.v_prev, m, x.s));
        fresh = false;
    } else if (o->warm_start) {                                            // given z^(1)
        const double gamma0 = beta_i <= beta_f ? o->gamma_init : o->gamma_final;
        HIPCHK(launch_divs(f_out, gamma0, S.u, n, x.s));
        HIPCHK(launch_divs(g_out, gamma0, S.v, m, x.s));
        HIPCHK(launch_copy(S.u, S.u_prev, n, x.s));
        HIPCHK(launch_copy(S.v, S.v_prev, m, x.s));
        fresh = false;
    }
    while (!done) {
        if (t > o->max_mdot) { status = EOT_ERR_NOT_CONVERGED; break; }
        done = (beta == beta_f);                                           // last temperature
        double eps_d = hmin / std::pow(beta, o->p);                        // projection tolerance
        if (done && eps_d > 0.5 * o->tol) eps_d = 0.5 * o->tol;
        HIPCHK(launch_smooth(r, o->w_r * eps_d, 1.0 / (double)n, S.rt, S.lrt, n, x.s));   // smoothing (Sec. 3.4)
        HIPCHK(launch_smooth(c, w_c * eps_d, 1.0 / (double)m, S.ct, S.lct, m, x.s));
        HIPCHK(launch_recip(S.ct, S.inv_ct, m, x.s));
        if (fresh) {                                                       // initial potentials
            HIPCHK(launch_copy(S.lrt, S.u, n, x.s));
            HIPCHK(launch_copy(S.lrt, S.u_prev, n, x.s));
            HIPCHK(launch_copy(S.lct, S.v, m, x.s));
            HIPCHK(launch_copy(S.lct, S.v_prev, m, x.s));
            fresh = false;
        }
        double dmin = INFINITY;                                            // projection
        const bool mixed = prec == EOT_PREC_MIXED;
        bool stalled = false;
        const bool sk = o->projection == EOT_PROJ_SINKHORN;
        const int32_t newton0 = st->newton_steps;
        ss.step = t;
        ss.start_err = 0.0;
        ss.sweeps = 0;
        ss.first_projection = true;
        status = sk ? sinkhorn_project(x, prec, beta, 0.5 * eps_d, ss, mixed, &stalled)
                    : tnp(x, prec, beta, 0.5 * eps_d, &rho0, &dmin, ss, mixed, &stalled);
        st->mixed_stalls += stalled ? 1 : 0;
        if (status == EOT_OK && done && mixed && o->verify_fp64) {
            double dmin64 = INFINITY;
            ss.first_projection = false;
            status = sk ? sinkhorn_project(x, EOT_PREC_FP64, beta, 0.5 * eps_d, ss)
                        : tnp(x, EOT_PREC_FP64, beta, 0.5 * eps_d, &rho0, &dmin64, ss);
        } else if (status == EOT_OK && done && stalled) {
            status = EOT_ERR_NOT_CONVERGED;
        }
        st->delta_min_last = dmin;
        st->mdot_steps = t;
        st->final_gamma = 1.0 / beta;
        if (status == EOT_OK && !done && o->adaptive_q) {                  // AdjustSchedule (Sec. 3.3)
            if (dmin > 0.95) q = std::min(2.0, q * q);
            else if (dmin < 0.8) q = std::sqrt(q);
        }
        if (trace) {
            const int32_t e = trace->n_steps;
            if (e < trace->cap_steps) {
                if (trace->beta) trace->beta[e] = beta;
                if (trace->eps_d) trace->eps_d[e] = eps_d;
                if (trace->start_err) trace->start_err[e] = ss.start_err;
                if (trace->delta_min) trace->delta_min[e] = dmin;
                if (trace->q) trace->q[e] = q;
                if (trace->newton) trace->newton[e] = st->newton_steps - newton0;
                if (trace->sweeps) trace->sweeps[e] = ss.sweeps;
            }
            trace->n_steps = e + 1;
        }
        if (o->verbose) {
            const double secs =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
            std::fprintf(stderr,
                         "[eot] mdot step %d: temperature %.3e, newton %d, cg %d, passes %lld, "
                         "%.1f s\n",
                         t, 1.0 / beta, st->newton_steps, st->cg_iters,
                         (long long)x.passes, secs);
            std::fflush(stderr);
        }
        if (status != EOT_OK || done) break;
        const double beta_next = std::min(q * beta, beta_f);               // next temperature
        const double ratio = (beta_next - beta) / (beta - beta_prev);      // extrapolation
        HIPCHK(launch_extrapolate(S.u, S.u_prev, ratio, n, x.s));
        HIPCHK(launch_extrapolate(S.v, S.v_prev, ratio, m, x.s));
        beta_prev = beta;
        beta = beta_next;
        ++t;
    }
    if (state_out) {
        state_out->t = t;
        state_out->beta = beta;
        state_out->beta_prev = beta_prev;
        state_out->q = q;
        state_out->rho0 = rho0;
        HIPCHK(launch_copy(S.u, state_out->u, n, x.s));
        HIPCHK(launch_copy(S.v, state_out->v, m, x.s));
        HIPCHK(launch_copy(S.u_prev, state_out->u_prev, n, x.s));
        HIPCHK(launch_copy(S.v_prev, state_out->v_prev, m, x.s));
    }
    if (status == EOT_OK || status == EOT_ERR_NOT_CONVERGED) {
        st->final_gamma = 1.0 / beta;
        eot_status rs = report(x, beta, r, c, st);
        if (rs != EOT_OK) return rs;
        HIPCHK(launch_scale(S.u, 1.0 / beta, f_out, n, x.s));
        HIPCHK(launch_scale(S.v, 1.0 / beta, g_out, m, x.s));
        HIPCHK(hipStreamSynchronize(x.s));
    }
    return status;
}

bool bad_gamma(double gamma) { return !(gamma > 0.0) || !std::isfinite(gamma); }

// Device address of the current GPU's copy of `scratch`, looked up once per
// device with that device current and kept.
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

eot_status noalloc_scratch(void** out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return EOT_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return EOT_ERR_HIP;
        }
        g_noalloc_ptr[dev] = ptr;
    }
    *out = g_noalloc_ptr[dev];
    return EOT_OK;
}

bool bad_opts(const eot_solve_opts& o)
{
    return bad_gamma(o.gamma_init) || bad_gamma(o.gamma_final) || !(o.tol > 0.0) ||
           !(o.p >= 1.0) || !(o.q1 > 1.0) || !(o.w_r > 0.0 && o.w_r < 0.5) || o.max_cg < 1 ||
           o.max_levels < 0 || o.max_backtrack < 0 || o.max_newton < 0 || o.max_sinkhorn < 0 ||
           o.max_mdot < 1 || (o.projection != EOT_PROJ_TNP && o.projection != EOT_PROJ_SINKHORN) ||
           (o.warm_start != 0 && o.warm_start != 1) ||
           (o.batch_persistent != 0 && o.batch_persistent != 1);
}

bool bad_state(const eot_solve_state* s, bool in)
{
    if (!s) return false;
    if (!s->u || !s->v || !s->u_prev || !s->v_prev) return true;
    if (!in) return false;
    return s->t < 1 || !(s->beta > 0.0) || !std::isfinite(s->beta) || !(s->beta_prev >= 0.0) ||
           !(s->beta_prev < s->beta) || !(s->q > 1.0) || !(s->rho0 >= 0.0 && s->rho0 < 1.0);
}

size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// One solve on `stream` with workspace ws (options already validated).
eot_status solve_one(const eot_cost* cost, const double* r, const double* c,
                     const eot_solve_opts* opts, double* f, double* g, eot_solve_stats* stats,
                     void* ws, size_t ws_bytes, void* stream,
                     const eot_solve_state* resume = nullptr,
                     eot_solve_state* state_out = nullptr, eot_solve_trace* trace = nullptr,
                     bool single_launch_cg = true)
{
    const auto t0 = std::chrono::steady_clock::now();
    Ctx x;
    x.cgp_ok = single_launch_cg;
    EOTCHK(setup(x, cost, EOT_OP_SOLVE, opts->precision, ws, ws_bytes, stream));
    eot_solve_stats st{};
    eot_status status = solve_impl(x, r, c, opts, resume, state_out, trace, f, g, &st);
    st.passes_other = x.passes - st.passes_newton - st.passes_linesearch - st.passes_sinkhorn -
                      st.passes_projection;
    st.status = status;
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return status;
}

// ---------------------------------------------------------------- gradients
// Derivatives of W and S at (f, g); see eot_gradient in eot.h for the
// formulas. Every pass is FP64 except the CG passes (precision prec).
eot_status gradient_impl(Ctx& x, double gamma, const double* f, const double* g, double w_W,
                         double w_S, double* grad_C, int64_t ldg, double* grad_X, double* grad_Y,
                         double* grad_r, double* grad_c, eot_grad_info* info, int prec)
{
    GradVecs& G = x.gv;
    NewtonVecs& V = x.nv;
    const int64_t n = x.n, m = x.m;
    const double beta = 1.0 / gamma;
    const bool pts = x.cost.kind == EOT_COST_SQEUCLID_POINTS;
    const double cs = pts ? 1.0 / x.cost.scale : 1.0;     // cost sums see |x - y|^2
    HIPCHK(launch_divs(f, gamma, G.u, n, x.s));
    HIPCHK(launch_divs(g, gamma, G.v, m, x.s));
    EOTCHK(row_max(x, G.u, G.v, beta, G.sh));
    // r(P), (P o C) 1, c(P), (P o C)^T 1 in one pass
    PassArgs A = make_args(x, G.u, G.sh, G.v, beta);
    HIPCHK(run_pass(x, A, EOT_PREC_FP64, 2, 2, R2_COST));
    x.passes += 1;
    HIPCHK(launch_merge_rows(x.sc.row_part, x.rtiles, n, 2, G.sh, V.rP, G.a, 0, x.s));
    HIPCHK(launch_merge_cols(x.sc.col_part, x.ctiles, m, 2, G.cP, G.bv, x.s));
    if (pts) {
        HIPCHK(launch_lincomb(G.a, n, cs, G.a, 0.0, nullptr, 0.0, x.s));
        HIPCHK(launch_lincomb(G.bv, m, cs, G.bv, 0.0, nullptr, 0.0, x.s));
    }
    HIPCHK(launch_log(V.rP, G.lr, n, x.s));
    double S = 0.0;
    EOTCHK(reduce_host(x, RED_SUM, G.a, nullptr, n, &S));
    eot_status status = EOT_OK;
    info->cg_iters = 0;
    info->cg_residual = 0.0;
    const double* lam = nullptr;
    const double* mu = nullptr;
    if (w_S != 0.0) {
        // s_i = sum_j P_ij^2 / c(P)_j and t = P (b / c(P)) in one row pass
        HIPCHK(launch_recip(G.cP, G.inv_c, m, x.s));
        HIPCHK(launch_div(G.bv, G.cP, G.tm, 1.0, m, x.s));
        PassArgs B = make_args(x, G.u, G.lr, G.v, beta);
        B.yw0 = G.tm;
        B.yw1 = G.inv_c;
        HIPCHK(run_pass(x, B, EOT_PREC_FP64, 2, 0, R2_SQUARE));
        x.passes += 1;
        HIPCHK(launch_merge_rows(x.sc.row_part, x.rtiles, n, 2, G.lr, V.grad, G.s, 1, x.s));
        // F_r(1) lam = a - P D(c(P))^-1 b
        HIPCHK(launch_lincomb(V.b, n, 1.0, G.a, -1.0, V.grad, 0.0, x.s));
        double bnorm = 0.0;
        EOTCHK(reduce_host(x, RED_L1, V.b, nullptr, n, &bnorm));
        CgScalars h{};
        if (bnorm > 0.0) {
            // FP64 row sums in every lane: this solve goes to a tight residual
            EOTCHK(device_pcg(x, prec, G.u, G.lr, G.v, beta, G.s, G.cP, 1.0, info->tol * bnorm,
                              info->max_cg, &h, true));
            info->cg_iters = h.iters;
            info->cg_residual = h.res_l1 / bnorm;
            if (h.broke || !(h.res_l1 <= info->tol * bnorm)) status = EOT_ERR_NOT_CONVERGED;
        } else {
            HIPCHK(launch_fill(V.dtry, 0.0, n, x.s));
        }
        lam = V.dtry;
        // mu = (b - P^T lam) / c(P)
        EOTCHK(col_pass(x, EOT_PREC_FP64, G.u, G.lr, G.v, beta, lam, G.tm));
        HIPCHK(launch_lincomb(G.mu, m, 1.0, G.bv, -1.0, G.tm, 0.0, x.s));
        HIPCHK(launch_div(G.mu, G.cP, G.mu, 1.0, m, x.s));
        mu = G.mu;
    }
    // G_ij = P_ij (ra_i + cb_j + kappa C_ij)
    HIPCHK(launch_lincomb(G.ra, n, w_S * beta, lam, 0.0, nullptr, w_W + w_S, x.s));
    HIPCHK(launch_lincomb(G.cb, m, w_S * beta, mu, 0.0, nullptr, 0.0, x.s));
    const double kappa = -w_S * beta;
    if (grad_C) HIPCHK(launch_plan_grad(A, G.ra, G.cb, kappa, grad_C, ldg, x.s));
    const int d = x.cost.d;
    if ((grad_X || grad_Y) && d > 3) {
        // high-dimensional points: the n x d (m x d) output is the accumulator
        if (grad_X) {
            HIPCHK(launch_fill(G.g0, 0.0, n, x.s));
            HIPCHK(launch_fill(grad_X, 0.0, n * d, x.s));
            HIPCHK(launch_points_grad_rows_hd(x.cost.X, x.cost.Y, d, n, m, G.u, G.v, beta * cs,
                                              G.ra, G.cb, kappa * cs, G.g0, grad_X, x.s));
            HIPCHK(launch_points_grad_finish_hd(x.cost.X, n, d, 2.0 * cs, G.g0, grad_X, x.s));
            x.passes += 1;
        }
        if (grad_Y) {
            HIPCHK(launch_fill(G.h0, 0.0, m, x.s));
            HIPCHK(launch_fill(grad_Y, 0.0, m * d, x.s));
            HIPCHK(launch_points_grad_rows_hd(x.cost.Y, x.cost.X, d, m, n, G.v, G.u, beta * cs,
                                              G.cb, G.ra, kappa * cs, G.h0, grad_Y, x.s));
            HIPCHK(launch_points_grad_finish_hd(x.cost.Y, m, d, 2.0 * cs, G.h0, grad_Y, x.s));
            x.passes += 1;
        }
    }
    if (grad_X && d <= 3) {
        double* acc[4] = {G.g0, G.gy0, G.gy1, G.gy2};
        for (double* p : acc) HIPCHK(launch_fill(p, 0.0, n, x.s));
        HIPCHK(launch_points_grad_rows(x.cost.X, x.cost.Y, d, n, m, G.u, G.v, beta * cs, G.ra,
                                       G.cb, kappa * cs, G.g0, G.gy0, G.gy1, G.gy2, x.s));
        HIPCHK(launch_points_grad_finish(x.cost.X, n, d, 2.0 * cs, G.g0, G.gy0, G.gy1, G.gy2,
                                         grad_X, x.s));
        x.passes += 1;
    }
    if (grad_Y && d <= 3) {
        double* acc[4] = {G.h0, G.hy0, G.hy1, G.hy2};
        for (double* p : acc) HIPCHK(launch_fill(p, 0.0, m, x.s));
        HIPCHK(launch_points_grad_rows(x.cost.Y, x.cost.X, d, m, n, G.v, G.u, beta * cs, G.cb,
                                       G.ra, kappa * cs, G.h0, G.hy0, G.hy1, G.hy2, x.s));
        HIPCHK(launch_points_grad_finish(x.cost.Y, m, d, 2.0 * cs, G.h0, G.hy0, G.hy1, G.hy2,
                                         grad_Y, x.s));
        x.passes += 1;
    }
    // marginal gradients, mean removed
    if (grad_r) {
        HIPCHK(launch_lincomb(grad_r, n, w_W, f, w_S, lam, 0.0, x.s));
        double sum = 0.0;
        EOTCHK(reduce_host(x, RED_SUM, grad_r, nullptr, n, &sum));
        HIPCHK(launch_lincomb(grad_r, n, 1.0, grad_r, 0.0, nullptr, -sum / (double)n, x.s));
    }
    if (grad_c) {
        HIPCHK(launch_lincomb(grad_c, m, w_W, g, w_S, mu, 0.0, x.s));
        double sum = 0.0;
        EOTCHK(reduce_host(x, RED_SUM, grad_c, nullptr, m, &sum));
        HIPCHK(launch_lincomb(grad_c, m, 1.0, grad_c, 0.0, nullptr, -sum / (double)m, x.s));
    }
    HIPCHK(hipStreamSynchronize(x.s));
    info->S = S;
    return status;
}

// ---------------------------------------------------------------- rounding
// Rounding of the plan onto U(r, c), the last step of Alg. 1; see eot_round in eot.h.
// All passes FP64. Uses the gradient's vectors: n-side u, sh, a (row sums of
// P o C), g0 (r(P)), ra (x), gy0 (er), gy1 (zeros); m-side v, cP, tm (column
// sums of D(x) P), cb (y), mu (ec), h0 (zeros).
eot_status round_impl(Ctx& x, double gamma, const double* f, const double* g, const double* r,
                      const double* c, double* xo, double* yo, double* ero, double* eco,
                      double* plan, int64_t ldp, eot_round_info* info)
{
    GradVecs& G = x.gv;
    const int64_t n = x.n, m = x.m;
    const double beta = 1.0 / gamma;
    const bool pts = x.cost.kind == EOT_COST_SQEUCLID_POINTS;
    const double cs = pts ? 1.0 / x.cost.scale : 1.0;
    double* xs = xo ? xo : G.ra;
    double* ys = yo ? yo : G.cb;
    double* er = ero ? ero : G.gy0;
    double* ec = eco ? eco : G.mu;
    HIPCHK(launch_divs(f, gamma, G.u, n, x.s));
    HIPCHK(launch_divs(g, gamma, G.v, m, x.s));
    EOTCHK(row_max(x, G.u, G.v, beta, G.sh));
    // r(P), (P o C) 1, c(P)
    PassArgs A = make_args(x, G.u, G.sh, G.v, beta);
    HIPCHK(run_pass(x, A, EOT_PREC_FP64, 2, 1, R2_COST));
    x.passes += 1;
    HIPCHK(launch_merge_rows(x.sc.row_part, x.rtiles, n, 2, G.sh, G.g0, G.a, 0, x.s));
    HIPCHK(launch_merge_cols(x.sc.col_part, x.ctiles, m, 1, G.cP, nullptr, x.s));
    double cost_plan = 0.0, err_r = 0.0, err_c = 0.0;
    EOTCHK(reduce_host(x, RED_SUM, G.a, nullptr, n, &cost_plan));
    HIPCHK(launch_round_err(r, nullptr, G.g0, er, n, x.s));
    EOTCHK(reduce_host(x, RED_L1, er, nullptr, n, &err_r));
    HIPCHK(launch_round_err(c, nullptr, G.cP, ec, m, x.s));
    EOTCHK(reduce_host(x, RED_L1, ec, nullptr, m, &err_c));
    // x = min(1, r / r(P)); column sums of D(x) P; y = min(1, c / that)
    HIPCHK(launch_round_scale(r, G.g0, xs, n, x.s));
    PassArgs B = make_args(x, G.u, G.sh, G.v, beta);
    B.xw0 = xs;
    HIPCHK(run_pass(x, B, EOT_PREC_FP64, 0, 1, R2_WEIGHT));
    x.passes += 1;
    HIPCHK(launch_merge_cols(x.sc.col_part, x.ctiles, m, 1, G.tm, nullptr, x.s));
    HIPCHK(launch_round_scale(c, G.tm, ys, m, x.s));
    HIPCHK(launch_round_err(c, ys, G.tm, ec, m, x.s));
    // row sums of P D(y) and of (P o C) D(y): er = r - x o P y, cost of D(x) P D(y)
    PassArgs D = make_args(x, G.u, G.sh, G.v, beta);
    D.yw0 = ys;
    D.yw1 = ys;
    HIPCHK(run_pass(x, D, EOT_PREC_FP64, 2, 0, R2_COST));
    x.passes += 1;
    HIPCHK(launch_merge_rows(x.sc.row_part, x.rtiles, n, 2, G.sh, G.g0, G.a, 0, x.s));
    HIPCHK(launch_round_err(r, xs, G.g0, er, n, x.s));
    double cost_scaled = 0.0, nr = 0.0;
    EOTCHK(reduce_host(x, RED_DOT, xs, G.a, n, &cost_scaled));
    EOTCHK(reduce_host(x, RED_L1, er, nullptr, n, &nr));
    // er^T C ec: a pass with beta = 0 and zero potentials, so every plan entry is 1
    double fix = 0.0;
    if (nr > 0.0) {
        HIPCHK(launch_fill(G.gy1, 0.0, n, x.s));
        HIPCHK(launch_fill(G.h0, 0.0, m, x.s));
        PassArgs Z = make_args(x, G.gy1, G.gy1, G.h0, 0.0);
        Z.yw1 = ec;
        HIPCHK(run_pass(x, Z, EOT_PREC_FP64, 2, 0, R2_COST));
        x.passes += 1;
        HIPCHK(launch_merge_rows(x.sc.row_part, x.rtiles, n, 2, G.gy1, nullptr, G.g0, 0, x.s));
        EOTCHK(reduce_host(x, RED_DOT, er, G.g0, n, &fix));
        fix /= nr;
    }
    if (plan) HIPCHK(launch_plan_round(A, xs, ys, er, ec, nr > 0.0 ? 1.0 / nr : 0.0, plan, ldp, x.s));
    HIPCHK(hipStreamSynchronize(x.s));
    info->cost_plan = cost_plan * cs;
    info->cost_round = (cost_scaled + fix) * cs;
    info->err_r = err_r;
    info->err_c = err_c;
    info->mass_fix = nr;
    return EOT_OK;
}

}  // namespace

namespace {

// ---------------------------------------------------------------- persistent batch
// Problems the persistent team solver takes (eot_team.hip): dense costs and 2-D /
// 3-D points with n, m <= kTeamMaxDim. Team kind: 0 dense FP32, 1 dense FP64,
// 2 / 3 points.
int team_kind(const eot_cost& c)
{
    if (c.n > kTeamMaxDim || c.m > kTeamMaxDim) return -1;
    if (c.kind == EOT_COST_DENSE_F32) return 0;
    if (c.kind == EOT_COST_DENSE_F64) return 1;
    if (c.kind == EOT_COST_SQEUCLID_POINTS && (c.d == 2 || c.d == 3)) return c.d;
    return -1;
}

// Workgroups per team from the largest problem: a team of K workgroups runs at
// about K / 4 compute units (4 workgroups of 256 threads per unit), so the
// largest problems get more of them; small ones still share the chip through
// many teams.
std::atomic<int> g_team_override{0};
std::atomic<int64_t> g_team_entries{0};

int team_size_for(int64_t max_nm)
{
    const int ov = g_team_override.load();
    if (ov > 0) return ov;
    if (max_nm >= (int64_t)4 << 20) return 16;
    if (max_nm >= (int64_t)1 << 20) return 8;
    if (max_nm >= (int64_t)1 << 18) return 4;
    if (max_nm >= (int64_t)1 << 16) return 2;
    return 1;
}

struct TeamPlan {
    int count = 0;                 // problems the team solver can take
    int K = 1;
    int64_t vstride = 0;
    size_t off_table = 0, off_order = 0, off_out = 0, off_vec = 0, off_priv = 0, off_sync = 0;
    size_t bytes = 0;
};

// Workspace layout of the persistent path (sized for the largest grid).
TeamPlan team_plan(int32_t nprob, const eot_batch_problem* probs)
{
    TeamPlan t;
    int64_t dim = 0, max_nm = 0;
    for (int32_t k = 0; k < nprob; ++k) {
        const eot_cost& c = probs[k].cost;
        if (team_kind(c) < 0) continue;
        t.count += 1;
        dim = std::max(dim, std::max(c.n, c.m));
        max_nm = std::max(max_nm, c.n * c.m);
    }
    if (t.count == 0) return t;
    t.K = team_size_for(max_nm);
    t.vstride = (dim + 63) / 64 * 64;
    const int64_t nteams = kTeamMaxGrid / t.K;
    size_t off = 0;
    auto take = [&](size_t b) { const size_t o = off; off += align_up(b); return o; };
    t.off_table = take(sizeof(TeamProblem) * (size_t)nprob);
    t.off_order = take(sizeof(int32_t) * (size_t)nprob);
    t.off_out = take(sizeof(eot_solve_stats) * (size_t)nprob);
    t.off_vec = take(sizeof(double) * (size_t)nteams * (size_t)team_doubles_of(t.vstride, t.K));
    t.off_priv = take(sizeof(double) * (size_t)kTeamMaxGrid * (kTeamPriv + kTeamColVecs) *
                      (size_t)t.vstride);
    t.off_sync = take(sizeof(uint32_t) * kTeamSyncWords * (size_t)kTeamMaxGrid + 256);
    t.bytes = off;
    return t;
}

// Solves the problems marked in `sel` with the persistent team kernel, one
// cooperative launch per cost kind, in order on `s`. Fills st_all / stats_all
// for them.
eot_status team_batch(int32_t nprob, const eot_batch_problem* probs,
                      const eot_solve_opts* opts, const std::vector<char>& sel, char* ws,
                      hipStream_t s, std::vector<eot_status>& st_all,
                      std::vector<eot_solve_stats>& stats_all)
{
    const TeamPlan tp = team_plan(nprob, probs);
    if (tp.count == 0) return EOT_OK;
    const size_t host_bytes = sizeof(TeamProblem) * (size_t)nprob +
                              sizeof(int32_t) * (size_t)nprob +
                              sizeof(eot_solve_stats) * (size_t)nprob;
    void* hbuf = nullptr;                          // pinned staging for the table and the stats
    HIPCHK(hipHostMalloc(&hbuf, host_bytes, hipHostMallocDefault));
    struct Free { void* p; ~Free() { (void)hipHostFree(p); } } free_guard{hbuf};
    TeamProblem* htab = static_cast<TeamProblem*>(hbuf);
    int32_t* hord = reinterpret_cast<int32_t*>(htab + nprob);
    eot_solve_stats* hout = reinterpret_cast<eot_solve_stats*>(hord + nprob);
    for (int32_t k = 0; k < nprob; ++k) {
        const eot_batch_problem& p = probs[k];
        TeamProblem& q = htab[k];
        q.kind = p.cost.kind;
        q.d = p.cost.d;
        q.n = p.cost.n;
        q.m = p.cost.m;
        q.ldc = p.cost.ldc;
        q.C = p.cost.C;
        q.X = p.cost.X;
        q.Y = p.cost.Y;
        q.scale = p.cost.scale;
        q.r = p.r;
        q.c = p.c;
        q.f = p.f;
        q.g = p.g;
    }
    TeamProblem* dtab = reinterpret_cast<TeamProblem*>(ws + tp.off_table);
    int32_t* dord = reinterpret_cast<int32_t*>(ws + tp.off_order);
    eot_solve_stats* dout = reinterpret_cast<eot_solve_stats*>(ws + tp.off_out);
    HIPCHK(hipMemcpyAsync(dtab, htab, sizeof(TeamProblem) * (size_t)nprob,
                          hipMemcpyHostToDevice, s));
    for (int kind = 0; kind < 4; ++kind) {
        std::vector<int32_t> order;
        for (int32_t k = 0; k < nprob; ++k)
            if (sel[(size_t)k] && team_kind(probs[k].cost) == kind) order.push_back(k);
        if (order.empty()) continue;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return probs[a].cost.n * probs[a].cost.m > probs[b].cost.n * probs[b].cost.m;
        });
        int bpc = 0, cus = 0;
        HIPCHK(team_max_grid(kind, &bpc, &cus));
        int K = tp.K;
        int grid = std::min(bpc * cus, kTeamMaxGrid);
        while (K > 1 && grid < 8 * K) K /= 2;
        // the team vectors were sized for kTeamMaxGrid / tp.K teams of tp.K members
        const int64_t alloc = (int64_t)(kTeamMaxGrid / tp.K) * team_doubles_of(tp.vstride, tp.K);
        grid = (int)std::min<int64_t>(grid, alloc / team_doubles_of(tp.vstride, K) * K);
        grid = grid / (8 * K) * (8 * K);
        if (grid < 8) return EOT_ERR_HIP;           // no co-resident team fits
        // wait for the table upload before the order array is overwritten
        HIPCHK(hipStreamSynchronize(s));
        std::memcpy(hord, order.data(), sizeof(int32_t) * order.size());
        HIPCHK(hipMemcpyAsync(dord, hord, sizeof(int32_t) * order.size(),
                              hipMemcpyHostToDevice, s));
        uint32_t* sync = reinterpret_cast<uint32_t*>(ws + tp.off_sync);
        const int nteams = grid / K;
        const size_t sync_words = kTeamSyncWords * (size_t)nteams + 64;
        HIPCHK(launch_fill(reinterpret_cast<double*>(sync), 0.0, (int64_t)(sync_words / 2), s));
        TeamLaunch L{};
        L.probs = dtab;
        L.order = dord;
        L.nprob = (int32_t)order.size();
        L.K = K;
        L.nteams = nteams;
        L.out = dout;
        L.vec = reinterpret_cast<double*>(ws + tp.off_vec);
        L.vstride = tp.vstride;
        L.team_doubles = team_doubles_of(tp.vstride, K);
        L.priv = reinterpret_cast<double*>(ws + tp.off_priv);
        L.sync = sync;
        L.queue = reinterpret_cast<int32_t*>(sync + kTeamSyncWords * (size_t)nteams);
        L.abort = L.queue + 16;
        L.opts = *opts;
        const int64_t epw = g_team_entries.load();
        L.entries_per_wg = epw > 0 ? epw : kTeamEntriesPerWg;
        HIPCHK(launch_team_solve(kind, L, grid, s));
        HIPCHK(hipMemcpyAsync(hout, dout, sizeof(eot_solve_stats) * (size_t)nprob,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int dev = 0, khz = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        for (int32_t k : order) {
            stats_all[(size_t)k] = hout[k];
            stats_all[(size_t)k].seconds = khz > 0 ? hout[k].seconds / (1e3 * khz) : 0.0;
            st_all[(size_t)k] = (eot_status)hout[k].status;
        }
    }
    return EOT_OK;
}

// Host workers: `nw` threads, each with its own non-blocking stream (default
// priority) and workspace slice wbase + w * slice, take the problems of
// `order` (already sorted) one at a time and run job(i, base, slice, stream);
// st_all[i] receives its status. The caller's stream is ordered before and
// after all of them. Returns EOT_ERR_HIP when the streams could not be set up
// (the problems no worker reached keep the status they had).
template <class Job>
eot_status run_host_workers(const std::vector<int32_t>& order, int nw, char* wbase, size_t slice,
                            hipStream_t caller, std::vector<eot_status>& st_all, Job job)
{
    const int32_t n_work = (int32_t)order.size();
    if (n_work == 0) return EOT_OK;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipEvent_t start;
    HIPCHK(hipEventCreateWithFlags(&start, hipEventDisableTiming));
    HIPCHK(hipEventRecord(start, caller));
    std::vector<hipStream_t> streams((size_t)nw, nullptr);
    std::vector<hipEvent_t> done((size_t)nw, nullptr);
    eot_status setup_err = EOT_OK;
    for (int w = 0; w < nw && setup_err == EOT_OK; ++w) {
        if (hipStreamCreateWithFlags(&streams[w], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&done[w], hipEventDisableTiming) != hipSuccess ||
            hipStreamWaitEvent(streams[w], start, 0) != hipSuccess)
            setup_err = EOT_ERR_HIP;
    }
    std::atomic<int32_t> next{0};
    auto work = [&](int w) {
        if (hipSetDevice(dev) != hipSuccess) return;
        char* base = wbase + (size_t)w * slice;
        for (;;) {
            const int32_t k = next.fetch_add(1);
            if (k >= n_work) break;
            const int32_t i = order[(size_t)k];
            st_all[(size_t)i] = job(i, base, slice, streams[w]);
        }
    };
    if (setup_err == EOT_OK) {
        std::vector<std::thread> pool;
        for (int w = 1; w < nw; ++w) pool.emplace_back(work, w);
        work(0);
        for (auto& t : pool) t.join();
    }
    for (int w = 0; w < nw; ++w) {
        if (streams[w]) {
            if (done[w] && hipEventRecord(done[w], streams[w]) == hipSuccess)
                (void)hipStreamWaitEvent(caller, done[w], 0);
        }
    }
    for (int w = 0; w < nw; ++w) {
        if (streams[w]) (void)hipStreamSynchronize(streams[w]);
        if (done[w]) (void)hipEventDestroy(done[w]);
        if (streams[w]) (void)hipStreamDestroy(streams[w]);
    }
    (void)hipEventDestroy(start);
    return setup_err;
}

// Arguments of one gradient (eot_gradient, each problem of eot_gradient_batched).
eot_status grad_check(const eot_cost* cost, double gamma, const double* f, const double* g,
                      double w_W, double w_S, const eot_grad_info* info, const double* grad_C,
                      int64_t ldg, const double* grad_X, const double* grad_Y)
{
    if (!f || !g || !info || bad_gamma(gamma)) return EOT_ERR_INVALID_ARG;
    if (!std::isfinite(w_W) || !std::isfinite(w_S)) return EOT_ERR_INVALID_ARG;
    if (w_S != 0.0 && (!(info->tol > 0.0) || info->max_cg < 1)) return EOT_ERR_INVALID_ARG;
    EOTCHK(check_cost(cost));
    const bool pts = cost->kind == EOT_COST_SQEUCLID_POINTS;
    if (grad_C && (pts || ldg < cost->m)) return EOT_ERR_INVALID_ARG;
    if ((grad_X || grad_Y) && !pts) return EOT_ERR_INVALID_ARG;
    return EOT_OK;
}

}  // namespace

extern "C" {

eot_status eot_workspace_size(int32_t op, const eot_cost* cost, int32_t prec, size_t* bytes)
{
    if (!bytes) return EOT_ERR_INVALID_ARG;
    eot_status cs = check_cost(cost);
    if (cs != EOT_OK) return cs;
    if (op < EOT_OP_MARGINALS || op > EOT_OP_ROUND) return EOT_ERR_INVALID_ARG;
    (void)prec;
    Ctx x;
    x.cost = *cost;
    x.n = cost->n;
    x.m = cost->m;
    layout(x);
    Arena dry;
    carve(dry, x, op);
    *bytes = dry.off + kAlign;
    return EOT_OK;
}

eot_status eot_marginals(const eot_cost* cost, double gamma, const double* f, const double* g,
                         const double* row_shift, double* log_rP, double* log_cP, double* mass,
                         const double* c_for_s, double* s, int32_t prec, void* ws,
                         size_t ws_bytes, void* stream)
{
    if (!f || !g || bad_gamma(gamma)) return EOT_ERR_INVALID_ARG;
    if (s && !c_for_s) return EOT_ERR_INVALID_ARG;
    if (!log_rP && !log_cP && !mass && !s) return EOT_ERR_INVALID_ARG;
    Ctx x;
    EOTCHK(setup(x, cost, EOT_OP_MARGINALS, prec, ws, ws_bytes, stream));
    const double beta = 1.0 / gamma;
    double* u = x.tmp_n[0];
    double* a = x.tmp_n[1];
    double* lr = log_rP ? log_rP : x.tmp_n[2];
    double* v = x.tmp_m[0];
    HIPCHK(launch_divs(f, gamma, u, x.n, x.s));
    HIPCHK(launch_divs(g, gamma, v, x.m, x.s));
    if (row_shift) HIPCHK(launch_copy(row_shift, a, x.n, x.s));
    else EOTCHK(row_max(x, u, v, beta, a));
    const bool rows = log_rP || mass || s;
    const int nr = rows ? (s ? 2 : 1) : 0;
    const int nc = log_cP ? 1 : 0;
    if (s) HIPCHK(launch_recip(c_for_s, x.tmp_m[1], x.m, x.s));
    PassArgs A = make_args(x, u, a, v, beta);
    A.yw1 = s ? x.tmp_m[1] : nullptr;
    HIPCHK(run_pass(x, A, prec, nr, nc, R2_SQUARE));
    if (rows) {
        HIPCHK(launch_log_row_from_sums(x.sc.row_part, x.rtiles, x.n, a, lr, x.sc.flags, x.s));
        if (s) HIPCHK(launch_merge_rows(x.sc.row_part, x.rtiles, x.n, 2, a, nullptr, s, 1, x.s));
        if (mass) {
            int nb = 0;
            HIPCHK(launch_reduce(RED_SUM_EXP, nullptr, lr, x.n, x.sc.red, &nb, x.s));
            HIPCHK(launch_finish_sum(x.sc.red, nb, mass, x.s));
        }
    }
    if (log_cP) {
        HIPCHK(launch_merge_cols(x.sc.col_part, x.ctiles, x.m, 1, x.tmp_m[2], nullptr, x.s));
        HIPCHK(launch_log(x.tmp_m[2], log_cP, x.m, x.s));
    }
    return EOT_OK;
}

eot_status eot_hvp(const eot_cost* cost, double gamma, const double* f, const double* g,
                   const double* row_shift, double rho, const double* xv, const double* yv,
                   double* Hx, double* Hy, int32_t prec, void* ws, size_t ws_bytes, void* stream)
{
    if (!f || !g || !xv || !yv || !Hx || !Hy || bad_gamma(gamma)) return EOT_ERR_INVALID_ARG;
    if (!(rho >= 0.0 && rho <= 1.0)) return EOT_ERR_INVALID_ARG;
    Ctx x;
    EOTCHK(setup(x, cost, EOT_OP_HVP, prec, ws, ws_bytes, stream));
    const double beta = 1.0 / gamma;
    double* u = x.tmp_n[0];
    double* a = x.tmp_n[1];
    double* v = x.tmp_m[0];
    HIPCHK(launch_divs(f, gamma, u, x.n, x.s));
    HIPCHK(launch_divs(g, gamma, v, x.m, x.s));
    if (row_shift) HIPCHK(launch_copy(row_shift, a, x.n, x.s));
    else EOTCHK(row_max(x, u, v, beta, a));
    // One pass: row weight x_i + sqrt(rho) y_j, column weight sqrt(rho) x_i + y_j.
    const double srho = std::sqrt(rho);
    double* sy = x.tmp_m[1];
    HIPCHK(launch_scale(yv, srho, sy, x.m, x.s));
    PassArgs A = make_args(x, u, a, v, beta);
    A.yw0 = sy;
    A.yw1 = yv;
    A.xw1 = xv;
    A.hvp_srho = srho;
    HIPCHK(run_pass(x, A, prec, 1, 1, R2_HVP));
    HIPCHK(launch_hvp_finish(x.sc.row_part, x.rtiles, x.sc.col_part, x.ctiles, x.n, x.m, a, Hx,
                             Hy, x.s));
    return EOT_OK;
}

eot_status eot_hvp_noalloc(const eot_cost* cost, double gamma, const double* f, const double* g,
                           const double* row_shift, double rho, const double* xv,
                           const double* yv, double* Hx, double* Hy, int32_t prec, void* stream)
{
    if (!f || !g || !xv || !yv || !Hx || !Hy || bad_gamma(gamma)) return EOT_ERR_INVALID_ARG;
    if (!(rho >= 0.0 && rho <= 1.0)) return EOT_ERR_INVALID_ARG;
    size_t need = 0;
    EOTCHK(eot_workspace_size(EOT_OP_HVP, cost, prec, &need));
    if (need > kNoAllocBytes) return EOT_ERR_WORKSPACE;
    void* ws = nullptr;
    EOTCHK(noalloc_scratch(&ws));
    return eot_hvp(cost, gamma, f, g, row_shift, rho, xv, yv, Hx, Hy, prec, ws, kNoAllocBytes,
                   stream);
}

eot_status eot_hvp_with_marginals(const eot_cost* cost, double gamma, const double* f,
                                  const double* g, const double* log_rP, const double* log_cP,
                                  double rho, const double* xv, const double* yv, double* Hx,
                                  double* Hy, int32_t prec, void* ws, size_t ws_bytes, void* stream)
{
    if (!f || !g || !log_rP || !log_cP || !xv || !yv || !Hx || !Hy || bad_gamma(gamma))
        return EOT_ERR_INVALID_ARG;
    if (!(rho >= 0.0 && rho <= 1.0)) return EOT_ERR_INVALID_ARG;
    Ctx x;
    EOTCHK(setup(x, cost, EOT_OP_HVP, prec, ws, ws_bytes, stream));
    const double beta = 1.0 / gamma;
    double* u = x.tmp_n[0];
    double* v = x.tmp_m[0];
    HIPCHK(launch_divs(f, gamma, u, x.n, x.s));
    HIPCHK(launch_divs(g, gamma, v, x.m, x.s));
    // One pass, one weighted sum per direction: (P y)_i over rows, (P^T x)_j over
    // columns; log r(P) doubles as the row shift. The diagonal blocks come from
    // the given marginals in the epilogue.
    PassArgs A = make_args(x, u, log_rP, v, beta);
    A.yw0 = yv;
    A.xw0 = xv;
    HIPCHK(run_pass(x, A, prec, 1, 1, R2_WEIGHT));
    HIPCHK(launch_hvp_finish_diag(x.sc.row_part, x.rtiles, x.sc.col_part, x.ctiles, x.n, x.m,
                                  log_rP, std::sqrt(rho), log_rP, log_cP, xv, yv, Hx, Hy, x.s));
    return EOT_OK;
}

eot_status eot_newton_cg(const eot_cost* cost, double gamma, const double* f, const double* g,
                         const double* r, const double* c, double eta, double rho0,
                         int32_t max_cg, int32_t max_levels, double* dir_f, double* dir_g,
                         eot_newton_stats* stats, int32_t prec, void* ws, size_t ws_bytes,
                         void* stream)
{
    if (!f || !g || !r || !c || !dir_f || !dir_g || bad_gamma(gamma)) return EOT_ERR_INVALID_ARG;
    if (!(eta > 0.0) || !(rho0 >= 0.0 && rho0 < 1.0) || max_cg < 1 || max_levels < 0)
        return EOT_ERR_INVALID_ARG;
    Ctx x;
    EOTCHK(setup(x, cost, EOT_OP_NEWTON_CG, prec, ws, ws_bytes, stream));
    const double beta = 1.0 / gamma;
    double* u = x.tmp_n[0];
    double* lr = x.tmp_n[1];
    double* s = x.tmp_n[2];
    double* a = x.tmp_n[3];
    double* v = x.tmp_m[0];
    double* inv_c = x.tmp_m[1];
    HIPCHK(launch_divs(f, gamma, u, x.n, x.s));
    HIPCHK(launch_divs(g, gamma, v, x.m, x.s));
    HIPCHK(launch_recip(c, inv_c, x.m, x.s));
    EOTCHK(row_max(x, u, v, beta, a));
    EOTCHK(row_pass(x, prec, u, a, v, beta, inv_c, lr, s));
    NewtonResult nr;
    double* du = a;                 // the row maxima are not needed past the row pass
    double* dv = x.tmp_m[2];
    EOTCHK(newton_solve(x, prec, u, v, beta, lr, s, r, c, eta, rho0, max_cg, max_levels, du, dv,
                        &nr));
    HIPCHK(launch_scale(du, gamma, dir_f, x.n, x.s));
    HIPCHK(launch_scale(dv, gamma, dir_g, x.m, x.s));
    HIPCHK(hipStreamSynchronize(x.s));
    if (stats) {
        stats->rho_out = nr.rho;
        stats->cg_iters = nr.cg_iters;
        stats->levels = nr.levels;
        stats->forcing_miss = nr.miss;
        stats->status = EOT_OK;
        stats->passes = x.passes;
        stats->forcing_ratio = nr.forcing_ratio;
    }
    return EOT_OK;
}

void eot_solve_opts_default(eot_solve_opts* o)
{
    if (!o) return;
    o->gamma_init = 1.0 / 32.0;
    o->gamma_final = 1e-3;
    o->tol = 1e-6;
    o->p = 1.5;
    o->q1 = 2.0;
    o->w_r = 0.45;
    o->adaptive_q = 1;
    o->adaptive_rho0 = 1;
    o->max_cg = 1000;
    o->max_levels = 30;
    o->max_backtrack = 60;
    o->max_newton = 200;
    o->max_sinkhorn = 10000;
    o->max_mdot = 500;
    o->precision = EOT_PREC_FP64;
    o->verify_fp64 = 1;
    o->projection = EOT_PROJ_TNP;
    o->cg_graph = 0;
    o->verbose = 0;
    o->warm_start = 0;
    o->batch_persistent = 1;
}

eot_status eot_solve(const eot_cost* cost, const double* r, const double* c,
                     const eot_solve_opts* opts, double* f, double* g, eot_solve_stats* stats,
                     void* ws, size_t ws_bytes, void* stream)
{
    if (!r || !c || !opts || !f || !g) return EOT_ERR_INVALID_ARG;
    if (bad_opts(*opts)) return EOT_ERR_INVALID_ARG;
    return solve_one(cost, r, c, opts, f, g, stats, ws, ws_bytes, stream);
}

eot_status eot_solve_ex(const eot_cost* cost, const double* r, const double* c,
                        const eot_solve_opts* opts, const eot_solve_state* resume,
                        eot_solve_state* state_out, eot_solve_trace* trace, double* f,
                        double* g, eot_solve_stats* stats, void* ws, size_t ws_bytes,
                        void* stream)
{
    if (!r || !c || !opts || !f || !g) return EOT_ERR_INVALID_ARG;
    if (bad_opts(*opts) || bad_state(resume, true) || bad_state(state_out, false))
        return EOT_ERR_INVALID_ARG;
    if (trace && (trace->cap_steps < 0 || trace->cap_newton < 0)) return EOT_ERR_INVALID_ARG;
    return solve_one(cost, r, c, opts, f, g, stats, ws, ws_bytes, stream, resume, state_out,
                     trace);
}

eot_status eot_workspace_size_batched(int32_t nprob, const eot_batch_problem* probs,
                                      int32_t workers, size_t* bytes)
{
    if (!bytes || nprob < 1 || !probs || workers < 1) return EOT_ERR_INVALID_ARG;
    size_t slice = 0;
    for (int32_t k = 0; k < nprob; ++k) {
        size_t b = 0;
        EOTCHK(eot_workspace_size(EOT_OP_SOLVE, &probs[k].cost, 0, &b));
        slice = std::max(slice, align_up(b));
    }
    const TeamPlan tp = team_plan(nprob, probs);
    *bytes = tp.bytes + slice * (size_t)std::min(workers, nprob) + kAlign;
    return EOT_OK;
}

eot_status eot_solve_batched(int32_t nprob, const eot_batch_problem* probs,
                             const eot_solve_opts* opts, int32_t workers,
                             eot_solve_stats* stats, int32_t* status, void* ws, size_t ws_bytes,
                             void* stream)
{
    if (nprob < 1 || !probs || !opts || workers < 1) return EOT_ERR_INVALID_ARG;
    if (bad_opts(*opts)) return EOT_ERR_INVALID_ARG;
    for (int32_t k = 0; k < nprob; ++k) {
        const eot_batch_problem& p = probs[k];
        if (!p.r || !p.c || !p.f || !p.g) return EOT_ERR_INVALID_ARG;
        EOTCHK(check_cost(&p.cost));
    }
    size_t need = 0;
    EOTCHK(eot_workspace_size_batched(nprob, probs, workers, &need));
    if (!ws || ws_bytes < need - kAlign || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0)
        return EOT_ERR_WORKSPACE;
    hipStream_t caller = static_cast<hipStream_t>(stream);
    // a problem no worker reached (a worker that could not select the device) reports EOT_ERR_HIP
    std::vector<eot_status> st_all((size_t)nprob, EOT_ERR_HIP);
    std::vector<eot_solve_stats> stats_all((size_t)nprob);
    // Persistent path: the problems the team kernel takes.
    const TeamPlan tp = team_plan(nprob, probs);
    std::vector<char> on_team((size_t)nprob, 0);
    const bool persistent = opts->batch_persistent != 0 && opts->projection == EOT_PROJ_TNP &&
                            opts->warm_start == 0;
    int32_t n_team = 0;
    if (persistent)
        for (int32_t k = 0; k < nprob; ++k)
            if (team_kind(probs[k].cost) >= 0 &&
                !(probs[k].cost.kind == EOT_COST_DENSE_F64 && opts->precision == EOT_PREC_MIXED)) {
                on_team[(size_t)k] = 1;
                ++n_team;
            }
    if (n_team > 0) {
        const eot_status ts = team_batch(nprob, probs, opts, on_team, static_cast<char*>(ws),
                                         caller, st_all, stats_all);
        if (ts != EOT_OK) return ts;
    }
    // Host workers for the rest.
    std::vector<int32_t> order;
    for (int32_t k = 0; k < nprob; ++k)
        if (!on_team[(size_t)k]) order.push_back(k);
    const int nw = std::min<int>(workers, std::max<int>(1, (int)order.size()));
    char* wbase = static_cast<char*>(ws) + tp.bytes;
    const size_t slice = (need - kAlign - tp.bytes) / (size_t)std::min(workers, nprob);
    // Longest first: problems in decreasing n m, dealt to whichever worker is free.
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return probs[a].cost.n * probs[a].cost.m > probs[b].cost.n * probs[b].cost.m;
    });
    const eot_status first = run_host_workers(
        order, nw, wbase, slice, caller, st_all,
        [&](int32_t i, char* base, size_t bytes, hipStream_t st) {
            const eot_batch_problem& p = probs[i];
            // no single-launch CG here: cooperative launches from 8 threads at once
            return solve_one(&p.cost, p.r, p.c, opts, p.f, p.g, &stats_all[(size_t)i], base, bytes,
                             st, nullptr, nullptr, nullptr, false);
        });
    for (int32_t i = 0; i < nprob; ++i) {
        if (status) status[i] = st_all[(size_t)i];
        if (stats) stats[i] = stats_all[(size_t)i];
    }
    if (first != EOT_OK) return first;
    for (int32_t i = 0; i < nprob; ++i)
        if (st_all[(size_t)i] != EOT_OK) return st_all[(size_t)i];
    return EOT_OK;
}

eot_status eot_gradient(const eot_cost* cost, double gamma, const double* f, const double* g,
                        double w_W, double w_S, double* grad_C, int64_t ldg, double* grad_X,
                        double* grad_Y, double* grad_r, double* grad_c, eot_grad_info* info,
                        int32_t prec, void* ws, size_t ws_bytes, void* stream)
{
    EOTCHK(grad_check(cost, gamma, f, g, w_W, w_S, info, grad_C, ldg, grad_X, grad_Y));
    Ctx x;
    EOTCHK(setup(x, cost, EOT_OP_GRADIENT, prec, ws, ws_bytes, stream));
    return gradient_impl(x, gamma, f, g, w_W, w_S, grad_C, ldg, grad_X, grad_Y, grad_r, grad_c,
                         info, prec);
}

eot_status eot_workspace_size_gradient_batched(int32_t nprob, const eot_grad_problem* probs,
                                               int32_t workers, size_t* bytes)
{
    if (!bytes || nprob < 1 || !probs || workers < 1) return EOT_ERR_INVALID_ARG;
    size_t slice = 0;
    for (int32_t k = 0; k < nprob; ++k) {
        size_t b = 0;
        EOTCHK(eot_workspace_size(EOT_OP_GRADIENT, &probs[k].cost, 0, &b));
        slice = std::max(slice, align_up(b));
    }
    *bytes = slice * (size_t)std::min(workers, nprob) + kAlign;
    return EOT_OK;
}

eot_status eot_gradient_batched(int32_t nprob, const eot_grad_problem* probs, double w_W,
                                double w_S, eot_grad_info* info, int32_t prec, int32_t workers,
                                int32_t* status, void* ws, size_t ws_bytes, void* stream)
{
    if (nprob < 1 || !probs || !info || workers < 1) return EOT_ERR_INVALID_ARG;
    for (int32_t k = 0; k < nprob; ++k) {
        const eot_grad_problem& p = probs[k];
        EOTCHK(grad_check(&p.cost, p.gamma, p.f, p.g, w_W, w_S, &info[k], p.grad_C, p.ldg,
                          p.grad_X, p.grad_Y));
    }
    size_t need = 0;
    EOTCHK(eot_workspace_size_gradient_batched(nprob, probs, workers, &need));
    if (!ws || ws_bytes < need - kAlign || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0)
        return EOT_ERR_WORKSPACE;
    std::vector<eot_status> st_all((size_t)nprob, EOT_ERR_HIP);
    std::vector<int32_t> order((size_t)nprob);
    for (int32_t k = 0; k < nprob; ++k) order[(size_t)k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return probs[a].cost.n * probs[a].cost.m > probs[b].cost.n * probs[b].cost.m;
    });
    const int nw = std::min<int>(workers, nprob);
    const size_t slice = (need - kAlign) / (size_t)nw;
    const eot_status first = run_host_workers(
        order, nw, static_cast<char*>(ws), slice, static_cast<hipStream_t>(stream), st_all,
        [&](int32_t i, char* base, size_t bytes, hipStream_t st) -> eot_status {
            const eot_grad_problem& p = probs[i];
            Ctx x;
            x.cgp_ok = false;                    // no cooperative launches from several threads
            EOTCHK(setup(x, &p.cost, EOT_OP_GRADIENT, prec, base, bytes, st));
            return gradient_impl(x, p.gamma, p.f, p.g, w_W, w_S, p.grad_C, p.ldg, p.grad_X,
                                 p.grad_Y, p.grad_r, p.grad_c, &info[i], prec);
        });
    if (status)
        for (int32_t i = 0; i < nprob; ++i) status[i] = st_all[(size_t)i];
    if (first != EOT_OK) return first;
    for (int32_t i = 0; i < nprob; ++i)
        if (st_all[(size_t)i] != EOT_OK) return st_all[(size_t)i];
    return EOT_OK;
}

eot_status eot_round(const eot_cost* cost, double gamma, const double* f, const double* g,
                     const double* r, const double* c, double* xo, double* yo, double* ero,
                     double* eco, double* plan, int64_t ldp, eot_round_info* info, void* ws,
                     size_t ws_bytes, void* stream)
{
    if (!f || !g || !r || !c || !info || bad_gamma(gamma)) return EOT_ERR_INVALID_ARG;
    EOTCHK(check_cost(cost));
    if (plan && (cost->kind == EOT_COST_SQEUCLID_POINTS || ldp < cost->m))
        return EOT_ERR_INVALID_ARG;
    Ctx x;
    EOTCHK(setup(x, cost, EOT_OP_ROUND, EOT_PREC_FP64, ws, ws_bytes, stream));
    return round_impl(x, gamma, f, g, r, c, xo, yo, ero, eco, plan, ldp, info);
}

eot_status eot_set_rows_per_tile(int32_t rows)
{
    if (rows != 0 && (rows < 8 || rows > kTileRows || (rows & (rows - 1)) != 0))
        return EOT_ERR_INVALID_ARG;
    g_rows_override.store(rows);
    return EOT_OK;
}

eot_status eot_set_cg_persist(int32_t enable, int32_t grid)
{
    if ((enable != 0 && enable != 1) || grid < 0 || grid > kCgpMaxGrid)
        return EOT_ERR_INVALID_ARG;
    g_cgp_mode.store(enable);
    g_cgp_grid.store(grid);
    return EOT_OK;
}

eot_status eot_set_team_size(int32_t k, int64_t entries_per_wg)
{
    if (k < 0 || k > kTeamMaxK || (k & (k - 1)) != 0 || entries_per_wg < 0)
        return EOT_ERR_INVALID_ARG;
    g_team_override.store(k);
    g_team_entries.store(entries_per_wg);
    return EOT_OK;
}

eot_status eot_pass_timing(int32_t enable)
{
    return set_pass_timing(enable != 0) == hipSuccess ? EOT_OK : EOT_ERR_HIP;
}

eot_status eot_pass_timing_read(int32_t nr, int32_t nc, int32_t prec, int32_t fused_hvp,
                                int64_t* launches, double* milliseconds)
{
    if (!launches || !milliseconds) return EOT_ERR_INVALID_ARG;
    return read_pass_timing(nr, nc, prec, fused_hvp, launches, milliseconds) == hipSuccess
               ? EOT_OK
               : EOT_ERR_HIP;
}

const char* eot_status_string(int32_t status)
{
    switch (status) {
        case EOT_OK: return "ok";
        case EOT_ERR_INVALID_ARG: return "invalid argument";
        case EOT_ERR_BAD_MARGINALS: return "marginals must be positive, finite and sum to 1";
        case EOT_ERR_NONFINITE: return "non-finite values that the range fallback could not repair";
        case EOT_ERR_NOT_CONVERGED: return "iteration cap reached; outputs hold the last iterate";
        case EOT_ERR_WORKSPACE: return "workspace missing, too small or not 256-byte aligned";
        case EOT_ERR_UNSUPPORTED: return "unsupported cost kind / precision combination";
        case EOT_ERR_HIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

const char* eot_version(void) { return "0.1.0 gfx950"; }

}  // extern "C"
