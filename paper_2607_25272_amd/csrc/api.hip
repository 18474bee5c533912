// Host driver and C ABI of the SPCG library: argument checking, handles,
// workspaces, the PCG stage runner and Algorithm 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "rng.hpp"
#include "spcg.h"

using namespace spcg;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t ensure(size_t bytes) {
        if (bytes <= n && p) return hipSuccess;
        release();
        if (bytes == 0) bytes = 256;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return e;
        }
        n = bytes;
        return hipSuccess;
    }
    template <typename T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

constexpr int MAX_TIMED = 256;

// Static scratch of spcg_pcg_stage_noalloc: product partials for at most
// NA_BLOCKS blocks of NA_DMAX columns (s and g), the per-block scalars, the
// d-space vectors and the PCG scalar record with its two counters.  Each
// device holds its own copy for the life of the process; host code reaches
// it only through the address that hipGetSymbolAddress returns on that
// device (na_scratch_address), never through the symbol itself.
constexpr int64_t NA_DMAX = 1024;
constexpr int64_t NA_BLOCKS = 256;
constexpr size_t NA_PART = (size_t)NA_BLOCKS * NA_DMAX;
constexpr size_t NA_DVEC = 5 * (size_t)NA_DMAX + 1024;
constexpr size_t NA_SCAL = 32;   // 256 bytes: PcgScalars and the counters
constexpr size_t NA_DOUBLES = 2 * NA_PART + 2 * (size_t)NA_BLOCKS + NA_DVEC + NA_SCAL;
__device__ __align__(256) double scratch[NA_DOUBLES];
static_assert(sizeof(PcgScalars) + 2 * sizeof(unsigned int) <= NA_SCAL * sizeof(double), "scalar slot");

constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mutex;
double* na_ptr[NA_MAX_DEVICES] = {};

// Device address of this device's scratch (the device must be current);
// looked up once per device.
hipError_t na_scratch_address(int device, double** out) {
    *out = nullptr;
    if (device < 0 || device >= NA_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(na_mutex);
    if (!na_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        na_ptr[device] = static_cast<double*>(p);
    }
    *out = na_ptr[device];
    return hipSuccess;
}

}  // namespace

namespace {
struct BatchWork;

// Per-kernel-class timing of an instrumented solve (time_products = 2):
// one start/end event pair per timed launch, recorded on the library stream.
constexpr int KT_MAX = 2048;
struct KTimer {
    hipEvent_t ev[2 * KT_MAX] = {};
    int cls[KT_MAX] = {};
    double bytes[KT_MAX] = {};
    int used = 0;
    bool ready = false;
    ~KTimer() {
        if (ready)
            for (auto& e : ev) (void)hipEventDestroy(e);
    }
};
}

struct spcg_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    std::string err;
    // product partials and d-space state
    DevBuf part_s, part_g, part_scal;
    DevBuf dvec;      // g z p s gt (5 * dpad) + blk (1024)
    DevBuf scal;      // PcgScalars + counters
    int64_t dvec_dpad = 0;
    DevBuf colx;      // one column of beta (column-by-column multi-RHS stages)
    // this device's copy of the allocation-free entry point's static scratch
    // (device address from hipGetSymbolAddress at context creation)
    double* na_scratch = nullptr;
    // sketch and preconditioner workspaces used by spcg_solve
    DevBuf zbuf, tables, wsB, wsBY, wsBh;
    DevBuf xlast;   // padded copy of the last input row (first transform pass)
    DevBuf wsR, wsMinv, dense_a, dense_b, dense_c, dense_q, dense_status, dense_w, dense_wd, dense_tmp;
    int64_t dense_w_elems = 0;
    // learned schedule: features and network outputs (4 x 8 floats), gradient partials
    DevBuf sched, mlp_part;
    int syncs = 0;   // stream synchronisations of the current solve
    // batched solves: per-problem sketches, preconditioners and buffers,
    // kept for reuse by later calls (allocation is slow next to a solve)
    BatchWork* batch = nullptr;
    // pinned copy of the Cholesky pivot status and its event
    DenseStatus* host_status = nullptr;
    hipEvent_t ev_status = nullptr;
    // the transform's output-slot tables are built on a side stream beside
    // its first pass (created on first use)
    hipStream_t side = nullptr;
    hipEvent_t ev_side_fork = nullptr, ev_side_join = nullptr;
    // a solve runs the response transform on the side stream too, beside
    // the preconditioner; y_pending until the library stream waits for it
    hipEvent_t ev_y = nullptr;
    bool y_pending = false;
    // events for timing
    hipEvent_t ev_phase[8] = {};
    hipEvent_t ev_prod[2 * MAX_TIMED] = {};
    bool events_ready = false;
    KTimer* kt = nullptr;   // created on the first instrumented solve
    bool kt_on = false;     // launches are being timed by class
};

struct spcg_sketch_s {
    spcg_ctx* ctx = nullptr;
    int64_t N = 0, Np = 0, d = 0, k = 0, r = 0, K = 0, ld = 0, ldy = 0;
    int L = 0;
    int dtype = DT_F32;    // transform and S_hat rows
    int bdtype = DT_F32;   // stage rows B
    uint64_t seed = 0;
    int64_t m[64] = {};
    int kind = SPCG_SKETCH_SRHT;
    int64_t off[64] = {};      // CountSketch: first row of stage i in B / BY
    double hat_c2 = 0.0;       // weight of the S_hat rows: 1/r (SRHT) or 1 (CountSketch)
    bool owns = true;
    DevBuf B, BY, Bh;          // owned storage (when owns)
    void* pB = nullptr;        // active pointers (owned or ctx workspace)
    double* pBY = nullptr;
    void* pBh = nullptr;
};

struct spcg_precond_s {
    int64_t d = 0;
    int passes = 0;
    bool owns = true;
    DevBuf R, Minv;
    double* pR = nullptr;
    double* pMinv = nullptr;
};

namespace {

int fail(spcg_ctx* ctx, int code, const char* fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess)                                                               \
            return fail((ctx), _e == hipErrorOutOfMemory ? SPCG_E_NOMEM : SPCG_E_HIP,       \
                        "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                        __LINE__);                                                          \
    } while (0)

int check_mat(spcg_ctx* ctx, const spcg_mat* M, const char* name) {
    if (!M) return fail(ctx, SPCG_E_INVALID_ARG, "%s is NULL", name);
    if (M->dtype < SPCG_F64 || M->dtype > SPCG_FP8E4M3)
        return fail(ctx, SPCG_E_DTYPE, "%s: unknown dtype %d", name, M->dtype);
    if (M->rows < 0 || M->cols < 1 || M->ld < M->cols)
        return fail(ctx, SPCG_E_SHAPE, "%s: bad shape rows=%lld cols=%lld ld=%lld", name,
                    (long long)M->rows, (long long)M->cols, (long long)M->ld);
    if (!M->data && M->rows > 0) return fail(ctx, SPCG_E_INVALID_ARG, "%s: data is NULL", name);
    if (M->dtype == SPCG_FP8E4M3 && !M->col_scale)
        return fail(ctx, SPCG_E_INVALID_ARG, "%s: FP8 storage needs col_scale", name);
    return SPCG_OK;
}

int ceil_log2(int64_t n) {
    int L = 0;
    while ((1ll << L) < n) ++L;
    return L < 1 ? 1 : L;
}

int ensure_events(spcg_ctx* ctx) {
    if (ctx->events_ready) return SPCG_OK;
    for (auto& e : ctx->ev_phase) HIP_TRY(ctx, hipEventCreate(&e));
    for (auto& e : ctx->ev_prod) HIP_TRY(ctx, hipEventCreate(&e));
    ctx->events_ready = true;
    return SPCG_OK;
}

// A timed launch of class cls with `bytes` algorithmic bytes: *idx is its
// record (start event already on the library stream unless `reserve`), or
// -1 when launches are not being timed or the records are used up.
int kt_begin(spcg_ctx* ctx, int cls, double bytes, int* idx, bool reserve = false) {
    *idx = -1;
    if (!ctx->kt_on || !ctx->kt || ctx->kt->used >= KT_MAX) return SPCG_OK;
    KTimer& t = *ctx->kt;
    const int i = t.used++;
    t.cls[i] = cls;
    t.bytes[i] = bytes;
    if (!reserve) HIP_TRY(ctx, hipEventRecord(t.ev[2 * i], ctx->stream));
    *idx = i;
    return SPCG_OK;
}
int kt_end(spcg_ctx* ctx, int idx) {
    if (idx >= 0) HIP_TRY(ctx, hipEventRecord(ctx->kt->ev[2 * idx + 1], ctx->stream));
    return SPCG_OK;
}
int kt_start(spcg_ctx* ctx) {
    if (!ctx->kt) ctx->kt = new (std::nothrow) KTimer();
    if (!ctx->kt) return fail(ctx, SPCG_E_NOMEM, "host allocation failed");
    if (!ctx->kt->ready) {
        for (auto& e : ctx->kt->ev) HIP_TRY(ctx, hipEventCreate(&e));
        ctx->kt->ready = true;
    }
    ctx->kt->used = 0;
    ctx->kt_on = true;
    return SPCG_OK;
}
// d-space phases, timed by class when an instrumented solve runs
int phase_a(spcg_ctx* ctx, const DspaceState& S, int variant, const double* part_s, const double* part_g,
            const double* part_scal, int nparts, int64_t dpad, double c2, double g_scale = 0.0) {
    int rc, i;
    if ((rc = kt_begin(ctx, SPCG_KT_PHASE_A, 0.0, &i)) != SPCG_OK) return rc;
    HIP_TRY(ctx, run_phase_a(ctx->stream, S, variant, part_s, part_g, part_scal, nparts, dpad, c2, g_scale));
    return kt_end(ctx, i);
}
int phase_b(spcg_ctx* ctx, const DspaceState& S, int init) {
    int rc, i;
    if ((rc = kt_begin(ctx, SPCG_KT_PHASE_B, 0.0, &i)) != SPCG_OK) return rc;
    HIP_TRY(ctx, run_phase_b(ctx->stream, S, init));
    return kt_end(ctx, i);
}

// ------------------------------------------------------------------ sketch

// Nested CountSketch (SPCG-CS): tables, the finest stage by a gather over
// its buckets, the coarser stages by folding, and S_hat by its own gather.
int countsketch_build(spcg_ctx* ctx, const spcg_mat* X, const spcg_mat* Y, spcg_sketch_t* sk, DevBuf& bB,
                      DevBuf& bBY, DevBuf& bBh) {
    const int64_t K = sk->K, ld = sk->ld, ldy = sk->ldy, Np = sk->Np;
    if (K && sk->k > 64) return fail(ctx, SPCG_E_SHAPE, "the CountSketch takes at most 64 right-hand sides");
    int64_t tot = 0;
    for (int64_t i = 0; i < K; ++i) {
        if (i > 0 && sk->m[i] % sk->m[i - 1] != 0)
            return fail(ctx, SPCG_E_SHAPE, "nested CountSketch sizes must divide each other");
        sk->off[i] = tot;
        tot += sk->m[i];
    }
    const size_t rowb = (size_t)ld * dtype_bytes(sk->bdtype);
    if (tot) {
        HIP_TRY(ctx, bB.ensure((size_t)tot * rowb));
        HIP_TRY(ctx, bBY.ensure((size_t)tot * ldy * 8));
    }
    HIP_TRY(ctx, bBh.ensure((size_t)sk->r * ld * dtype_bytes(sk->dtype)));
    sk->pB = tot ? bB.p : nullptr;
    sk->pBY = tot ? bBY.as<double>() : nullptr;
    sk->pBh = bBh.p;
    // bucket tables, then the round tables of their two bijections
    HIP_TRY(ctx, ctx->tables.ensure(((size_t)2 * Np + 2 * (size_t)feistel_table_size(sk->L)) * sizeof(int32_t)));
    int32_t* tbl = ctx->tables.as<int32_t>();
    int32_t* tbl_hat = tbl + Np;
    uint32_t* rt = reinterpret_cast<uint32_t*>(tbl + 2 * Np);
    // scratch (grown before any launch below uses it): the FP32 working copy
    // of the stage folds and the segment partials of S_hat
    const size_t seg_bytes = (size_t)64 * sk->r * ld * dtype_bytes(sk->dtype);
    HIP_TRY(ctx, ctx->zbuf.ensure(std::max(seg_bytes, K ? (size_t)sk->m[K - 1] * ld * 4 : (size_t)0)));
    hipStream_t st = ctx->stream;
    HIP_TRY(ctx, launch_cs_tables(st, sk->seed, sk->L, K ? tbl : nullptr, tbl_hat, rt));
    CsJob j{};
    j.x = X->data;
    j.in_dtype = X->dtype;
    j.N = sk->N;
    j.d = sk->d;
    j.ldx = X->ld;
    j.col_scale = X->col_scale;
    j.Np = Np;
    j.ld = ld;
    if (K) {
        const bool f64 = sk->dtype == DT_F64;
        const bool direct = sk->bdtype == sk->dtype;   // stage rows kept in the sum type
        // the finest stage and up to 3 coarser ones come from one gather
        // (while the sizes halve; one coarser at a ratio of 4); the rest by
        // folding with each step's own ratio
        const int g = K > 1 ? (int)(sk->m[K - 1] / sk->m[K - 2]) : 2;
        int J = 0;
        if (K > 1 && g == 2)
            while (J < 3 && J < K - 1 && sk->m[K - 1 - J] == 2 * sk->m[K - 2 - J]) ++J;
        if (K > 1 && g == 4) J = 1;
        const int64_t lowest = K - 1 - J;   // coarsest stage written by the gather
        char* Bb = static_cast<char*>(sk->pB);
        void* work = nullptr;
        if (!direct && lowest > 0) work = ctx->zbuf.p;   // m[lowest] x ld FP32, sized above
        CsTreeJob t{};
        t.base = j;
        t.base.y = static_cast<const double*>(Y->data);
        t.base.ldy_in = Y->ld;
        t.base.k = sk->k;
        t.base.tbl = tbl;
        t.base.nbk = sk->m[K - 1];
        t.base.out_dtype = sk->bdtype;
        t.base.ldoy = ldy;
        t.growth = g;
        t.levels = J;
        for (int l = 0; l <= J; ++l) {
            const int64_t i = K - 1 - l;
            t.out[l] = Bb + (size_t)sk->off[i] * rowb;
            t.outy[l] = sk->pBY + (size_t)sk->off[i] * ldy;
            t.m[l] = sk->m[i];
        }
        t.work = work;
        HIP_TRY(ctx, run_cs_gather_tree(st, t));
        for (int64_t i = lowest - 1; i >= 0; --i) {
            const void* src = direct ? static_cast<const void*>(Bb + (size_t)sk->off[i + 1] * rowb) : work;
            const int gi = (int)(sk->m[i + 1] / sk->m[i]);
            HIP_TRY(ctx, run_cs_fold(st, f64, src, direct ? nullptr : work, Bb + (size_t)sk->off[i] * rowb,
                                     sk->bdtype, ld, sk->m[i], gi, sk->pBY + (size_t)sk->off[i + 1] * ldy,
                                     sk->pBY + (size_t)sk->off[i] * ldy, ldy, sk->k));
        }
    }
    CsJob h = j;
    h.tbl = tbl_hat;
    h.nbk = sk->r;
    h.out = sk->pBh;
    h.out_dtype = sk->dtype;
    // segment partials of the few S_hat buckets (at most 64 per bucket; the
    // buffer was sized before the first launch)
    h.scratch = ctx->zbuf.p;
    h.scratch_bytes = seg_bytes;
    HIP_TRY(ctx, run_cs_gather(st, h));
    return SPCG_OK;
}

// Order the library stream after a response transform left on the side
// stream (host = true: wait on the host, before buffers it uses may be
// reallocated).
int y_join(spcg_ctx* ctx, bool host) {
    if (!ctx->y_pending) return SPCG_OK;
    if (host)
        HIP_TRY(ctx, hipEventSynchronize(ctx->ev_y));
    else
        HIP_TRY(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_y, 0));
    ctx->y_pending = false;
    return SPCG_OK;
}

// defer_y: run the response transform on the side stream and leave it
// pending (the caller joins with y_join before reading the sketched
// responses).
int sketch_build(spcg_ctx* ctx, const spcg_mat* X, const spcg_mat* Y, const spcg_sketch_opts* o,
                 bool borrow, spcg_sketch_t* sk, bool defer_y = false) {
    int rc;
    if ((rc = y_join(ctx, true)) != SPCG_OK) return rc;
    if ((rc = check_mat(ctx, X, "X")) != SPCG_OK) return rc;
    const bool hat_only = o && o->hat_only;
    if (!hat_only) {
        if ((rc = check_mat(ctx, Y, "Y")) != SPCG_OK) return rc;
        if (Y->dtype != SPCG_F64) return fail(ctx, SPCG_E_DTYPE, "Y must be SPCG_F64");
        if (Y->rows != X->rows) return fail(ctx, SPCG_E_SHAPE, "Y has %lld rows, X has %lld",
                                            (long long)Y->rows, (long long)X->rows);
    }
    const int64_t N = X->rows, d = X->cols;
    if (N <= d) return fail(ctx, SPCG_E_SHAPE, "need N > d (N=%lld, d=%lld)", (long long)N, (long long)d);
    if (d > product_max_d(X->dtype))
        return fail(ctx, SPCG_E_SHAPE, "d=%lld exceeds the supported maximum %lld", (long long)d,
                    (long long)product_max_d(X->dtype));
    const int L = ceil_log2(N);
    if (L > 30) return fail(ctx, SPCG_E_SHAPE, "N too large (2^30 rows max)");
    const int64_t Np = 1ll << L;
    const int64_t m0 = (o && o->m0 > 0) ? o->m0 : 4 * d;
    const int64_t growth = (o && o->growth > 0) ? o->growth : 2;
    const int64_t r = (o && o->r > 0) ? o->r : 6 * d;
    if (growth < 2) return fail(ctx, SPCG_E_INVALID_ARG, "growth must be >= 2");
    if (r < d || r > Np) return fail(ctx, SPCG_E_SHAPE, "need d <= r <= N' (r=%lld)", (long long)r);
    sk->ctx = ctx;
    sk->N = N;
    sk->Np = Np;
    sk->d = d;
    sk->L = L;
    sk->r = r;
    sk->seed = o ? o->seed : 0;
    sk->dtype = X->dtype == SPCG_F64 ? DT_F64 : DT_F32;
    sk->ld = sketch_ld(d, sk->dtype == DT_F64);
    const int want = o ? o->stage_dtype : 0;
    if (sk->dtype == DT_F64) {
        if (want != 0 && want != SPCG_F64) return fail(ctx, SPCG_E_DTYPE, "FP64 input keeps FP64 stage rows");
        sk->bdtype = DT_F64;
    } else if (want == 0) {
        sk->bdtype = (X->dtype == SPCG_BF16 || X->dtype == SPCG_FP8E4M3) ? DT_BF16 : DT_F32;
    } else if (want == SPCG_F32 || want == SPCG_BF16) {
        sk->bdtype = want == SPCG_F32 ? DT_F32 : DT_BF16;
    } else {
        return fail(ctx, SPCG_E_DTYPE, "stage_dtype must be 0, SPCG_F32 or SPCG_BF16");
    }
    sk->K = 0;
    sk->k = 0;
    if (!hat_only && o && o->m_list_len > 0) {
        if (!o->m_list) return fail(ctx, SPCG_E_INVALID_ARG, "m_list is NULL");
        if (o->m_list_len > 64) return fail(ctx, SPCG_E_SHAPE, "more than 64 stages");
        for (int i = 0; i < o->m_list_len; ++i) {
            const int64_t m = o->m_list[i];
            if (m <= d || m >= N || (i > 0 && m <= o->m_list[i - 1]))
                return fail(ctx, SPCG_E_SHAPE, "m_list must increase strictly within (d, N)");
            sk->m[sk->K++] = m;
        }
        sk->k = Y->cols;
    } else if (!hat_only) {
        if (m0 <= d) return fail(ctx, SPCG_E_SHAPE, "need m_1 > d (m_1=%lld)", (long long)m0);
        const int64_t limit = (o && o->m_max > 0) ? std::min<int64_t>(o->m_max, N - 1) : N - 1;
        for (int64_t m = m0; m <= limit; m *= growth) {
            if (sk->K >= 64) return fail(ctx, SPCG_E_SHAPE, "more than 64 stages");
            sk->m[sk->K++] = m;
        }
        if (sk->K == 0) return fail(ctx, SPCG_E_SHAPE, "no sketch size fits: m_1=%lld >= N", (long long)m0);
        sk->k = Y->cols;
    }
    const int64_t mK = sk->K ? sk->m[sk->K - 1] : 0;
    const size_t es = sk->dtype == DT_F64 ? 8 : 4;
    sk->ldy = sketch_ldy(sk->k);
    sk->owns = !borrow;
    DevBuf& bB = borrow ? ctx->wsB : sk->B;
    DevBuf& bBY = borrow ? ctx->wsBY : sk->BY;
    DevBuf& bBh = borrow ? ctx->wsBh : sk->Bh;
    const int kind = o ? o->kind : SPCG_SKETCH_SRHT;
    if (kind != SPCG_SKETCH_SRHT && kind != SPCG_SKETCH_COUNT)
        return fail(ctx, SPCG_E_INVALID_ARG, "sketch kind must be SPCG_SKETCH_SRHT or SPCG_SKETCH_COUNT");
    sk->kind = kind;
    sk->hat_c2 = kind == SPCG_SKETCH_COUNT ? 1.0 : 1.0 / (double)r;
    if (kind == SPCG_SKETCH_COUNT) return countsketch_build(ctx, X, Y, sk, bB, bBY, bBh);
    if (mK) {
        HIP_TRY(ctx, bB.ensure((size_t)mK * sk->ld * dtype_bytes(sk->bdtype)));
        HIP_TRY(ctx, bBY.ensure((size_t)mK * sk->ldy * 8));
    }
    HIP_TRY(ctx, bBh.ensure((size_t)r * sk->ld * es));
    sk->pB = mK ? bB.p : nullptr;
    sk->pBY = mK ? bBY.as<double>() : nullptr;
    sk->pBh = bBh.p;
    // randomness tables and transform scratch (always context workspace)
    // randomness tables, then the round tables of the three Feistel streams
    // the 11-bit half-tile-staged last pass also reads both output slots per
    // row in tile order (pair table after the round tables)
    const int seg = o ? o->transform_segment : 0;
    if (seg != 0 && seg != 64 && seg != 128 && seg != 256 && seg != -64 && seg != -32)
        return fail(ctx, SPCG_E_INVALID_ARG, "transform_segment must be 0, 64, 128, 256, -32 or -64");
    const int split = fwht_split_tables(X->dtype == SPCG_F64 ? DT_F64 : DT_F32, L, sk->ld, seg);
    const size_t tsz = (size_t)3 * Np + 3 * (size_t)feistel_table_size(L);
    const size_t tpad = (size_t)round_up((int64_t)(tsz * sizeof(int32_t)), 16);
    const size_t psz = (split & 2) ? (size_t)Np * sizeof(int2) : 0;
    HIP_TRY(ctx, ctx->tables.ensure(tpad + psz + ((split & 1) ? (size_t)Np / 4 : 0)));
    int32_t* perm_sign = ctx->tables.as<int32_t>();
    int32_t* inv_slot = perm_sign + Np;
    int32_t* inv_hat = perm_sign + 2 * Np;
    uint32_t* rt = reinterpret_cast<uint32_t*>(perm_sign + 3 * Np);
    int2* pair_t = (split & 2) ? reinterpret_cast<int2*>(ctx->tables.as<char>() + tpad) : nullptr;
    uint32_t* row_masks = (split & 1) ? reinterpret_cast<uint32_t*>(ctx->tables.as<char>() + tpad + psz) : nullptr;
    const size_t zx = (size_t)Np * sk->ld * es;
    const size_t zy = (size_t)Np * sk->ldy * 8;
    HIP_TRY(ctx, ctx->zbuf.ensure(std::max(zx, zy)));
    hipStream_t st = ctx->stream;
    // the round tables of the three Feistel streams (one launch) and the
    // permutation first; the output-slot tables (only the last pass needs
    // them) on the side stream, beside the first pass
    if (!ctx->side) {
        HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
        HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->ev_side_fork, hipEventDisableTiming));
        HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->ev_side_join, hipEventDisableTiming));
        HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->ev_y, hipEventDisableTiming));
    }
    HIP_TRY(ctx, launch_sketch_round_tables(st, sk->seed, L, rt));
    HIP_TRY(ctx, hipEventRecord(ctx->ev_side_fork, st));
    HIP_TRY(ctx, launch_sketch_tables(st, sk->seed, L, mK, r, perm_sign, nullptr, nullptr, rt, nullptr, 0, row_masks,
                                      N));
    HIP_TRY(ctx, hipStreamWaitEvent(ctx->side, ctx->ev_side_fork, 0));
    HIP_TRY(ctx, launch_sketch_tables(ctx->side, sk->seed, L, mK, r, nullptr, mK ? inv_slot : nullptr, inv_hat, rt,
                                      pair_t, L / 2));
    HIP_TRY(ctx, hipEventRecord(ctx->ev_side_join, ctx->side));
    FwhtJob jx{};
    jx.x = X->data;
    // rows whose byte stride is a multiple of 4 but not of 16: a padded copy
    // of the last row lets the first pass stage every row with 16-byte loads
    if (X->dtype != SPCG_F64 && N >= 2) {
        const int64_t eb = dtype_bytes(X->dtype), rowb = d * eb;
        const bool a16 = (uintptr_t)X->data % 16 == 0 && (X->ld * eb) % 16 == 0;
        const bool a4 = (uintptr_t)X->data % 4 == 0 && (X->ld * eb) % 4 == 0;
        if (!a16 && a4) {
            HIP_TRY(ctx, ctx->xlast.ensure((size_t)round_up(rowb, 16) + 16));
            HIP_TRY(ctx, hipMemcpyAsync(ctx->xlast.p, static_cast<const char*>(X->data) + (N - 1) * X->ld * eb,
                                        (size_t)rowb, hipMemcpyDeviceToDevice, st));
            jx.x_last = ctx->xlast.p;
        }
    }
    jx.in_dtype = X->dtype;
    jx.N = N;
    jx.d = d;
    jx.ldx = X->ld;
    jx.col_scale = X->col_scale;
    jx.L = L;
    jx.perm_sign = perm_sign;
    jx.inv_slot = mK ? inv_slot : nullptr;
    jx.inv_hat = inv_hat;
    jx.zbuf = ctx->zbuf.p;
    jx.ldz = sk->ld;
    jx.B = sk->pB;
    jx.ldb = sk->ld;
    jx.Bh = sk->pBh;
    jx.ldbh = sk->ld;
    jx.b_bf16 = sk->bdtype == DT_BF16;
    jx.seg_bytes = seg;
    jx.narrow = 0;
    jx.stream = 1;
    jx.num_cu = ctx->num_cu;
    jx.wait_before_last = ctx->ev_side_join;
    jx.slot_pairs = pair_t;
    jx.row_masks = row_masks;
    if (ctx->kt_on) {
        // algorithmic bytes of each pass (used columns only)
        const int np = fwht_passes(L);
        const double eX = (double)dtype_bytes(X->dtype), eB = (double)dtype_bytes(sk->bdtype);
        const double zrow = (double)d * (double)es, outb = (double)mK * d * eB + (double)r * d * (double)es;
        for (int pi = 0; pi < np && pi < 3; ++pi) {
            const double in = pi == 0 ? (double)N * d * eX : (double)Np * zrow;
            const double outp = pi == np - 1 ? outb : (double)Np * zrow;
            int idx;
            if ((rc = kt_begin(ctx, pi == 0 ? SPCG_KT_TRANSFORM_FIRST : SPCG_KT_TRANSFORM_REST, in + outp, &idx,
                               true)) != SPCG_OK)
                return rc;
            if (idx >= 0) {
                jx.pass_ev[2 * pi] = ctx->kt->ev[2 * idx];
                jx.pass_ev[2 * pi + 1] = ctx->kt->ev[2 * idx + 1];
            }
        }
    }
    HIP_TRY(ctx, run_fwht(st, jx));
    if (mK) {
        FwhtJob jy{};
        jy.x = Y->data;
        jy.in_dtype = DT_F64;
        jy.N = N;
        jy.d = sk->k;
        jy.ldx = Y->ld;
        jy.L = L;
        jy.perm_sign = perm_sign;
        jy.inv_slot = inv_slot;
        jy.inv_hat = nullptr;
        jy.zbuf = ctx->zbuf.p;
        jy.ldz = sk->ldy;
        jy.B = sk->pBY;
        jy.ldb = sk->ldy;
        jy.narrow = sk->k == 1;
        // rows of 8 or 16 columns: the tiled passes take that segment width
        jy.seg_bytes = sk->ldy > 1 && sk->ldy < 32 ? (int)sk->ldy * 8 : 0;
        if (defer_y) {
            HIP_TRY(ctx, hipEventRecord(ctx->ev_side_fork, st));
            HIP_TRY(ctx, hipStreamWaitEvent(ctx->side, ctx->ev_side_fork, 0));
            HIP_TRY(ctx, run_fwht(ctx->side, jy));
            HIP_TRY(ctx, hipEventRecord(ctx->ev_y, ctx->side));
            ctx->y_pending = true;
        } else {
            HIP_TRY(ctx, run_fwht(st, jy));
        }
    }
    return SPCG_OK;
}

// --------------------------------------------------------- preconditioner

// Cholesky of G with its pivot status copied to pinned host memory behind
// it; the caller waits for the copy with chol_status_wait (and may queue
// more work first).
int chol_enqueue(spcg_ctx* ctx, double* G, int64_t d, DenseStatus* dev_status, DenseStatus* host_dst = nullptr) {
    hipStream_t st = ctx->stream;
    if (!ctx->host_status) {
        HIP_TRY(ctx, hipHostMalloc((void**)&ctx->host_status, sizeof(DenseStatus), hipHostMallocDefault));
        HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->ev_status, hipEventDisableTiming));
    }
    HIP_TRY(ctx, dense_status_reset(st, dev_status));
    HIP_TRY(ctx, cholesky_upper(st, G, d, d, dev_status, ctx->dense_wd.as<double>(), ctx->dense_tmp.as<double>(),
                                ctx->dense_w.as<double>(), ctx->dense_w_elems));
    HIP_TRY(ctx, hipMemcpyAsync(host_dst ? host_dst : ctx->host_status, dev_status, sizeof(DenseStatus),
                                hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipEventRecord(ctx->ev_status, st));
    return SPCG_OK;
}

int chol_status_wait(spcg_ctx* ctx, DenseStatus* host) {
    HIP_TRY(ctx, hipEventSynchronize(ctx->ev_status));
    ctx->syncs++;
    *host = *ctx->host_status;
    return SPCG_OK;
}

int chol_checked(spcg_ctx* ctx, double* G, int64_t d, DenseStatus* dev_status, DenseStatus* host) {
    int rc;
    if ((rc = chol_enqueue(ctx, G, d, dev_status)) != SPCG_OK) return rc;
    return chol_status_wait(ctx, host);
}

// split-K workspace of the dense kernels (8 partial d x d or r x 64
// products), the diagonal-block inverses (d x d) and a d x d (at least
// 64-column) scratch
int ensure_dense_work(spcg_ctx* ctx, int64_t d, int64_t r) {
    const int64_t elems = 8 * std::max<int64_t>(d * d, r * 64);
    if (ctx->dense_w_elems < elems) {
        HIP_TRY(ctx, ctx->dense_w.ensure((size_t)elems * 8));
        ctx->dense_w_elems = elems;
    }
    HIP_TRY(ctx, ctx->dense_wd.ensure((size_t)d * d * 8));
    HIP_TRY(ctx, ctx->dense_tmp.ensure((size_t)std::max(std::max(r, d) * 64, d * d + 64) * 8));
    return SPCG_OK;
}

// R -> (R, M = R^{-1} R^{-T}); diag_inv: the inverses of R's 64 x 64
// diagonal blocks when the Cholesky that produced R left them (d x d, or
// null)
int precond_finish(spcg_ctx* ctx, spcg_precond_t* pc, const double* diag_inv = nullptr) {
    const int64_t d = pc->d;
    hipStream_t st = ctx->stream;
    int rc;
    if ((rc = ensure_dense_work(ctx, d, d)) != SPCG_OK) return rc;
    double* wk = ctx->dense_w.as<double>();
    const int64_t we = ctx->dense_w_elems;
    HIP_TRY(ctx, ctx->dense_a.ensure((size_t)d * d * 8));
    double* W = ctx->dense_a.as<double>();
    HIP_TRY(ctx, tri_inverse_upper(st, pc->pR, d, d, W, diag_inv, ctx->dense_tmp.as<double>(), wk, we));
    HIP_TRY(ctx, gemm_f64(st, d, d, d, 1.0, W, 0, d, 1, W, 0, 1, d, 0.0, pc->pMinv, d, 0, wk, we));
    return SPCG_OK;
}

int precond_alloc(spcg_ctx* ctx, spcg_precond_t* pc, int64_t d, bool borrow) {
    pc->d = d;
    pc->owns = !borrow;
    DevBuf& bR = borrow ? ctx->wsR : pc->R;
    DevBuf& bM = borrow ? ctx->wsMinv : pc->Minv;
    HIP_TRY(ctx, bR.ensure((size_t)d * d * 8));
    HIP_TRY(ctx, bM.ensure((size_t)d * d * 8));
    pc->pR = bR.as<double>();
    pc->pMinv = bM.as<double>();
    return SPCG_OK;
}

// a one-pass factor is kept when the Cholesky succeeded and (mode 0) its
// diagonal spans at most five decades
bool precond_status_ok(const DenseStatus& hs, int mode) {
    const bool ok = hs.fail == 0 && hs.min_diag > 0.0;
    const double ratio = ok ? hs.max_diag / hs.min_diag : INFINITY;
    return ok && (mode == 1 || ratio <= 1e5);
}

// deferred (pinned host memory, modes 0 and 1 only): queue the one-pass
// factor and M, copy the pivot status to *deferred behind them and return
// without waiting; the caller checks it with precond_status_ok once the
// stream has passed the copy and builds again (without deferral) when it
// fails.
int precond_build(spcg_ctx* ctx, const spcg_sketch_t* sk, const spcg_precond_opts* o, bool borrow,
                  spcg_precond_t* pc, DenseStatus* deferred = nullptr) {
    int rc;
    const int64_t d = sk->d, r = sk->r, ld = sk->ld;
    const int mode = o ? o->qr_passes : 0;
    if (mode < 0 || mode > 3) return fail(ctx, SPCG_E_INVALID_ARG, "qr_passes must be 0..3");
    if ((rc = precond_alloc(ctx, pc, d, borrow)) != SPCG_OK) return rc;
    hipStream_t st = ctx->stream;
    const int bf32 = sk->dtype == DT_F32;
    HIP_TRY(ctx, ctx->dense_status.ensure(sizeof(DenseStatus)));
    DenseStatus* dst = ctx->dense_status.as<DenseStatus>();
    DenseStatus hs{};
    double* R = pc->pR;
    const double inv_r = sk->hat_c2;   // S_hat X = sqrt(hat_c2) * (stored rows)
    if ((rc = ensure_dense_work(ctx, d, r)) != SPCG_OK) return rc;
    double* wk = ctx->dense_w.as<double>();
    const int64_t we = ctx->dense_w_elems;
    // Gram of S_hat X = B_hat / sqrt(r): upper 64x64 tiles only
    auto gram_hat = [&](double* C) {
        return gemm_f64(st, d, d, r, inv_r, sk->pBh, bf32, 1, ld, sk->pBh, bf32, ld, 1, 0.0, C, d, 1, wk, we);
    };
    if (mode == 0 || mode == 1) {
        HIP_TRY(ctx, gram_hat(R));
        // M is formed right behind the factor while the host waits for the
        // pivot status (no idle gap); a failed or badly scaled factor is
        // redone below, which overwrites R and M
        if ((rc = chol_enqueue(ctx, R, d, dst, deferred)) != SPCG_OK) return rc;
        if ((rc = precond_finish(ctx, pc, ctx->dense_wd.as<double>())) != SPCG_OK) return rc;
        if (deferred) {
            pc->passes = 1;
            return SPCG_OK;
        }
        if ((rc = chol_status_wait(ctx, &hs)) != SPCG_OK) return rc;
        if (precond_status_ok(hs, mode)) {
            pc->passes = 1;
            return SPCG_OK;
        }
        if (mode == 1)
            return fail(ctx, SPCG_E_RANK, "Cholesky of the sketched Gram failed at pivot %d", hs.fail);
    }
    // CholeskyQR2 (mode 2) or shifted CholeskyQR3 (mode 0 fallback, 3)
    const int passes = mode == 2 ? 2 : 3;
    HIP_TRY(ctx, ctx->dense_b.ensure((size_t)d * d * 8));
    HIP_TRY(ctx, ctx->dense_c.ensure((size_t)d * d * 8));
    HIP_TRY(ctx, ctx->dense_q.ensure((size_t)r * d * 8));
    double* R1 = ctx->dense_b.as<double>();
    double* R2 = ctx->dense_c.as<double>();
    double* Q = ctx->dense_q.as<double>();
    HIP_TRY(ctx, ctx->dense_a.ensure((size_t)d * d * 8));
    double* T = ctx->dense_a.as<double>();
    HIP_TRY(ctx, gram_hat(R1));
    if (passes == 3) {
        const double u = std::ldexp(1.0, -53);
        HIP_TRY(ctx, dense_add_trace_shift(st, R1, d, 11.0 * ((double)r * d + (double)d * (d + 1)) * u));
    }
    if ((rc = chol_checked(ctx, R1, d, dst, &hs)) != SPCG_OK) return rc;
    if (hs.fail) return fail(ctx, SPCG_E_RANK, "Cholesky of the (shifted) sketched Gram failed");
    HIP_TRY(ctx, dense_convert(st, sk->pBh, bf32, r, d, ld, std::sqrt(inv_r), Q, d));
    HIP_TRY(ctx, trsm_right_upper(st, Q, r, d, d, R1, d, ctx->dense_wd.as<double>(), ctx->dense_tmp.as<double>(),
                                  wk, we));
    // second pass
    HIP_TRY(ctx, gemm_f64(st, d, d, r, 1.0, Q, 0, 1, d, Q, 0, d, 1, 0.0, R2, d, 1, wk, we));
    if ((rc = chol_checked(ctx, R2, d, dst, &hs)) != SPCG_OK) return rc;
    if (hs.fail || hs.min_pivot < 1e-12)
        return fail(ctx, SPCG_E_RANK, "S_hat X is numerically rank deficient (pivot %.3g)", hs.min_pivot);
    if (passes == 3) {
        HIP_TRY(ctx, trsm_right_upper(st, Q, r, d, d, R2, d, ctx->dense_wd.as<double>(),
                                      ctx->dense_tmp.as<double>(), wk, we));
        HIP_TRY(ctx, gemm_f64(st, d, d, r, 1.0, Q, 0, 1, d, Q, 0, d, 1, 0.0, R, d, 1, wk, we));
        if ((rc = chol_checked(ctx, R, d, dst, &hs)) != SPCG_OK) return rc;
        if (hs.fail || hs.min_pivot < 1e-12)
            return fail(ctx, SPCG_E_RANK, "S_hat X is numerically rank deficient (pivot %.3g)", hs.min_pivot);
        // R <- R3 R2 R1
        HIP_TRY(ctx, gemm_f64(st, d, d, d, 1.0, R, 0, d, 1, R2, 0, d, 1, 0.0, T, d, 0, wk, we));
        HIP_TRY(ctx, gemm_f64(st, d, d, d, 1.0, T, 0, d, 1, R1, 0, d, 1, 0.0, R, d, 0, wk, we));
    } else {
        HIP_TRY(ctx, gemm_f64(st, d, d, d, 1.0, R2, 0, d, 1, R1, 0, d, 1, 0.0, R, d, 0, wk, we));
    }
    pc->passes = passes;
    return precond_finish(ctx, pc);
}

// -------------------------------------------------------------- PCG stage

struct StageRun {
    int iters_done = 0;
    bool converged = false;
    PcgScalars sc{};
};

// Workspace of one PCG solve: the product partials (one row of dpad
// doubles per product block) and the d-space state.  Filled from the
// context's cached buffers (ensure_stage_ws) or from the static area of the
// allocation-free entry point (static_stage_ws).
struct StageWs {
    DspaceState S{};
    double* part_s = nullptr;
    double* part_g = nullptr;
    double* part_scal = nullptr;
    int num_cu = 256;   // product launches use at most this many blocks
};

// d-vector block g z p s gt (5 dpad) + per-block scalars (1024), then the
// PcgScalars record and its two last-block counters
void stage_ws_layout(StageWs* W, double* v, int64_t stride, void* scal, double* x, const double* Minv,
                     int64_t d) {
    DspaceState& S = W->S;
    S.x = x;
    S.g = v;
    S.z = v + stride;
    S.p = v + 2 * stride;
    S.s = v + 3 * stride;
    S.gt = v + 4 * stride;
    S.blk = v + 5 * stride;
    S.sc = static_cast<PcgScalars*>(scal);
    S.counters = reinterpret_cast<unsigned int*>(static_cast<char*>(scal) + sizeof(PcgScalars));
    S.Minv = Minv;
    S.d = d;
}

int ensure_stage_ws(spcg_ctx* ctx, int64_t d, StageWs* W, double* x, const double* Minv) {
    const int64_t dpad = round_up(d, 64);
    const size_t mb = (size_t)product_max_blocks(ctx->num_cu);
    HIP_TRY(ctx, ctx->part_s.ensure(mb * dpad * 8));
    HIP_TRY(ctx, ctx->part_g.ensure(mb * dpad * 8));
    HIP_TRY(ctx, ctx->part_scal.ensure(mb * 2 * 8));
    if (ctx->dvec_dpad < dpad || !ctx->dvec.p) {
        HIP_TRY(ctx, ctx->dvec.ensure((size_t)(5 * dpad + 1024) * 8));
        ctx->dvec_dpad = dpad;
    }
    if (!ctx->scal.p) {
        HIP_TRY(ctx, ctx->scal.ensure(sizeof(PcgScalars) + 64));
        HIP_TRY(ctx, run_counters_reset(ctx->stream,
                                        reinterpret_cast<unsigned int*>(ctx->scal.as<char>() + sizeof(PcgScalars)), 16));
    }
    stage_ws_layout(W, ctx->dvec.as<double>(), ctx->dvec_dpad, ctx->scal.p, x, Minv, d);
    W->part_s = ctx->part_s.as<double>();
    W->part_g = ctx->part_g.as<double>();
    W->part_scal = ctx->part_scal.as<double>();
    W->num_cu = ctx->num_cu;
    return SPCG_OK;
}

int read_scalars(spcg_ctx* ctx, const DspaceState& S, PcgScalars* out) {
    HIP_TRY(ctx, hipMemcpyAsync(out, S.sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    ctx->syncs++;
    return SPCG_OK;
}

bool stop_test(const PcgScalars& sc, double tol) {
    if (sc.exact) return true;
    return std::sqrt(std::max(sc.rho, 0.0)) <= tol * std::sqrt(std::max(sc.ax2, 0.0));
}

struct ProductTimer {
    spcg_ctx* ctx = nullptr;
    int used = 0;
};

int product_pass(spcg_ctx* ctx, const spcg_mat* A, const spcg_mat* b, const StageWs& W, int mode,
                 int* nparts, ProductTimer* timer) {
    ProdJob j{};
    j.A = A->data;
    j.dtype = A->dtype;
    j.m = A->rows;
    j.d = A->cols;
    j.lda = A->ld;
    j.dmem = A->reserved == 1 ? A->ld : A->cols;
    j.col_scale = A->col_scale;
    j.b = b ? static_cast<const double*>(b->data) : nullptr;
    j.ldbv = b ? b->ld : 0;
    j.x = W.S.x;
    j.p = W.S.p;
    j.mode = mode;
    j.part_s = W.part_s;
    j.part_g = W.part_g;
    j.part_scal = W.part_scal;
    j.dpad = round_up(A->cols, 64);
    j.num_cu = W.num_cu;
    j.gate = W.S.gate;
    j.gmin = W.S.gmin;
    const bool timed = timer && timer->used < MAX_TIMED;
    if (timed) HIP_TRY(ctx, hipEventRecord(ctx->ev_prod[2 * timer->used], ctx->stream));
    const double e = (double)dtype_bytes(A->dtype);
    const double bytes = mode == PM_S ? (double)A->rows * A->cols * e : (double)A->rows * (A->cols * e + 8.0);
    int rc, ki;
    if ((rc = kt_begin(ctx, mode == PM_S ? SPCG_KT_PROD_S : mode == PM_G ? SPCG_KT_PROD_G : SPCG_KT_PROD_SG, bytes,
                       &ki)) != SPCG_OK)
        return rc;
    HIP_TRY(ctx, run_product(ctx->stream, j, nparts));
    if ((rc = kt_end(ctx, ki)) != SPCG_OK) return rc;
    if (timed) {
        HIP_TRY(ctx, hipEventRecord(ctx->ev_prod[2 * timer->used + 1], ctx->stream));
        timer->used++;
    }
    return SPCG_OK;
}

// Work done at the start of a tested stage for the schedule network:
// Stage II features (when fpre is set) and, with weights, the network's
// prediction of the iteration count; both come back with the first test,
// as do the listed device-to-host copies.  With t1_host set, the stage's
// iteration budget is capped at t_total - *t1_host once that copy is in.
struct StageHooks {
    const float* fpre = nullptr;   // device: pre-Stage-I features
    float* fii = nullptr;          // device: Stage II features (8)
    const float* W = nullptr;      // device: network weights (learned schedule)
    float* out = nullptr;          // device: network outputs (8)
    int margin = 1;
    struct Copy {
        void* dst;
        const void* src;
        size_t bytes;
    };
    Copy copies[6] = {};
    int ncopy = 0;
    void add_copy(void* dst, const void* src, size_t bytes) {
        if (ncopy < 6 && bytes > 0) copies[ncopy++] = Copy{dst, src, bytes};
    }
    const int32_t* t1_host = nullptr;
    int t_total = 0;
    // results
    float host_fii[8] = {};
    float host_out[8] = {};
    double s_pred = 0.0;
    int unchecked = 0;
    bool fallback = false;
    PcgScalars start{};
};

// PCG(A, b, c2, M, x, iters) with optional stopping test; x is device
// memory.  W: a prepared workspace (the context's when null).
int stage_run(spcg_ctx* ctx, const spcg_mat* A, const spcg_mat* b, double c2, const spcg_precond_t* pc,
              double* x, int iters, double tol, bool refresh, int check_every, StageRun* out,
              ProductTimer* timer, StageHooks* hooks = nullptr, const StageWs* W_in = nullptr) {
    int rc;
    StageWs Wl;
    if (!W_in) {
        if ((rc = ensure_stage_ws(ctx, A->cols, &Wl, x, pc->pMinv)) != SPCG_OK) return rc;
        W_in = &Wl;
    }
    const StageWs& W = *W_in;
    const DspaceState& S = W.S;
    hipStream_t st = ctx->stream;
    const int64_t dpad = round_up(A->cols, 64);
    int np = 0;
    // stage start: g = c2 A^T (b - A x), z = M g, p = z, rho = g^T z
    if ((rc = product_pass(ctx, A, b, W, PM_G, &np, nullptr)) != SPCG_OK) return rc;
    if ((rc = phase_a(ctx, S, PA_START, nullptr, W.part_g, W.part_scal, np, dpad, c2)) != SPCG_OK) return rc;
    if ((rc = phase_b(ctx, S, 1)) != SPCG_OK) return rc;
    const bool testing = tol > 0.0;
    if (check_every < 1) check_every = 1;
    out->iters_done = 0;
    out->converged = false;
    int unchecked = 0;
    if (testing) {
        if (hooks) {
            for (int i = 0; i < hooks->ncopy; ++i)
                HIP_TRY(ctx, hipMemcpyAsync(hooks->copies[i].dst, hooks->copies[i].src, hooks->copies[i].bytes,
                                            hipMemcpyDeviceToHost, st));
        }
        if (hooks && hooks->fpre) {
            HIP_TRY(ctx, run_features_ii(st, hooks->fpre, S.sc, tol, hooks->fii));
            HIP_TRY(ctx, hipMemcpyAsync(hooks->host_fii, hooks->fii, 8 * sizeof(float), hipMemcpyDeviceToHost, st));
            if (hooks->W) {
                HIP_TRY(ctx, run_mlp_forward(st, hooks->W, hooks->fii, 1, hooks->out));
                HIP_TRY(ctx,
                        hipMemcpyAsync(hooks->host_out, hooks->out, MLP_O * sizeof(float), hipMemcpyDeviceToHost, st));
            }
        }
        if ((rc = read_scalars(ctx, S, &out->sc)) != SPCG_OK) return rc;
        if (hooks) hooks->start = out->sc;
        if (hooks && hooks->t1_host) iters = std::max(0, std::min(iters, hooks->t_total - *hooks->t1_host));
        if (out->sc.breakdown) return fail(ctx, SPCG_E_BREAKDOWN, "PCG breakdown at stage start");
        if (stop_test(out->sc, tol)) {
            out->converged = true;
            return SPCG_OK;
        }
        if (hooks && hooks->W) {
            hooks->s_pred = (double)hooks->host_out[MLP_NA + 2] * MLP_S_SCALE;
            const double rs = std::isfinite(hooks->s_pred) ? std::round(hooks->s_pred) : 0.0;
            const double k = std::min(std::max(rs - (double)hooks->margin, 0.0), (double)iters);
            unchecked = (int)k;
            hooks->unchecked = unchecked;
        }
    }
    const int pmode = refresh ? PM_SG : PM_S;
    for (int it = 0; it < iters; ++it) {
        if ((rc = product_pass(ctx, A, b, W, pmode, &np, timer)) != SPCG_OK) return rc;
        if ((rc = phase_a(ctx, S, refresh ? PA_REFRESH : PA_STEP, W.part_s, W.part_g, W.part_scal, np, dpad, c2)) !=
            SPCG_OK)
            return rc;
        if ((rc = phase_b(ctx, S, 0)) != SPCG_OK) return rc;
        out->iters_done = it + 1;
        const int done = it + 1;
        if (testing && done >= unchecked && ((done - unchecked) % check_every == 0 || done == iters)) {
            if ((rc = read_scalars(ctx, S, &out->sc)) != SPCG_OK) return rc;
            if (out->sc.breakdown) return fail(ctx, SPCG_E_BREAKDOWN, "PCG breakdown: p^T s <= 0 or non-finite");
            if (stop_test(out->sc, tol)) {
                out->converged = true;
                return SPCG_OK;
            }
            if (hooks && unchecked > 0 && done == unchecked) hooks->fallback = true;
        }
    }
    if (!testing) {
        if ((rc = read_scalars(ctx, S, &out->sc)) != SPCG_OK) return rc;
        if (out->sc.breakdown) return fail(ctx, SPCG_E_BREAKDOWN, "PCG breakdown: p^T s <= 0 or non-finite");
        out->converged = out->sc.exact != 0;
    }
    return SPCG_OK;
}

// m_prev > 0: the previous stage ran on the first m_prev rows of this
// prefix view (nested sketches) and left its final gradient in the state;
// the starting gradient then needs a G pass over the new rows only.
//
// stage_start_nosync / stage_iter_nosync: the stage start (starting
// gradient, z, p, rho) and one PCG iteration of a sketched stage, without
// host synchronisation.  W may carry a launch gate (W.S.gate): every kernel
// then returns at once unless the decision word is >= W.S.gmin.
int stage_start_nosync(spcg_ctx* ctx, const spcg_mat* A, const spcg_mat* b, double c2, const StageWs& W,
                       int64_t m_prev) {
    int rc;
    const DspaceState& S = W.S;
    const int64_t dpad = round_up(A->cols, 64);
    int np = 0;
    if (m_prev > 0 && m_prev < A->rows) {
        spcg_mat dA = *A, db = *b;
        dA.data = static_cast<const char*>(A->data) + (size_t)m_prev * A->ld * dtype_bytes(A->dtype);
        dA.rows = A->rows - m_prev;
        db.data = static_cast<const double*>(b->data) + (size_t)m_prev * b->ld;
        db.rows = dA.rows;
        if ((rc = product_pass(ctx, &dA, &db, W, PM_G, &np, nullptr)) != SPCG_OK) return rc;
        if ((rc = phase_a(ctx, S, PA_START_NESTED, nullptr, W.part_g, W.part_scal, np, dpad, c2,
                          (double)m_prev / (double)A->rows)) != SPCG_OK)
            return rc;
    } else {
        if ((rc = product_pass(ctx, A, b, W, PM_G, &np, nullptr)) != SPCG_OK) return rc;
        if ((rc = phase_a(ctx, S, PA_START, nullptr, W.part_g, W.part_scal, np, dpad, c2)) != SPCG_OK) return rc;
    }
    return phase_b(ctx, S, 1);
}

int stage_iter_nosync(spcg_ctx* ctx, const spcg_mat* A, const spcg_mat* b, double c2, const StageWs& W) {
    int rc, np = 0;
    const int64_t dpad = round_up(A->cols, 64);
    if ((rc = product_pass(ctx, A, b, W, PM_S, &np, nullptr)) != SPCG_OK) return rc;
    if ((rc = phase_a(ctx, W.S, PA_STEP, W.part_s, nullptr, nullptr, np, dpad, c2)) != SPCG_OK) return rc;
    return phase_b(ctx, W.S, 0);
}

StageWs gated(const StageWs& W, const int32_t* gate, int gmin) {
    StageWs G = W;
    G.S.gate = gate;
    G.S.gmin = gmin;
    return G;
}

int stage_run_nosync(spcg_ctx* ctx, const spcg_mat* A, const spcg_mat* b, double c2,
                     const spcg_precond_t* pc, double* x, int iters, int64_t m_prev = 0) {
    int rc;
    StageWs W;
    if ((rc = ensure_stage_ws(ctx, A->cols, &W, x, pc->pMinv)) != SPCG_OK) return rc;
    if ((rc = stage_start_nosync(ctx, A, b, c2, W, m_prev)) != SPCG_OK) return rc;
    for (int it = 0; it < iters; ++it)
        if ((rc = stage_iter_nosync(ctx, A, b, c2, W)) != SPCG_OK) return rc;
    return SPCG_OK;
}

int check_stage_args(spcg_ctx* ctx, const spcg_mat* A, const spcg_mat* b, const spcg_precond_t* pc,
                     const double* beta) {
    int rc;
    if ((rc = check_mat(ctx, A, "A")) != SPCG_OK) return rc;
    if ((rc = check_mat(ctx, b, "b")) != SPCG_OK) return rc;
    if (!pc) return fail(ctx, SPCG_E_INVALID_ARG, "preconditioner is NULL");
    if (!beta) return fail(ctx, SPCG_E_INVALID_ARG, "beta is NULL");
    if (b->dtype != SPCG_F64) return fail(ctx, SPCG_E_DTYPE, "b must be SPCG_F64");
    if (b->rows != A->rows) return fail(ctx, SPCG_E_SHAPE, "b has %lld rows, A has %lld",
                                        (long long)b->rows, (long long)A->rows);
    if (A->cols != pc->d) return fail(ctx, SPCG_E_SHAPE, "A has %lld columns, preconditioner %lld",
                                      (long long)A->cols, (long long)pc->d);
    if (b->cols < 1) return fail(ctx, SPCG_E_SHAPE, "b needs at least one column");
    if (A->cols > product_max_d(A->dtype)) return fail(ctx, SPCG_E_SHAPE, "d too large");
    return SPCG_OK;
}

// a_i of Theorems 3.3 / 3.4 for the stage sizes m[0..n) actually run.
std::vector<int> theory_a(const int64_t* m, int n, int64_t d, double omega) {
    std::vector<int> a(n, 1);
    auto bound = [&](double r) { return std::log(((1.0 + omega) * r + 1.0) / omega) / std::log(4.0); };
    auto ratio = [&](int64_t mp, int64_t mc) { return std::sqrt((double)(mc - d) / (double)(mp - d)); };
    for (int i = 0; i < n; ++i) {
        const double r = n < 2 ? 1.0 : (i == 0 ? ratio(m[0], m[1]) : ratio(m[i - 1], m[i]));
        a[i] = std::max(1, (int)std::ceil(bound(r) - 1e-12));
    }
    return a;
}

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return ms;
}

// --------------------------------------------------- batched / multi-RHS

struct BatchWork {
    std::vector<spcg_sketch_t*> sk;
    std::vector<spcg_precond_t*> pc;
    DevBuf vecs, scal, probs, tasks, part_s, part_g, part_scal, bestx;
    DevBuf probs2, tasks2;   // a second task list (the nested stage starts' G pass)
    DevBuf rpart;   // per problem: the z slices' shares of g^T z
    // one stream per launch bucket (row-width class x k range: the bucket
    // launches of a pass run concurrently), a private stream for graph
    // capture, fork/join events
    hipStream_t cls[MR_NBUCKET] = {};
    hipStream_t cap = nullptr;
    hipEvent_t fork = nullptr, join[MR_NBUCKET] = {}, tune[2] = {};
    int tasks_per_cu[4] = {};   // autotuned task granularity per storage type (0: not yet)
    int shape[4][MR_NBUCKET] = {};   // autotuned tile shape per storage type and bucket (0: not yet)
    int shape1[4][MR_NBUCKET] = {};  // the same for the Stage I passes over sketch rows
    bool tuned1[4] = {};             // Stage I shapes tuned for this storage type
    // per-problem setup (sketch, preconditioner) is spread over NLANE lanes,
    // each a context of its own (stream and workspaces), so the small
    // transforms and the latency-bound factor chains of different problems
    // overlap; one pinned pivot status per problem
    static constexpr int NLANE = 8;
    spcg_ctx* lane[NLANE] = {};
    hipEvent_t lane_join[NLANE] = {};
    DenseStatus* hstat = nullptr;
    size_t hstat_n = 0;
    // executable graphs kept across solves, by slot (Stage I stage i: slot
    // i; Stage II active set j: slots 64 + 2 j (products) and 65 + 2 j
    // (d-space)); a later solve updates them in place
    std::vector<hipGraphExec_t> gcache;
    bool gcache_busy = false;   // a solve launched cached graphs and did not finish normally
    ~BatchWork() {
        for (auto e : gcache)
            if (e) (void)hipGraphExecDestroy(e);
        for (auto* p : sk) delete p;
        for (auto* p : pc) delete p;
        for (auto* c : lane) {
            if (!c) continue;
            hipStream_t q = c->stream;
            (void)spcg_ctx_destroy(c);
            (void)hipStreamDestroy(q);
        }
        for (auto& e : lane_join)
            if (e) (void)hipEventDestroy(e);
        if (hstat) (void)hipHostFree(hstat);
        for (auto& q : cls)
            if (q) (void)hipStreamDestroy(q);
        if (cap) (void)hipStreamDestroy(cap);
        if (fork) (void)hipEventDestroy(fork);
        for (auto& e : join)
            if (e) (void)hipEventDestroy(e);
        for (auto& e : tune)
            if (e) (void)hipEventDestroy(e);
    }
};

int batch_lanes(spcg_ctx* ctx, BatchWork& W) {
    if (W.lane[0]) return SPCG_OK;
    for (int i = 0; i < BatchWork::NLANE; ++i) {
        hipStream_t q = nullptr;
        HIP_TRY(ctx, hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
        const int rc = spcg_ctx_create(ctx->device, q, &W.lane[i]);
        if (rc != SPCG_OK) {
            (void)hipStreamDestroy(q);
            W.lane[i] = nullptr;
            return fail(ctx, rc, "lane context creation failed");
        }
        HIP_TRY(ctx, hipEventCreateWithFlags(&W.lane_join[i], hipEventDisableTiming));
    }
    return SPCG_OK;
}

// lane streams wait for what is queued on st / st waits for the lanes
int lanes_fork(spcg_ctx* ctx, BatchWork& W, hipStream_t st) {
    HIP_TRY(ctx, hipEventRecord(W.fork, st));
    for (auto* c : W.lane) HIP_TRY(ctx, hipStreamWaitEvent(c->stream, W.fork, 0));
    return SPCG_OK;
}
int lanes_join(spcg_ctx* ctx, BatchWork& W, hipStream_t st) {
    for (int i = 0; i < BatchWork::NLANE; ++i) {
        HIP_TRY(ctx, hipEventRecord(W.lane_join[i], W.lane[i]->stream));
        HIP_TRY(ctx, hipStreamWaitEvent(st, W.lane_join[i], 0));
    }
    return SPCG_OK;
}
// a lane's error becomes the caller's
int lane_fail(spcg_ctx* ctx, spcg_ctx* lane, int rc) {
    ctx->err = lane->err;
    return rc;
}

// The order in which the setup work of the problems is queued: round r
// queues the r-th problem of every lane.  Problems go to lanes longest
// first onto the least loaded lane by an estimate of their cost (what a
// problem computes does not depend on its lane).
std::vector<std::pair<int, int>> lane_schedule(const std::vector<double>& cost) {
    constexpr int NL = BatchWork::NLANE;
    const int n = (int)cost.size();
    std::vector<int> order(n);
    for (int p = 0; p < n; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<std::vector<int>> lanes(NL);
    double load[NL] = {};
    for (int p : order) {
        int best = 0;
        for (int i = 1; i < NL; ++i)
            if (load[i] < load[best]) best = i;
        lanes[best].push_back(p);
        load[best] += cost[p];
    }
    std::vector<std::pair<int, int>> q;   // (problem, lane)
    for (size_t r = 0;; ++r) {
        bool any = false;
        for (int i = 0; i < NL; ++i)
            if (r < lanes[i].size()) {
                q.emplace_back(lanes[i][r], i);
                any = true;
            }
        if (!any) break;
    }
    return q;
}

int batch_streams(spcg_ctx* ctx, BatchWork& W) {
    if (W.cap) return SPCG_OK;
    for (auto& q : W.cls) HIP_TRY(ctx, hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    HIP_TRY(ctx, hipStreamCreateWithFlags(&W.cap, hipStreamNonBlocking));
    HIP_TRY(ctx, hipEventCreateWithFlags(&W.fork, hipEventDisableTiming));
    for (auto& e : W.join) HIP_TRY(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto& e : W.tune) HIP_TRY(ctx, hipEventCreate(&e));
    return SPCG_OK;
}

constexpr int MR_VECS = 6;   // X G Z P S Gt

// Tasks grouped by launch bucket (row-width class x k range, one product
// launch per bucket); the tasks of a problem are contiguous, [t0, t1).
// one_launch puts every problem into the widest class that can read it
// (one launch per pass).  Returns the task count or a negative class error.
int build_tasks(int dtype, const std::vector<MrhsProblem>& hp, std::vector<MrhsTask>& tasks,
                std::vector<MrhsProblem>& out, int64_t target_tasks, int* seg, bool one_launch) {
    tasks.clear();
    out = hp;
    std::vector<int> bkt(hp.size(), -1);
    int64_t bucket_rows[MR_NBUCKET] = {};
    for (size_t p = 0; p < hp.size(); ++p) {
        out[p].t0 = out[p].t1 = 0;
        out[p].lshift = 0;
        if (!hp[p].active) continue;
        int c = mrhs_class(dtype, hp[p].A, hp[p].m, hp[p].lda, hp[p].dmem, hp[p].d);
        if (c < 0) return -1;
        // one launch: the 4-byte, 8-load class reads every row that a
        // direct-load class can (4-byte aligned, its 4-byte vectors within
        // the readable part of the row: implied by either load width; at
        // most 2 KB of data)
        if (one_launch && c != MR_CLASS_GENERIC) c = MR_CLASS_4x8;
        // 16-byte classes of rows that are only 4-byte aligned shift the
        // last row's loads
        out[p].lshift = (c == MR_CLASS_16x1 || c == MR_CLASS_16x2)
                            ? mrhs_row_shift(dtype, hp[p].A, hp[p].m, hp[p].lda, hp[p].dmem, hp[p].d)
                            : 0;
        bkt[p] = one_launch ? mrhs_bucket(c, 0) : mrhs_bucket(c, hp[p].k);
        bucket_rows[bkt[p]] += hp[p].m;
    }
    for (int c = 0; c < MR_NBUCKET; ++c) {
        seg[c] = (int)tasks.size();
        // each bucket is its own launch: split its rows into about
        // target_tasks tasks so that every launch fills the device
        const int64_t rows_per_task = std::max<int64_t>(256, round_up(ceil_div(bucket_rows[c], target_tasks), 16));
        for (size_t p = 0; p < hp.size(); ++p) {
            if (bkt[p] != c) continue;
            out[p].t0 = (int)tasks.size();
            // rows that are not 16-byte aligned: the last row is a task of
            // its own (the 16-byte loads of rows that are only 4-byte
            // aligned load it shifted; the 4-byte and 16-byte classes then
            // split such rows alike, so their sums round alike)
            const int es = dtype == DT_F32 ? 4 : 2;
            const bool split_last =
                hp[p].m > 1 && ((hp[p].lda * es) % 16 != 0 || (uintptr_t)hp[p].A % 16 != 0);
            const int64_t mb = split_last ? hp[p].m - 1 : hp[p].m;
            for (int64_t r = 0; r < mb; r += rows_per_task) {
                MrhsTask t{};
                t.prob = (int)p;
                t.r0 = r;
                t.r1 = std::min<int64_t>(mb, r + rows_per_task);
                tasks.push_back(t);
            }
            if (mb < hp[p].m) {
                MrhsTask t{};
                t.prob = (int)p;
                t.r0 = mb;
                t.r1 = hp[p].m;
                tasks.push_back(t);
            }
            out[p].t1 = (int)tasks.size();
        }
    }
    seg[MR_NBUCKET] = (int)tasks.size();
    return (int)tasks.size();
}

// The task list of one active set, uploaded once and reused by every pass
// over that set (stream synchronisations before the buffers may grow and
// after the upload: the host arrays are pageable).
struct BatchPlan {
    int nt = 0;
    int nprob = 0;
    int seg[MR_NBUCKET + 1] = {};
    int shape[MR_NBUCKET] = {};   // tile shape of each bucket's launch
    bool one_launch = false;
    int set = 0;   // 0: the task and problem buffers tasks / probs, 1: tasks2 / probs2
};
DevBuf& plan_tasks(BatchWork& W, const BatchPlan& plan) { return plan.set ? W.tasks2 : W.tasks; }
DevBuf& plan_probs(BatchWork& W, const BatchPlan& plan) { return plan.set ? W.probs2 : W.probs; }

// tile shape of every bucket: forced (> 0), else the context's tuned one,
// else the two-tile pipeline with 3 slots
void plan_shapes(const BatchWork& W, int dtype, int forced, BatchPlan& plan, bool stage_rows = false) {
    for (int b = 0; b < MR_NBUCKET; ++b) {
        const int tuned = stage_rows ? W.shape1[dtype & 3][b] : W.shape[dtype & 3][b];
        plan.shape[b] = forced > 0 ? forced : tuned > 0 ? tuned : MR_SHAPE_PIPE3;
    }
}

int batched_setup(spcg_ctx* ctx, BatchWork& W, int dtype, const std::vector<MrhsProblem>& hp, int64_t target_tasks,
                  BatchPlan& plan) {
    // earlier passes (or graphs) may still read the buffers that grow below
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<MrhsTask> tasks;
    std::vector<MrhsProblem> probs;
    const int nt = build_tasks(dtype, hp, tasks, probs, target_tasks, plan.seg, plan.one_launch);
    if (nt < 0) return fail(ctx, SPCG_E_SHAPE, "a batched matrix has an unsupported row layout");
    plan.nt = nt;
    plan.nprob = (int)probs.size();
    const size_t per_task = (size_t)mrhs_max_d() * mrhs_max_k();
    DevBuf& tbuf = plan_tasks(W, plan);
    DevBuf& pbuf = plan_probs(W, plan);
    HIP_TRY(ctx, tbuf.ensure(std::max<size_t>(1, tasks.size()) * sizeof(MrhsTask)));
    HIP_TRY(ctx, pbuf.ensure(probs.size() * sizeof(MrhsProblem)));
    HIP_TRY(ctx, W.part_s.ensure((size_t)std::max(nt, 1) * per_task * 4));
    HIP_TRY(ctx, W.part_g.ensure((size_t)std::max(nt, 1) * per_task * 4));
    HIP_TRY(ctx, W.part_scal.ensure((size_t)std::max(nt, 1) * 2 * mrhs_max_k() * 4));
    hipStream_t st = ctx->stream;
    if (nt)
        HIP_TRY(ctx, hipMemcpyAsync(tbuf.p, tasks.data(), tasks.size() * sizeof(MrhsTask), hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipMemcpyAsync(pbuf.p, probs.data(), probs.size() * sizeof(MrhsProblem), hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    return SPCG_OK;
}

// The product launches of one pass on stream st: each bucket (row-width
// class x k range) on its own stream (the buckets write disjoint task
// partials), joined back into st; only_bucket >= 0 launches that bucket
// alone.  Launches only: safe to capture.
int batched_products(spcg_ctx* ctx, BatchWork& W, hipStream_t st, int dtype, int mode, const BatchPlan& plan,
                     int only_bucket = -1) {
    int used = 0;
    for (int c = 0; c < MR_NBUCKET; ++c)
        used += plan.seg[c + 1] > plan.seg[c] && (only_bucket < 0 || c == only_bucket);
    if (used > 1) HIP_TRY(ctx, hipEventRecord(W.fork, st));
    for (int c = 0; c < MR_NBUCKET; ++c) {
        const int n = plan.seg[c + 1] - plan.seg[c];
        if (n <= 0 || (only_bucket >= 0 && c != only_bucket)) continue;
        hipStream_t sc = st;
        if (used > 1) {
            sc = W.cls[c];
            HIP_TRY(ctx, hipStreamWaitEvent(sc, W.fork, 0));
        }
        HIP_TRY(ctx, run_mrhs_product(sc, dtype, mode, c / MR_KB, plan.shape[c], plan_tasks(W, plan).as<MrhsTask>(),
                                      plan.seg[c], n, plan_probs(W, plan).as<MrhsProblem>(), W.part_s.as<float>(),
                                      W.part_g.as<float>(), W.part_scal.as<float>()));
        if (used > 1) {
            HIP_TRY(ctx, hipEventRecord(W.join[c], sc));
            HIP_TRY(ctx, hipStreamWaitEvent(st, W.join[c], 0));
        }
    }
    return SPCG_OK;
}

int batched_dspace(spcg_ctx* ctx, BatchWork& W, hipStream_t st, int variant, const BatchPlan& plan) {
    HIP_TRY(ctx, run_mrhs_dspace(st, variant, plan_probs(W, plan).as<MrhsProblem>(), plan.nprob, W.part_s.as<float>(),
                                 W.part_g.as<float>(), W.part_scal.as<float>()));
    return SPCG_OK;
}

// Captures the launches of body(stream) into an executable graph, recorded
// on the private capture stream (the library stream may be the null stream,
// which cannot be captured).  *exec stays null when capture is unavailable;
// the caller then launches directly.  With slot >= 0 the executable graph
// of that slot from an earlier solve is updated in place with the new
// capture (hipGraphExecUpdate: the same topology with new kernel arguments
// needs no instantiation) and stays cached; a failed update instantiates
// anew.  Cached graphs are idle here: every solve ends with a stream
// synchronisation after its last graph launch, and slots are unique
// within a solve.
template <class F>
int capture_graph(spcg_ctx* ctx, BatchWork& W, F&& body, hipGraphExec_t* exec, int slot = -1) {
    *exec = nullptr;
    if (hipStreamBeginCapture(W.cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return SPCG_OK;
    }
    const int rc = body(W.cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(W.cap, &g);
    if (rc != SPCG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        return SPCG_OK;
    }
    if (slot >= 0) {
        if ((int)W.gcache.size() <= slot) W.gcache.resize((size_t)slot + 1, nullptr);
        hipGraphExec_t& c = W.gcache[(size_t)slot];
        if (c) {
            hipGraphNode_t err_node = nullptr;
            hipGraphExecUpdateResult res = hipGraphExecUpdateError;
            if (hipGraphExecUpdate(c, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
                (void)hipGraphDestroy(g);
                *exec = c;
                return SPCG_OK;
            }
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(c);
            c = nullptr;
        }
        if (hipGraphInstantiate(&c, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGetLastError();
            c = nullptr;
        }
        (void)hipGraphDestroy(g);
        *exec = c;
        return SPCG_OK;
    }
    const hipError_t ei = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        (void)hipGetLastError();
        *exec = nullptr;
    }
    return SPCG_OK;
}

// Runs body once: as a captured graph of the given cache slot launched on
// the library stream when graphs are on (*launched counts it), else
// directly on the library stream.
template <class F>
int run_captured(spcg_ctx* ctx, BatchWork& W, bool graphs, F&& body, int slot, int* launched) {
    if (graphs) {
        hipGraphExec_t ex = nullptr;
        int rc;
        if ((rc = capture_graph(ctx, W, body, &ex, slot)) != SPCG_OK) return rc;
        if (ex) {
            HIP_TRY(ctx, hipGraphLaunch(ex, ctx->stream));
            ++*launched;
            return SPCG_OK;
        }
    }
    return body(ctx->stream);
}

int batched_solve(spcg_ctx* ctx, int nprob, const spcg_mat* X, const spcg_mat* Y, const spcg_solve_opts* opts,
                  double* const* beta, spcg_solve_stats* stats) {
    int rc;
    if (nprob < 1 || !X || !Y || !beta || !opts) return fail(ctx, SPCG_E_INVALID_ARG, "bad batched arguments");
    const int dtype = X[0].dtype;
    if (dtype != SPCG_F32 && dtype != SPCG_BF16)
        return fail(ctx, SPCG_E_DTYPE, "the batched form needs SPCG_F32 or SPCG_BF16 storage");
    if (opts->a_rule != SPCG_A_FIXED)
        return fail(ctx, SPCG_E_INVALID_ARG, "the batched form takes a fixed a / a_list");
    for (int p = 0; p < nprob; ++p) {
        if ((rc = check_mat(ctx, &X[p], "X[p]")) != SPCG_OK) return rc;
        if ((rc = check_mat(ctx, &Y[p], "Y[p]")) != SPCG_OK) return rc;
        if (X[p].dtype != dtype) return fail(ctx, SPCG_E_DTYPE, "all X[p] must share one storage type");
        if (Y[p].dtype != SPCG_F64) return fail(ctx, SPCG_E_DTYPE, "Y[p] must be SPCG_F64");
        if (Y[p].rows != X[p].rows) return fail(ctx, SPCG_E_SHAPE, "X[%d] and Y[%d] row counts differ", p, p);
        if (X[p].cols > mrhs_max_d()) return fail(ctx, SPCG_E_SHAPE, "batched form: d <= %d", mrhs_max_d());
        if (Y[p].cols > mrhs_max_k()) return fail(ctx, SPCG_E_SHAPE, "batched form: k <= %d", mrhs_max_k());
        if (!beta[p]) return fail(ctx, SPCG_E_INVALID_ARG, "beta[%d] is NULL", p);
    }
    if (opts->method != SPCG_METHOD_SPCG && opts->method != SPCG_METHOD_FULL_PCG)
        return fail(ctx, SPCG_E_INVALID_ARG, "unknown method %d", opts->method);
    const int a = opts->a > 0 ? opts->a : 3;
    const int T = opts->T > 0 ? opts->T : 100;
    const double tol = opts->tol > 0.0 ? opts->tol : 5e-7;
    hipStream_t st = ctx->stream;
    const bool timing = opts->time_phases != 0;
    if (timing || opts->time_products) {
        if ((rc = ensure_events(ctx)) != SPCG_OK) return rc;
    }
    if (timing) HIP_TRY(ctx, hipEventRecord(ctx->ev_phase[0], st));
    ProductTimer timer;
    timer.ctx = ctx;
    double timed_bytes = 0.0;
    const int64_t es = dtype_bytes(dtype);
    if (!ctx->batch) ctx->batch = new (std::nothrow) BatchWork();
    if (!ctx->batch) return fail(ctx, SPCG_E_NOMEM, "host allocation failed");
    BatchWork& W = *ctx->batch;
    while ((int)W.sk.size() < nprob) {
        W.sk.push_back(new (std::nothrow) spcg_sketch_t());
        W.pc.push_back(new (std::nothrow) spcg_precond_t());
        if (!W.sk.back() || !W.pc.back()) return fail(ctx, SPCG_E_NOMEM, "host allocation failed");
    }
    spcg_sketch_opts so = opts->sketch;
    so.hat_only = opts->method == SPCG_METHOD_FULL_PCG ? 1 : 0;
    // sketches and one-pass preconditioners of the problems on the lanes
    // (problem p on lane p mod NLANE), each phase joined back into st
    if ((rc = batch_streams(ctx, W)) != SPCG_OK) return rc;
    if ((rc = batch_lanes(ctx, W)) != SPCG_OK) return rc;
    // The sketches keep problem p on lane p mod NLANE: their phase keeps the
    // GPU busy throughout, and balancing their estimated bytes over the lanes
    // measured no faster.  The preconditioners are chains of small dependent
    // kernels (a chain grows with the 64-column panels), balanced over the
    // lanes below.
    if ((rc = lanes_fork(ctx, W, st)) != SPCG_OK) return rc;
    for (int p = 0; p < nprob; ++p) {
        spcg_ctx* ln = W.lane[p % BatchWork::NLANE];
        if ((rc = sketch_build(ln, &X[p], &Y[p], &so, false, W.sk[p])) != SPCG_OK) return lane_fail(ctx, ln, rc);
    }
    if ((rc = lanes_join(ctx, W, st)) != SPCG_OK) return rc;
    std::vector<double> cost_pc(nprob);
    for (int p = 0; p < nprob; ++p) cost_pc[p] = 1.0 + (double)ceil_div(X[p].cols, 64);
    if (timing) HIP_TRY(ctx, hipEventRecord(ctx->ev_phase[1], st));
    const int qmode = opts->precond.qr_passes;
    const bool defer = qmode == 0 || qmode == 1;
    if (defer && W.hstat_n < (size_t)nprob) {
        if (W.hstat) HIP_TRY(ctx, hipHostFree(W.hstat));
        W.hstat = nullptr;
        W.hstat_n = 0;
        HIP_TRY(ctx, hipHostMalloc((void**)&W.hstat, (size_t)nprob * sizeof(DenseStatus), hipHostMallocDefault));
        W.hstat_n = (size_t)nprob;
    }
    if ((rc = lanes_fork(ctx, W, st)) != SPCG_OK) return rc;
    for (const auto& pl : lane_schedule(cost_pc)) {
        const int p = pl.first;
        spcg_ctx* ln = W.lane[pl.second];
        if ((rc = precond_build(ln, W.sk[p], &opts->precond, false, W.pc[p], defer ? &W.hstat[p] : nullptr)) !=
            SPCG_OK)
            return lane_fail(ctx, ln, rc);
    }
    if ((rc = lanes_join(ctx, W, st)) != SPCG_OK) return rc;
    if (defer) {
        // the pivot statuses: a factor that failed or is badly scaled is
        // built again here, with the fallback of a single solve
        HIP_TRY(ctx, hipStreamSynchronize(st));
        ctx->syncs++;
        for (int p = 0; p < nprob; ++p) {
            if (precond_status_ok(W.hstat[p], qmode)) continue;
            if ((rc = precond_build(ctx, W.sk[p], &opts->precond, false, W.pc[p])) != SPCG_OK) return rc;
        }
    }
    if (timing) HIP_TRY(ctx, hipEventRecord(ctx->ev_phase[2], st));
    const int64_t ldv = mrhs_max_d();
    const int kmax = mrhs_max_k();
    HIP_TRY(ctx, W.vecs.ensure((size_t)nprob * MR_VECS * kmax * ldv * 8));
    HIP_TRY(ctx, W.scal.ensure((size_t)nprob * kmax * sizeof(MrhsScalars)));
    HIP_TRY(ctx, W.rpart.ensure((size_t)nprob * MR_ZSLICES * kmax * 8));
    HIP_TRY(ctx, hipMemsetAsync(W.vecs.p, 0, (size_t)nprob * MR_VECS * kmax * ldv * 8, st));
    HIP_TRY(ctx, hipMemsetAsync(W.scal.p, 0, (size_t)nprob * kmax * sizeof(MrhsScalars), st));
    std::vector<MrhsProblem> hp(nprob);
    int64_t maxK = 0;
    for (int p = 0; p < nprob; ++p) {
        MrhsProblem& q = hp[p];
        std::memset(&q, 0, sizeof q);
        double* base = W.vecs.as<double>() + (size_t)p * MR_VECS * kmax * ldv;
        q.d = (int)X[p].cols;
        q.k = (int)Y[p].cols;
        q.ldv = ldv;
        q.X = base;
        q.G = base + 1 * kmax * ldv;
        q.Z = base + 2 * kmax * ldv;
        q.P = base + 3 * kmax * ldv;
        q.S = base + 4 * kmax * ldv;
        q.Gt = base + 5 * kmax * ldv;
        q.Minv = W.pc[p]->pMinv;
        q.sc = W.scal.as<MrhsScalars>() + (size_t)p * kmax;
        q.rho_part = W.rpart.as<double>() + (size_t)p * MR_ZSLICES * kmax;
        maxK = std::max<int64_t>(maxK, W.sk[p]->K);
    }
    // tasks per launch in Stage I: about 4 per CU, never fewer than 256 rows each
    const int64_t target_tasks = 4 * (int64_t)ctx->num_cu;
    const bool graphs_on = opts->batch_direct == 0;
    if ((rc = batch_streams(ctx, W)) != SPCG_OK) return rc;
    int graphs_launched = 0;
    // cached graphs may still run if an earlier solve returned early
    if (graphs_on && W.gcache_busy) HIP_TRY(ctx, hipStreamSynchronize(st));
    W.gcache_busy = graphs_on;
    std::vector<int> t1(nprob, 0), t2(nprob, 0), conv(nprob, 0);
    // Stage I: stage i of every problem that has one; its G pass and a_i S
    // passes form one graph.  Nested SRHT prefixes: a problem that ran
    // stage i - 1 starts stage i from its previous gradient plus a G pass
    // over the new prefix rows only (as the single-problem path does).
    std::vector<char> ran_prev(nprob, 0);
    // the stage at which the Stage I shapes are tuned: the largest one that
    // every problem with a sketch has
    int64_t i_tune = maxK - 1;
    for (int p = 0; p < nprob; ++p)
        if (W.sk[p]->K > 0) i_tune = std::min<int64_t>(i_tune, W.sk[p]->K - 1);
    for (int64_t i = 0; i < maxK; ++i) {
        int ai = a;
        if (opts->a_list_len > 0) ai = opts->a_list[std::min<int64_t>(i, opts->a_list_len - 1)];
        bool any = false;
        for (int p = 0; p < nprob; ++p) {
            MrhsProblem& q = hp[p];
            q.active = i < W.sk[p]->K && t1[p] + ai <= T;
            if (!q.active) continue;
            any = true;
            spcg_mat A{}, b{};
            double c2 = 1.0;
            spcg_sketch_view(W.sk[p], (int)i, &A, &b, &c2);
            q.A = A.data;
            q.m = A.rows;
            q.lda = A.ld;
            q.dmem = A.ld;   // sketch rows are zero-padded to ld
            q.b = static_cast<const double*>(b.data);
            q.ldb = b.ld;
            q.c2 = c2;
            q.gscale = 0.0;
        }
        if (!any) continue;
        // stage rows: every problem's sketch has the same element type
        const int sdt = W.sk[0]->bdtype;
        BatchPlan plan;
        plan.one_launch = opts->batch_one_launch != 0;
        if ((rc = batched_setup(ctx, W, sdt, hp, target_tasks, plan)) != SPCG_OK) return rc;
        // Stage I tile shapes: tuned once per context and storage type at the
        // largest stage every problem has, by timing three S passes of each
        // bucket alone in every shape its class has (the partials are
        // overwritten by the stage's own passes; iterates are unaffected)
        if (opts->batch_shape <= 0 && !W.tuned1[sdt & 3] && i == i_tune) {
            plan_shapes(W, sdt, 0, plan, true);
            for (int b = 0; b < MR_NBUCKET; ++b) {
                if (plan.seg[b + 1] <= plan.seg[b] || b / MR_KB == MR_CLASS_GENERIC) continue;
                double best_ms = INFINITY;
                int best = MR_SHAPE_PIPE3;
                for (int sh = MR_SHAPE_PLAIN; sh < MR_NSHAPE; ++sh) {
                    if (!mrhs_shape_native(b / MR_KB, sh)) continue;
                    plan.shape[b] = sh;
                    if ((rc = batched_products(ctx, W, st, sdt, PM_S, plan, b)) != SPCG_OK) return rc;   // warm-up
                    HIP_TRY(ctx, hipEventRecord(W.tune[0], st));
                    for (int rep = 0; rep < 3; ++rep)
                        if ((rc = batched_products(ctx, W, st, sdt, PM_S, plan, b)) != SPCG_OK) return rc;
                    HIP_TRY(ctx, hipEventRecord(W.tune[1], st));
                    HIP_TRY(ctx, hipEventSynchronize(W.tune[1]));
                    const double ms = elapsed_ms(W.tune[0], W.tune[1]) / 3.0;
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = sh;
                    }
                }
                W.shape1[sdt & 3][b] = best;
            }
            W.tuned1[sdt & 3] = true;
        }
        plan_shapes(W, sdt, opts->batch_shape, plan, true);
        // the starting G pass: over the new prefix rows [m_{i-1}, m_i) of the
        // problems that can reuse their gradient, over all rows otherwise
        BatchPlan gplan;
        bool nested = false;
        if (opts->nested_gradient && i > 0) {
            std::vector<MrhsProblem> hg = hp;
            for (int p = 0; p < nprob; ++p) {
                MrhsProblem& g = hg[p];
                if (!g.active || !ran_prev[p] || W.sk[p]->kind != SPCG_SKETCH_SRHT) continue;
                const int64_t mprev = W.sk[p]->m[i - 1];
                if (mprev <= 0 || mprev >= g.m) continue;
                g.A = static_cast<const char*>(g.A) + (size_t)mprev * g.lda * dtype_bytes(sdt);
                g.b += (size_t)mprev * g.ldb;
                g.m -= mprev;
                g.gscale = (double)mprev / (double)hp[p].m;
                nested = true;
            }
            if (nested) {
                gplan.set = 1;
                gplan.one_launch = plan.one_launch;
                if ((rc = batched_setup(ctx, W, sdt, hg, target_tasks, gplan)) != SPCG_OK) return rc;
                plan_shapes(W, sdt, opts->batch_shape, gplan, true);
            }
        }
        auto stage = [&](hipStream_t s) -> int {
            int r;
            if (nested) {
                if ((r = batched_products(ctx, W, s, sdt, PM_G, gplan)) != SPCG_OK) return r;
                if ((r = batched_dspace(ctx, W, s, PA_START_NESTED, gplan)) != SPCG_OK) return r;
            } else {
                if ((r = batched_products(ctx, W, s, sdt, PM_G, plan)) != SPCG_OK) return r;
                if ((r = batched_dspace(ctx, W, s, PA_START, plan)) != SPCG_OK) return r;
            }
            for (int it = 0; it < ai; ++it) {
                if ((r = batched_products(ctx, W, s, sdt, PM_S, plan)) != SPCG_OK) return r;
                if ((r = batched_dspace(ctx, W, s, PA_STEP, plan)) != SPCG_OK) return r;
            }
            return SPCG_OK;
        };
        if ((rc = run_captured(ctx, W, graphs_on, stage, (int)i, &graphs_launched)) != SPCG_OK) return rc;
        for (int p = 0; p < nprob; ++p) {
            if (hp[p].active) t1[p] += ai;
            ran_prev[p] = hp[p].active ? 1 : 0;
        }
    }
    if (timing) HIP_TRY(ctx, hipEventRecord(ctx->ev_phase[3], st));
    // Stage II on the full data; every problem stops on its own test
    for (int p = 0; p < nprob; ++p) {
        MrhsProblem& q = hp[p];
        q.active = 1;
        q.A = X[p].data;
        q.m = X[p].rows;
        q.lda = X[p].ld;
        q.dmem = X[p].cols;
        q.b = static_cast<const double*>(Y[p].data);
        q.ldb = Y[p].ld;
        q.c2 = 1.0;
    }
    // task granularity of the full-data passes: fixed, cached, or tuned now
    // by timing one product pass per candidate (the partials are discarded:
    // the d-space step is not run, so the iterates are unaffected)
    int tpc = opts->batch_tasks_per_cu > 0 ? opts->batch_tasks_per_cu : W.tasks_per_cu[dtype & 3];
    // tile shape per bucket: tuned once per context and storage type, by
    // timing three product passes of each bucket alone in every shape its
    // class has (at the tuned granularity, else 4 tasks per CU)
    bool shapes_tuned = false;
    float tune_ms[MR_NBUCKET * 4] = {};
    if (opts->batch_shape <= 0) {
        for (int b = 0; b < MR_NBUCKET; ++b) shapes_tuned = shapes_tuned || W.shape[dtype & 3][b] > 0;
    }
    if (opts->batch_shape <= 0 && !shapes_tuned) {
        BatchPlan tp;
        tp.one_launch = opts->batch_one_launch != 0;
        if ((rc = batched_setup(ctx, W, dtype, hp, (int64_t)(tpc > 0 ? tpc : 4) * ctx->num_cu, tp)) != SPCG_OK)
            return rc;
        plan_shapes(W, dtype, 0, tp);
        for (int b = 0; b < MR_NBUCKET; ++b) {
            if (tp.seg[b + 1] <= tp.seg[b] || b / MR_KB == MR_CLASS_GENERIC) continue;
            double best_ms = INFINITY;
            int best = MR_SHAPE_PIPE3;
            for (int sh = MR_SHAPE_PLAIN; sh < MR_NSHAPE; ++sh) {
                if (!mrhs_shape_native(b / MR_KB, sh)) continue;
                tp.shape[b] = sh;
                if ((rc = batched_products(ctx, W, st, dtype, PM_SG, tp, b)) != SPCG_OK) return rc;   // warm-up
                HIP_TRY(ctx, hipEventRecord(W.tune[0], st));
                for (int rep = 0; rep < 3; ++rep)
                    if ((rc = batched_products(ctx, W, st, dtype, PM_SG, tp, b)) != SPCG_OK) return rc;
                HIP_TRY(ctx, hipEventRecord(W.tune[1], st));
                HIP_TRY(ctx, hipEventSynchronize(W.tune[1]));
                const double ms = elapsed_ms(W.tune[0], W.tune[1]) / 3.0;
                tune_ms[b * 4 + sh - 1] = (float)ms;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = sh;
                }
            }
            W.shape[dtype & 3][b] = best;
        }
    }
    if (tpc <= 0) {
        double best_ms = INFINITY;
        for (int cand : {2, 4, 8}) {
            BatchPlan tp;
            tp.one_launch = opts->batch_one_launch != 0;
            if ((rc = batched_setup(ctx, W, dtype, hp, (int64_t)cand * ctx->num_cu, tp)) != SPCG_OK) return rc;
            plan_shapes(W, dtype, opts->batch_shape, tp);
            if ((rc = batched_products(ctx, W, st, dtype, PM_SG, tp)) != SPCG_OK) return rc;   // warm-up
            HIP_TRY(ctx, hipEventRecord(W.tune[0], st));
            if ((rc = batched_products(ctx, W, st, dtype, PM_SG, tp)) != SPCG_OK) return rc;
            HIP_TRY(ctx, hipEventRecord(W.tune[1], st));
            HIP_TRY(ctx, hipEventSynchronize(W.tune[1]));
            const double ms = elapsed_ms(W.tune[0], W.tune[1]);
            if (ms < best_ms) {
                best_ms = ms;
                tpc = cand;
            }
        }
        W.tasks_per_cu[dtype & 3] = tpc;
    }
    const int64_t full_tasks = (int64_t)tpc * ctx->num_cu;
    std::vector<MrhsScalars> hs((size_t)nprob * kmax);
    // Divergence guard: the FP32 products have an accuracy floor; a problem
    // whose stopping ratio climbs well above its best value (iterating past
    // the floor) stops, keeping the best iterate seen.
    std::vector<double> best(nprob, INFINITY);
    DevBuf& bestx = W.bestx;
    HIP_TRY(ctx, bestx.ensure((size_t)nprob * kmax * ldv * 8));
    bool set_changed = true;
    auto check = [&](int* n_active) -> int {
        HIP_TRY(ctx, hipMemcpyAsync(hs.data(), W.scal.p, hs.size() * sizeof(MrhsScalars), hipMemcpyDeviceToHost, st));
        HIP_TRY(ctx, hipStreamSynchronize(st));
        int act = 0;
        for (int p = 0; p < nprob; ++p) {
            if (!hp[p].active) continue;
            bool done = true;
            double worst = 0.0;
            for (int c = 0; c < hp[p].k; ++c) {
                const MrhsScalars& s = hs[(size_t)p * kmax + c];
                if (s.breakdown) return fail(ctx, SPCG_E_BREAKDOWN, "PCG breakdown in problem %d", p);
                const double ratio = s.exact ? 0.0 : std::sqrt(std::max(s.rho, 0.0)) /
                                                         std::max(std::sqrt(std::max(s.ax2, 0.0)), 1e-300);
                worst = std::max(worst, ratio);
                done = done && ratio <= tol;
            }
            double* xp = W.vecs.as<double>() + (size_t)p * MR_VECS * kmax * ldv;
            double* bp = bestx.as<double>() + (size_t)p * kmax * ldv;
            const bool diverging = worst > 100.0 * best[p];
            if (worst < best[p]) {
                best[p] = worst;
                HIP_TRY(ctx, hipMemcpyAsync(bp, xp, (size_t)kmax * ldv * 8, hipMemcpyDeviceToDevice, st));
            }
            if (done) {
                conv[p] = 1;
                hp[p].active = 0;
                set_changed = true;
            } else if (diverging || t1[p] + t2[p] >= T) {
                hp[p].active = 0;
                set_changed = true;
                HIP_TRY(ctx, hipMemcpyAsync(xp, bp, (size_t)kmax * ldv * 8, hipMemcpyDeviceToDevice, st));
            } else {
                ++act;
            }
        }
        *n_active = act;
        return SPCG_OK;
    };
    int act = 0;
    BatchPlan plan;
    plan.one_launch = opts->batch_one_launch != 0;
    if ((rc = batched_setup(ctx, W, dtype, hp, full_tasks, plan)) != SPCG_OK) return rc;
    plan_shapes(W, dtype, opts->batch_shape, plan);
    set_changed = false;
    if ((rc = batched_products(ctx, W, st, dtype, PM_G, plan)) != SPCG_OK) return rc;
    if ((rc = batched_dspace(ctx, W, st, PA_START, plan)) != SPCG_OK) return rc;
    if ((rc = check(&act)) != SPCG_OK) return rc;
    // one graph for the product launches and one for the d-space launch of
    // each active set, replayed every iteration (events around the product
    // graph time the products alone)
    hipGraphExec_t gprod = nullptr, gds = nullptr;
    int set_index = 0;   // active sets of this Stage II, for the graph cache slots
    while (act > 0) {
        if (set_changed) {
            if ((rc = batched_setup(ctx, W, dtype, hp, full_tasks, plan)) != SPCG_OK) return rc;
            plan_shapes(W, dtype, opts->batch_shape, plan);
            set_changed = false;
            gprod = gds = nullptr;
            if (graphs_on) {
                const int slot = 64 + 2 * set_index++;
                if ((rc = capture_graph(ctx, W, [&](hipStream_t s) { return batched_products(ctx, W, s, dtype, PM_SG, plan); },
                                        &gprod, slot)) != SPCG_OK)
                    return rc;
                if ((rc = capture_graph(ctx, W, [&](hipStream_t s) { return batched_dspace(ctx, W, s, PA_REFRESH, plan); },
                                        &gds, slot + 1)) != SPCG_OK)
                    return rc;
            }
        }
        const bool timed = opts->time_products && timer.used < MAX_TIMED;
        if (timed) {
            for (int p = 0; p < nprob; ++p)
                if (hp[p].active) timed_bytes += (double)hp[p].m * (hp[p].d * es + hp[p].k * 8);
            HIP_TRY(ctx, hipEventRecord(ctx->ev_prod[2 * timer.used], st));
        }
        if (gprod) {
            HIP_TRY(ctx, hipGraphLaunch(gprod, st));
            ++graphs_launched;
        } else if ((rc = batched_products(ctx, W, st, dtype, PM_SG, plan)) != SPCG_OK) {
            return rc;
        }
        if (timed) {
            HIP_TRY(ctx, hipEventRecord(ctx->ev_prod[2 * timer.used + 1], st));
            timer.used++;
        }
        if (gds) {
            HIP_TRY(ctx, hipGraphLaunch(gds, st));
            ++graphs_launched;
        } else if ((rc = batched_dspace(ctx, W, st, PA_REFRESH, plan)) != SPCG_OK) {
            return rc;
        }
        for (int p = 0; p < nprob; ++p)
            if (hp[p].active) ++t2[p];
        if ((rc = check(&act)) != SPCG_OK) return rc;
    }
    if (timing) HIP_TRY(ctx, hipEventRecord(ctx->ev_phase[4], st));
    // beta[p] (d x k row-major) <- X (column by column)
    for (int p = 0; p < nprob; ++p)
        HIP_TRY(ctx, hipMemcpy2DAsync(beta[p], (size_t)hp[p].k * 8, hp[p].X, 8, 8, hp[p].d, hipMemcpyDeviceToDevice, st));
    for (int p = 0; p < nprob; ++p)
        for (int c = 1; c < hp[p].k; ++c)
            HIP_TRY(ctx, hipMemcpy2DAsync(beta[p] + c, (size_t)hp[p].k * 8, hp[p].X + (size_t)c * ldv, 8, 8, hp[p].d,
                                          hipMemcpyDeviceToDevice, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    W.gcache_busy = false;
    double prod_ms = 0.0;
    for (int i = 0; i < timer.used; ++i) prod_ms += elapsed_ms(ctx->ev_prod[2 * i], ctx->ev_prod[2 * i + 1]);
    bool all = true;
    for (int p = 0; p < nprob; ++p) {
        all = all && conv[p];
        if (stats) {
            spcg_solve_stats& s = stats[p];
            std::memset(&s, 0, sizeof s);
            if (p == 0 && opts->time_products) {
                s.product_launches = timer.used;
                s.product_ms_sum = prod_ms;
                s.product_bytes = timed_bytes;
            }
            s.K = (int32_t)W.sk[p]->K;
            s.T_stage1 = t1[p];
            s.T_stage2 = t2[p];
            s.converged = conv[p];
            s.qr_passes = W.pc[p]->passes;
            s.batch_tasks_per_cu = tpc;
            s.batch_graphs = graphs_launched;
            for (int b = 0; b < MR_NBUCKET && b < 16; ++b)
                s.batch_shapes[b] = plan.seg[b + 1] > plan.seg[b] ? plan.shape[b] : 0;
            for (int b = 0; b < MR_NBUCKET * 4 && b < 64; ++b) s.batch_tune_ms[b] = tune_ms[b];
            s.rho_final = hs[(size_t)p * kmax].rho;
            s.ax_norm = std::sqrt(std::max(hs[(size_t)p * kmax].ax2, 0.0));
            if (timing) {
                s.t_sketch_ms = elapsed_ms(ctx->ev_phase[0], ctx->ev_phase[1]);
                s.t_precond_ms = elapsed_ms(ctx->ev_phase[1], ctx->ev_phase[2]);
                s.t_stage1_ms = elapsed_ms(ctx->ev_phase[2], ctx->ev_phase[3]);
                s.t_stage2_ms = elapsed_ms(ctx->ev_phase[3], ctx->ev_phase[4]);
                s.t_total_ms = elapsed_ms(ctx->ev_phase[0], ctx->ev_phase[4]);
            }
        }
    }
    if (!all) {
        fail(ctx, SPCG_W_NOT_CONVERGED, "some problems did not meet tol=%g within T=%d", tol, T);
        return SPCG_W_NOT_CONVERGED;
    }
    return SPCG_OK;
}



// ------------------------------------------- one PCG solve, k right-hand sides

// The k columns of beta (d x k row-major) <-> the column-major d-space
// vectors of a multi-RHS problem (column c at v + c ldv).
int beta_to_cols(spcg_ctx* ctx, const double* beta, int64_t d, int64_t k, double* v, int64_t ldv) {
    for (int64_t c = 0; c < k; ++c)
        HIP_TRY(ctx, hipMemcpy2DAsync(v + c * ldv, 8, beta + c, (size_t)k * 8, 8, d, hipMemcpyDeviceToDevice,
                                      ctx->stream));
    return SPCG_OK;
}
int cols_to_beta(spcg_ctx* ctx, const double* v, int64_t ldv, int64_t d, int64_t k, double* beta) {
    for (int64_t c = 0; c < k; ++c)
        HIP_TRY(ctx, hipMemcpy2DAsync(beta + c, (size_t)k * 8, v + c * ldv, 8, 8, d, hipMemcpyDeviceToDevice,
                                      ctx->stream));
    return SPCG_OK;
}

// True when the matrix-core multi-RHS product takes A (FP32 or BF16 rows of
// a supported layout, d <= 512, k <= 16); other stages run column by column.
bool mrhs_stage_ok(const spcg_mat* A, int64_t k) {
    if (A->dtype != SPCG_F32 && A->dtype != SPCG_BF16) return false;
    if (A->cols > mrhs_max_d() || k > mrhs_max_k()) return false;
    const int64_t dmem = A->reserved == 1 ? A->ld : A->cols;
    return mrhs_class(A->dtype, A->data, A->rows, A->ld, dmem, (int)A->cols) >= 0;
}

// PCG(A, b, c2, M, beta, iters) for the k columns of b at once: every
// product pass reads A once for all columns (MFMA tiles, FP32 accumulation,
// FP64 residuals), the d-space step runs per column, and the stopping test
// passes when every column passes.  sc0: column 0's scalars at the end;
// resid0: c2 ||b - A beta||^2 of column 0 at the start.
int mrhs_stage_run(spcg_ctx* ctx, const spcg_mat* A, const spcg_mat* b, double c2, const spcg_precond_t* pc,
                   double* beta, int iters, double tol, bool refresh, int check_every, StageRun* out,
                   MrhsScalars* sc0, double* resid0) {
    int rc;
    if (!ctx->batch) ctx->batch = new (std::nothrow) BatchWork();
    if (!ctx->batch) return fail(ctx, SPCG_E_NOMEM, "host allocation failed");
    BatchWork& W = *ctx->batch;
    if ((rc = batch_streams(ctx, W)) != SPCG_OK) return rc;
    hipStream_t st = ctx->stream;
    const int64_t d = A->cols, k = b->cols;
    const int64_t ldv = mrhs_max_d();
    const int kmax = mrhs_max_k();
    // the vectors may still be read by an earlier batched call's graphs
    HIP_TRY(ctx, hipStreamSynchronize(st));
    HIP_TRY(ctx, W.vecs.ensure((size_t)MR_VECS * kmax * ldv * 8));
    HIP_TRY(ctx, W.scal.ensure((size_t)kmax * sizeof(MrhsScalars)));
    HIP_TRY(ctx, W.rpart.ensure((size_t)MR_ZSLICES * kmax * 8));
    HIP_TRY(ctx, hipMemsetAsync(W.vecs.p, 0, (size_t)MR_VECS * kmax * ldv * 8, st));
    HIP_TRY(ctx, hipMemsetAsync(W.scal.p, 0, (size_t)kmax * sizeof(MrhsScalars), st));
    std::vector<MrhsProblem> hp(1);
    MrhsProblem& q = hp[0];
    std::memset(&q, 0, sizeof q);
    double* base = W.vecs.as<double>();
    q.d = (int)d;
    q.k = (int)k;
    q.ldv = ldv;
    q.X = base;
    q.G = base + 1 * kmax * ldv;
    q.Z = base + 2 * kmax * ldv;
    q.P = base + 3 * kmax * ldv;
    q.S = base + 4 * kmax * ldv;
    q.Gt = base + 5 * kmax * ldv;
    q.Minv = pc->pMinv;
    q.sc = W.scal.as<MrhsScalars>();
    q.rho_part = W.rpart.as<double>();
    q.A = A->data;
    q.m = A->rows;
    q.lda = A->ld;
    q.dmem = A->reserved == 1 ? A->ld : A->cols;
    q.b = static_cast<const double*>(b->data);
    q.ldb = b->ld;
    q.c2 = c2;
    q.active = 1;
    if ((rc = beta_to_cols(ctx, beta, d, k, q.X, ldv)) != SPCG_OK) return rc;
    BatchPlan plan;
    if ((rc = batched_setup(ctx, W, A->dtype, hp, 4 * (int64_t)ctx->num_cu, plan)) != SPCG_OK) return rc;
    plan_shapes(W, A->dtype, 0, plan);
    std::vector<MrhsScalars> hs(kmax);
    auto read = [&]() -> int {
        HIP_TRY(ctx, hipMemcpyAsync(hs.data(), W.scal.p, (size_t)k * sizeof(MrhsScalars), hipMemcpyDeviceToHost, st));
        HIP_TRY(ctx, hipStreamSynchronize(st));
        ctx->syncs++;
        for (int64_t c = 0; c < k; ++c)
            if (hs[c].breakdown) return fail(ctx, SPCG_E_BREAKDOWN, "PCG breakdown in column %lld", (long long)c);
        return SPCG_OK;
    };
    auto all_pass = [&]() {
        for (int64_t c = 0; c < k; ++c) {
            const MrhsScalars& s = hs[c];
            if (s.exact) continue;
            if (!(std::sqrt(std::max(s.rho, 0.0)) <= tol * std::sqrt(std::max(s.ax2, 0.0)))) return false;
        }
        return true;
    };
    auto finish = [&](int code) -> int {
        int r2;
        if ((r2 = cols_to_beta(ctx, q.X, ldv, d, k, beta)) != SPCG_OK) return r2;
        *sc0 = hs[0];
        return code;
    };
    out->iters_done = 0;
    out->converged = false;
    if ((rc = batched_products(ctx, W, st, A->dtype, PM_G, plan)) != SPCG_OK) return rc;
    if ((rc = batched_dspace(ctx, W, st, PA_START, plan)) != SPCG_OK) return rc;
    if ((rc = read()) != SPCG_OK) return finish(rc);
    *resid0 = hs[0].resid2;
    const bool testing = tol > 0.0;
    if (check_every < 1) check_every = 1;
    if (testing && all_pass()) {
        out->converged = true;
        return finish(SPCG_OK);
    }
    const int pmode = refresh ? PM_SG : PM_S;
    for (int it = 0; it < iters; ++it) {
        if ((rc = batched_products(ctx, W, st, A->dtype, pmode, plan)) != SPCG_OK) return rc;
        if ((rc = batched_dspace(ctx, W, st, refresh ? PA_REFRESH : PA_STEP, plan)) != SPCG_OK) return rc;
        out->iters_done = it + 1;
        if (testing && ((it + 1) % check_every == 0 || it + 1 == iters)) {
            if ((rc = read()) != SPCG_OK) return finish(rc);
            if (all_pass()) {
                out->converged = true;
                return finish(SPCG_OK);
            }
        }
    }
    if (!testing) {
        if ((rc = read()) != SPCG_OK) return finish(rc);
        bool ex = true;
        for (int64_t c = 0; c < k; ++c) ex = ex && hs[c].exact;
        out->converged = ex;
    }
    return finish(SPCG_OK);
}
}  // namespace

// ================================================================== C ABI

extern "C" {

const char* spcg_version(void) { return "spcg-mi355x 0.1 (gfx950)"; }

int spcg_ctx_create(int device, void* hip_stream, spcg_ctx** out) {
    if (!out) return SPCG_E_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SPCG_E_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return SPCG_E_HIP;
    spcg_ctx* c = new (std::nothrow) spcg_ctx();
    if (!c) return SPCG_E_NOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cu = prop.multiProcessorCount;
    if (na_scratch_address(device, &c->na_scratch) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return SPCG_E_HIP;
    }

    *out = c;
    return SPCG_OK;
}

int spcg_ctx_destroy(spcg_ctx* ctx) {
    if (!ctx) return SPCG_E_INVALID_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->events_ready) {
        for (auto& e : ctx->ev_phase) (void)hipEventDestroy(e);
        for (auto& e : ctx->ev_prod) (void)hipEventDestroy(e);
    }
    delete ctx->batch;
    delete ctx->kt;
    if (ctx->side) {
        (void)hipStreamSynchronize(ctx->side);
        (void)hipStreamDestroy(ctx->side);
    }
    if (ctx->host_status) (void)hipHostFree(ctx->host_status);
    if (ctx->ev_status) (void)hipEventDestroy(ctx->ev_status);
    if (ctx->ev_side_fork) (void)hipEventDestroy(ctx->ev_side_fork);
    if (ctx->ev_side_join) (void)hipEventDestroy(ctx->ev_side_join);
    if (ctx->ev_y) (void)hipEventDestroy(ctx->ev_y);
    delete ctx;
    return SPCG_OK;
}

const char* spcg_last_error(const spcg_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int spcg_sketch(spcg_ctx* ctx, const spcg_mat* X, const spcg_mat* Y, const spcg_sketch_opts* opts,
                spcg_sketch_t** out) {
    if (!ctx || !out) return SPCG_E_INVALID_ARG;
    *out = nullptr;
    spcg_sketch_t* sk = new (std::nothrow) spcg_sketch_t();
    if (!sk) return fail(ctx, SPCG_E_NOMEM, "host allocation failed");
    const int rc = sketch_build(ctx, X, Y, opts, false, sk);
    if (rc != SPCG_OK) {
        delete sk;
        return rc;
    }
    *out = sk;
    return SPCG_OK;
}

int spcg_sketch_get_info(const spcg_sketch_t* sk, spcg_sketch_info* info) {
    if (!sk || !info) return SPCG_E_INVALID_ARG;
    std::memset(info, 0, sizeof *info);
    info->N = sk->N;
    info->Np = sk->Np;
    info->d = sk->d;
    info->k = sk->k;
    info->r = sk->r;
    info->K = sk->K;
    info->L = sk->L;
    info->sketch_dtype = sk->bdtype;
    info->ld = sk->ld;
    for (int64_t i = 0; i < sk->K; ++i) info->m[i] = sk->m[i];
    info->kind = sk->kind;
    return SPCG_OK;
}

int spcg_sketch_view(const spcg_sketch_t* sk, int stage, spcg_mat* A, spcg_mat* b, double* c2) {
    if (!sk || !A) return SPCG_E_INVALID_ARG;
    if (stage < -1 || stage >= sk->K) return SPCG_E_INVALID_ARG;
    const int64_t rows = stage < 0 ? sk->r : sk->m[stage];
    const bool cs = sk->kind == SPCG_SKETCH_COUNT;
    const int64_t row0 = (cs && stage >= 0) ? sk->off[stage] : 0;
    A->data = stage < 0 ? sk->pBh : static_cast<char*>(sk->pB) + (size_t)row0 * sk->ld * dtype_bytes(sk->bdtype);
    A->dtype = stage < 0 ? sk->dtype : sk->bdtype;
    A->reserved = 1;   // zero-padded rows: columns up to ld may be read
    A->rows = rows;
    A->cols = sk->d;
    A->ld = sk->ld;
    A->col_scale = nullptr;
    if (b) {
        b->data = stage < 0 ? nullptr : sk->pBY + (size_t)row0 * sk->ldy;
        b->dtype = SPCG_F64;
        b->reserved = 0;
        b->rows = stage < 0 ? 0 : rows;
        b->cols = sk->k < 1 ? 1 : sk->k;
        b->ld = sk->ldy;
        b->col_scale = nullptr;
    }
    if (c2) *c2 = stage < 0 ? sk->hat_c2 : (cs ? 1.0 : 1.0 / (double)rows);
    return SPCG_OK;
}

int spcg_sketch_export(spcg_ctx* ctx, const spcg_sketch_t* sk, int32_t* slot_rows, int32_t* hat_rows,
                       int32_t* input_perm, uint8_t* sign_bits) {
    if (!ctx || !sk) return SPCG_E_INVALID_ARG;
    if (sk->kind != SPCG_SKETCH_SRHT) return fail(ctx, SPCG_E_INVALID_ARG, "export covers SRHT sketches only");
    const int64_t mK = sk->K ? sk->m[sk->K - 1] : 0;
    const size_t n_slot = (size_t)mK, n_hat = (size_t)sk->r, n_perm = (size_t)sk->Np,
                 n_sign = (size_t)(sk->Np / 8 > 0 ? sk->Np / 8 : 1);
    DevBuf buf;
    HIP_TRY(ctx, buf.ensure((n_slot + n_hat + n_perm) * 4 + n_sign + 64));
    int32_t* d_slot = buf.as<int32_t>();
    int32_t* d_hat = d_slot + n_slot;
    int32_t* d_perm = d_hat + n_hat;
    uint8_t* d_sign = reinterpret_cast<uint8_t*>(d_perm + n_perm);
    hipStream_t st = ctx->stream;
    HIP_TRY(ctx, launch_sketch_export(st, sk->seed, sk->L, mK, sk->r, slot_rows ? d_slot : nullptr,
                                      hat_rows ? d_hat : nullptr, input_perm ? d_perm : nullptr,
                                      sign_bits ? d_sign : nullptr));
    if (slot_rows && n_slot) HIP_TRY(ctx, hipMemcpyAsync(slot_rows, d_slot, n_slot * 4, hipMemcpyDeviceToHost, st));
    if (hat_rows) HIP_TRY(ctx, hipMemcpyAsync(hat_rows, d_hat, n_hat * 4, hipMemcpyDeviceToHost, st));
    if (input_perm) HIP_TRY(ctx, hipMemcpyAsync(input_perm, d_perm, n_perm * 4, hipMemcpyDeviceToHost, st));
    if (sign_bits) HIP_TRY(ctx, hipMemcpyAsync(sign_bits, d_sign, (size_t)(sk->Np / 8), hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    return SPCG_OK;
}

void spcg_sketch_free(spcg_sketch_t* sk) { delete sk; }

int spcg_sketch_tables_host(uint64_t seed, int32_t L, int64_t m, int64_t r, int32_t* slot_rows,
                            int32_t* hat_rows, int32_t* input_perm, uint8_t* sign_bits) {
    if (L < 1 || L > 30 || m < 0 || r < 0) return SPCG_E_INVALID_ARG;
    const int64_t np = 1ll << L;
    if (m > np || r > np) return SPCG_E_SHAPE;
    if (slot_rows)
        for (int64_t t = 0; t < m; ++t) slot_rows[t] = (int32_t)feistel_fwd((uint64_t)t, L, seed, STREAM_PI);
    if (hat_rows)
        for (int64_t t = 0; t < r; ++t) hat_rows[t] = (int32_t)feistel_fwd((uint64_t)t, L, seed, STREAM_PIHAT);
    if (input_perm)
        for (int64_t k = 0; k < np; ++k) input_perm[k] = (int32_t)feistel_fwd((uint64_t)k, L, seed, STREAM_P);
    if (sign_bits)
        for (int64_t i = 0; i < np / 8; ++i) {
            uint32_t byte = 0;
            for (int b = 0; b < 8; ++b) byte |= sign_bit(seed, (uint64_t)(i * 8 + b)) << b;
            sign_bits[i] = (uint8_t)byte;
        }
    return SPCG_OK;
}

int spcg_precond_build(spcg_ctx* ctx, const spcg_sketch_t* sk, const spcg_precond_opts* opts,
                       spcg_precond_t** out) {
    if (!ctx || !sk || !out) return SPCG_E_INVALID_ARG;
    *out = nullptr;
    spcg_precond_t* pc = new (std::nothrow) spcg_precond_t();
    if (!pc) return fail(ctx, SPCG_E_NOMEM, "host allocation failed");
    const int rc = precond_build(ctx, sk, opts, false, pc);
    if (rc != SPCG_OK) {
        delete pc;
        return rc;
    }
    *out = pc;
    return SPCG_OK;
}

int spcg_precond_from_r(spcg_ctx* ctx, const double* R, int64_t d, spcg_precond_t** out) {
    if (!ctx || !R || !out || d < 1) return SPCG_E_INVALID_ARG;
    *out = nullptr;
    spcg_precond_t* pc = new (std::nothrow) spcg_precond_t();
    if (!pc) return fail(ctx, SPCG_E_NOMEM, "host allocation failed");
    int rc = precond_alloc(ctx, pc, d, false);
    if (rc == SPCG_OK) {
        hipError_t e = hipMemcpyAsync(pc->pR, R, (size_t)d * d * 8, hipMemcpyDeviceToDevice, ctx->stream);
        if (e != hipSuccess) rc = fail(ctx, SPCG_E_HIP, "copy of R failed: %s", hipGetErrorString(e));
    }
    if (rc == SPCG_OK) rc = precond_finish(ctx, pc);
    if (rc != SPCG_OK) {
        delete pc;
        return rc;
    }
    pc->passes = 0;
    *out = pc;
    return SPCG_OK;
}

int spcg_precond_export(spcg_ctx* ctx, const spcg_precond_t* pc, double* R_host, int32_t* passes) {
    if (!ctx || !pc) return SPCG_E_INVALID_ARG;
    if (R_host) {
        HIP_TRY(ctx, hipMemcpyAsync(R_host, pc->pR, (size_t)pc->d * pc->d * 8, hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (passes) *passes = pc->passes;
    return SPCG_OK;
}

void spcg_precond_free(spcg_precond_t* pc) { delete pc; }

int spcg_pcg_stage(spcg_ctx* ctx, const spcg_mat* A, const spcg_mat* b, double c2, const spcg_precond_t* pc,
                   double* beta, const spcg_stage_opts* opts, spcg_stage_stats* stats) {
    if (!ctx) return SPCG_E_INVALID_ARG;
    int rc;
    if ((rc = check_stage_args(ctx, A, b, pc, beta)) != SPCG_OK) return rc;
    if (!opts || opts->iters < 0 || opts->tol < 0.0 || !(c2 > 0.0))
        return fail(ctx, SPCG_E_INVALID_ARG, "bad stage options (iters >= 0, tol >= 0, c2 > 0)");
    const int64_t d = A->cols, k = b->cols;
    const bool refresh = opts->refresh_gradient || opts->tol > 0.0;
    StageRun run;
    PcgScalars sc{};   // column 0 at the end
    double resid0 = 0.0;
    bool conv = true;
    int iters_max = 0;
    if (k == 1) {
        StageWs W;
        if ((rc = ensure_stage_ws(ctx, d, &W, beta, pc->pMinv)) != SPCG_OK) return rc;
        HIP_TRY(ctx, run_scalars_reset(ctx->stream, W.S.sc));
        rc = stage_run(ctx, A, b, c2, pc, beta, opts->iters, opts->tol, refresh, opts->check_every, &run, nullptr,
                       nullptr, &W);
        sc = run.sc;
        resid0 = run.sc.resid2_0;
        conv = run.converged;
        iters_max = run.iters_done;
    } else if (mrhs_stage_ok(A, k)) {
        MrhsScalars m0{};
        rc = mrhs_stage_run(ctx, A, b, c2, pc, beta, opts->iters, opts->tol, refresh, opts->check_every, &run, &m0,
                            &resid0);
        sc.rho0 = m0.rho0;
        sc.rho = m0.rho;
        sc.ax2 = m0.ax2;
        conv = run.converged;
        iters_max = run.iters_done;
    } else {
        // column by column on the single-RHS kernels (FP64 and FP8 rows,
        // d > 512 or k > 16): one PCG per column, each from its warm start
        HIP_TRY(ctx, ctx->colx.ensure((size_t)d * 8));
        double* x = ctx->colx.as<double>();
        StageWs W;
        if ((rc = ensure_stage_ws(ctx, d, &W, x, pc->pMinv)) != SPCG_OK) return rc;
        rc = SPCG_OK;
        for (int64_t c = 0; c < k && rc == SPCG_OK; ++c) {
            spcg_mat bc = *b;
            bc.data = static_cast<const double*>(b->data) + c;
            bc.cols = 1;
            HIP_TRY(ctx, hipMemcpy2DAsync(x, 8, beta + c, (size_t)k * 8, 8, d, hipMemcpyDeviceToDevice, ctx->stream));
            HIP_TRY(ctx, run_scalars_reset(ctx->stream, W.S.sc));
            StageRun rcol;
            rc = stage_run(ctx, A, &bc, c2, pc, x, opts->iters, opts->tol, refresh, opts->check_every, &rcol,
                           nullptr, nullptr, &W);
            // the column's last good iterate is returned on breakdown too
            HIP_TRY(ctx, hipMemcpy2DAsync(beta + c, (size_t)k * 8, x, 8, 8, d, hipMemcpyDeviceToDevice, ctx->stream));
            if (c == 0) {
                sc = rcol.sc;
                resid0 = rcol.sc.resid2_0;
            }
            conv = conv && rcol.converged;
            iters_max = std::max(iters_max, rcol.iters_done);
        }
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (stats) {
        stats->iters = iters_max;
        stats->converged = conv;
        stats->rho0 = sc.rho0;
        stats->rho = sc.rho;
        stats->ax_norm = std::sqrt(std::max(sc.ax2, 0.0));
        stats->resid_norm2 = resid0;
    }
    if (rc != SPCG_OK) return rc;
    if (opts->tol > 0.0 && !conv) {
        fail(ctx, SPCG_W_NOT_CONVERGED, "stopping test not met in %d iterations", opts->iters);
        return SPCG_W_NOT_CONVERGED;
    }
    return SPCG_OK;
}

int spcg_pcg_stage_noalloc(spcg_ctx* ctx, const spcg_mat* A, const spcg_mat* b, double c2,
                           const spcg_precond_t* pc, double* beta, const spcg_stage_opts* opts,
                           spcg_stage_stats* stats) {
    if (!ctx) return SPCG_E_INVALID_ARG;
    int rc;
    if ((rc = check_stage_args(ctx, A, b, pc, beta)) != SPCG_OK) return rc;
    if (!opts || opts->iters < 0 || opts->tol < 0.0 || !(c2 > 0.0))
        return fail(ctx, SPCG_E_INVALID_ARG, "bad stage options (iters >= 0, tol >= 0, c2 > 0)");
    if (b->cols != 1) return fail(ctx, SPCG_E_SHAPE, "spcg_pcg_stage_noalloc takes one right-hand side");
    if (A->cols > NA_DMAX)
        return fail(ctx, SPCG_E_SHAPE, "spcg_pcg_stage_noalloc: d = %lld exceeds its static scratch (d <= %lld)",
                    (long long)A->cols, (long long)NA_DMAX);
    if (!ctx->na_scratch) return fail(ctx, SPCG_E_HIP, "static scratch address unavailable");
    const int64_t d = A->cols;
    // layout of the static scratch (see scratch above); every call reuses
    // it, so the counters and the scalar record are cleared by kernels first
    StageWs W;
    double* base = ctx->na_scratch;
    W.part_s = base;
    W.part_g = base + NA_PART;
    W.part_scal = base + 2 * NA_PART;
    double* dv = W.part_scal + 2 * NA_BLOCKS;
    stage_ws_layout(&W, dv, NA_DMAX, dv + NA_DVEC, beta, pc->pMinv, d);
    W.num_cu = (int)std::min<int64_t>(ctx->num_cu, NA_BLOCKS);
    HIP_TRY(ctx, run_counters_reset(ctx->stream, W.S.counters, 2));
    HIP_TRY(ctx, run_scalars_reset(ctx->stream, W.S.sc));
    StageRun run;
    const bool refresh = opts->refresh_gradient || opts->tol > 0.0;
    rc = stage_run(ctx, A, b, c2, pc, beta, opts->iters, opts->tol, refresh, opts->check_every, &run, nullptr,
                   nullptr, &W);
    if (stats) {
        stats->iters = run.iters_done;
        stats->converged = run.converged;
        stats->rho0 = run.sc.rho0;
        stats->rho = run.sc.rho;
        stats->ax_norm = std::sqrt(std::max(run.sc.ax2, 0.0));
        stats->resid_norm2 = run.sc.resid2_0;
    }
    if (rc != SPCG_OK) return rc;
    if (opts->tol > 0.0 && !run.converged) {
        fail(ctx, SPCG_W_NOT_CONVERGED, "stopping test not met in %d iterations", opts->iters);
        return SPCG_W_NOT_CONVERGED;
    }
    return SPCG_OK;
}

int spcg_solve_batched(spcg_ctx* ctx, int nprob, const spcg_mat* X, const spcg_mat* Y,
                       const spcg_solve_opts* opts, double* const* beta, spcg_solve_stats* stats) {
    if (!ctx) return SPCG_E_INVALID_ARG;
    if (opts && opts->schedule != SPCG_SCHEDULE_PLAIN)
        return fail(ctx, SPCG_E_INVALID_ARG, "the batched form runs the plain schedule only");
    return batched_solve(ctx, nprob, X, Y, opts, beta, stats);
}

void spcg_solve_opts_default(spcg_solve_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->sketch.seed = 1;
    o->sketch.growth = 2;
    o->method = SPCG_METHOD_SPCG;
    o->a = 3;
    o->T = 100;
    o->check_every = 1;
    o->tol = 5e-7;
    o->nested_gradient = 1;
}

int spcg_solve(spcg_ctx* ctx, const spcg_mat* X, const spcg_mat* Y, const spcg_solve_opts* opts,
               double* beta, spcg_solve_stats* stats) {
    if (!ctx || !opts) return SPCG_E_INVALID_ARG;
    int rc;
    if ((rc = check_mat(ctx, X, "X")) != SPCG_OK) return rc;
    if ((rc = check_mat(ctx, Y, "Y")) != SPCG_OK) return rc;
    if (!beta) return fail(ctx, SPCG_E_INVALID_ARG, "beta is NULL");
    if (Y->dtype != SPCG_F64) return fail(ctx, SPCG_E_DTYPE, "Y must be SPCG_F64");
    if (Y->rows != X->rows) return fail(ctx, SPCG_E_SHAPE, "X and Y row counts differ");
    if (Y->cols > 1) {
        if (opts->schedule != SPCG_SCHEDULE_PLAIN)
            return fail(ctx, SPCG_E_INVALID_ARG, "the learned schedule takes one right-hand side");
        double* const b1[1] = {beta};
        return batched_solve(ctx, 1, X, Y, opts, b1, stats);
    }
    if (opts->method != SPCG_METHOD_SPCG && opts->method != SPCG_METHOD_FULL_PCG)
        return fail(ctx, SPCG_E_INVALID_ARG, "unknown method %d", opts->method);
    if (opts->a < 0 || opts->T < 0 || opts->tol < 0.0 || opts->a_list_len < 0 ||
        (opts->a_list_len > 0 && !opts->a_list) || opts->stage_stride < 0 || opts->stage_stride > 2 ||
        (opts->a_rule != SPCG_A_FIXED && opts->a_rule != SPCG_A_THEORY) || opts->omega < 0.0 || opts->omega >= 1.0 ||
        opts->stage_limit < 0)
        return fail(ctx, SPCG_E_INVALID_ARG, "bad solve options");
    const bool learned = opts->schedule == SPCG_SCHEDULE_LEARNED;
    if (opts->schedule != SPCG_SCHEDULE_PLAIN && !learned)
        return fail(ctx, SPCG_E_INVALID_ARG, "unknown schedule %d", opts->schedule);
    if (learned && (!opts->schedule_weights || opts->method != SPCG_METHOD_SPCG))
        return fail(ctx, SPCG_E_INVALID_ARG, "the learned schedule needs weights and method SPCG");
    const bool features = learned || opts->record_features;
    int a = opts->a > 0 ? opts->a : 3;
    const int stride = learned ? 1 : (opts->stage_stride > 0 ? opts->stage_stride : 1);
    const int T = opts->T > 0 ? opts->T : 100;
    const double tol = opts->tol > 0.0 ? opts->tol : 5e-7;
    const bool timing = opts->time_phases != 0;
    if (timing || opts->time_products) {
        if ((rc = ensure_events(ctx)) != SPCG_OK) return rc;
    }
    // time_products = 2: every launch timed by kernel class (switched off
    // again on every return)
    const bool by_class = opts->time_products == 2;
    struct KtOff {
        spcg_ctx* c;
        ~KtOff() { c->kt_on = false; }
    } kt_off{ctx};
    if (by_class && (rc = kt_start(ctx)) != SPCG_OK) return rc;
    ctx->syncs = 0;
    hipStream_t st = ctx->stream;
    if (timing) HIP_TRY(ctx, hipEventRecord(ctx->ev_phase[0], st));
    spcg_sketch_opts so = opts->sketch;
    so.hat_only = opts->method == SPCG_METHOD_FULL_PCG ? 1 : 0;
    spcg_sketch_t sk;
    // the response transform runs beside the preconditioner (which needs
    // only S_hat X); the stages wait for it below
    if ((rc = sketch_build(ctx, X, Y, &so, true, &sk, true)) != SPCG_OK) return rc;
    if (timing) HIP_TRY(ctx, hipEventRecord(ctx->ev_phase[1], st));
    spcg_precond_t pc;
    if ((rc = precond_build(ctx, &sk, &opts->precond, true, &pc)) != SPCG_OK) return rc;
    if ((rc = y_join(ctx, false)) != SPCG_OK) return rc;
    const int64_t d = X->cols;
    // planned stages: the prefixes K-1, K-1-stride, ... in increasing order
    // (every prefix for the learned schedule); stage_limit keeps the first
    std::vector<int64_t> stages;
    for (int64_t i = sk.K - 1; i >= 0; i -= stride) stages.push_back(i);
    std::reverse(stages.begin(), stages.end());
    const int Kplan = (int)stages.size();
    if (learned && Kplan > SCHED_KMAX)
        return fail(ctx, SPCG_E_INVALID_ARG, "the learned schedule takes at most %d stages", SCHED_KMAX);
    const int Krun = (!learned && opts->stage_limit > 0) ? std::min(Kplan, (int)opts->stage_limit) : Kplan;
    // schedule scratch (floats): base features, Stage II features, Stage II
    // outputs, then per planned stage its features and network outputs, then
    // the decision words
    constexpr int SF_BASE = 0, SF_II = 8, SF_OUT_II = 24, SF_STAGE = 32, SF_SOUT = SF_STAGE + 8 * SCHED_KMAX,
                  SF_CTL = SF_SOUT + 8 * SCHED_KMAX;
    float* sched = nullptr;
    int32_t* ctl = nullptr;
    float host_fpre[8] = {};
    if (features) {
        HIP_TRY(ctx, ctx->sched.ensure((size_t)(SF_CTL + sched_ctl_words(SCHED_KMAX)) * sizeof(float)));
        sched = ctx->sched.as<float>();
        ctl = reinterpret_cast<int32_t*>(sched + SF_CTL);
        HIP_TRY(ctx, run_features_pre(st, X->data, X->dtype, X->rows, d, X->ld, X->col_scale, pc.pR, d,
                                      sched + SF_BASE));
    }
    // stage features known on the host: size, Theorem 3.3 bound (omega =
    // 1/2) over the planned sizes, position
    auto stage_fixed = [&](int si, float* f2, float* f5, float* f7) {
        const double m = (double)sk.m[stages[si]], dd = (double)d;
        auto bound = [&](double mp, double mc) {
            const double r = std::sqrt((mc - dd) / (mp - dd));
            return std::log((1.5 * r + 1.0) / 0.5) / std::log(4.0);
        };
        double B;
        if (Kplan == 1) B = std::log(5.0) / std::log(4.0);
        else if (si == 0) B = bound((double)sk.m[stages[0]], (double)sk.m[stages[1]]);
        else B = bound((double)sk.m[stages[si - 1]], m);
        *f2 = (float)(std::log2(m / dd) / 8.0 - 1.0);
        *f5 = (float)(B / 4.0);
        *f7 = (float)((double)si / (double)Kplan);
    };
    if (timing) HIP_TRY(ctx, hipEventRecord(ctx->ev_phase[2], st));
    StageWs SW;
    if ((rc = ensure_stage_ws(ctx, d, &SW, beta, pc.pMinv)) != SPCG_OK) return rc;
    HIP_TRY(ctx, run_scalars_reset(st, SW.S.sc));
    HIP_TRY(ctx, run_fill(st, beta, d, 0.0));
    std::vector<int> a_th;
    if (!learned && opts->a_rule == SPCG_A_THEORY) {
        std::vector<int64_t> ms;
        for (int64_t i : stages) ms.push_back(sk.m[i]);
        a_th = theory_a(ms.data(), (int)ms.size(), d, opts->omega > 0.0 ? opts->omega : 0.5);
    }
    if (learned) HIP_TRY(ctx, run_sched_init(st, ctl, Kplan));
    std::vector<int> iters_run(Kplan, -1);
    int t1 = 0, a_used = a;
    for (int si = 0; si < Krun; ++si) {
        spcg_mat A{}, b{};
        double c2 = 1.0;
        spcg_sketch_view(&sk, (int)stages[si], &A, &b, &c2);
        // nested prefixes: reuse the previous stage's gradient (SRHT only)
        const int64_t m_prev = (opts->nested_gradient && si > 0 && sk.kind == SPCG_SKETCH_SRHT)
                                   ? sk.m[stages[si - 1]] : 0;
        float f2 = 0.f, f5 = 0.f, f7 = 0.f;
        if (features) stage_fixed(si, &f2, &f5, &f7);
        float* frow = features ? sched + SF_STAGE + 8 * si : nullptr;
        if (learned) {
            // every launch of the stage is queued; the decision words switch
            // off what the network does not choose
            if ((rc = stage_start_nosync(ctx, &A, &b, c2, gated(SW, ctl + si, 1), m_prev)) != SPCG_OK) return rc;
            float* orow = sched + SF_SOUT + 8 * si;
            HIP_TRY(ctx, run_features_stage(st, sched + SF_BASE, SW.S.sc, f2, f5, f7, ctl + si, frow));
            HIP_TRY(ctx, run_mlp_forward(st, opts->schedule_weights, frow, 1, orow));
            HIP_TRY(ctx, run_sched_decide(st, orow, ctl, si, Kplan, T - 1));
            for (int it = 0; it < MLP_NA - 1; ++it)
                if ((rc = stage_iter_nosync(ctx, &A, &b, c2, gated(SW, ctl + Kplan + 1 + si, it + 1))) != SPCG_OK)
                    return rc;
            continue;
        }
        int ai = a;
        if (opts->a_list_len > 0) ai = opts->a_list[std::min<int64_t>(si, opts->a_list_len - 1)];
        if (!a_th.empty()) ai = a_th[si];
        if (ai < 0) return fail(ctx, SPCG_E_INVALID_ARG, "negative a_i");
        if (t1 + ai > T) ai = std::max(0, T - t1);
        a_used = ai;
        if ((rc = stage_start_nosync(ctx, &A, &b, c2, SW, m_prev)) != SPCG_OK) return rc;
        if (features) HIP_TRY(ctx, run_features_stage(st, sched + SF_BASE, SW.S.sc, f2, f5, f7, nullptr, frow));
        for (int it = 0; it < ai; ++it)
            if ((rc = stage_iter_nosync(ctx, &A, &b, c2, SW)) != SPCG_OK) return rc;
        iters_run[si] = ai;
        t1 += ai;
    }
    if (timing) HIP_TRY(ctx, hipEventRecord(ctx->ev_phase[3], st));
    // Stage II: full data, refreshed gradient, stopping test
    ProductTimer timer;
    timer.ctx = ctx;
    StageRun run;
    StageHooks hooks;
    std::vector<int32_t> host_ctl(learned ? sched_ctl_words(Kplan) : 0);
    std::vector<float> host_sf(features ? 8 * SCHED_FREC : 0), host_so(learned ? 8 * SCHED_FREC : 0);
    const int nrec = std::min(Krun, SCHED_FREC);
    if (features) {
        // the base features come back with the first stopping test (a copy
        // to pageable host memory here would stall the host before Stage I)
        hooks.fpre = sched + SF_BASE;
        hooks.fii = sched + SF_II;
        hooks.add_copy(host_fpre, sched + SF_BASE, 8 * sizeof(float));
        if (nrec > 0) hooks.add_copy(host_sf.data(), sched + SF_STAGE, (size_t)nrec * 8 * sizeof(float));
    }
    if (learned) {
        hooks.W = opts->schedule_weights;
        hooks.out = sched + SF_OUT_II;
        hooks.margin = opts->schedule_margin == 0 ? 1 : std::max(0, opts->schedule_margin);
        hooks.add_copy(host_so.data(), sched + SF_SOUT, (size_t)nrec * 8 * sizeof(float));
        // the Stage I decisions come back with the first stopping test, which
        // then caps Stage II at T minus the Stage I iterations
        hooks.add_copy(host_ctl.data(), ctl, host_ctl.size() * sizeof(int32_t));
        hooks.t1_host = &host_ctl[2 * Kplan + 1];
        hooks.t_total = T;
    }
    rc = stage_run(ctx, X, Y, 1.0, &pc, beta, learned ? T : std::max(0, T - t1), tol, true, opts->check_every,
                   &run, opts->time_products == 1 ? &timer : nullptr, &hooks);
    if (timing) HIP_TRY(ctx, hipEventRecord(ctx->ev_phase[4], st));
    if (rc != SPCG_OK && rc != SPCG_E_BREAKDOWN) return rc;
    const int rc_stage = rc;
    if (learned) {
        // the copies ran before the first stopping test (stage_run always
        // tests at the Stage II start)
        t1 = host_ctl[2 * Kplan + 1];
        for (int si = 0; si < Kplan; ++si) {
            iters_run[si] = host_ctl[Kplan + 1 + si];
            if (iters_run[si] >= 0) a_used = iters_run[si];
        }
    }
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        int started = 0;
        for (int v : iters_run) started += v >= 0 ? 1 : 0;
        stats->K = started;
        stats->T_stage1 = t1;
        stats->T_stage2 = run.iters_done;
        stats->converged = run.converged;
        stats->qr_passes = pc.passes;
        stats->rho_final = run.sc.rho;
        stats->ax_norm = std::sqrt(std::max(run.sc.ax2, 0.0));
        const int64_t es = dtype_bytes(X->dtype);
        stats->product_bytes = (double)X->rows * X->cols * es + (double)X->rows * 8.0;
        stats->policy_a = a_used;
        stats->policy_stride = stride;
        stats->unchecked_iters = hooks.unchecked;
        stats->fallback = hooks.fallback ? 1 : 0;
        stats->s_pred = (float)hooks.s_pred;
        stats->rho_ii0 = hooks.start.rho;
        stats->ax2_ii0 = hooks.start.ax2;
        stats->resid2_ii0 = hooks.start.resid2;
        stats->stages_planned = std::min(Kplan, SCHED_KMAX);
        for (int si = 0; si < SCHED_KMAX; ++si) stats->stage_iters[si] = si < Kplan ? iters_run[si] : -1;
        for (int i = 0; i < (int)host_sf.size() && i < 8 * nrec; ++i) stats->stage_features[i] = host_sf[i];
        for (int i = 0; i < (int)host_so.size() && i < 8 * nrec; ++i) stats->stage_out[i] = host_so[i];
        if (timing || opts->time_products) {
            HIP_TRY(ctx, hipStreamSynchronize(st));
        }
        stats->host_syncs = ctx->syncs;
        for (int i = 0; i < 8; ++i) {
            stats->features_pre[i] = host_fpre[i];
            stats->features_ii[i] = hooks.host_fii[i];
            stats->out_ii[i] = hooks.host_out[i];
        }
        if (timing) {
            stats->t_sketch_ms = elapsed_ms(ctx->ev_phase[0], ctx->ev_phase[1]);
            stats->t_precond_ms = elapsed_ms(ctx->ev_phase[1], ctx->ev_phase[2]);
            stats->t_stage1_ms = elapsed_ms(ctx->ev_phase[2], ctx->ev_phase[3]);
            stats->t_stage2_ms = elapsed_ms(ctx->ev_phase[3], ctx->ev_phase[4]);
            stats->t_total_ms = elapsed_ms(ctx->ev_phase[0], ctx->ev_phase[4]);
        }
        if (opts->time_products == 1) {
            double sum = 0.0;
            for (int i = 0; i < timer.used; ++i) sum += elapsed_ms(ctx->ev_prod[2 * i], ctx->ev_prod[2 * i + 1]);
            stats->product_ms_sum = sum;
            stats->product_launches = timer.used;
        }
        if (by_class) {
            const KTimer& t = *ctx->kt;
            for (int i = 0; i < t.used; ++i) {
                const int c = t.cls[i];
                stats->kernel_ms[c] += elapsed_ms(t.ev[2 * i], t.ev[2 * i + 1]);
                stats->kernel_bytes[c] += t.bytes[i];
                stats->kernel_launches[c] += 1;
            }
            // the full-data dual passes, as time_products = 1 reports them
            stats->product_ms_sum = stats->kernel_ms[SPCG_KT_PROD_SG];
            stats->product_launches = stats->kernel_launches[SPCG_KT_PROD_SG];
        }
    }
    if (rc_stage == SPCG_E_BREAKDOWN) return rc_stage;
    if (!run.converged) {
        fail(ctx, SPCG_W_NOT_CONVERGED, "Stage II did not meet tol=%g within T=%d", tol, T);
        return SPCG_W_NOT_CONVERGED;
    }
    return SPCG_OK;
}

// ---------------------------------------------------- schedule network

int spcg_mlp_forward(spcg_ctx* ctx, const float* W, const float* feats, int64_t n, float* out) {
    if (!ctx) return SPCG_E_INVALID_ARG;
    if (n < 0 || (n > 0 && (!W || !feats || !out))) return fail(ctx, SPCG_E_INVALID_ARG, "bad network arguments");
    HIP_TRY(ctx, run_mlp_forward(ctx->stream, W, feats, n, out));
    return SPCG_OK;
}

int spcg_mlp_loss_grad(spcg_ctx* ctx, const float* W, const float* feats, const int32_t* a_label,
                       const int32_t* g_label, const float* s_label, const float* w_a, const float* w_s, int64_t n,
                       float* grad, float* loss) {
    if (!ctx) return SPCG_E_INVALID_ARG;
    if (n < 0 || !W || !grad || (n > 0 && (!feats || !a_label || !g_label || !s_label || !w_a || !w_s)))
        return fail(ctx, SPCG_E_INVALID_ARG, "bad network arguments");
    const int nb = mlp_grad_blocks(n);
    HIP_TRY(ctx, ctx->mlp_part.ensure((size_t)nb * (MLP_PARAMS + 1) * sizeof(float)));
    HIP_TRY(ctx, run_mlp_loss_grad(ctx->stream, W, feats, n, a_label, g_label, s_label, w_a, w_s,
                                   ctx->mlp_part.as<float>(), grad, loss));
    return SPCG_OK;
}

int spcg_mlp_adam(spcg_ctx* ctx, float* W, const float* grad, float* m, float* v, int64_t n, int32_t step,
                  float lr, float beta1, float beta2, float eps) {
    if (!ctx) return SPCG_E_INVALID_ARG;
    if (n < 0 || step < 1 || (n > 0 && (!W || !grad || !m || !v)) || !(beta1 >= 0.f && beta1 < 1.f) ||
        !(beta2 >= 0.f && beta2 < 1.f))
        return fail(ctx, SPCG_E_INVALID_ARG, "bad Adam arguments");
    const double c1 = 1.0 - std::pow((double)beta1, (double)step);
    const double c2 = 1.0 - std::pow((double)beta2, (double)step);
    HIP_TRY(ctx, run_adam(ctx->stream, W, grad, m, v, n, lr, beta1, beta2, eps, (float)c1, (float)c2));
    return SPCG_OK;
}

}  // extern "C"
