/*
 * spcg.h - C ABI of the MI355X (gfx950) SPCG library.
 *
 * SPCG solves the ordinary least-squares problem of the linear model
 * Y = X beta + zeta (Sec. 1, eqs. (model) and (ols) of Chen, Xie, Yang,
 * Zheng, "Sequential Preconditioned Conjugate Gradient Method for Linear
 * Statistical Models"):
 *
 *     beta_hat = argmin_u 1/2 ||Y - X u||^2,   X: N x d, full column rank.
 *
 * Algorithm 1: Stage I runs a_i PCG iterations on each sketched problem
 * (S_i X, S_i Y), i = 1..K, with nested SRHT sketches of doubling size,
 * warm-starting every stage from the previous one; Stage II runs PCG on
 * the full problem.  All PCG solves share one preconditioner
 * H_hat = (S_hat X)^T (S_hat X) = R^T R built from an independent sketch.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Matrices are row-major: element (i, j) of an spcg_mat lives at
 *   data + (i * ld + j) * sizeof(element).  ld >= cols.  The allocation
 *   behind a matrix spans rows * ld elements: kernels may read (never
 *   write) the row padding between cols and ld, whose contents are ignored.
 * - All data pointers (matrix data, beta, col_scale, R) are DEVICE
 *   pointers on the context's device unless a parameter says "host".
 * - The caller owns X, Y and beta; the library never writes X or Y.
 *   Handles (spcg_ctx, spcg_sketch_t, spcg_precond_t) and the workspaces they
 *   hold are owned by the library and released by the matching *_free /
 *   spcg_ctx_destroy call.
 * - Work is queued on the context's HIP stream; a call returns after its
 *   work is queued, except where it must read a device scalar (stopping
 *   tests, error checks), which synchronises that stream.
 * - Return value: SPCG_OK (0) on success, a positive warning
 *   (SPCG_W_NOT_CONVERGED: beta is still written) or a negative error
 *   code.  spcg_last_error() gives a message for the last failing call on
 *   that context.  No C++ exception crosses this interface.
 * - One context per host thread; calls on one context are not reentrant.
 */
#ifndef SPCG_H
#define SPCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define SPCG_OK 0
#define SPCG_W_NOT_CONVERGED 1   /* budget T exhausted before the stopping test passed */
#define SPCG_E_INVALID_ARG (-1)  /* null handle/pointer or out-of-range option */
#define SPCG_E_SHAPE (-2)        /* N <= d, m_1 <= d, r < d, k < 1, mismatched sizes */
#define SPCG_E_DTYPE (-3)        /* unsupported or mismatched element type */
#define SPCG_E_RANK (-4)         /* S_hat X numerically rank deficient (QR pivot test) */
#define SPCG_E_BREAKDOWN (-5)    /* PCG breakdown: p^T s <= 0 or a non-finite scalar */
#define SPCG_E_HIP (-6)          /* a HIP runtime call failed */
#define SPCG_E_NOMEM (-7)        /* device allocation failed */

/* ---- element types ----------------------------------------------------- */
#define SPCG_F64 0      /* IEEE binary64 */
#define SPCG_F32 1      /* IEEE binary32 */
#define SPCG_BF16 2     /* bfloat16 (upper half of binary32) */
#define SPCG_FP8E4M3 3  /* OCP float8 e4m3fn (bias 7, max 448, no inf), value = decode * col_scale[j] */

typedef struct spcg_ctx spcg_ctx;
typedef struct spcg_sketch_s spcg_sketch_t;
typedef struct spcg_precond_s spcg_precond_t;

/* A dense row-major matrix view.  col_scale is used only for SPCG_FP8E4M3
 * (device array of cols floats, must be non-null then) and ignored
 * otherwise.  Any ld >= cols is accepted.  The direct-load kernels take
 * rows whose start address and byte stride are multiples of 4 (multiples
 * of 16 read fastest; dense rows, ld == cols, that are only 4-byte aligned
 * also take 16-byte loads, which may read up to 12 bytes into the next
 * row); other layouts run on slower element-wise kernels. */
typedef struct spcg_mat {
    const void* data;
    int32_t dtype;
    int32_t reserved;   /* callers set 0; spcg_sketch_view sets 1: the row padding
                           up to ld holds zeros and may be read */
    int64_t rows;
    int64_t cols;
    int64_t ld;
    const float* col_scale;
} spcg_mat;

/* ---- context ----------------------------------------------------------- */

/* Creates a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL selects the null stream).  The stream is borrowed,
 * not owned. */
int spcg_ctx_create(int device, void* hip_stream, spcg_ctx** out);
/* Releases the context and every workspace it holds.  Outstanding
 * sketches and preconditioners created on it must be freed first. */
int spcg_ctx_destroy(spcg_ctx* ctx);
/* Message of the last failing call on ctx ("" if none).  The pointer is
 * valid until the next call on ctx. */
const char* spcg_last_error(const spcg_ctx* ctx);
/* Library version string (static storage). */
const char* spcg_version(void);

/* ---- sketch (Sec. 2.1 SRHT, Sec. 2.2 nested construction) --------------- */

typedef struct spcg_sketch_opts {
    uint64_t seed;    /* key of the Philox4x64-10 streams drawing D, P, pi, pi_hat */
    int64_t m0;       /* m_1, the first sketch size (0: 4 d) */
    int64_t m_max;    /* largest allowed m_K (0: largest m0 * growth^j < N) */
    int64_t r;        /* rows of S_hat, the preconditioner sketch (0: 6 d) */
    int32_t growth;   /* m_{i+1} / m_i (0: 2) */
    int32_t hat_only; /* 1: build only S_hat X (what full-data PCG needs); K = 0 */
    int32_t stage_dtype; /* element type of the stored stage rows B: 0 selects
                            SPCG_F64 for F64 input, SPCG_BF16 for BF16/FP8 input
                            and SPCG_F32 for F32 input; SPCG_F32 or SPCG_BF16
                            may be forced for non-F64 input.  The transform and
                            the preconditioner rows S_hat X stay FP32 (FP64 for
                            F64 input); BF16 rows are rounded to nearest even. */
    int32_t transform_segment; /* tuning: 0 = library default (10- and 9-bit passes
                                  stream 128- or 256-byte row segments through LDS
                                  in persistent blocks; the 11-bit passes of
                                  N' = 2^21 and 2^22 transforms work on tiles of
                                  2048 rows x 128 bytes, staging quarter tiles in
                                  a ring of two buffers); -32 selects the same,
                                  -64 stages half tiles instead; 64, 128 or 256
                                  selects one tile per block with at most that
                                  many bytes per row segment.  Any other value is
                                  SPCG_E_INVALID_ARG.  Results are bit-identical
                                  either way. */
    int32_t kind;     /* SPCG_SKETCH_SRHT (0) or SPCG_SKETCH_COUNT (SPCG-CS, Sec. 4.3) */
    int32_t reserved; /* set to 0 */
    const int64_t* m_list; /* optional HOST array of the stage sizes m_1 < ... < m_K (replaces
                              m0 / growth / m_max), e.g. the tuned schedule of Sec. 4.3:
                              2^10 ... 2^16, then 2^20.  d < m_1, m_K < N, K <= 64; for a
                              CountSketch each size must divide the next. */
    int32_t m_list_len;
    int32_t reserved2; /* set to 0 */
} spcg_sketch_opts;

/* Sketch operators.  SRHT: Sec. 2.1 / 2.2, the method's default.  COUNT:
 * the CountSketch of the SPCG-CS variant (Sec. 4.3).  With N' = 2^L as for
 * the SRHT, row k goes to bucket q(k) mod m with sign s(k), where q is a
 * keyed Feistel bijection of [0, N') (Philox stream 5) and s is D's sign
 * (stream 1); bucket b of S M is the sum of s(k) M[k] over its rows, so
 * every bucket holds floor(N'/m) or ceil(N'/m) padded rows and no scaling is
 * applied (E[S^T S] = I).  Stage i has m_i buckets (m_i divides m_{i+1}:
 * S_i M is S_{i+1} M with buckets b + t m_i added).  S_hat draws its own
 * bijection (stream 6) and signs (stream 7) and has r buckets. */
#define SPCG_SKETCH_SRHT 0
#define SPCG_SKETCH_COUNT 1

/* Shape of a built sketch. */
typedef struct spcg_sketch_info {
    int64_t N, Np, d, k, r, K;
    int32_t L;              /* Np = 2^L, the padded row count */
    int32_t sketch_dtype;   /* element type of the stage rows B (see stage_dtype) */
    int64_t ld;             /* leading dimension of the stored sketch rows */
    int64_t m[64];          /* m_1 .. m_K */
    int32_t kind;           /* SPCG_SKETCH_SRHT or SPCG_SKETCH_COUNT */
    int32_t reserved;
} spcg_sketch_info;

/* Nested SRHT of (X, Y).  With N' = 2^ceil(log2 N) and X, Y zero-padded to
 * N' rows, computes Z = H_un D P [X | Y] once (H_un the unnormalised
 * Walsh-Hadamard matrix, D random signs, P a random permutation) and keeps
 * the rows pi(0..m_K) (nested prefixes: S_i X = rows 0..m_i, scaled by
 * 1/sqrt(m_i)) and pi_hat(0..r) (S_hat X, scaled by 1/sqrt(r)).
 * With opts.kind = SPCG_SKETCH_COUNT the nested CountSketch above is built
 * instead: one stored block of m_i rows per stage (bucket sums in a fixed
 * order, reading every row of X once per sketch) and r bucket rows of S_hat;
 * k <= 64.
 * X: N x d, any element type.  Y: N x k, SPCG_F64, k >= 1.
 * Errors: SHAPE if N <= d, m_1 <= d, r < d or r > N', k < 1, or Y.rows != N.
 * The handle owns the sketch rows; release with spcg_sketch_free. */
int spcg_sketch(spcg_ctx* ctx, const spcg_mat* X, const spcg_mat* Y,
                const spcg_sketch_opts* opts, spcg_sketch_t** out);
int spcg_sketch_get_info(const spcg_sketch_t* sk, spcg_sketch_info* info);
/* Stage view: A = rows 0..m_i of the stored sketch of X (unscaled),
 * b = the same rows of the sketch of Y, *c2 = 1 / m_i, so that
 * c2 A^T A = (S_i X)^T (S_i X).  stage in [0, K); stage = -1 returns the
 * preconditioner sketch rows (b->data = NULL, *c2 = 1 / r).  For a
 * CountSketch, A is stage i's block of m_i bucket rows and *c2 = 1 (also
 * for stage -1).  Views borrow the sketch's memory. */
int spcg_sketch_view(const spcg_sketch_t* sk, int stage, spcg_mat* A, spcg_mat* b, double* c2);
/* Copies the sketch randomness to HOST arrays for reproducibility checks
 * (any pointer may be NULL): slot_rows[t] = pi(t) for t < m_K,
 * hat_rows[t] = pi_hat(t) for t < r, input_perm[k] = p(k) for k < N'
 * (W[k] = sign(k) * X[p(k)]), sign_bits[k/8] bit (k%8) set when D_kk = -1.
 * SRHT sketches only (INVALID_ARG for a CountSketch).  Synchronises the
 * stream. */
int spcg_sketch_export(spcg_ctx* ctx, const spcg_sketch_t* sk, int32_t* slot_rows,
                       int32_t* hat_rows, int32_t* input_perm, uint8_t* sign_bits);
void spcg_sketch_free(spcg_sketch_t* sk);

/* Same randomness computed by the library's host code (no device needed):
 * fills any non-null HOST array exactly as spcg_sketch_export would for a
 * sketch with these parameters (Np = 2^L, m_K = m, r rows). */
int spcg_sketch_tables_host(uint64_t seed, int32_t L, int64_t m, int64_t r, int32_t* slot_rows,
                            int32_t* hat_rows, int32_t* input_perm, uint8_t* sign_bits);

/* ---- preconditioner (Sec. 2.2 H_hat; Sec. 4: applied through QR) -------- */

typedef struct spcg_precond_opts {
    int32_t qr_passes; /* 0: auto (1 if the Gram's Cholesky succeeds with a
                          diagonal ratio below 1e5, else 3); 1: Cholesky of the
                          Gram; 2: CholeskyQR2; 3: shifted CholeskyQR3 */
    int32_t reserved;
} spcg_precond_opts;

/* FP64 QR of S_hat X = Q R (diag(R) > 0) from the sketch's S_hat rows, and
 * the operator H_hat^{-1} = R^{-1} R^{-T} it applies.
 * Errors: RANK when a Cholesky pivot of the orthogonalised Gram falls
 * below 1e-12 (relative) or is not positive. */
int spcg_precond_build(spcg_ctx* ctx, const spcg_sketch_t* sk, const spcg_precond_opts* opts,
                       spcg_precond_t** out);
/* Preconditioner from a caller-supplied upper-triangular R (DEVICE, d x d
 * row-major FP64, diag(R) != 0); the library copies it. */
int spcg_precond_from_r(spcg_ctx* ctx, const double* R, int64_t d, spcg_precond_t** out);
/* Copies R (d x d row-major, zero below the diagonal) to a HOST array,
 * and the number of QR passes used (may be NULL).  Synchronises. */
int spcg_precond_export(spcg_ctx* ctx, const spcg_precond_t* pc, double* R_host, int32_t* passes);
void spcg_precond_free(spcg_precond_t* pc);

/* ---- one PCG solve (Sec. 2.2: PCG(A, b, H_hat, beta_init, a)) ---------- */

typedef struct spcg_stage_opts {
    int32_t iters;            /* iteration count (the maximum if tol > 0) */
    int32_t refresh_gradient; /* 1: every product pass also recomputes
                                 g = c2 A^T (b - A x) with FP64 accumulation and
                                 the next gradient is that minus alpha s */
    double tol;               /* 0: exactly `iters` iterations; > 0: stop once
                                 sqrt(g^T H^-1 g) <= tol * ||sqrt(c2) A x|| */
    int32_t check_every;      /* iterations between stopping tests (0: 1) */
    int32_t reserved;
} spcg_stage_opts;

typedef struct spcg_stage_stats {
    int32_t iters;       /* iterations taken */
    int32_t converged;   /* stopping test passed (or rho reached exactly 0) */
    double rho0;         /* g^T H^-1 g at the start (RHS 0) */
    double rho;          /* at the end (RHS 0) */
    double ax_norm;      /* ||sqrt(c2) A x|| at the last product pass (RHS 0) */
    double resid_norm2;  /* c2 ||b - A x_start||^2 (RHS 0) */
} spcg_stage_stats;

/* PCG on c2 A^T A x = c2 A^T b, x = beta (DEVICE, d x k row-major FP64: in =
 * warm start, out = iterate), preconditioned by pc.  A: m x d (any element
 * type), b: m x k SPCG_F64, k >= 1: the k columns are k independent PCG
 * solves that share A.  With k > 1, FP32 or BF16 rows, d <= 512 and
 * k <= 16, every product pass reads A once for all columns on the matrix
 * cores (FP32 accumulation, FP64 residuals and d-space work); otherwise the
 * columns run one after another on the single-right-hand-side kernels.  A
 * stopping test (tol > 0) passes when it passes for every column.  stats
 * may be NULL; it reports column 0, with iters the largest count over the
 * columns.  Returns BREAKDOWN (beta holds the last good iterate) or
 * W_NOT_CONVERGED when tol > 0 was not met within iters. */
int spcg_pcg_stage(spcg_ctx* ctx, const spcg_mat* A, const spcg_mat* b, double c2,
                   const spcg_precond_t* pc, double* beta, const spcg_stage_opts* opts,
                   spcg_stage_stats* stats);

/* spcg_pcg_stage for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same PCG, kernels and results as spcg_pcg_stage with one
 * right-hand side, but every workspace (product partials, d-space vectors,
 * scalars and counters) lives in a static device array of about 4.3 MB that
 * each device holds from the first context created on it until the process
 * ends; the call itself allocates nothing.  Limits: k = 1 and d <= 1024
 * (SHAPE otherwise); at most 256 product blocks.  All calls on one device
 * share that array, so calls that overlap in time on one device (from any
 * context or stream) race and must not be issued; each call clears the
 * counters and the scalar record it needs before use.  Stopping tests still
 * read the scalars back with one stream synchronisation each. */
int spcg_pcg_stage_noalloc(spcg_ctx* ctx, const spcg_mat* A, const spcg_mat* b, double c2,
                           const spcg_precond_t* pc, double* beta, const spcg_stage_opts* opts,
                           spcg_stage_stats* stats);

/* ---- whole solve (Algorithm 1) ------------------------------------------ */

#define SPCG_METHOD_SPCG 0      /* Algorithm 1 */
#define SPCG_METHOD_FULL_PCG 1  /* full-data PCG from beta = 0, same preconditioner */

typedef struct spcg_solve_opts {
    spcg_sketch_opts sketch;
    spcg_precond_opts precond;
    int32_t method;       /* SPCG_METHOD_* */
    int32_t a;            /* a_i for every sketched stage (0: 3) */
    int32_t T;            /* total PCG iteration budget, Stage I + II (0: 100) */
    int32_t check_every;  /* Stage II stopping-test interval (0: 1) */
    double tol;           /* Stage II stopping tolerance (0: 5e-7) */
    const int32_t* a_list;/* optional HOST array of per-stage a_i (length a_list_len) */
    int32_t a_list_len;
    int32_t time_phases;  /* 1: record phase times (adds stream syncs) */
    int32_t time_products;/* 1: time every full-data product launch with events;
                             2: time every launch of the kernel classes SPCG_KT_*
                             (SRHT sketch passes over X, every product pass and
                             the d-space phases) into the stats' kernel_* fields
                             (events around each launch: an instrumented run) */
    int32_t stage_stride; /* 1: every prefix m_1..m_K; 2: every other prefix, ending
                             at m_K, so sketch sizes grow by 4 per stage (0: 1) */
    int32_t schedule;     /* SPCG_SCHEDULE_PLAIN or SPCG_SCHEDULE_LEARNED */
    const float* schedule_weights; /* learned: DEVICE array of SPCG_MLP_PARAMS floats */
    int32_t schedule_margin;  /* learned: iterations taken off the predicted Stage II
                                 count before the unchecked run (0: 1, < 0: none) */
    int32_t record_features;  /* 1: also compute the schedule features under the
                                 plain schedule (returned in the stats) */
    int32_t batch_direct;     /* batched form: 1 launches every pass directly; 0 (default)
                                 captures each Stage I stage, and the Stage II product and
                                 d-space launches of each active set, in hipGraphs, which the
                                 context keeps and later calls update in place */
    int32_t batch_tasks_per_cu; /* batched form, full-data passes: tasks per CU of each
                                   row-width class launch; 0 (default) autotunes it once per
                                   context and storage type, timing one product pass with
                                   2, 4 and 8 (results are discarded) */
    int32_t a_rule;           /* SPCG_A_FIXED (a / a_list) or SPCG_A_THEORY (below) */
    int32_t nested_gradient;  /* 1: SRHT stages after the first start from the previous
                                 stage's gradient: g = (m_prev / m_i) g_prev
                                 + (1/m_i) dA^T (db - dA x) over the new prefix rows only
                                 (the sketches are nested prefixes, Sec. 2.2), so each
                                 stage-start pass reads m_i - m_prev rows instead of m_i.
                                 Ignored for a CountSketch (its stages are not prefixes).
                                 Single, multi-RHS and batched solves alike (batched:
                                 per problem that ran the previous stage).
                                 spcg_solve_opts_default sets 1. */
    double omega;             /* SPCG_A_THEORY: the stagewise accuracy factor (0: 0.5) */
    int32_t stage_limit;      /* plain schedule: run only the first stage_limit of the
                                 planned stages (after stage_stride), Stage II next;
                                 0: all.  A zero entry of a_list runs the stage's
                                 start (its gradient) and no PCG iteration. */
    int32_t batch_shape;      /* batched form: tile shape of the product launches.
                                 0 (default) autotunes it once per context and storage
                                 type for every launch bucket (row-width class x
                                 k <= 8 / k > 8), timing three product passes of the
                                 bucket in each shape (results are discarded), once
                                 for the Stage II passes over X (SG) and once for the
                                 Stage I passes over sketch rows (S, at the largest
                                 stage every problem has); 1: three
                                 barriers per 16-row tile, 3 LDS slots; 2: two tiles
                                 software-pipelined (the W reduction of one beside the
                                 first GEMM of the next), 3 slots; 3: as 2 with 4 slots
                                 (rows of at most 1 KB; wider rows use 2).  Results are
                                 bit-identical in every shape. */
    int32_t batch_one_launch; /* batched form: 1 runs every task of a pass in one launch
                                 of the widest row-width class (a comparison point for
                                 the per-bucket launches).  The tasks are then split
                                 over one launch instead of one per bucket, so the
                                 partial sums round differently. */
} spcg_solve_opts;

/* a_i rules.  THEORY takes the stage iteration counts from Theorems 3.3
 * and 3.4 for the stage sizes actually run (after stage_stride): with
 * r_{i-1,i} = sqrt((m_i - d) / (m_{i-1} - d)),
 *   a_i = ceil(ln{[(1 + omega) r_{i-1,i} + 1] / omega} / ln 4)   (i >= 2),
 *   a_1 = ceil(alpha), alpha the same expression with r_{1,2} (the bound
 *         Theorem 3.4 gives for every stage; r = 1 when K = 1). */
#define SPCG_A_FIXED 0
#define SPCG_A_THEORY 1

/* Plain schedule: Algorithm 1 as written (a_i = a, every prefix, stopping
 * test after every check_every Stage II iterations).
 * Learned schedule: the network below decides on the device, per stage,
 * with no stream synchronisation in Stage I.  The planned stages are every
 * prefix m_0 < ... < m_{K-1} of the sketch (stage_stride, a, a_list and
 * a_rule are ignored).  At the start of planned stage i (after its
 * starting-gradient pass) the device computes the stage features, runs the
 * network and takes a_i = arg-max of outputs 0..4 (PCG iterations of the
 * stage, 0..4) and stop = arg-max of outputs 5..6; with stop = 1 the later
 * stages are skipped entirely and Stage II follows.  The launches of every
 * planned stage are queued up front; the kernels of a skipped start or
 * iteration read the decision and return at once.  Stage I iterations are
 * capped so that they total at most T - 1.  At the start of Stage II the
 * network runs on the Stage II features, read with the scalars of the
 * first stopping test; s_hat = 10 * output 7.  Stage II then runs
 * max(0, round(s_hat) - margin) iterations without host synchronisation,
 * applies the stopping test once, and, if it fails, continues with the
 * plain test (the fallback) up to the budget T.  The result always
 * passes the same stopping test as the plain schedule. */
#define SPCG_SCHEDULE_PLAIN 0
#define SPCG_SCHEDULE_LEARNED 1

typedef struct spcg_solve_stats {
    int32_t K;              /* sketched stages run */
    int32_t T_stage1;       /* Sum a_i */
    int32_t T_stage2;       /* full-data iterations */
    int32_t converged;
    int32_t qr_passes;
    int32_t product_launches;   /* full-data product launches timed */
    double rho_final;
    double ax_norm;
    double t_sketch_ms, t_precond_ms, t_stage1_ms, t_stage2_ms, t_total_ms;
    double product_ms_sum;      /* summed duration of the timed product launches */
    double product_bytes;       /* algorithmic bytes of one full-data product launch */
    int32_t host_syncs;         /* stream synchronisations made inside the solve */
    int32_t policy_a;           /* a of the last Stage I stage run */
    int32_t policy_stride;      /* stage stride used (1 for the learned schedule) */
    int32_t unchecked_iters;    /* Stage II iterations run before the first test after the start */
    int32_t fallback;           /* learned: the plain test had to continue after the unchecked run */
    float s_pred;               /* learned: 10 * output 6 of the Stage II evaluation */
    double rho_ii0, ax2_ii0, resid2_ii0; /* Stage II start: g^T H^-1 g, ||X b||^2, ||Y - X b||^2 */
    float features_pre[8];      /* schedule features (learned, or record_features) */
    float features_ii[8];
    float out_pre[8];           /* unused (zero) */
    float out_ii[8];            /* network outputs at the Stage II start (learned) */
    int32_t batch_tasks_per_cu; /* batched form: task granularity used in Stage II */
    int32_t batch_graphs;       /* batched form: executable graphs launched */
    /* time_products = 2 (single-problem solves): per kernel class, the
     * summed duration in ms of the timed launches, their summed algorithmic
     * bytes (the class comments below) and their number */
    double kernel_ms[8];
    double kernel_bytes[8];
    int32_t kernel_launches[8];
    /* Stage I per planned stage i < stages_planned (<= 64): PCG iterations
     * run (-1: stage not started), and for i < 16 the stage features and
     * network outputs (learned; features also with record_features) */
    int32_t stages_planned;
    int32_t stage_iters[64];
    float stage_features[16 * 8];
    float stage_out[16 * 8];
    int32_t batch_shapes[16];   /* batched form: tile shape of each launch bucket
                                   (class * 2 + (k > 8)) in Stage II, 0 if unused */
    float batch_tune_ms[16 * 4];/* batched form, the solve that autotuned the Stage II
                                   shapes: one SG product pass of bucket b alone in
                                   shape s (mean of three) at [b * 4 + s - 1], in ms
                                   (0: not timed) */
} spcg_solve_stats;

/* Kernel classes of spcg_solve_stats.kernel_*.  Algorithmic bytes count
 * the d used columns of each row (not the row padding) and elem = the
 * element size of the matrix streamed. */
#define SPCG_KT_TRANSFORM_FIRST 0 /* first SRHT pass over X: N d elem_X (read X) + N' d z (write Z),
                                     z = 8 for FP64 input, else 4 */
#define SPCG_KT_TRANSFORM_REST 1  /* later passes: N' d z (read Z) + N' d z (write Z), or, for the
                                     last pass, m_K d elem_B (write B) + r d z (write S_hat X) */
#define SPCG_KT_PROD_S 2          /* s = c2 A^T (A p): m d elem */
#define SPCG_KT_PROD_G 3          /* stage-start gradient: m (d elem + 8) */
#define SPCG_KT_PROD_SG 4         /* dual pass (s and the refreshed gradient): m (d elem + 8) */
#define SPCG_KT_PHASE_A 5         /* d-space phase A (latency-bound: no bytes counted) */
#define SPCG_KT_PHASE_B 6         /* d-space phase B (latency-bound: no bytes counted) */
#define SPCG_KT_N 8

/* beta (DEVICE, d x k row-major FP64) <- Algorithm 1 (or full-data PCG)
 * for (X, Y).  X: N x d any element type; Y: N x k SPCG_F64 (k > 1 takes
 * the batched form with one problem, see spcg_solve_batched).  Stage II
 * stops when sqrt(g^T H^-1 g) <= tol ||X beta|| or at T total iterations.
 * Workspaces are cached in ctx and reused by later solves of the same or
 * smaller size. */
int spcg_solve(spcg_ctx* ctx, const spcg_mat* X, const spcg_mat* Y, const spcg_solve_opts* opts,
               double* beta, spcg_solve_stats* stats);

/* Batched / multi-right-hand-side form.  Solves nprob independent problems
 * (X[p], Y[p]) with the same options: every PCG step of all problems is one
 * product launch over a queue of (problem, row range) tasks on the matrix
 * cores plus one d-space launch (one block per problem), and Stage II stops
 * per problem.  Requirements: X[p] SPCG_F32 or SPCG_BF16 (all the same),
 * d <= 512, 1 <= k <= 16 right-hand sides (Y[p] is N x k SPCG_F64), beta[p]
 * DEVICE d x k row-major FP64.  Products accumulate in FP32.  stats may be
 * NULL or an array of nprob entries.  With opts.time_products, stats[0]
 * holds the launches timed (the full-data product passes of Stage II), their
 * summed duration and, in product_bytes, their summed algorithmic bytes
 * (sum over the active problems of m (d elem + 8 k) per launch).  Returns the
 * worst code over the problems (W_NOT_CONVERGED if any problem missed tol
 * within T).  The per-problem sketches, preconditioners and buffers stay in
 * ctx for reuse by later batched calls and are freed by spcg_ctx_destroy. */
int spcg_solve_batched(spcg_ctx* ctx, int nprob, const spcg_mat* X, const spcg_mat* Y,
                       const spcg_solve_opts* opts, double* const* beta, spcg_solve_stats* stats);

/* Default option values (all zero fields mean "default"). */
void spcg_solve_opts_default(spcg_solve_opts* opts);

/* ---- learned schedule network -------------------------------------------
 * The paper fixes a_i = 3 and a doubling schedule (Sec. 4.1) and names the
 * automatic choice of the schedule an open problem (Sec. 4.3).  This
 * library learns it: a dense network F -> H -> H -> O with ReLU after the
 * first two layers, all FP32.  Parameters are one flat array, in order
 * W1 (H x F row-major), b1 (H), W2 (H x H), b2 (H), W3 (O x H), b3 (O).
 * Outputs: 0..4 logits of a_i (a stage's PCG iterations), 5..6 logits of
 * stop (Stage I ends after this stage), 7 the Stage II count divided by
 * SPCG_MLP_S_SCALE.
 *
 * Features (FP32, computed on the device; every value scale-free):
 *   base (before Stage I): f0 = log10 N - 5, f1 = log10 d - 2,
 *   f2 = log2(N / d) / 8 - 1,
 *   f3 = log10(max|R_jj| / min|R_jj|) / 3 - 1 (3 if a diagonal entry is 0),
 *   f4 = log10(max q / mean q) / 2 over q_j = ||x_j||^2 of the rows
 *        floor((2t + 1) N / 512), t < 256 (every row if N < 256; 0 if all q are 0),
 *   f5 = f6 = f7 = 0;
 *   start of planned stage i of K (sizes m_0 < ... < m_{K-1}; res and fit
 *   the residual and fit norms of the rows the starting-gradient pass
 *   read: all m_i rows, or the new rows m_{i-1}..m_i of a nested start):
 *   f2 = log2(m_i / d) / 8 - 1,
 *   f5 = B_i / 4, B_i = ln{[1.5 r + 1] / 0.5} / ln 4 the Theorem 3.3 bound at
 *        omega = 1/2, r = sqrt((m_i - d) / (m_{i-1} - d)) (i = 0: the pair
 *        m_0, m_1; r = 1 if K = 1),
 *   f6 = clamp(log10(res / fit) / 6, -2, 2) (-2 if res <= 0, 2 if fit <= 0),
 *   f7 = i / K, the others as the base;
 *   Stage II start (rho = g^T H^-1 g, fit = ||X beta||^2, res = ||Y - X beta||^2):
 *   f5 = clamp(log10(sqrt(rho) / (tol sqrt(fit))) / 3, -3, 3) (-3 if rho <= 0, 3 if fit <= 0),
 *   f6 = clamp(log10(res / fit) / 6, -2, 2) (-2 if res <= 0, 2 if fit <= 0), f7 = 1,
 *   the others as the base.
 *
 * Training loss of n samples with labels a in 0..4, g in 0..1, s >= 0 and
 * weights w_a, w_s:
 *   (1/n) sum [ w_a (CE(out[0:5], a) + CE(out[5:7], g))
 *               + w_s SPCG_MLP_LAMBDA (out[7] - s / SPCG_MLP_S_SCALE)^2 ]
 * with CE the softmax cross-entropy. */
#define SPCG_MLP_F 8
#define SPCG_MLP_H 64
#define SPCG_MLP_O 8
#define SPCG_MLP_PARAMS (SPCG_MLP_H * SPCG_MLP_F + SPCG_MLP_H + SPCG_MLP_H * SPCG_MLP_H + SPCG_MLP_H + \
                         SPCG_MLP_O * SPCG_MLP_H + SPCG_MLP_O)
#define SPCG_MLP_S_SCALE 10.0
#define SPCG_MLP_LAMBDA 0.5

/* out (DEVICE, n x O FP32) <- network(W, feats (DEVICE, n x F FP32)). */
int spcg_mlp_forward(spcg_ctx* ctx, const float* W, const float* feats, int64_t n, float* out);
/* grad (DEVICE, SPCG_MLP_PARAMS FP32) <- gradient of the mean loss above;
 * *loss (DEVICE, one FP32, may be NULL) <- the loss.  Labels and weights
 * are DEVICE arrays of n entries; a is clamped to 0..4 and g taken mod 2.
 * Sums run in a fixed order (identical bits on repeated calls). */
int spcg_mlp_loss_grad(spcg_ctx* ctx, const float* W, const float* feats, const int32_t* a_label,
                       const int32_t* g_label, const float* s_label, const float* w_a,
                       const float* w_s, int64_t n, float* grad, float* loss);
/* One Adam step (Kingma and Ba) on n DEVICE parameters: m <- b1 m + (1 - b1) g,
 * v <- b2 v + (1 - b2) g^2, W <- W - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps);
 * step = t >= 1. */
int spcg_mlp_adam(spcg_ctx* ctx, float* W, const float* grad, float* m, float* v, int64_t n,
                  int32_t step, float lr, float beta1, float beta2, float eps);

#ifdef __cplusplus
}
#endif

#endif /* SPCG_H */
