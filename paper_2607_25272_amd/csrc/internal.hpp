// Internal launch interface between the host driver (api.hip) and the
// kernel files.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "spcg.h"

namespace spcg {

// ---------------------------------------------------------------- sketch
// Per-row randomness tables for a padded size Np = 2^L (each output may be
// null and is then skipped):
//   perm_sign[k] = p(k) | (sign_bit(k) << 31)
//   inv_slot[k]  = pi^{-1}(k)     if < mK, else -1
//   inv_hat[k]   = pi_hat^{-1}(k) if < r,  else -1
// rt: the round tables of the p, pi and pi_hat streams (written by
// launch_sketch_round_tables before).  1 <= L <= 30.
// pair_t (optional, with inv_slot or inv_hat): both output slots of row k
// at index (k mod 2^plo) 2^(L - plo) + k / 2^plo, so that a last transform
// pass over bits [plo, L) finds the slots of one tile's rows contiguously.
// row_masks (optional, with perm_sign; N = the unpadded row count): for each
// group of 16 rows k = 16 g + t, bit t = sign bit of row k and bit 16 + t =
// (p(k) < N), so that a first transform pass reads one word per 16 rows.
hipError_t launch_sketch_tables(hipStream_t st, uint64_t seed, int L, int64_t mK, int64_t r,
                                int32_t* perm_sign, int32_t* inv_slot, int32_t* inv_hat, const uint32_t* rt,
                                int2* pair_t = nullptr, int plo = 0, uint32_t* row_masks = nullptr,
                                int64_t N = 0);
// Round tables of the p, pi and pi_hat streams: 3 feistel_table_size(L)
// words, one launch.
hipError_t launch_sketch_round_tables(hipStream_t st, uint64_t seed, int L, uint32_t* rt);
// Round tables of n <= 3 Feistel streams, table i at rt + i
// feistel_table_size(L); one launch.
hipError_t launch_feistel_tables(hipStream_t st, uint64_t seed, int L, int n, const uint64_t* streams, uint32_t* rt);
// Forward maps for export (device arrays, any may be null).
hipError_t launch_sketch_export(hipStream_t st, uint64_t seed, int L, int64_t mK, int64_t r,
                                int32_t* slot_rows, int32_t* hat_rows, int32_t* input_perm,
                                uint8_t* sign_bits);

struct FwhtJob {
    const void* x;          // N x d input rows, element type in_dtype, leading dim ldx
    const void* x_last;     // null, or a copy of row N - 1 readable to 16 bytes past
                            // round_up(d * elem, 16) (lets rows that are only 4-byte
                            // aligned take 16-byte direct loads in the first pass)
    int in_dtype;           // DT_*; TZ is double for DT_F64, float otherwise
    int64_t N, d, ldx;
    const float* col_scale; // FP8 only
    int L;
    const int32_t* perm_sign;
    const int32_t* inv_slot;  // may be null (no stage sketch output)
    const int32_t* inv_hat;   // may be null (no S_hat output)
    void* zbuf;               // Np x ldz scratch of TZ (unused when L fits one pass)
    int64_t ldz;
    void* B;                  // mK x ldb of TZ (rows pi(t)), or null
    int64_t ldb;
    void* Bh;                 // r x ldbh of TZ (rows pi_hat(t)), or null
    int64_t ldbh;
    int narrow;               // 1: single-column FP64 transform (the response vector)
    int b_bf16;               // 1: store the B rows as BF16 (round to nearest even)
    int seg_bytes;            // 0: default column segment; 64 / 128 / 256: at most this
                              // (one tile per block); -32 / -64: quarter- / half-tile
                              // staging in the 11-bit passes (0: quarter tiles)
    int stream;               // 1: 10- and 11-bit FP32-precision passes use the streaming
                              // kernel (persistent blocks, next tile prefetched)
    int num_cu;               // compute units (grid of the streaming kernel)
    hipEvent_t wait_before_last;  // if set: the last pass waits for it (the
                                  // output-slot tables are built beside the
                                  // first pass)
    hipEvent_t pass_ev[6];        // optional timing events: pass i (< 3) is
                                  // bracketed by pass_ev[2i] and pass_ev[2i+1]
    const uint32_t* row_masks;    // optional: launch_sketch_tables' row_masks (sign and
                                  // validity of 16 rows per word) for the split first pass
    const int2* slot_pairs;       // optional: (inv_slot, inv_hat) per row in the order of
                                  // launch_sketch_tables' pair_t with plo = the last pass's
                                  // first bit (lets 11-bit last passes stage them in LDS)
};
// Tables that the half-tile-staged 11-bit passes of an N' = 2^L transform
// read (FP32 working precision, two passes, the first of 11 bits): bit 0
// FwhtJob::row_masks (first pass), bit 1 FwhtJob::slot_pairs (an 11-bit
// last pass, plo = 11).  0: run_fwht does not use that kernel.
int fwht_split_tables(int in_dtype, int L, int64_t ldz, int seg_bytes);
// Widest column chunk of the transform (256-byte row segments): every row
// width used by a job (ldz, ldb, ldbh) must be equal and a multiple of it.
inline int fwht_chunk_cols(int in_dtype, int narrow) {
    return narrow ? 1 : (in_dtype == DT_F64 ? 32 : 64);
}
// Row padding of the stored sketch rows (multiple of every chunk width).
inline int64_t sketch_ld(int64_t d, bool f64) { return round_up(d, f64 ? 32 : 64); }
// Row stride of the FP64 sketched responses and of their transform scratch:
// one column, 8 or 16 columns (64- or 128-byte row segments) for up to 8 or
// 16 right-hand sides, else a multiple of the 32-column chunk.
inline int64_t sketch_ldy(int64_t k) { return k == 1 ? 1 : k <= 8 ? 8 : k <= 16 ? 16 : round_up(k, 32); }
hipError_t run_fwht(hipStream_t st, const FwhtJob& job);
// Number of passes run_fwht makes over an N' = 2^L row transform.
int fwht_passes(int L);

// ----------------------------------------------------------- CountSketch
// Bucket tables for a padded size Np = 2^L: entry y holds the row k with
// q(k) = y (q the bucket bijection) and its sign in bit 31.  Bucket b of an
// m-bucket sketch gathers the entries y = b, b + m, b + 2m, ... < Np.
// rt: workspace of 2 feistel_table_size(L) words (round tables of the two
// bucket bijections).
hipError_t launch_cs_tables(hipStream_t st, uint64_t seed, int L, int32_t* tbl, int32_t* tbl_hat, uint32_t* rt);

struct CsJob {
    const void* x;            // N x d input rows, element type in_dtype, leading dim ldx
    int in_dtype;             // DT_*; sums are FP64 for DT_F64 input, FP32 otherwise
    int64_t N, d, ldx;
    const float* col_scale;   // FP8 only
    const double* y;          // N x k FP64 responses (may be null)
    int64_t ldy_in, k;
    const int32_t* tbl;       // bucket table (see launch_cs_tables)
    int64_t Np, nbk;          // padded rows; buckets
    void* out;                // nbk x ld rows (element type out_dtype), zero beyond d
    int out_dtype;            // DT_F64, DT_F32 or DT_BF16
    void* work;               // optional nbk x ld copy in the sum type, or null
    int64_t ld;
    double* outy;             // nbk x ldoy sketched responses, or null
    int64_t ldoy;
    void* scratch;            // optional: lets few, long buckets be split into
    size_t scratch_bytes;     // segments (partial sums, reduced in segment order)
};
hipError_t run_cs_gather(hipStream_t st, const CsJob& job);
// The finest stage and up to 3 coarser ones in one gather: a wave takes a
// bucket c of the coarsest produced level (m[levels] buckets) and its
// growth^levels finest buckets c + t m[levels], and adds them level by
// level in the folding order (bit-identical to gathering the finest stage
// and folding).  base.nbk = m[0]; out[l] / outy[l] take level l (0 finest);
// work (optional) the coarsest produced level in the sum type.
struct CsTreeJob {
    CsJob base;
    int growth, levels;
    void* out[4];
    double* outy[4];
    int64_t m[4];
    void* work;
};
hipError_t run_cs_gather_tree(hipStream_t st, const CsTreeJob& job);
// Folding to a coarser nested sketch: dst[b] = sum_{t < g} src[b + t mc]
// (ascending t) for b < mc.  src and work hold rows in the sum type (FP64 for
// f64, else FP32; work may equal src); dst takes out_dtype.  Also the
// sketched responses (FP64) when ysrc is set.
hipError_t run_cs_fold(hipStream_t st, bool f64, const void* src, void* work, void* dst, int out_dtype, int64_t ld,
                       int64_t mc, int g, const double* ysrc, double* ydst, int64_t ldy, int64_t k);

// --------------------------------------------------------------- product
enum ProdMode : int { PM_S = 0, PM_G = 1, PM_SG = 2 };

struct ProdJob {
    const void* A;
    int dtype;
    int64_t m, d, lda;
    int64_t dmem;            // columns readable in every row (>= d; padding of library buffers)
    const float* col_scale;  // FP8 only
    const double* b;         // m rows (G/SG), stride ldbv
    int64_t ldbv;
    const double* x;         // d (G/SG)
    const double* p;         // d (S/SG)
    int mode;
    double* part_s;          // [nblocks][dpad]
    double* part_g;          // [nblocks][dpad]
    double* part_scal;       // [nblocks][2]: sum (b - a.x)^2, sum (a.x)^2
    int64_t dpad;
    int num_cu;
    const int32_t* gate = nullptr;   // optional: the launch does nothing unless *gate >= gmin
    int32_t gmin = 0;
};
// Chooses the launch shape, returns the number of blocks (partials) used.
hipError_t run_product(hipStream_t st, const ProdJob& job, int* nblocks_out);
int64_t product_max_blocks(int num_cu);
int64_t product_max_d(int dtype);

// ---------------------------------------------------------------- d-space
struct PcgScalars {
    double rho;       // g^T H^-1 g (current)
    double alpha;
    double pts;       // p^T s
    double resid2;    // c2 ||b - A x||^2 from the last G/SG pass
    double ax2;       // c2 ||A x||^2 from the last G/SG pass
    double rho0;
    double resid2_0;  // c2 ||b - A x||^2 at the stage start
    int32_t exact;    // rho reached exactly zero in this stage
    int32_t breakdown;// sticky: p^T s <= 0 or non-finite
    int32_t iters;
    int32_t pad;
};

struct DspaceState {
    double* x;        // d (caller beta for k = 1)
    double* g;        // d
    double* z;        // d
    double* p;        // d
    double* s;        // d
    double* gt;       // d (refreshed gradient)
    double* blk;      // per-block partial scalars (>= 1024)
    unsigned int* counters;  // 2 counters, zero between launches
    PcgScalars* sc;
    const double* Minv;  // d x d
    int64_t d;
    // optional launch gate: the phase kernels return at once unless
    // *gate >= gmin (a decision written earlier on the same stream)
    const int32_t* gate = nullptr;
    int32_t gmin = 0;
};
// phase A: reduce the product partials; start / step / refresh variants
// PA_START_NESTED: g = g_scale * g + c2 * (reduced partials), the starting
// gradient of a larger nested prefix from the previous stage's gradient and
// a G pass over the new rows only.
enum PhaseA : int { PA_START = 0, PA_STEP = 1, PA_REFRESH = 2, PA_START_NESTED = 3 };
hipError_t run_phase_a(hipStream_t st, const DspaceState& S, int variant, const double* part_s,
                       const double* part_g, const double* part_scal, int nparts, int64_t dpad,
                       double c2, double g_scale = 0.0);
// phase B: z = H^-1 g, rho' = g^T z, p update (init or CG step)
hipError_t run_phase_b(hipStream_t st, const DspaceState& S, int init);
hipError_t run_scalars_reset(hipStream_t st, PcgScalars* sc);
hipError_t run_fill(hipStream_t st, double* v, int64_t n, double value);
hipError_t run_counters_reset(hipStream_t st, unsigned int* c, int n);

// ------------------------------------------------- multi-RHS / batched
// One independent least-squares problem of a batch (or one problem with
// k right-hand sides).  d-space vectors are stored column by column:
// v[c * ldv + j], c < 16.
struct MrhsScalars {
    double rho, rho0, alpha, pts, resid2, ax2;
    int32_t exact, breakdown;
};
struct MrhsProblem {
    const void* A;          // m x d row-major (FP32 or BF16), leading dim lda
    int64_t m, lda;
    int64_t dmem;           // columns readable in every row (>= d)
    int d, k;
    const double* b;        // m x k row-major, leading dim ldb
    int64_t ldb;
    double c2;
    int64_t ldv;            // stride between d-space columns
    double* X;              // iterate
    double* G;
    double* Z;
    double* P;
    double* S;
    double* Gt;
    const double* Minv;     // d x d
    MrhsScalars* sc;        // k entries
    double* rho_part;       // per 128-row slice of z, 16 shares of g^T z
    double gscale;          // PA_START_NESTED: weight of the previous gradient (0: plain start)
    int t0, t1;             // tasks of this problem in the current launch
    int active;             // 0: skip (converged or no stage)
    int lshift;             // 16-byte loads of rows only 4-byte aligned: the last row's loads start this many bytes early
};
struct MrhsTask {
    int prob;
    int pad;
    int64_t r0, r1;
};
int mrhs_max_d();
int mrhs_max_k();
constexpr int MR_ZSLICES = 4;   // 128-row slices of z = M g (d <= 512)
// Row-width classes of the product launches: load width (16 or 4 bytes) x
// loads per row (a power of two); MR_CLASS_GENERIC reads element by element
// (any row stride).
enum MrhsClass : int { MR_CLASS_16x1 = 0, MR_CLASS_16x2, MR_CLASS_4x1, MR_CLASS_4x2, MR_CLASS_4x4, MR_CLASS_4x8,
                       MR_CLASS_GENERIC, MR_NCLASS };
int mrhs_class(int dtype, const void* A, int64_t m, int64_t lda, int64_t dmem, int d);
// Bytes by which the 16-byte loads of the matrix's last row start early
// (rows only 4-byte aligned), 0 for aligned rows, -1 when 16-byte loads
// cannot read the rows.
int mrhs_row_shift(int dtype, const void* A, int64_t m, int64_t lda, int64_t dmem, int d);
// Tile shapes of a product launch: MR_SHAPE_PLAIN runs GEMM1, the W
// reduction and GEMM2 of each 16-row tile between three barriers with 3 LDS
// slots; MR_SHAPE_PIPE3 / PIPE4 software-pipeline two tiles (two barriers
// per tile) with 3 / 4 slots.  PIPE4 exists for rows of at most 1 KB
// (classes 16x1, 4x1, 4x2, 4x4); elsewhere it runs as PIPE3.
enum MrhsShape : int { MR_SHAPE_PLAIN = 1, MR_SHAPE_PIPE3 = 2, MR_SHAPE_PIPE4 = 3, MR_NSHAPE = 4 };
bool mrhs_shape_native(int cls, int shape);
// launch buckets: row-width class x (k <= 8, k > 8)
constexpr int MR_KB = 2;
constexpr int MR_NBUCKET = MR_NCLASS * MR_KB;
inline int mrhs_bucket(int cls, int k) { return cls * MR_KB + (k > 8 ? 1 : 0); }
// One launch over tasks[task0 .. task0 + ntasks), all of class cls, in tile
// shape `shape`; task t writes partial block t.
hipError_t run_mrhs_product(hipStream_t st, int dtype, int mode, int cls, int shape, const MrhsTask* tasks,
                            int task0, int ntasks, const MrhsProblem* probs, float* part_s, float* part_g,
                            float* part_scal);
// The d-space step of all k columns of every problem, three launches: the
// partial sums, alpha and the x, g updates (one block per problem); z = M g
// in 128-row slices (one block per slice and problem); rho and p (one block
// per problem).  variant: PA_START (g, z, p, rho from the G partials),
// PA_START_NESTED (the same from g = gscale g + c2 (partials of the new
// prefix rows), per problem; gscale 0: PA_START),
// PA_STEP, PA_REFRESH.
hipError_t run_mrhs_dspace(hipStream_t st, int variant, const MrhsProblem* probs, int nprob,
                           const float* part_s, const float* part_g, const float* part_scal);

// --------------------------------------------------------- dense FP64
struct DenseStatus {
    int32_t fail;        // first failing pivot index + 1, 0 if none
    int32_t pad;
    double min_diag, max_diag;   // of the computed factor
    double min_pivot;            // smallest pivot (before sqrt)
};
// C = alpha op(A) op(B) + beta C; A(i,l) = A[i*sai + l*sal], B(l,j) = B[l*sbl + j*sbj]
// upper = 1: only 64x64 tiles on or above the block diagonal are computed.
// work (work_elems doubles, may be null) enables split-K for short-and-wide
// products; the chunks are summed in a fixed order.
hipError_t gemm_f64(hipStream_t st, int64_t M, int64_t N, int64_t K, double alpha, const void* A,
                    int a_f32, int64_t sai, int64_t sal, const void* B, int b_f32, int64_t sbl,
                    int64_t sbj, double beta, double* C, int64_t ldc, int upper, double* work,
                    int64_t work_elems);
// `batch` FP64 products of one shape in one launch: entry z reads A + z bsa
// and B + z bsb and writes C + z bsc (bsc != 0); the last entry has N = n_last
// and K = k_last where those are > 0.  No split-K unless batch = 1.
hipError_t gemm_f64_batched(hipStream_t st, int64_t batch, int64_t M, int64_t N, int64_t K, double alpha,
                            const double* A, int64_t sai, int64_t sal, int64_t bsa, const double* B,
                            int64_t sbl, int64_t sbj, int64_t bsb, double beta, double* C, int64_t ldc,
                            int64_t bsc, int64_t n_last, int64_t k_last, double* work, int64_t work_elems);
// In-place upper Cholesky G = U^T U (row-major d x d, ld; the upper part
// of G is read); lower part zeroed; the inverses of the 64 x 64 diagonal
// blocks of U go to the same positions of W (d x d, ld).  One fused launch
// per 64-row panel.  The remaining arguments are unused.
hipError_t cholesky_upper(hipStream_t st, double* G, int64_t d, int64_t ld, DenseStatus* status,
                          double* W, double* panel, double* work, int64_t work_elems);
// W = U^{-1} (d x d, ld) for upper-triangular U: diagonal-block inverses
// (taken from diag_inv, same layout, when given; computed otherwise), then
// block recursive doubling W12 = -W11 U12 W22 over 64, 128, ... column
// blocks, all pairs of a level in one batched launch per product.  tmp: d * d
// doubles; work: split-K workspace (as for gemm_f64, may be null).
hipError_t tri_inverse_upper(hipStream_t st, const double* U, int64_t d, int64_t ld, double* W,
                             const double* diag_inv, double* tmp, double* work, int64_t work_elems);
// Inverses of the 64 x 64 diagonal blocks of an upper-triangular U into W.
hipError_t trtri_diag_blocks(hipStream_t st, const double* U, int64_t d, int64_t ld, double* W);
// In-place A <- A U^{-1} for A (n x d, lda), upper-triangular U (d x d,
// ldu) whose diagonal-block inverses are in W (same layout); tmp: n x 64.
hipError_t trsm_right_upper(hipStream_t st, double* A, int64_t n, int64_t d, int64_t lda,
                            const double* U, int64_t ldu, const double* W, double* tmp, double* work,
                            int64_t work_elems);
hipError_t dense_fill_identity(hipStream_t st, double* A, int64_t d);
hipError_t dense_convert(hipStream_t st, const void* src, int src_f32, int64_t rows, int64_t cols,
                         int64_t lds, double scale, double* dst, int64_t ldd);
hipError_t dense_add_trace_shift(hipStream_t st, double* G, int64_t d, double factor);
hipError_t dense_status_reset(hipStream_t st, DenseStatus* status);

// ------------------------------------------------------ learned schedule
constexpr int MLP_F = SPCG_MLP_F, MLP_H = SPCG_MLP_H, MLP_O = SPCG_MLP_O;
constexpr int MLP_PARAMS = SPCG_MLP_PARAMS;
constexpr double MLP_S_SCALE = SPCG_MLP_S_SCALE;
constexpr double MLP_LAMBDA = SPCG_MLP_LAMBDA;
constexpr int MLP_SAMPLE_ROWS = 256;
// Partial-gradient blocks used for n samples (each holds MLP_PARAMS + 1 floats).
int mlp_grad_blocks(int64_t n);
hipError_t run_mlp_forward(hipStream_t st, const float* W, const float* feats, int64_t n, float* out);
hipError_t run_mlp_loss_grad(hipStream_t st, const float* W, const float* feats, int64_t n, const int32_t* la,
                             const int32_t* lg, const float* ls, const float* wa, const float* ws, float* partial,
                             float* grad, float* loss);
// One Adam step; c1 = 1 - b1^t and c2 = 1 - b2^t are the bias corrections.
hipError_t run_adam(hipStream_t st, float* W, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                    float b2, float eps, float c1, float c2);
hipError_t run_features_pre(hipStream_t st, const void* X, int dtype, int64_t N, int64_t d, int64_t ld,
                            const float* col_scale, const double* R, int64_t ldr, float* f);
hipError_t run_features_ii(hipStream_t st, const float* fpre, const PcgScalars* sc, double tol, float* f);

// Per-stage decisions of the learned schedule.  Control words of K planned
// stages (2 K + 2 int32): ctl[i] (i <= K) = 1 if stage i starts,
// ctl[K + 1 + i] = PCG iterations of stage i (-1 before its decision or if
// it never starts), ctl[2 K + 1] = Stage I iterations so far.
constexpr int MLP_NA = 5;          // a_i choices 0..4 (outputs 0..4), stop (5..6), s_II (7)
constexpr int SCHED_KMAX = 64;     // planned stages with recorded decisions
constexpr int SCHED_FREC = 16;     // stages whose features / outputs are recorded
__host__ __device__ inline int sched_ctl_words(int K) { return 2 * K + 2; }
hipError_t run_sched_init(hipStream_t st, int32_t* ctl, int K);
// Stage features: f = base with f2, f5, f7 replaced (host-computed from the
// planned sizes) and f6 from the stage-start scalars; skipped unless
// gate is null or *gate >= 1.
hipError_t run_features_stage(hipStream_t st, const float* fbase, const PcgScalars* sc, float f2, float f5, float f7,
                              const int32_t* gate, float* f);
// Decision of stage s from the network outputs (skipped unless ctl[s] >= 1):
// a = first arg-max of out[0..4], capped so that Stage I totals at most
// t_cap; ctl[s + 1] = 1 unless out[6] > out[5] (stop).
hipError_t run_sched_decide(hipStream_t st, const float* out, int32_t* ctl, int s, int K, int t_cap);

}  // namespace spcg
