// Multi-right-hand-side and batched PCG products on gfx950 matrix cores.
//
// With k right-hand sides the two products of a PCG iteration become
// skinny GEMMs: W = A_t P (rows x k) and S += A_t^T W (d x k) for every
// row tile A_t of A, P in R^{d x k}.  Each PCG column is independent (one
// set of scalars per right-hand side); only the reads of A are shared.
// At k = 16 a FP32 row costs 4k = 64 flops per 4 bytes, beyond what the
// vector units sustain at HBM speed, so both GEMMs run on
// v_mfma_f32_16x16x4_f32 (16 x 16 output, K = 4):
//   A operand: lane l holds A[l % 16][l / 16]
//   B operand: lane l holds B[l / 16][l % 16]
//   result   : lane l, register v holds C[4 (l / 16) + v][l % 16].
//
// Work is a list of tasks (problem, first row, last row); one launch covers
// every task of a batch of independent problems.  A task's block stages
// 16-row tiles of its problem's A in LDS (widened to FP32); the 4 waves
// split the first GEMM along d and combine their 16 x 16 partials through
// LDS; each wave then owns a quarter of the d / 16 output tiles of the
// second GEMM, with the accumulators in registers.  The task writes one
// FP32 partial d x 16 block per output; the per-problem d-space kernel sums
// the partials of its tasks in a fixed order.
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace spcg {

namespace {

constexpr int MT = 16;          // rows per tile (MFMA M)
constexpr int KP = 16;          // right-hand sides per MFMA (N)
constexpr int MR_DMAX = 512;    // columns supported by the staged path
constexpr int MR_WAVES = 4;
constexpr int AT_LD = MR_DMAX + 4;

typedef float mv4f __attribute__((ext_vector_type(4)));

template <typename TS>
__device__ __forceinline__ float widen1(const void* A, int64_t idx);
template <>
__device__ __forceinline__ float widen1<float>(const void* A, int64_t idx) {
    return static_cast<const float*>(A)[idx];
}
template <>
__device__ __forceinline__ float widen1<bf16_t>(const void* A, int64_t idx) {
    return bf16_bits_to_f32(static_cast<const uint16_t*>(A)[idx]);
}

template <typename TS, int MODE>
__global__ __launch_bounds__(64 * MR_WAVES) void mrhs_product_kernel(const MrhsTask* __restrict__ tasks,
                                                                     const MrhsProblem* __restrict__ probs,
                                                                     float* part_s, float* part_g,
                                                                     float* part_scal) {
    constexpr bool DO_S = MODE != PM_G;
    constexpr bool DO_G = MODE != PM_S;
    __shared__ float At[MT][AT_LD];
    __shared__ float Ps[DO_S ? MR_DMAX : 1][KP];
    __shared__ float Xs[DO_G ? MR_DMAX : 1][KP];    // x rounded to FP32
    __shared__ float Xl[DO_G ? MR_DMAX : 1][KP];    // x - Xs, the low part
    __shared__ float Wp[MR_WAVES][MT][KP + 1];
    __shared__ float Wgp[DO_G ? MR_WAVES : 1][MT][KP + 1];
    __shared__ float Wlp[DO_G ? MR_WAVES : 1][MT][KP + 1];

    const MrhsTask task = tasks[blockIdx.x];
    const MrhsProblem pb = probs[task.prob];
    const int d = pb.d, k = pb.k;
    const int dt = (d + 15) / 16;          // 16-column tiles of d
    const int d4 = (d + 3) / 4;            // K steps of the first GEMM
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;

    // Stage P (FP32) and x as an FP32 pair (hi + lo, ~48 bits), padded with
    // zeros.  A x = A x_hi + A x_lo: the high product only changes when x_hi
    // does, so steps far below FP32 resolution of x still move the residual
    // (through the low product) and the refreshed gradient keeps seeing
    // them.
    for (int e = threadIdx.x; e < MR_DMAX * KP; e += 64 * MR_WAVES) {
        const int j = e / KP, c = e % KP;
        const bool ok = j < d && c < k;
        if (DO_S) Ps[j][c] = ok ? (float)pb.P[(int64_t)c * pb.ldv + j] : 0.f;
        if (DO_G) {
            const double xv = ok ? pb.X[(int64_t)c * pb.ldv + j] : 0.0;
            const float hi = (float)xv;
            Xs[j][c] = hi;
            Xl[j][c] = (float)(xv - (double)hi);
        }
    }
    // this wave's output tiles of the second GEMM: mt = wave, wave + 4, ...
    constexpr int MAXT = MR_DMAX / 16 / MR_WAVES;
    mv4f accS[MAXT], accG[MAXT];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        accS[t] = mv4f{0.f, 0.f, 0.f, 0.f};
        accG[t] = mv4f{0.f, 0.f, 0.f, 0.f};
    }
    float r2 = 0.f, ax2 = 0.f;   // per lane: column li, rows of its groups
    // first-GEMM K range of this wave
    const int kq = (d4 + MR_WAVES - 1) / MR_WAVES;
    const int ks0 = wave * kq, ks1 = min(d4, ks0 + kq);

    for (int64_t row0 = task.r0; row0 < task.r1; row0 += MT) {
        __syncthreads();   // previous tile fully consumed
        for (int e = threadIdx.x; e < MT * MR_DMAX; e += 64 * MR_WAVES) {
            const int rr = e / MR_DMAX, j = e % MR_DMAX;
            const int64_t row = row0 + rr;
            At[rr][j] = (row < task.r1 && j < d) ? widen1<TS>(pb.A, row * pb.lda + j) : 0.f;
        }
        __syncthreads();
        // first GEMM: partial W over this wave's K range
        mv4f ws = mv4f{0.f, 0.f, 0.f, 0.f}, wg = mv4f{0.f, 0.f, 0.f, 0.f}, wl = mv4f{0.f, 0.f, 0.f, 0.f};
        for (int s = ks0; s < ks1; ++s) {
            const float av = At[li][4 * s + lg];
            if (DO_S) ws = __builtin_amdgcn_mfma_f32_16x16x4f32(av, Ps[4 * s + lg][li], ws, 0, 0, 0);
            if (DO_G) {
                wg = __builtin_amdgcn_mfma_f32_16x16x4f32(av, Xs[4 * s + lg][li], wg, 0, 0, 0);
                wl = __builtin_amdgcn_mfma_f32_16x16x4f32(av, Xl[4 * s + lg][li], wl, 0, 0, 0);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            Wp[wave][4 * lg + v][li] = ws[v];
            if (DO_G) {
                Wgp[wave][4 * lg + v][li] = wg[v];
                Wlp[wave][4 * lg + v][li] = wl[v];
            }
        }
        __syncthreads();
        // B operands of the second GEMM: W[4 s + lg][li], s = 0..3, summed over waves
        float wb[4], gb[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int rr = 4 * s + lg;
            float t0 = 0.f, t1 = 0.f, tl = 0.f;
#pragma unroll
            for (int w = 0; w < MR_WAVES; ++w) {
                t0 += Wp[w][rr][li];
                if (DO_G) {
                    t1 += Wgp[w][rr][li];
                    tl += Wlp[w][rr][li];
                }
            }
            wb[s] = t0;
            if (DO_G) {
                const int64_t row = row0 + rr;
                const bool ok = row < task.r1 && li < k;
                const double bv = ok ? pb.b[row * pb.ldb + li] : 0.0;
                const double res = ok ? (bv - (double)t1) - (double)tl : 0.0;
                gb[s] = (float)res;
                if (wave == 0) {
                    r2 = fmaf((float)res, (float)res, r2);
                    ax2 = fmaf(t1, t1, ax2);
                }
            }
        }
        // second GEMM: S[:, tile mt] += A_t^T W
#pragma unroll
        for (int t = 0; t < MAXT; ++t) {
            const int mt = wave + MR_WAVES * t;
            if (mt < dt) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const float av = At[4 * s + lg][16 * mt + li];
                    if (DO_S) accS[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, wb[s], accS[t], 0, 0, 0);
                    if (DO_G) accG[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, gb[s], accG[t], 0, 0, 0);
                }
            }
        }
    }
    // partial outputs: part[task][col][c] (c < 16)
    const int64_t base = (int64_t)blockIdx.x * MR_DMAX * KP;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        const int mt = wave + MR_WAVES * t;
        if (mt < dt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int col = 16 * mt + 4 * lg + v;
                if (DO_S) part_s[base + (int64_t)col * KP + li] = accS[t][v];
                if (DO_G) part_g[base + (int64_t)col * KP + li] = accG[t][v];
            }
        }
    }
    if (DO_G) {
        // reduce the per-lane norms of wave 0 over its 4 lane groups
        __shared__ float nrm[2][4][KP];
        if (wave == 0) {
            nrm[0][lg][li] = r2;
            nrm[1][lg][li] = ax2;
        }
        __syncthreads();
        if (threadIdx.x < KP) {
            const int c = threadIdx.x;
            part_scal[(int64_t)blockIdx.x * 2 * KP + c] = ((nrm[0][0][c] + nrm[0][1][c]) + nrm[0][2][c]) + nrm[0][3][c];
            part_scal[(int64_t)blockIdx.x * 2 * KP + KP + c] =
                ((nrm[1][0][c] + nrm[1][1][c]) + nrm[1][2][c]) + nrm[1][3][c];
        }
    }
}

}  // namespace

int mrhs_max_d() { return MR_DMAX; }
int mrhs_max_k() { return KP; }

hipError_t run_mrhs_product(hipStream_t st, int dtype, int mode, const MrhsTask* tasks, int ntasks,
                            const MrhsProblem* probs, float* part_s, float* part_g, float* part_scal) {
    if (ntasks <= 0) return hipSuccess;
    dim3 grid(ntasks), block(64 * MR_WAVES);
#define SPCG_MR_LAUNCH(TS)                                                                                    \
    switch (mode) {                                                                                           \
        case PM_S: mrhs_product_kernel<TS, PM_S><<<grid, block, 0, st>>>(tasks, probs, part_s, part_g, part_scal); break; \
        case PM_G: mrhs_product_kernel<TS, PM_G><<<grid, block, 0, st>>>(tasks, probs, part_s, part_g, part_scal); break; \
        default: mrhs_product_kernel<TS, PM_SG><<<grid, block, 0, st>>>(tasks, probs, part_s, part_g, part_scal); break; \
    }
    if (dtype == DT_F32) {
        SPCG_MR_LAUNCH(float)
    } else if (dtype == DT_BF16) {
        SPCG_MR_LAUNCH(bf16_t)
    } else {
        return hipErrorInvalidValue;
    }
#undef SPCG_MR_LAUNCH
    return hipGetLastError();
}

}  // namespace spcg

namespace spcg {

namespace {

constexpr int DS_THREADS = 256;

__device__ __forceinline__ bool dfinite(double v) { return __builtin_isfinite(v); }

// Column sums over j of a[j][c] * b[j][c] for every c < 16, fixed order.
__device__ void colwise_dot(const double* a, const double* b, int64_t ldv, int d, int k, double* out,
                            double (*red)[KP + 1]) {
    const int c = threadIdx.x % KP, q = threadIdx.x / KP;   // 16 lanes per column
    double t = 0.0;
    if (c < k)
        for (int j = q; j < d; j += DS_THREADS / KP) t = fma(a[(int64_t)c * ldv + j], b[(int64_t)c * ldv + j], t);
    red[q][c] = t;
    __syncthreads();
    if (threadIdx.x < KP) {
        double s = 0.0;
        for (int w = 0; w < DS_THREADS / KP; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

__global__ __launch_bounds__(DS_THREADS) void mrhs_dspace_kernel(int variant, const MrhsProblem* __restrict__ probs,
                                                                  const float* __restrict__ part_s,
                                                                  const float* __restrict__ part_g,
                                                                  const float* __restrict__ part_scal) {
    __shared__ double red[DS_THREADS / KP][KP + 1];
    __shared__ double colv[KP], colw[KP];
    __shared__ double alpha_sh[KP], gamma_sh[KP];
    __shared__ int step_sh[KP];
    const MrhsProblem pb = probs[blockIdx.x];
    if (!pb.active) return;
    const int d = pb.d, k = pb.k;
    const int64_t ldv = pb.ldv;
    const bool want_s = variant != PA_START, want_g = variant != PA_STEP;
    // 1. reduce the task partials (fixed task order)
    for (int e = threadIdx.x; e < d * KP; e += DS_THREADS) {
        const int j = e / KP, c = e % KP;
        if (c >= k) continue;
        double ss = 0.0, gg = 0.0;
        for (int t = pb.t0; t < pb.t1; ++t) {
            const int64_t off = (int64_t)t * MR_DMAX * KP + (int64_t)j * KP + c;
            if (want_s) ss += (double)part_s[off];
            if (want_g) gg += (double)part_g[off];
        }
        if (variant == PA_START) pb.G[c * ldv + j] = gg * pb.c2;
        else {
            pb.S[c * ldv + j] = ss * pb.c2;
            if (variant == PA_REFRESH) pb.Gt[c * ldv + j] = gg * pb.c2;
        }
    }
    if (want_g && threadIdx.x < KP) {
        double r2 = 0.0, ax2 = 0.0;
        for (int t = pb.t0; t < pb.t1; ++t) {
            r2 += (double)part_scal[(int64_t)t * 2 * KP + threadIdx.x];
            ax2 += (double)part_scal[(int64_t)t * 2 * KP + KP + threadIdx.x];
        }
        colv[threadIdx.x] = r2 * pb.c2;
        colw[threadIdx.x] = ax2 * pb.c2;
    }
    __syncthreads();
    if (want_g && threadIdx.x < k) {
        pb.sc[threadIdx.x].resid2 = colv[threadIdx.x];
        pb.sc[threadIdx.x].ax2 = colw[threadIdx.x];
    }
    // 2. step: alpha = rho / p^T s; x += alpha p; g = (g or g_true) - alpha s
    if (variant != PA_START) {
        colwise_dot(pb.P, pb.S, ldv, d, k, colv, red);
        if (threadIdx.x < KP) {
            const int c = threadIdx.x;
            int doit = 0;
            double al = 0.0;
            if (c < k) {
                MrhsScalars& sc = pb.sc[c];
                const double pts = colv[c], rho = sc.rho;
                sc.pts = pts;
                if (sc.breakdown || sc.exact) {
                } else if (rho == 0.0) {
                    sc.exact = 1;
                } else if (!(pts > 0.0) || !dfinite(pts) || !dfinite(rho)) {
                    sc.breakdown = 1;
                } else {
                    al = rho / pts;
                    doit = 1;
                }
                sc.alpha = al;
            }
            alpha_sh[c] = al;
            step_sh[c] = doit;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < d * KP; e += DS_THREADS) {
            const int j = e / KP, c = e % KP;
            if (c >= k || !step_sh[c]) continue;
            const int64_t o = c * ldv + j;
            pb.X[o] = fma(alpha_sh[c], pb.P[o], pb.X[o]);
            const double gb = variant == PA_REFRESH ? pb.Gt[o] : pb.G[o];
            pb.G[o] = fma(-alpha_sh[c], pb.S[o], gb);
        }
        __syncthreads();
    } else if (threadIdx.x < k) {
        pb.sc[threadIdx.x].exact = 0;
    }
    __syncthreads();
    // 3. z = M g for every column (thread per row of M)
    for (int i = threadIdx.x; i < d; i += DS_THREADS) {
        double acc[KP];
#pragma unroll
        for (int c = 0; c < KP; ++c) acc[c] = 0.0;
        const double* row = pb.Minv + (int64_t)i * d;
        for (int j = 0; j < d; ++j) {
            const double m = row[j];
#pragma unroll
            for (int c = 0; c < KP; ++c)
                if (c < k) acc[c] = fma(m, pb.G[c * ldv + j], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < KP; ++c)
            if (c < k) pb.Z[c * ldv + i] = acc[c];
    }
    __syncthreads();
    // 4. rho' = g^T z; p = z (start) or z + (rho'/rho) p
    colwise_dot(pb.G, pb.Z, ldv, d, k, colv, red);
    if (threadIdx.x < KP) {
        const int c = threadIdx.x;
        int mode = 0;
        double gm = 0.0;
        if (c < k) {
            MrhsScalars& sc = pb.sc[c];
            const double rn = colv[c];
            const bool skip = sc.breakdown || (variant != PA_START && sc.exact);
            if (!skip) {
                if (!dfinite(rn)) {
                    sc.breakdown = 1;
                } else if (variant == PA_START) {
                    sc.rho = rn;
                    sc.rho0 = rn;
                    sc.exact = rn == 0.0;
                    mode = 1;
                } else {
                    gm = rn / sc.rho;
                    sc.rho = rn;
                    if (rn == 0.0) sc.exact = 1;
                    mode = 2;
                }
            }
        }
        gamma_sh[c] = gm;
        step_sh[c] = mode;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < d * KP; e += DS_THREADS) {
        const int j = e / KP, c = e % KP;
        if (c >= k || step_sh[c] == 0) continue;
        const int64_t o = c * ldv + j;
        pb.P[o] = step_sh[c] == 1 ? pb.Z[o] : fma(gamma_sh[c], pb.P[o], pb.Z[o]);
    }
}

}  // namespace

hipError_t run_mrhs_dspace(hipStream_t st, int variant, const MrhsProblem* probs, int nprob,
                           const float* part_s, const float* part_g, const float* part_scal) {
    if (nprob <= 0) return hipSuccess;
    mrhs_dspace_kernel<<<nprob, DS_THREADS, 0, st>>>(variant, probs, part_s, part_g, part_scal);
    return hipGetLastError();
}

}  // namespace spcg
