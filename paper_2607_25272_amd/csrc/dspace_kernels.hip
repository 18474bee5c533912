// d-space part of a PCG iteration on gfx950 (all FP64).
//
// Phase A reduces the per-block product partials in a fixed order and
// performs the step  alpha = rho / (p^T s),  x += alpha p,  g -= alpha s
// (or g = g_true - alpha s when the product pass refreshed the gradient).
// Phase B applies the preconditioner, z = H_hat^{-1} g = R^{-1} R^{-T} g,
// as one symmetric matrix-vector product with the precomputed FP64
// operator M = R^{-1} R^{-T}, and performs  rho' = g^T z,
// p = z + (rho'/rho) p.  Both phases spread the O(d) / O(d^2) work over
// many blocks and let the last block to finish (device-scope counter) form
// the scalars, so a whole PCG iteration is three kernel launches and no
// host synchronisation.
//
// Guard rules (shared with the oracle's PCG): rho == 0 means the current
// iterate is exact and no step is taken; p^T s <= 0 or a non-finite scalar
// is a breakdown: the step is skipped, x keeps its last good value and a
// sticky flag is raised for the host.
#include "common.hpp"
#include "internal.hpp"

namespace spcg {

namespace {

constexpr int A_COLS = 16;   // columns per phase-A block
constexpr int B_ROWS = 4;    // rows of M per phase-B wave and sweep
constexpr int B_GRID = 32;   // at most this many phase-B blocks (few device-scope hand-offs)

struct PhaseAArgs {
    DspaceState S;
    const double* part_s;
    const double* part_g;
    const double* part_scal;
    int nparts;
    int64_t dpad;
    double c2;
    double g_scale;   // PA_START_NESTED: weight of the previous gradient
    int variant;
};

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// Hand-off to the last block: every wave waits for its own global stores,
// the block barrier orders them before thread 0, and thread 0 alone
// releases at device scope and counts the block.  A device-scope fence
// costs tens of nanoseconds and fences of different blocks serialize, so
// one fence per block (not one per wave) and few blocks keep the hand-off
// short.  Returns true in the last block, after its acquire.
__device__ __forceinline__ bool last_block_arrive(unsigned int* counter, int* is_last) {
    __builtin_amdgcn_s_waitcnt((0x7 << 4) | (0xf << 8));   // vmcnt(0)
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev = atomicAdd(counter, 1u);
        *is_last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (!*is_last) return false;
    __threadfence();
    return true;
}

__global__ __launch_bounds__(256) void phase_a_kernel(PhaseAArgs a) {
    // 16 columns x 16 partial lanes per block; lane ty sums partials
    // ty + 16 v into four running sums (v mod 4), combined in a fixed order.
    // All loads of the first 256 partials are issued before any is used.
    __shared__ double sh_s[16][A_COLS + 1];
    __shared__ double sh_g[16][A_COLS + 1];
    __shared__ double sh_r[256];
    __shared__ double sh_t[256];
    __shared__ double sh_b[256];
    __shared__ int is_last;
    const DspaceState& S = a.S;
    if (S.gate && *S.gate < S.gmin) return;   // switched off on the device (uniform)
    const int tx = threadIdx.x & (A_COLS - 1), ty = threadIdx.x / A_COLS;
    const int64_t col = (int64_t)blockIdx.x * A_COLS + tx;
    const bool start = a.variant == PA_START || a.variant == PA_START_NESTED;
    const bool want_s = !start;
    const bool want_g = a.variant != PA_STEP;
    double ss[4] = {0.0, 0.0, 0.0, 0.0}, gg[4] = {0.0, 0.0, 0.0, 0.0};
    double pc = 0.0;
    if (col < S.d) {
        if (want_s) pc = S.p[col];
        double vs[16], vg[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int b = ty + 16 * v;
            const int64_t off = (int64_t)b * a.dpad + col;
            vs[v] = (want_s && b < a.nparts) ? a.part_s[off] : 0.0;
            vg[v] = (want_g && b < a.nparts) ? a.part_g[off] : 0.0;
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            ss[v & 3] += vs[v];
            gg[v & 3] += vg[v];
        }
        for (int b = ty + 256, u = 0; b < a.nparts; b += 16, u = (u + 1) & 3) {
            const int64_t off = (int64_t)b * a.dpad + col;
            if (want_s) ss[u] += a.part_s[off];
            if (want_g) gg[u] += a.part_g[off];
        }
    }
    sh_s[ty][tx] = (ss[0] + ss[1]) + (ss[2] + ss[3]);
    sh_g[ty][tx] = (gg[0] + gg[1]) + (gg[2] + gg[3]);
    __syncthreads();
    double dot = 0.0;
    if (ty == 0 && col < S.d) {
        double s_col = 0.0, g_col = 0.0;
        for (int q = 0; q < 16; ++q) {
            s_col += sh_s[q][tx];
            g_col += sh_g[q][tx];
        }
        s_col *= a.c2;
        g_col *= a.c2;
        if (a.variant == PA_START) {
            S.g[col] = g_col;
        } else if (a.variant == PA_START_NESTED) {
            S.g[col] = fma(a.g_scale, S.g[col], g_col);
        } else {
            S.s[col] = s_col;
            dot = pc * s_col;
            if (a.variant == PA_REFRESH) S.gt[col] = g_col;
        }
    }
    if (ty == 0) {
        dot = group_sum<A_COLS>(dot);
        if (tx == 0) S.blk[blockIdx.x] = dot;
    }
    if (!last_block_arrive(&S.counters[0], &is_last)) return;

    // ---- last block: scalars and the x / g update.  The block partials of
    // p^T s, the norm partials and the vectors of the update are all
    // requested together.
    PcgScalars* sc = S.sc;
    const unsigned nblk = gridDim.x;
    double t0 = 0.0, t1 = 0.0;
    if (want_g) {
        for (int b = threadIdx.x; b < a.nparts; b += 256) {
            t0 += a.part_scal[2 * b];
            t1 += a.part_scal[2 * b + 1];
        }
    }
    if (threadIdx.x < nblk) sh_b[threadIdx.x] = S.blk[threadIdx.x];
    // norm partials: DPP sums per wave, then the four waves in order (one
    // barrier instead of a shared-memory tree)
    if (want_g) {
        const double wr = wave_sum(t0), wt = wave_sum(t1);
        if ((threadIdx.x & 63) == 0) {
            sh_r[threadIdx.x >> 6] = wr;
            sh_t[threadIdx.x >> 6] = wt;
        }
    }
    __syncthreads();
    if (want_g && threadIdx.x == 0) {
        sh_r[0] = (sh_r[0] + sh_r[1]) + (sh_r[2] + sh_r[3]);
        sh_t[0] = (sh_t[0] + sh_t[1]) + (sh_t[2] + sh_t[3]);
    }
    __shared__ double alpha_sh;
    __shared__ int do_step;
    if (threadIdx.x == 0) {
        if (want_g) {
            sc->resid2 = sh_r[0] * a.c2;
            sc->ax2 = sh_t[0] * a.c2;
        }
        do_step = 0;
        if (start) {
            sc->resid2_0 = sh_r[0] * a.c2;
            sc->exact = 0;
        } else {
            double pts = 0.0;
            for (unsigned b = 0; b < nblk; ++b) pts += b < 256 ? sh_b[b] : S.blk[b];
            sc->pts = pts;
            const double rho = sc->rho;
            if (sc->breakdown || sc->exact) {
                sc->alpha = 0.0;
            } else if (rho == 0.0) {
                sc->exact = 1;
                sc->alpha = 0.0;
            } else if (!(pts > 0.0) || !finite(pts) || !finite(rho)) {
                sc->breakdown = 1;
                sc->alpha = 0.0;
            } else {
                alpha_sh = rho / pts;
                sc->alpha = alpha_sh;
                do_step = 1;
            }
        }
        S.counters[0] = 0u;
    }
    __syncthreads();
    if (do_step) {
        const double al = alpha_sh;
        const bool refresh = a.variant == PA_REFRESH;
        for (int64_t c = threadIdx.x; c < S.d; c += 256) {
            S.x[c] = fma(al, S.p[c], S.x[c]);
            const double gbase = refresh ? S.gt[c] : S.g[c];
            S.g[c] = fma(-al, S.s[c], gbase);
        }
    }
}

__global__ __launch_bounds__(256) void phase_b_kernel(DspaceState S, int init) {
    __shared__ double sh[4];
    __shared__ double red[4];
    __shared__ int is_last;
    if (S.gate && *S.gate < S.gmin) return;   // switched off on the device (uniform)
    PcgScalars* sc = S.sc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // wave w of block b takes rows b*4 + w + k * stride, k = 0..B_ROWS-1 per
    // sweep (stride = 4 * gridDim.x); the row loads of a sweep are all
    // issued before any is used, and they do not wait for the guard flags
    // (a skipped iteration computes and discards)
    const bool skip = sc->breakdown || (!init && sc->exact);
    const int64_t stride = (int64_t)gridDim.x * 4;
    double gz = 0.0;
    for (int64_t i0 = (int64_t)blockIdx.x * 4 + wave; i0 < S.d; i0 += B_ROWS * stride) {
        double acc4[B_ROWS][2];
#pragma unroll
        for (int k = 0; k < B_ROWS; ++k) acc4[k][0] = acc4[k][1] = 0.0;
        for (int64_t j0 = lane; j0 < S.d; j0 += 512) {
            double gv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t j = j0 + 64 * u;
                gv[u] = j < S.d ? S.g[j] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < B_ROWS; ++k) {
                const int64_t i = i0 + k * stride;
                const double* row = S.Minv + min(i, S.d - 1) * S.d;
                double mv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int64_t j = j0 + 64 * u;
                    mv[u] = (i < S.d && j < S.d) ? row[j] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) acc4[k][u & 1] = fma(mv[u], gv[u], acc4[k][u & 1]);
            }
        }
#pragma unroll
        for (int k = 0; k < B_ROWS; ++k) {
            const int64_t i = i0 + k * stride;
            const double acc = wave_sum(acc4[k][0] + acc4[k][1]);
            if (!skip && i < S.d && lane == 0) {
                S.z[i] = acc;
                gz += S.g[i] * acc;
            }
        }
    }
    if (lane == 0) sh[wave] = gz;
    __syncthreads();
    if (threadIdx.x == 0) S.blk[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    if (!last_block_arrive(&S.counters[1], &is_last)) return;
    // fixed-order reduction of the block partials: DPP sums per wave, then
    // the four waves in order
    double t = 0.0;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += 256) t += S.blk[b];
    t = wave_sum(t);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    __shared__ double gamma_sh;
    __shared__ int mode;  // 0 skip, 1 p = z, 2 p = z + gamma p
    if (threadIdx.x == 0) {
        const double rho_new = (red[0] + red[1]) + (red[2] + red[3]);
        mode = 0;
        if (!skip) {
            if (!finite(rho_new)) {
                sc->breakdown = 1;
            } else if (init) {
                sc->rho = rho_new;
                sc->rho0 = rho_new;
                sc->exact = rho_new == 0.0;
                mode = 1;
            } else {
                gamma_sh = rho_new / sc->rho;
                sc->rho = rho_new;
                if (rho_new == 0.0) sc->exact = 1;
                mode = 2;
            }
        }
        S.counters[1] = 0u;
    }
    __syncthreads();
    if (mode == 1) {
        for (int64_t c = threadIdx.x; c < S.d; c += 256) S.p[c] = S.z[c];
    } else if (mode == 2) {
        const double gm = gamma_sh;
        for (int64_t c = threadIdx.x; c < S.d; c += 256) S.p[c] = fma(gm, S.p[c], S.z[c]);
    }
}

__global__ void scalars_reset_kernel(PcgScalars* sc) {
    sc->rho = 0.0;
    sc->alpha = 0.0;
    sc->pts = 0.0;
    sc->resid2 = 0.0;
    sc->ax2 = 0.0;
    sc->rho0 = 0.0;
    sc->resid2_0 = 0.0;
    sc->exact = 0;
    sc->breakdown = 0;
    sc->iters = 0;
    sc->pad = 0;
}

__global__ void fill_kernel(double* v, int64_t n, double value) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = value;
}

__global__ void counters_reset_kernel(unsigned int* c, int n) {
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0u;
}

}  // namespace

hipError_t run_scalars_reset(hipStream_t st, PcgScalars* sc) {
    scalars_reset_kernel<<<1, 1, 0, st>>>(sc);
    return hipGetLastError();
}

hipError_t run_fill(hipStream_t st, double* v, int64_t n, double value) {
    if (n <= 0) return hipSuccess;
    fill_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(v, n, value);
    return hipGetLastError();
}

hipError_t run_counters_reset(hipStream_t st, unsigned int* c, int n) {
    counters_reset_kernel<<<1, 64, 0, st>>>(c, n);
    return hipGetLastError();
}

hipError_t run_phase_a(hipStream_t st, const DspaceState& S, int variant, const double* part_s,
                       const double* part_g, const double* part_scal, int nparts, int64_t dpad,
                       double c2, double g_scale) {
    PhaseAArgs a;
    a.g_scale = g_scale;
    a.S = S;
    a.part_s = part_s;
    a.part_g = part_g;
    a.part_scal = part_scal;
    a.nparts = nparts;
    a.dpad = dpad;
    a.c2 = c2;
    a.variant = variant;
    const int64_t grid = ceil_div(S.d, A_COLS);
    phase_a_kernel<<<(unsigned)grid, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t run_phase_b(hipStream_t st, const DspaceState& S, int init) {
    const int64_t grid = std::min<int64_t>(ceil_div(S.d, 4 * B_ROWS), B_GRID);
    phase_b_kernel<<<(unsigned)grid, 256, 0, st>>>(S, init);
    return hipGetLastError();
}

}  // namespace spcg
