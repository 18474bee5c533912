// Learned schedule on gfx950: the features of a problem and of each
// sketched stage, a three-layer FP32 network (forward, loss gradient, Adam)
// that maps them to a stage's iteration count, whether Stage I stops after
// it, and the Stage II iteration count, and the per-stage decision kernels.
//
// The network is tiny (5191 parameters), so the kernels keep all weights in
// LDS and give each sample eight threads (eight hidden units each).  The
// loss gradient is summed over the samples in a fixed order: each block
// walks a fixed set of 32-sample chunks and writes one partial gradient,
// and one reduction kernel adds the partials block by block, so repeated
// calls give identical bits.
#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace spcg {

namespace {

constexpr int F = MLP_F, H = MLP_H, O = MLP_O;
constexpr int OW1 = 0, OB1 = H * F, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + O * H;
constexpr int NP = OB3 + O;
static_assert(NP == MLP_PARAMS, "parameter layout");
constexpr int NT = 256;              // threads per block
constexpr int CH = 32;               // samples per chunk
constexpr int TPS = NT / CH;         // threads per sample
constexpr int UPT = H / TPS;         // hidden units per thread
constexpr int GPT = (NP + NT - 1) / NT;  // gradient entries per thread
// one LDS row per sample: x | h1 | h2 | d1 | d2 | dout (odd stride: no bank conflicts)
constexpr int RX = 0, RH1 = 8, RH2 = RH1 + H, RD1 = RH2 + H, RD2 = RD1 + H, RDO = RD2 + H;
constexpr int RS = RDO + 8 + 1;
constexpr int MAX_GRAD_BLOCKS = 512;

template <bool GRAD>
__global__ __launch_bounds__(NT) void mlp_kernel(const float* __restrict__ W, const float* __restrict__ feats,
                                                 int64_t n, const int32_t* __restrict__ la,
                                                 const int32_t* __restrict__ lg, const float* __restrict__ ls,
                                                 const float* __restrict__ wa, const float* __restrict__ ws,
                                                 float inv_n, float* __restrict__ out,
                                                 float* __restrict__ partial) {
    __shared__ float sW[NP];
    __shared__ float rows[CH * RS];
    __shared__ float sloss[CH];
    const int tid = threadIdx.x;
    for (int i = tid; i < NP; i += NT) sW[i] = W[i];
    const int s = tid / TPS;
    const int q = tid % TPS;
    float* row = rows + s * RS;
    float gacc[GRAD ? GPT : 1];
#pragma unroll
    for (int r = 0; r < (GRAD ? GPT : 1); ++r) gacc[r] = 0.f;
    float lacc = 0.f;
    const int64_t nchunks = ceil_div(n, CH);
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t smp = c * CH + s;
        const bool valid = smp < n;
        __syncthreads();
        if (q == 0) {
#pragma unroll
            for (int i = 0; i < F; ++i) row[RX + i] = valid ? feats[smp * F + i] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            const int j = q * UPT + u;
            float z = sW[OB1 + j];
#pragma unroll
            for (int i = 0; i < F; ++i) z = fmaf(sW[OW1 + j * F + i], row[RX + i], z);
            row[RH1 + j] = fmaxf(z, 0.f);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            const int j = q * UPT + u;
            float z = sW[OB2 + j];
#pragma unroll 16
            for (int k = 0; k < H; ++k) z = fmaf(sW[OW2 + j * H + k], row[RH1 + k], z);
            row[RH2 + j] = fmaxf(z, 0.f);
        }
        __syncthreads();
        if (q < O) {
            float z = sW[OB3 + q];
#pragma unroll 16
            for (int k = 0; k < H; ++k) z = fmaf(sW[OW3 + q * H + k], row[RH2 + k], z);
            row[RDO + q] = z;
            if (!GRAD && valid) out[smp * O + q] = z;
        }
        if constexpr (GRAD) {
            __syncthreads();
            if (q == 0) {
                float l = 0.f;
                float o[O];
#pragma unroll
                for (int i = 0; i < O; ++i) o[i] = row[RDO + i];
                if (valid) {
                    // outputs 0..NA-1: a_i logits, NA..NA+1: stop logits, NA+2: s_II
                    constexpr int NA = MLP_NA;
                    static_assert(NA + 3 == O, "output layout");
                    const int a = min(max(la[smp], 0), NA - 1), g = lg[smp] & 1;
                    const float t = ls[smp] * (float)(1.0 / MLP_S_SCALE);
                    const float w1 = wa[smp], w2 = ws[smp];
                    float ma = o[0];
#pragma unroll
                    for (int i = 1; i < NA; ++i) ma = fmaxf(ma, o[i]);
                    float ea[NA], sa = 0.f;
#pragma unroll
                    for (int i = 0; i < NA; ++i) {
                        ea[i] = expf(o[i] - ma);
                        sa += ea[i];
                    }
                    const float mg = fmaxf(o[NA], o[NA + 1]);
                    const float eg0 = expf(o[NA] - mg), eg1 = expf(o[NA + 1] - mg);
                    const float sg = eg0 + eg1;
                    float oa = 0.f;
#pragma unroll
                    for (int i = 0; i < NA; ++i) oa = i == a ? o[i] : oa;
                    const float og = g == 0 ? o[NA] : o[NA + 1];
                    const float ce = (ma + logf(sa) - oa) + (mg + logf(sg) - og);
                    const float rr = o[NA + 2] - t;
                    l = w1 * ce + w2 * (float)MLP_LAMBDA * rr * rr;
                    const float ka = w1 * inv_n;
#pragma unroll
                    for (int i = 0; i < NA; ++i) row[RDO + i] = ka * (ea[i] / sa - (i == a ? 1.f : 0.f));
                    row[RDO + NA] = ka * (eg0 / sg - (g == 0 ? 1.f : 0.f));
                    row[RDO + NA + 1] = ka * (eg1 / sg - (g == 1 ? 1.f : 0.f));
                    row[RDO + NA + 2] = w2 * (float)(2.0 * MLP_LAMBDA) * rr * inv_n;
                } else {
#pragma unroll
                    for (int i = 0; i < O; ++i) row[RDO + i] = 0.f;
                }
                sloss[s] = l;
            }
            __syncthreads();
            // d2 = (dout W3) * [h2 > 0]
#pragma unroll
            for (int u = 0; u < UPT; ++u) {
                const int j = q * UPT + u;
                float acc = 0.f;
#pragma unroll
                for (int i = 0; i < O; ++i) acc = fmaf(row[RDO + i], sW[OW3 + i * H + j], acc);
                row[RD2 + j] = row[RH2 + j] > 0.f ? acc : 0.f;
            }
            __syncthreads();
            // d1 = (d2 W2) * [h1 > 0]
#pragma unroll
            for (int u = 0; u < UPT; ++u) {
                const int k = q * UPT + u;
                float acc = 0.f;
#pragma unroll 16
                for (int j = 0; j < H; ++j) acc = fmaf(row[RD2 + j], sW[OW2 + j * H + k], acc);
                row[RD1 + k] = row[RH1 + k] > 0.f ? acc : 0.f;
            }
            __syncthreads();
            // parameter gradients summed over the chunk, samples in order
#pragma unroll
            for (int r = 0; r < GPT; ++r) {
                const int e = tid + r * NT;
                if (e < NP) {
                    int ua, ub;  // row offsets of the two factors (ub < 0: bias)
                    if (e < OB1) {
                        ua = RD1 + e / F;
                        ub = RX + e % F;
                    } else if (e < OW2) {
                        ua = RD1 + (e - OB1);
                        ub = -1;
                    } else if (e < OB2) {
                        ua = RD2 + (e - OW2) / H;
                        ub = RH1 + (e - OW2) % H;
                    } else if (e < OW3) {
                        ua = RD2 + (e - OB2);
                        ub = -1;
                    } else if (e < OB3) {
                        ua = RDO + (e - OW3) / H;
                        ub = RH2 + (e - OW3) % H;
                    } else {
                        ua = RDO + (e - OB3);
                        ub = -1;
                    }
                    float acc = 0.f;
                    if (ub >= 0) {
#pragma unroll 4
                        for (int s2 = 0; s2 < CH; ++s2) acc = fmaf(rows[s2 * RS + ua], rows[s2 * RS + ub], acc);
                    } else {
#pragma unroll 4
                        for (int s2 = 0; s2 < CH; ++s2) acc += rows[s2 * RS + ua];
                    }
                    gacc[r] += acc;
                }
            }
            if (tid == 0) {
                for (int s2 = 0; s2 < CH; ++s2) lacc += sloss[s2];
            }
        }
    }
    if constexpr (GRAD) {
        float* dst = partial + (int64_t)blockIdx.x * (NP + 1);
#pragma unroll
        for (int r = 0; r < GPT; ++r) {
            const int e = tid + r * NT;
            if (e < NP) dst[e] = gacc[r];
        }
        if (tid == 0) dst[NP] = lacc;
    }
}

__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ partial, int nb, float inv_n,
                                                          float* __restrict__ grad, float* __restrict__ loss) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e > NP) return;
    float acc = 0.f;
    for (int b = 0; b < nb; ++b) acc += partial[(int64_t)b * (NP + 1) + e];
    if (e < NP) {
        grad[e] = acc;
    } else if (loss) {
        *loss = acc * inv_n;
    }
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ W, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t n,
                                                   float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    W[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

template <typename TS>
__device__ __forceinline__ double load_elem(const TS* p, int64_t i, const float* cs, int64_t c);
template <>
__device__ __forceinline__ double load_elem<double>(const double* p, int64_t i, const float*, int64_t) {
    return p[i];
}
template <>
__device__ __forceinline__ double load_elem<float>(const float* p, int64_t i, const float*, int64_t) {
    return (double)p[i];
}
template <>
__device__ __forceinline__ double load_elem<bf16_t>(const bf16_t* p, int64_t i, const float*, int64_t) {
    return (double)bf16_bits_to_f32(p[i].bits);
}
template <>
__device__ __forceinline__ double load_elem<fp8_t>(const fp8_t* p, int64_t i, const float* cs, int64_t c) {
    return (double)fp8e4m3_bits_to_f32(p[i].bits) * (double)cs[c];
}

// Features known before Stage I (one block of 16 waves): the problem
// shape, the spread of diag(R) and the row-norm spread over 256 evenly
// spaced rows.  Wave w takes the sampled rows w, w + 16, ...; its lanes
// read a row's columns in stride (coalesced), the squared norm is summed
// per lane and across the wave.
template <typename TS>
__global__ __launch_bounds__(1024) void features_pre_kernel(const TS* __restrict__ X, int64_t N, int64_t d,
                                                            int64_t ld, const float* __restrict__ cs,
                                                            const double* __restrict__ R, int64_t ldr,
                                                            float* __restrict__ f) {
    __shared__ double s_q[MLP_SAMPLE_ROWS];
    __shared__ double s_max[1024], s_sum[1024], s_dmin[1024], s_dmax[1024];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const bool all = N >= MLP_SAMPLE_ROWS;
    const int nrows = all ? MLP_SAMPLE_ROWS : (int)N;
    for (int r = wave; r < nrows; r += 16) {
        const int64_t j = all ? ((2 * (int64_t)r + 1) * N) / (2 * MLP_SAMPLE_ROWS) : r;
        double q = 0.0;
        for (int64_t c = lane; c < d; c += 64) {
            const double v = load_elem<TS>(X, j * ld + c, cs, c);
            q = fma(v, v, q);
        }
        for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o);
        if (lane == 0) s_q[r] = q;
    }
    __syncthreads();
    double mn = INFINITY, mx = 0.0;
    for (int64_t c = t; c < d; c += 1024) {
        const double r = fabs(R[c * ldr + c]);
        mn = fmin(mn, r);
        mx = fmax(mx, r);
    }
    const double q = t < nrows ? s_q[t] : 0.0;
    s_max[t] = q;
    s_sum[t] = q;
    s_dmin[t] = mn;
    s_dmax[t] = mx;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (t < o) {
            s_max[t] = fmax(s_max[t], s_max[t + o]);
            s_sum[t] += s_sum[t + o];
            s_dmin[t] = fmin(s_dmin[t], s_dmin[t + o]);
            s_dmax[t] = fmax(s_dmax[t], s_dmax[t + o]);
        }
        __syncthreads();
    }
    if (t == 0) {
        const double cnt = (double)nrows;
        const double sum = s_sum[0];
        f[0] = (float)(log10((double)N) - 5.0);
        f[1] = (float)(log10((double)d) - 2.0);
        f[2] = (float)(log2((double)N / (double)d) / 8.0 - 1.0);
        f[3] = (float)(s_dmin[0] <= 0.0 ? 3.0 : log10(s_dmax[0] / s_dmin[0]) / 3.0 - 1.0);
        f[4] = (float)(sum <= 0.0 ? 0.0 : log10(s_max[0] / (sum / cnt)) / 2.0);
        f[5] = 0.f;
        f[6] = 0.f;
        f[7] = 0.f;
    }
}

// Features at the start of Stage II: the pre-Stage-I ones plus the distance
// of the stopping test from its threshold and the residual-to-fit ratio.
__global__ void features_ii_kernel(const float* __restrict__ fpre, const PcgScalars* __restrict__ sc, double tol,
                                   float* __restrict__ f) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double rho = sc->rho, ax2 = sc->ax2, r2 = sc->resid2;
    double f5, f6;
    if (!(rho > 0.0)) {
        f5 = -3.0;
    } else if (!(ax2 > 0.0)) {
        f5 = 3.0;
    } else {
        f5 = log10(sqrt(rho) / (tol * sqrt(ax2))) / 3.0;
    }
    if (!(r2 > 0.0)) {
        f6 = -2.0;
    } else if (!(ax2 > 0.0)) {
        f6 = 2.0;
    } else {
        f6 = log10(r2 / ax2) / 6.0;
    }
    for (int i = 0; i < 5; ++i) f[i] = fpre[i];
    f[5] = (float)fmin(fmax(f5, -3.0), 3.0);
    f[6] = (float)fmin(fmax(f6, -2.0), 2.0);
    f[7] = 1.f;
}

// Features at the start of a sketched stage: the base features with the
// stage size, the Theorem 3.3 bound and the position (host-computed), and
// the residual-to-fit ratio of the rows the starting-gradient pass read.
__global__ void features_stage_kernel(const float* __restrict__ fb, const PcgScalars* __restrict__ sc, float f2,
                                      float f5, float f7, const int32_t* __restrict__ gate, float* __restrict__ f) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (gate && *gate < 1) return;
    const double ax2 = sc->ax2, r2 = sc->resid2;
    double f6;
    if (!(r2 > 0.0)) {
        f6 = -2.0;
    } else if (!(ax2 > 0.0)) {
        f6 = 2.0;
    } else {
        f6 = log10(r2 / ax2) / 6.0;
    }
    f[0] = fb[0];
    f[1] = fb[1];
    f[2] = f2;
    f[3] = fb[3];
    f[4] = fb[4];
    f[5] = f5;
    f[6] = (float)fmin(fmax(f6, -2.0), 2.0);
    f[7] = f7;
}

__global__ void sched_init_kernel(int32_t* ctl, int K) {
    for (int i = threadIdx.x; i < sched_ctl_words(K); i += blockDim.x) {
        int v;
        if (i <= K) v = i == 0 ? 1 : 0;           // start flags: stage 0 starts
        else if (i <= 2 * K) v = -1;              // iterations: not decided
        else v = 0;                               // Stage I iterations so far
        ctl[i] = v;
    }
}

__global__ void sched_decide_kernel(const float* __restrict__ out, int32_t* __restrict__ ctl, int s, int K,
                                    int t_cap) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (ctl[s] < 1) return;
    int a = 0;
    for (int i = 1; i < MLP_NA; ++i)
        if (out[i] > out[a]) a = i;
    const int used = ctl[2 * K + 1];
    a = max(0, min(a, t_cap - used));
    const bool stop = out[MLP_NA + 1] > out[MLP_NA];
    ctl[K + 1 + s] = a;
    ctl[2 * K + 1] = used + a;
    ctl[s + 1] = stop ? 0 : 1;   // ctl[K] is a sentinel
}

}  // namespace

hipError_t run_sched_init(hipStream_t st, int32_t* ctl, int K) {
    if (K < 1) return hipErrorInvalidValue;
    sched_init_kernel<<<1, 128, 0, st>>>(ctl, K);
    return hipGetLastError();
}

hipError_t run_features_stage(hipStream_t st, const float* fbase, const PcgScalars* sc, float f2, float f5, float f7,
                              const int32_t* gate, float* f) {
    features_stage_kernel<<<1, 64, 0, st>>>(fbase, sc, f2, f5, f7, gate, f);
    return hipGetLastError();
}

hipError_t run_sched_decide(hipStream_t st, const float* out, int32_t* ctl, int s, int K, int t_cap) {
    if (s < 0 || s >= K) return hipErrorInvalidValue;
    sched_decide_kernel<<<1, 64, 0, st>>>(out, ctl, s, K, t_cap);
    return hipGetLastError();
}

int mlp_grad_blocks(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>(ceil_div(n, CH), 1), MAX_GRAD_BLOCKS); }

hipError_t run_mlp_forward(hipStream_t st, const float* W, const float* feats, int64_t n, float* out) {
    if (n <= 0) return hipSuccess;
    const int nb = (int)std::min<int64_t>(ceil_div(n, CH), 65535);
    mlp_kernel<false><<<nb, NT, 0, st>>>(W, feats, n, nullptr, nullptr, nullptr, nullptr, nullptr, 0.f, out,
                                         nullptr);
    return hipGetLastError();
}

hipError_t run_mlp_loss_grad(hipStream_t st, const float* W, const float* feats, int64_t n, const int32_t* la,
                             const int32_t* lg, const float* ls, const float* wa, const float* ws, float* partial,
                             float* grad, float* loss) {
    const int nb = mlp_grad_blocks(n);
    const float inv_n = n > 0 ? (float)(1.0 / (double)n) : 0.f;
    mlp_kernel<true><<<nb, NT, 0, st>>>(W, feats, n, la, lg, ls, wa, ws, inv_n, nullptr, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    mlp_reduce_kernel<<<(int)ceil_div(NP + 1, 256), 256, 0, st>>>(partial, nb, inv_n, grad, loss);
    return hipGetLastError();
}

hipError_t run_adam(hipStream_t st, float* W, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                    float b2, float eps, float c1, float c2) {
    if (n <= 0) return hipSuccess;
    adam_kernel<<<(int)ceil_div(n, 256), 256, 0, st>>>(W, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t run_features_pre(hipStream_t st, const void* X, int dtype, int64_t N, int64_t d, int64_t ld,
                            const float* col_scale, const double* R, int64_t ldr, float* f) {
    switch (dtype) {
        case DT_F64:
            features_pre_kernel<double><<<1, 1024, 0, st>>>(static_cast<const double*>(X), N, d, ld, col_scale, R,
                                                           ldr, f);
            break;
        case DT_F32:
            features_pre_kernel<float><<<1, 1024, 0, st>>>(static_cast<const float*>(X), N, d, ld, col_scale, R, ldr,
                                                          f);
            break;
        case DT_BF16:
            features_pre_kernel<bf16_t><<<1, 1024, 0, st>>>(static_cast<const bf16_t*>(X), N, d, ld, col_scale, R,
                                                           ldr, f);
            break;
        case DT_FP8:
            features_pre_kernel<fp8_t><<<1, 1024, 0, st>>>(static_cast<const fp8_t*>(X), N, d, ld, col_scale, R, ldr,
                                                          f);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t run_features_ii(hipStream_t st, const float* fpre, const PcgScalars* sc, double tol, float* f) {
    features_ii_kernel<<<1, 64, 0, st>>>(fpre, sc, tol, f);
    return hipGetLastError();
}

}  // namespace spcg
