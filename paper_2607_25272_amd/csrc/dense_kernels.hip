// FP64 dense kernels for the preconditioner build on gfx950.
//
// The preconditioner of Sec. 2.2 is H_hat = (S_hat X)^T (S_hat X), applied
// "through a QR factorization" (Sec. 4): with S_hat X = Q R,
// H_hat^{-1} = R^{-1} R^{-T}.  R is obtained from Cholesky factorizations of
// Gram matrices (CholeskyQR; the shifted three-pass form of Fukaya,
// Kannan, Nakatsukasa, Yamamoto, Yanagisawa, "Shifted Cholesky QR for
// computing the QR factorization of ill-conditioned matrices", SISC 2020),
// which maps onto GPU-friendly pieces: a tiled GEMM, a blocked right-looking
// Cholesky and a blocked triangular solve.
#include <algorithm>
#include <type_traits>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace spcg {

namespace {

constexpr int GT = 64;   // GEMM tile
constexpr int GK = 16;   // GEMM k step
constexpr int CB = 64;   // Cholesky / TRSM panel width

struct GemmArgs {
    int64_t M, N, K;
    double alpha, beta;
    const void* A;
    int64_t sai, sal;
    const void* B;
    int64_t sbl, sbj;
    double* C;
    int64_t ldc;
    int upper;
    int64_t kchunk;     // K range per blockIdx.z
    double* part;       // split-K: [gridDim.z][M][N] partial products (or null)
    // batched products (bsc != 0): blockIdx.z selects entry z, whose A, B and
    // C start bsa, bsb and bsc elements after entry 0's; no split-K.  The
    // last entry may be narrower: N = n_last, K = k_last where those are > 0
    int64_t bsa, bsb, bsc;
    int64_t n_last, k_last;
};

template <bool F32>
__device__ __forceinline__ double ld_elem(const void* p, int64_t idx) {
    if (F32) return (double)static_cast<const float*>(p)[idx];
    return static_cast<const double*>(p)[idx];
}

// TT x TT output tile per block of 256 threads (16 x 16, each a P x P
// patch, P = TT / 16); K in steps of GK through LDS.  TT = 64 for large
// products; TT = 32 gives 4x the blocks for the small ones, whose time is
// set by how many CUs they occupy.
template <bool AF32, bool BF32, int TT>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    constexpr int P = TT / 16;
    constexpr int NL = TT * GK / 256;   // loads per thread per operand and k step
    const int64_t ti = blockIdx.y, tj = blockIdx.x;
    if (g.upper && ti > tj) return;
    __shared__ double As[GK][TT + 1];
    __shared__ double Bs[GK][TT + 1];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int64_t i0 = ti * TT, j0 = tj * TT;
    double acc[P][P];
#pragma unroll
    for (int r = 0; r < P; ++r)
#pragma unroll
        for (int c = 0; c < P; ++c) acc[r][c] = 0.0;
    const bool a_icontig = g.sai == 1;
    const bool b_jcontig = g.sbj == 1;
    const bool batched = g.bsc != 0;
    const int64_t oa = batched ? (int64_t)blockIdx.z * g.bsa : 0;
    const int64_t ob = batched ? (int64_t)blockIdx.z * g.bsb : 0;
    const bool lastz = batched && blockIdx.z + 1 == gridDim.z;
    const int64_t gN = lastz && g.n_last > 0 ? g.n_last : g.N;
    const int64_t gK = lastz && g.k_last > 0 ? g.k_last : g.K;
    const int64_t kbeg = batched ? 0 : (int64_t)blockIdx.z * g.kchunk;
    const int64_t kend = batched ? gK : min(g.K, kbeg + g.kchunk);
    for (int64_t l0 = kbeg; l0 < kend; l0 += GK) {
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int e = tid + q * 256;
            int i, l;
            if (a_icontig) {
                i = e % TT;
                l = e / TT;
            } else {
                l = e % GK;
                i = e / GK;
            }
            const int64_t gi = i0 + i, gl = l0 + l;
            As[l][i] = (gi < g.M && gl < kend) ? ld_elem<AF32>(g.A, oa + gi * g.sai + gl * g.sal) : 0.0;
            int j;
            if (b_jcontig) {
                j = e % TT;
                l = e / TT;
            } else {
                l = e % GK;
                j = e / GK;
            }
            const int64_t gj = j0 + j, gl2 = l0 + l;
            Bs[l][j] = (gj < gN && gl2 < kend) ? ld_elem<BF32>(g.B, ob + gl2 * g.sbl + gj * g.sbj) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < GK; ++l) {
            double av[P], bv[P];
#pragma unroll
            for (int r = 0; r < P; ++r) av[r] = As[l][ty * P + r];
#pragma unroll
            for (int c = 0; c < P; ++c) bv[c] = Bs[l][tx * P + c];
#pragma unroll
            for (int r = 0; r < P; ++r)
#pragma unroll
                for (int c = 0; c < P; ++c) acc[r][c] = fma(av[r], bv[c], acc[r][c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const int64_t gi = i0 + ty * P + r;
        if (gi >= g.M) continue;
#pragma unroll
        for (int c = 0; c < P; ++c) {
            const int64_t gj = j0 + tx * P + c;
            if (gj >= gN) continue;
            if (g.part) {
                g.part[((int64_t)blockIdx.z * g.M + gi) * g.N + gj] = acc[r][c];
                continue;
            }
            double* cp = g.C + (batched ? (int64_t)blockIdx.z * g.bsc : 0) + gi * g.ldc + gj;
            const double v = g.alpha * acc[r][c];
            *cp = g.beta == 0.0 ? v : fma(g.beta, *cp, v);
        }
    }
}

// The same tiling (64 x 64 output per block, K in steps of GK through LDS)
// with the products on the FP64 matrix cores: each of the 4 waves owns a
// 32 x 32 quarter as 2 x 2 tiles of v_mfma_f64_16x16x4f64.  Per 16 x 16 x 4
// step a lane feeds A[i][k] with i = lane mod 16, k = lane / 16 and B[k][j]
// with j = lane mod 16, k = lane / 16, and holds D[lane / 16 + 4 v][lane mod
// 16] in register v (rows interleaved, unlike the FP32 16x16x4 form; checked
// on the device).  Per K step a wave reads 4 doubles per lane from
// LDS for 16 instructions (1024 FMA each), against 8 reads per 16 FMA of the
// register-tiled kernel.
typedef double gemm_v4d __attribute__((ext_vector_type(4)));

template <bool AF32, bool BF32>
// (at least 4 waves per SIMD: 3 blocks per CU left the k-step load latency exposed)
__global__ __launch_bounds__(256, 4) void gemm_mfma_kernel(GemmArgs g) {
    const int64_t ti = blockIdx.y, tj = blockIdx.x;
    if (g.upper && ti > tj) return;
    constexpr int NL = GT * GK / 256;   // elements per thread per operand and k step
    __shared__ double As[GK][GT + 1];
    __shared__ double Bs[GK][GT + 1];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int64_t i0 = ti * GT, j0 = tj * GT;
    gemm_v4d acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = gemm_v4d{0.0, 0.0, 0.0, 0.0};
    const bool a_icontig = g.sai == 1;
    const bool b_jcontig = g.sbj == 1;
    const bool batched = g.bsc != 0;
    const int64_t oa = batched ? (int64_t)blockIdx.z * g.bsa : 0;
    const int64_t ob = batched ? (int64_t)blockIdx.z * g.bsb : 0;
    const bool lastz = batched && blockIdx.z + 1 == gridDim.z;
    const int64_t gN = lastz && g.n_last > 0 ? g.n_last : g.N;
    const int64_t gK = lastz && g.k_last > 0 ? g.k_last : g.K;
    const int64_t kbeg = batched ? 0 : (int64_t)blockIdx.z * g.kchunk;
    const int64_t kend = batched ? gK : min(g.K, kbeg + g.kchunk);
    // the (row or column, k) slots this thread loads for either operand
    int ai[NL], al[NL], bj[NL], bl[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int e = tid + q * 256;
        ai[q] = a_icontig ? e % GT : e / GK;
        al[q] = a_icontig ? e / GT : e % GK;
        bj[q] = b_jcontig ? e % GT : e / GK;
        bl[q] = b_jcontig ? e / GT : e % GK;
    }
    double ra[NL], rb[NL];
    auto fetch = [&](int64_t l0) {
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int64_t gi = i0 + ai[q], gl = l0 + al[q];
            ra[q] = (gi < g.M && gl < kend) ? ld_elem<AF32>(g.A, oa + gi * g.sai + gl * g.sal) : 0.0;
            const int64_t gj = j0 + bj[q], gl2 = l0 + bl[q];
            rb[q] = (gj < gN && gl2 < kend) ? ld_elem<BF32>(g.B, ob + gl2 * g.sbl + gj * g.sbj) : 0.0;
        }
    };
    // software pipeline: the loads of k step l0 + GK are in flight while
    // step l0 runs on the matrix cores
    if (kbeg < kend) fetch(kbeg);
    for (int64_t l0 = kbeg; l0 < kend; l0 += GK) {
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            As[al[q]][ai[q]] = ra[q];
            Bs[bl[q]][bj[q]] = rb[q];
        }
        __syncthreads();
        if (l0 + GK < kend) fetch(l0 + GK);
#pragma unroll
        for (int ks = 0; ks < GK / 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            double av[2], bv[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                av[t] = As[kk][wr * 32 + t * 16 + (lane & 15)];
                bv[t] = Bs[kk][wc * 32 + t * 16 + (lane & 15)];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gi = i0 + wr * 32 + a * 16 + (lane >> 4) + 4 * v;
                const int64_t gj = j0 + wc * 32 + b * 16 + (lane & 15);
                if (gi >= g.M || gj >= gN) continue;
                const double r = acc[a][b][v];
                if (g.part) {
                    g.part[((int64_t)blockIdx.z * g.M + gi) * g.N + gj] = r;
                    continue;
                }
                double* cp = g.C + (batched ? (int64_t)blockIdx.z * g.bsc : 0) + gi * g.ldc + gj;
                const double val = g.alpha * r;
                *cp = g.beta == 0.0 ? val : fma(g.beta, *cp, val);
            }
}

// C = alpha * sum_z part[z] + beta * C (fixed order over z)
__global__ void splitk_reduce_kernel(const double* part, int nz, int64_t M, int64_t N, double alpha,
                                     double beta, double* C, int64_t ldc, int upper) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= M * N) return;
    const int64_t i = e / N, j = e - i * N;
    if (upper && (i / GT) > (j / GT)) return;
    double s = 0.0;
    for (int z = 0; z < nz; ++z) s += part[(int64_t)z * M * N + e];
    double* cp = C + i * ldc + j;
    const double v = alpha * s;
    *cp = beta == 0.0 ? v : fma(beta, *cp, v);
}

// Upper Cholesky of the nb x nb diagonal block at (k0, k0) of G, in place
// (strict lower part zeroed).
// 256 threads in a 16 x 16 grid; each keeps a 4 x 4 patch of the block in
// registers.  Step j needs only w = row j of U right of the diagonal
// (w[l] = U[j][l] for l > j, 0 otherwise): every patch then takes
// a[i][l] -= w[i] w[l] without conditions (rows i <= j see w[i] = 0; the
// strict lower part collects values that are never used).  The 16 threads
// of a patch row share one wave, so the wave that owns row j + 1 reads its
// pivot with a lane broadcast right after its own update, scales the row
// and publishes w through LDS (double-buffered): one barrier per step.  The
// step loop is unrolled by 4 so that the row inside a patch is static.
__device__ __forceinline__ double bcast_lane(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// a: this thread's 4 x 4 patch (rows 4 ty + r, columns 4 tx + c) of the
// nb x nb block; only the upper part (diagonal included) is read.  On
// return the upper part holds U; pivs[0..nb) the pivots.
__device__ __forceinline__ void potrf_patch(double (&a)[4][4], int nb, double (*rows)[CB], double* pivs) {
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // row j = 4 jb + JR: scale it in place and publish w (wave jb / 4 only)
    auto publish = [&](int jb, auto jr_c) __attribute__((always_inline)) {
        constexpr int JR = decltype(jr_c)::value;
        const int j = 4 * jb + JR;
        if (wave != (jb >> 2)) return;
        // the pivot (j, j) sits in patch (jb, jb) at (JR, JR): lane 16 (jb mod 4) + jb
        const double piv = bcast_lane(a[JR][JR], (jb & 3) * 16 + jb);
        const bool bad = !(piv > 0.0) || !__builtin_isfinite(piv);
        // 1 / sqrt(piv) from the hardware estimate and two Newton steps,
        // then sqrt(piv) = piv / sqrt(piv) with one Newton correction: a
        // shorter dependent chain than a square root and a division
        const double p1 = bad ? 1.0 : piv;
        double y = __builtin_amdgcn_rsq(p1);
        y = fma(0.5 * y, fma(-p1 * y, y, 1.0), y);
        y = fma(0.5 * y, fma(-p1 * y, y, 1.0), y);
        double u = p1 * y;
        u = fma(fma(-u, u, p1), 0.5 * y, u);
        const double ru = y;
        if (ty == jb) {
            double w[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const bool right = tx > jb || (tx == jb && c > JR);
                const bool diag = tx == jb && c == JR;
                const double v = a[JR][c] * ru;
                a[JR][c] = diag ? u : (right ? v : a[JR][c]);
                w[c] = right ? v : 0.0;
            }
            *reinterpret_cast<double2*>(&rows[j & 1][tx * 4]) = make_double2(w[0], w[1]);
            *reinterpret_cast<double2*>(&rows[j & 1][tx * 4 + 2]) = make_double2(w[2], w[3]);
            if (tx == jb) pivs[j] = piv;
        }
    };
    auto update = [&](int j) __attribute__((always_inline)) {
        const double* w = rows[j & 1];
        const double2 wi0 = *reinterpret_cast<const double2*>(&w[ty * 4]);
        const double2 wi1 = *reinterpret_cast<const double2*>(&w[ty * 4 + 2]);
        const double2 wl0 = *reinterpret_cast<const double2*>(&w[tx * 4]);
        const double2 wl1 = *reinterpret_cast<const double2*>(&w[tx * 4 + 2]);
        const double wi[4] = {wi0.x, wi0.y, wi1.x, wi1.y};
        const double wl[4] = {wl0.x, wl0.y, wl1.x, wl1.y};
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) a[r][c] = fma(-wi[r], wl[c], a[r][c]);
    };
    using C0 = std::integral_constant<int, 0>;
    using C1 = std::integral_constant<int, 1>;
    using C2 = std::integral_constant<int, 2>;
    using C3 = std::integral_constant<int, 3>;
    publish(0, C0{});
    for (int jb = 0; 4 * jb < nb; ++jb) {
        const int j = 4 * jb;
        __syncthreads();
        update(j);
        if (j + 1 >= nb) break;
        publish(jb, C1{});
        __syncthreads();
        update(j + 1);
        if (j + 2 >= nb) break;
        publish(jb, C2{});
        __syncthreads();
        update(j + 2);
        if (j + 3 >= nb) break;
        publish(jb, C3{});
        __syncthreads();
        update(j + 3);
        if (j + 4 >= nb) break;
        publish(jb + 1, C0{});
    }
    __syncthreads();   // pivs complete
}

// running pivot statistics of the factorization: one wave, lane j takes
// pivot j (nb <= 64); a NaN pivot never lowers the minimum, and the first
// failure is the smallest failing index
__device__ __forceinline__ void potrf_status(const double* pivs, int nb, int64_t k0, DenseStatus* st) {
    const int j = threadIdx.x & 63;
    const bool in = j < nb;
    const double p = in ? pivs[j] : 1.0;
    const bool bad = in && (!(p > 0.0) || !__builtin_isfinite(p));
    const double u = bad ? 1.0 : sqrt(p);
    const double inf = __builtin_huge_val();
    double mp = (in && p == p) ? p : inf;
    double mn = in ? u : inf, mx = in ? u : -inf;
    int ff = bad ? j : 64;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double a = __shfl_xor(mp, o), b = __shfl_xor(mn, o), c = __shfl_xor(mx, o);
        const int f = __shfl_xor(ff, o);
        mp = a < mp ? a : mp;
        mn = b < mn ? b : mn;
        mx = c > mx ? c : mx;
        ff = f < ff ? f : ff;
    }
    if (j == 0) {
        if (mp < st->min_pivot) st->min_pivot = mp;
        if (mn < st->min_diag) st->min_diag = mn;
        if (mx > st->max_diag) st->max_diag = mx;
        if (st->fail == 0 && ff < 64) st->fail = (int)(k0 + ff) + 1;
    }
}

// One doubling round of trtri_lds: for each pair of neighbouring SZ x SZ
// diagonal blocks, W12 = -W11 (U12 W22).  W is upper triangular with its
// strict lower part zero, so the products run over the full SZ range: the
// extra terms are exact zeros added after (first product) or before (second)
// the triangular ones, and the fixed trip count lets the LDS loads batch.
template <int SZ>
__device__ __forceinline__ void trtri_round(double (*T)[CB + 1], double (*Wl)[CB + 1], double (*Tmp)[CB + 1]) {
    constexpr int OUTS = (CB / (2 * SZ)) * SZ * SZ;
    static_assert(OUTS % 256 == 0, "whole rounds per thread");
    const int tid = threadIdx.x;
#pragma unroll
    for (int e0 = 0; e0 < OUTS; e0 += 256) {
        const int e = e0 + tid;
        const int p = e / (SZ * SZ), rem = e % (SZ * SZ), i = rem / SZ, j = rem % SZ;
        const int s0 = p * 2 * SZ, s1 = s0 + SZ;
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < SZ; ++l) acc = fma(T[s0 + i][s1 + l], Wl[s1 + l][s1 + j], acc);
        Tmp[s0 + i][s1 + j] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int e0 = 0; e0 < OUTS; e0 += 256) {
        const int e = e0 + tid;
        const int p = e / (SZ * SZ), rem = e % (SZ * SZ), i = rem / SZ, j = rem % SZ;
        const int s0 = p * 2 * SZ, s1 = s0 + SZ;
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < SZ; ++l) acc = fma(Wl[s0 + i][s0 + l], Tmp[s0 + l][s1 + j], acc);
        Wl[s0 + i][s1 + j] = -acc;
    }
    __syncthreads();
}

// The same round on the FP64 matrix cores, for SZ = 16 (two pairs) and 32
// (one pair): each product has at most four 16 x 16 output tiles, one per
// wave.  Per step of 4 in K, lane l feeds A[l mod 16][l / 16] and
// B[l / 16][l mod 16] and holds D[l / 16 + 4 v][l mod 16] in register v.
template <int SZ>
__device__ __forceinline__ void trtri_round_mfma(double (*T)[CB + 1], double (*Wl)[CB + 1],
                                                 double (*Tmp)[CB + 1]) {
    constexpr int TS = SZ / 16;                   // tiles per side of a pair's block
    constexpr int TILES = (CB / (2 * SZ)) * TS * TS;
    static_assert(SZ % 16 == 0 && TILES <= 4, "one tile per wave");
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int li = lane & 15, lk = lane >> 4;
    const bool active = wave < TILES;             // uniform over the wave
    const int pr = wave / (TS * TS), t = wave % (TS * TS);
    const int ti = (t / TS) * 16, tj = (t % TS) * 16;
    const int s0 = pr * 2 * SZ, s1 = s0 + SZ;
    if (active) {   // Tmp = U12 W22
        gemm_v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k0 = 0; k0 < SZ; k0 += 4)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(T[s0 + ti + li][s1 + k0 + lk], Wl[s1 + k0 + lk][s1 + tj + li],
                                                       acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) Tmp[s0 + ti + lk + 4 * v][s1 + tj + li] = acc[v];
    }
    __syncthreads();
    if (active) {   // W12 = -W11 Tmp
        gemm_v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k0 = 0; k0 < SZ; k0 += 4)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Wl[s0 + ti + li][s0 + k0 + lk], Tmp[s0 + k0 + lk][s1 + tj + li],
                                                       acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) Wl[s0 + ti + lk + 4 * v][s1 + tj + li] = -acc[v];
    }
    __syncthreads();
}

// Inverse of the upper-triangular CB x CB block in T (identity past the
// used size) into Wl, by recursive doubling in LDS: invert the eight 8 x 8
// diagonal blocks by back substitution, then for s = 8, 16, 32 combine
// neighbouring s x s inverses with W12 = -W11 U12 W22 (s = 16, 32 on the
// matrix cores).  Tmp is scratch.  Expects T complete (caller synchronizes);
// Wl is complete on return.
__device__ __forceinline__ void trtri_lds(double (*T)[CB + 1], double (*Wl)[CB + 1], double (*Tmp)[CB + 1]) {
    static_assert(CB == 64, "three doubling rounds");
    const int tid = threadIdx.x;
    for (int e = tid; e < CB * CB; e += 256) Wl[e >> 6][e & 63] = 0.0;
    __syncthreads();
    if (tid < CB) {   // 8 x 8 diagonal blocks: thread = (block, column)
        const int b0 = (tid >> 3) * 8, c = tid & 7;
        double w[8];
#pragma unroll
        for (int i = 7; i >= 0; --i) {
            double acc = (i == c) ? 1.0 : 0.0;
#pragma unroll
            for (int l = i + 1; l < 8; ++l) acc = fma(-T[b0 + i][b0 + l], w[l], acc);
            w[i] = (i <= c) ? acc / T[b0 + i][b0 + i] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) Wl[b0 + i][b0 + c] = w[i];
    }
    __syncthreads();
    trtri_round<8>(T, Wl, Tmp);
    trtri_round_mfma<16>(T, Wl, Tmp);
    trtri_round_mfma<32>(T, Wl, Tmp);
}

// Inverses of CB x CB diagonal blocks of an upper-triangular U, starting at
// block `first` (one block of 256 threads per diagonal block).  A partial
// last block is padded with the identity.
__global__ __launch_bounds__(256) void trtri_blocks_kernel(const double* U, int64_t d, int64_t ld, double* W,
                                                           int64_t first) {
    __shared__ double T[CB][CB + 1];
    __shared__ double Wl[CB][CB + 1];
    __shared__ double Tmp[CB][CB + 1];
    const int tid = threadIdx.x;
    const int64_t k0 = (first + (int64_t)blockIdx.x) * CB;
    const int nb = (int)min((int64_t)CB, d - k0);
    {
        constexpr int NQ = CB * CB / 256;
        double v[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {   // all loads in flight first
            const int e = tid + q * 256, i = e >> 6, j = e & 63;
            if (i < nb && j < nb) v[q] = (j >= i) ? U[(k0 + i) * ld + k0 + j] : 0.0;
            else v[q] = (i == j) ? 1.0 : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = tid + q * 256;
            T[e >> 6][e & 63] = v[q];
        }
    }
    __syncthreads();
    trtri_lds(T, Wl, Tmp);
    for (int e = tid; e < CB * CB; e += 256) {
        const int i = e >> 6, j = e & 63;
        if (i < nb && j < nb) W[(k0 + i) * ld + k0 + j] = Wl[i][j];
    }
}

// ---- fused blocked Cholesky (upper, G = U^T U) ------------------------------
//
// chol_first_kernel factors the first diagonal block; then one
// chol_step_kernel per panel k (rows k0 .. k0 + CB) does, for every tile
// pair ti <= tj of the trailing part (one block each):
//   P_i = W_kk^T G[k, ti],  P_j = W_kk^T G[k, tj]   (columns of U_k,trailing)
//   G[ti, tj] -= P_i^T P_j
// with W_kk = U_kk^{-1}.  The diagonal-pair blocks keep their P_j as U's row
// panel, stored transposed in the (otherwise unused) strict lower triangle
// so that no block overwrites rows another block still reads; the block of
// the first trailing diagonal tile then factors it in place (potrf on its
// register patch, which has exactly the update's layout) and inverts it:
// U and W of panel k + 1.  chol_finish_kernel moves the row panels to the
// upper triangle and clears the lower one.  Per panel: one launch instead
// of a factor, an inverse, a panel product, a copy and a trailing update.
__device__ __forceinline__ void store_factor_and_inverse(double (&a)[4][4], int nb, double* G, int64_t ld,
                                                         int64_t k0, double* Wd, double (*T)[CB + 1],
                                                         double (*Wl)[CB + 1], double (*Tmp)[CB + 1],
                                                         double (*rows)[CB], double* pivs, DenseStatus* st) {
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    potrf_patch(a, nb, rows, pivs);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = ty * 4 + r, j = tx * 4 + c;
            const double u = (j >= i) ? a[r][c] : 0.0;
            if (i < nb && j < nb) G[(k0 + i) * ld + k0 + j] = u;
            T[i][j] = (i < nb && j < nb) ? u : (i == j ? 1.0 : 0.0);
        }
    if (tid < 64) potrf_status(pivs, nb, k0, st);   // wave 0
    __syncthreads();
    trtri_lds(T, Wl, Tmp);
    for (int e = tid; e < CB * CB; e += 256) {
        const int i = e >> 6, j = e & 63;
        if (i < nb && j < nb) Wd[(k0 + i) * ld + k0 + j] = Wl[i][j];
    }
}

__global__ __launch_bounds__(256) void chol_first_kernel(double* G, int64_t d, int64_t ld, double* Wd,
                                                         DenseStatus* st) {
    __shared__ double T[CB][CB + 1];
    __shared__ double Wl[CB][CB + 1];
    __shared__ double Tmp[CB][CB + 1];
    __shared__ __align__(16) double rows[2][CB];
    __shared__ double pivs[CB];
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    const int nb = (int)min((int64_t)CB, d);
    double a[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = ty * 4 + r, j = tx * 4 + c;
            a[r][c] = (i < nb && j < nb && j >= i) ? G[i * ld + j] : 0.0;
        }
    store_factor_and_inverse(a, nb, G, ld, 0, Wd, T, Wl, Tmp, rows, pivs, st);
}

__global__ __launch_bounds__(256) void chol_step_kernel(double* G, int64_t d, int64_t ld, int64_t k0, double* Wd,
                                                        DenseStatus* st) {
    __shared__ double S0[CB][CB + 1];   // W_kk; then T of the next factor
    __shared__ double S1[CB][CB + 1];   // G[k, ti] -> P_i; then the inverse
    __shared__ double S2[CB][CB + 1];   // G[k, tj] -> P_j; then scratch
    __shared__ __align__(16) double rows[2][CB];
    __shared__ double pivs[CB];
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    const int64_t k1 = k0 + CB;
    const int64_t nt = (d - k1 + CB - 1) / CB;
    // block -> (ti, tj), ti <= tj, row by row over the upper triangle
    int64_t b = blockIdx.x, ti = 0;
    while (b >= nt - ti) {
        b -= nt - ti;
        ++ti;
    }
    const int64_t tj = ti + b;
    const bool diag = ti == tj;
    const int64_t i0 = k1 + ti * CB, j0 = k1 + tj * CB;
    const int ni = (int)min((int64_t)CB, d - i0), nj = (int)min((int64_t)CB, d - j0);
    // every global load is issued before the first LDS store (a rolled
    // load-store loop would wait for each load in turn), the trailing tile
    // G[ti, tj] included: no block of this step writes it (the kept row
    // panels go to panel k's columns)
    double acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = ty * 4 + r, j = tx * 4 + c;
            acc[r][c] = (i < ni && j < nj) ? G[(i0 + i) * ld + j0 + j] : 0.0;
        }
    {
        constexpr int NQ = CB * CB / 256;
        double l0[NQ], l1[NQ], l2[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = tid + q * 256, r = e >> 6, c = e & 63;
            l0[q] = c >= r ? Wd[(k0 + r) * ld + k0 + c] : 0.0;
            l1[q] = c < ni ? G[(k0 + r) * ld + i0 + c] : 0.0;
            l2[q] = (!diag && c < nj) ? G[(k0 + r) * ld + j0 + c] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = tid + q * 256, r = e >> 6, c = e & 63;
            S0[r][c] = l0[q];
            S1[r][c] = l1[q];
            if (!diag) S2[r][c] = l2[q];
        }
    }
    __syncthreads();
    // P = W_kk^T A: P[r][c] = sum_{l <= r} W[l][r] A[l][c]
    double pi[4][4], pj[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            pi[r][c] = 0.0;
            pj[r][c] = 0.0;
        }
    // diagonal pairs (ti = tj, the critical block among them) form P_i only
    auto panel = [&](auto both_c) __attribute__((always_inline)) {
        constexpr bool BOTH = decltype(both_c)::value;
#pragma unroll 8
        for (int l = 0; l < CB; ++l) {
            double wv[4], av[4], bv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) wv[r] = S0[l][ty * 4 + r];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                av[c] = S1[l][tx * 4 + c];
                bv[c] = BOTH ? S2[l][tx * 4 + c] : 0.0;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    pi[r][c] = fma(wv[r], av[c], pi[r][c]);
                    if constexpr (BOTH) pj[r][c] = fma(wv[r], bv[c], pj[r][c]);
                }
        }
    };
    if (diag)
        panel(std::false_type{});
    else
        panel(std::true_type{});
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            S1[ty * 4 + r][tx * 4 + c] = pi[r][c];
            if (!diag) S2[ty * 4 + r][tx * 4 + c] = pj[r][c];
        }
    // the diagonal-pair blocks keep U's row panel (transposed, lower triangle)
    if (diag) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int pr = ty * 4 + r, pc = tx * 4 + c;
                if (pc < nj) G[(j0 + pc) * ld + k0 + pr] = pi[r][c];
            }
    }
    __syncthreads();
    // trailing update of this tile: G[ti, tj] -= P_i^T P_j
    const double (*Pj)[CB + 1] = diag ? S1 : S2;
#pragma unroll 8
    for (int l = 0; l < CB; ++l) {
        double pv[4], qv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) pv[r] = S1[l][ty * 4 + r];
#pragma unroll
        for (int c = 0; c < 4; ++c) qv[c] = Pj[l][tx * 4 + c];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = fma(-pv[r], qv[c], acc[r][c]);
    }
    if (ti == 0 && tj == 0) {
        // the next diagonal block: factor and invert it
        __syncthreads();   // S0..S2 are reused below
        store_factor_and_inverse(acc, ni, G, ld, k1, Wd, S0, S1, S2, rows, pivs, st);
        return;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = ty * 4 + r, j = tx * 4 + c;
            if (i < ni && j < nj) G[(i0 + i) * ld + j0 + j] = acc[r][c];
        }
}

// upper triangle <- the row panels kept in the lower triangle; lower <- 0
__global__ void chol_finish_kernel(double* G, int64_t d, int64_t ld) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= d * d) return;
    const int64_t i = e / d, j = e - i * d;
    if (j <= i) return;
    // (i, j) upper, (j, i) its mirror
    if (i / CB != j / CB) G[i * ld + j] = G[j * ld + i];
    G[j * ld + i] = 0.0;
}

__global__ void copy2d_kernel(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                              int64_t cols) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cols) return;
    const int64_t i = e / cols, j = e - i * cols;
    dst[i * ldd + j] = src[i * lds + j];
}

// W = the 64 x 64 diagonal blocks of D, zeros elsewhere
__global__ void blockdiag_copy_kernel(const double* D, int64_t d, int64_t ld, double* W) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= d * d) return;
    const int64_t i = e / d, j = e - i * d;
    W[i * ld + j] = (i / CB == j / CB) ? D[i * ld + j] : 0.0;
}

__global__ void identity_kernel(double* A, int64_t d) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= d * d) return;
    const int64_t i = e / d, j = e - i * d;
    A[e] = i == j ? 1.0 : 0.0;
}

template <bool F32>
__global__ void convert_kernel(const void* src, int64_t rows, int64_t cols, int64_t lds, double scale,
                               double* dst, int64_t ldd) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cols) return;
    const int64_t i = e / cols, j = e - i * cols;
    dst[i * ldd + j] = ld_elem<F32>(src, i * lds + j) * scale;
}

__global__ __launch_bounds__(256) void trace_shift_kernel(double* G, int64_t d, double factor) {
    __shared__ double red[256];
    double t = 0.0;
    for (int64_t i = threadIdx.x; i < d; i += 256) t += G[i * d + i];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double shift = factor * red[0];
    for (int64_t i = threadIdx.x; i < d; i += 256) G[i * d + i] += shift;
}

__global__ void status_reset_kernel(DenseStatus* st) {
    st->fail = 0;
    st->pad = 0;
    st->min_diag = __builtin_inf();
    st->max_diag = 0.0;
    st->min_pivot = __builtin_inf();
}

}  // namespace

namespace {
template <int TT>
hipError_t gemm_launch(hipStream_t st, const GemmArgs& g, int a_f32, int b_f32, dim3 grid) {
    const dim3 block(256);
    if constexpr (TT == GT) {
        if (a_f32 && b_f32)
            gemm_mfma_kernel<true, true><<<grid, block, 0, st>>>(g);
        else if (a_f32)
            gemm_mfma_kernel<true, false><<<grid, block, 0, st>>>(g);
        else if (b_f32)
            gemm_mfma_kernel<false, true><<<grid, block, 0, st>>>(g);
        else
            gemm_mfma_kernel<false, false><<<grid, block, 0, st>>>(g);
        return hipGetLastError();
    }
    if (a_f32 && b_f32)
        gemm_kernel<true, true, TT><<<grid, block, 0, st>>>(g);
    else if (a_f32)
        gemm_kernel<true, false, TT><<<grid, block, 0, st>>>(g);
    else if (b_f32)
        gemm_kernel<false, true, TT><<<grid, block, 0, st>>>(g);
    else
        gemm_kernel<false, false, TT><<<grid, block, 0, st>>>(g);
    return hipGetLastError();
}

}  // namespace

hipError_t gemm_f64(hipStream_t st, int64_t M, int64_t N, int64_t K, double alpha, const void* A,
                    int a_f32, int64_t sai, int64_t sal, const void* B, int b_f32, int64_t sbl,
                    int64_t sbj, double beta, double* C, int64_t ldc, int upper, double* work,
                    int64_t work_elems) {
    if (M <= 0 || N <= 0) return hipSuccess;
    // products with few 64 x 64 tiles (not the upper-tile Gram) use 32 x 32
    // tiles: their time is set by how many CUs they occupy
    const bool small = !upper && ceil_div(M, GT) * ceil_div(N, GT) < 64;
    const int64_t tt = small ? 32 : GT;
    const int64_t ti = ceil_div(M, tt), tj = ceil_div(N, tt);
    const int64_t tiles = upper ? (ti * (ti + 1)) / 2 : ti * tj;
    // split K until there are about 512 blocks (2048 for the matrix-core
    // tiles, several per CU, so that their k loops overlap), keeping >= 64
    // per chunk
    const int64_t target = small ? 512 : 2048;
    int64_t nz = 1;
    while (work && tiles * nz * 2 <= target && K / (nz * 2) >= 64 && (nz * 2) * M * N <= work_elems) nz *= 2;
    const int64_t kchunk = round_up(ceil_div(K, nz), GK);
    nz = ceil_div(K, kchunk);
    if (nz < 1) nz = 1;
    GemmArgs g{M, N, K, alpha, beta, A, sai, sal, B, sbl, sbj, C, ldc, upper,
               kchunk, nz > 1 ? work : nullptr};
    const dim3 grid((unsigned)tj, (unsigned)ti, (unsigned)nz);
    hipError_t e = small ? gemm_launch<32>(st, g, a_f32, b_f32, grid) : gemm_launch<GT>(st, g, a_f32, b_f32, grid);
    if (e != hipSuccess || nz == 1) return e;
    splitk_reduce_kernel<<<(unsigned)ceil_div(M * N, 256), 256, 0, st>>>(work, (int)nz, M, N, alpha,
                                                                         beta, C, ldc, upper);
    return hipGetLastError();
}

// `batch` FP64 products of one shape (the last may have N = n_last and
// K = k_last, where those are > 0), entry z at A + z bsa, B + z bsb and
// C + z bsc (row-major strides as for gemm_f64); one launch, no split-K.
// A single entry goes through gemm_f64 (which may split K into work).
hipError_t gemm_f64_batched(hipStream_t st, int64_t batch, int64_t M, int64_t N, int64_t K, double alpha,
                            const double* A, int64_t sai, int64_t sal, int64_t bsa, const double* B,
                            int64_t sbl, int64_t sbj, int64_t bsb, double beta, double* C, int64_t ldc,
                            int64_t bsc, int64_t n_last, int64_t k_last, double* work, int64_t work_elems) {
    if (M <= 0 || N <= 0 || batch <= 0 || n_last < 0 || n_last > N || k_last < 0 || k_last > K)
        return M <= 0 || N <= 0 || batch <= 0 ? hipSuccess : hipErrorInvalidValue;
    if (batch == 1)
        return gemm_f64(st, M, n_last > 0 ? n_last : N, k_last > 0 ? k_last : K, alpha, A, 0, sai, sal, B, 0, sbl,
                        sbj, beta, C, ldc, 0, work, work_elems);
    if (bsc == 0 || batch > 65535) return hipErrorInvalidValue;
    const bool small = ceil_div(M, GT) * ceil_div(N, GT) * batch < 64;
    const int64_t tt = small ? 32 : GT;
    GemmArgs g{M, N, K, alpha, beta, A, sai, sal, B, sbl, sbj, C, ldc, 0, round_up(K, GK), nullptr,
               bsa, bsb, bsc, n_last, k_last};
    const dim3 grid((unsigned)ceil_div(N, tt), (unsigned)ceil_div(M, tt), (unsigned)batch);
    return small ? gemm_launch<32>(st, g, 0, 0, grid) : gemm_launch<GT>(st, g, 0, 0, grid);
}

hipError_t copy2d(hipStream_t st, const double* src, int64_t lds, double* dst, int64_t ldd,
                  int64_t rows, int64_t cols) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    copy2d_kernel<<<(unsigned)ceil_div(rows * cols, 256), 256, 0, st>>>(src, lds, dst, ldd, rows, cols);
    return hipGetLastError();
}

hipError_t cholesky_upper(hipStream_t st, double* G, int64_t d, int64_t ld, DenseStatus* status,
                          double* W, double*, double*, int64_t) {
    hipError_t e;
    chol_first_kernel<<<1, 256, 0, st>>>(G, d, ld, W, status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int64_t k0 = 0; k0 + CB < d; k0 += CB) {
        const int64_t nt = ceil_div(d - k0 - CB, CB);
        chol_step_kernel<<<(unsigned)(nt * (nt + 1) / 2), 256, 0, st>>>(G, d, ld, k0, W, status);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    chol_finish_kernel<<<(unsigned)ceil_div(d * d, 256), 256, 0, st>>>(G, d, ld);
    return hipGetLastError();
}

hipError_t trtri_diag_blocks(hipStream_t st, const double* U, int64_t d, int64_t ld, double* W) {
    trtri_blocks_kernel<<<(unsigned)ceil_div(d, CB), 256, 0, st>>>(U, d, ld, W, 0);
    return hipGetLastError();
}

hipError_t trsm_right_upper(hipStream_t st, double* A, int64_t n, int64_t d, int64_t lda,
                            const double* U, int64_t ldu, const double* W, double* tmp, double* work,
                            int64_t work_elems) {
    hipError_t e;
    for (int64_t k0 = 0; k0 < d; k0 += CB) {
        const int nb = (int)std::min<int64_t>(CB, d - k0);
        if (k0 > 0) {
            e = gemm_f64(st, n, nb, k0, -1.0, A, 0, lda, 1, U + k0, 0, ldu, 1, 1.0, A + k0, lda, 0,
                         work, work_elems);
            if (e != hipSuccess) return e;
        }
        // A[:, k] <- A[:, k] U_kk^{-1}
        e = gemm_f64(st, n, nb, nb, 1.0, A + k0, 0, lda, 1, W + k0 * ldu + k0, 0, ldu, 1, 0.0, tmp, nb, 0,
                     nullptr, 0);
        if (e != hipSuccess) return e;
        if ((e = copy2d(st, tmp, nb, A + k0, lda, n, nb)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t tri_inverse_upper(hipStream_t st, const double* U, int64_t d, int64_t ld, double* W,
                             const double* diag_inv, double* tmp, double* work, int64_t work_elems) {
    hipError_t e;
    if (diag_inv) {
        blockdiag_copy_kernel<<<(unsigned)ceil_div(d * d, 256), 256, 0, st>>>(diag_inv, d, ld, W);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        if ((e = dense_fill_identity(st, W, d)) != hipSuccess) return e;
        if ((e = trtri_diag_blocks(st, U, d, ld, W)) != hipSuccess) return e;
    }
    // recursive doubling over block columns: [W11 W12; 0 W22] with
    // W12 = -W11 (U12 W22), neighbouring s-blocks per level, s = CB, 2 CB, ...
    // All pairs of a level (pair p at columns 2 p s; the last one may be
    // narrower, min(s, d - 2 p s - s)) go in one batched launch per product,
    // each with its own s x s slice of tmp: ceil((d - s) / 2s) s^2 < d^2
    // elements.
    for (int64_t s = CB; s < d; s *= 2) {
        const int64_t pairs = ceil_div(d - s, 2 * s);
        const int64_t s2 = std::min<int64_t>(s, d - (pairs - 1) * 2 * s - s);   // last pair's width, in (0, s]
        const int64_t nl = s2 < s ? s2 : 0;
        const int64_t step = 2 * s * (ld + 1);   // from pair p to pair p + 1 along the diagonal
        e = gemm_f64_batched(st, pairs, s, s, s, 1.0, U + s, ld, 1, step, W + s * ld + s, ld, 1, step, 0.0, tmp, s,
                             s * s, nl, nl, work, work_elems);
        if (e != hipSuccess) return e;
        e = gemm_f64_batched(st, pairs, s, s, s, -1.0, W, ld, 1, step, tmp, s, 1, s * s, 0.0, W + s, ld, step, nl,
                             0, work, work_elems);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t dense_fill_identity(hipStream_t st, double* A, int64_t d) {
    identity_kernel<<<(unsigned)ceil_div(d * d, 256), 256, 0, st>>>(A, d);
    return hipGetLastError();
}

hipError_t dense_convert(hipStream_t st, const void* src, int src_f32, int64_t rows, int64_t cols,
                         int64_t lds, double scale, double* dst, int64_t ldd) {
    const unsigned grid = (unsigned)ceil_div(rows * cols, 256);
    if (src_f32)
        convert_kernel<true><<<grid, 256, 0, st>>>(src, rows, cols, lds, scale, dst, ldd);
    else
        convert_kernel<false><<<grid, 256, 0, st>>>(src, rows, cols, lds, scale, dst, ldd);
    return hipGetLastError();
}

hipError_t dense_add_trace_shift(hipStream_t st, double* G, int64_t d, double factor) {
    trace_shift_kernel<<<1, 256, 0, st>>>(G, d, factor);
    return hipGetLastError();
}

hipError_t dense_status_reset(hipStream_t st, DenseStatus* status) {
    status_reset_kernel<<<1, 1, 0, st>>>(status);
    return hipGetLastError();
}

}  // namespace spcg
