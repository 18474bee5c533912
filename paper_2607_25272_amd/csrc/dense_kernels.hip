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
};

template <bool F32>
__device__ __forceinline__ double ld_elem(const void* p, int64_t idx) {
    if (F32) return (double)static_cast<const float*>(p)[idx];
    return static_cast<const double*>(p)[idx];
}

template <bool AF32, bool BF32>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    const int64_t ti = blockIdx.y, tj = blockIdx.x;
    if (g.upper && ti > tj) return;
    __shared__ double As[GK][GT + 1];
    __shared__ double Bs[GK][GT + 1];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int64_t i0 = ti * GT, j0 = tj * GT;
    double acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
    const bool a_icontig = g.sai == 1;
    const bool b_jcontig = g.sbj == 1;
    const int64_t kbeg = (int64_t)blockIdx.z * g.kchunk;
    const int64_t kend = min(g.K, kbeg + g.kchunk);
    for (int64_t l0 = kbeg; l0 < kend; l0 += GK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * 256;
            int i, l;
            if (a_icontig) {
                i = e & 63;
                l = e >> 6;
            } else {
                l = e & 15;
                i = e >> 4;
            }
            const int64_t gi = i0 + i, gl = l0 + l;
            As[l][i] = (gi < g.M && gl < kend) ? ld_elem<AF32>(g.A, gi * g.sai + gl * g.sal) : 0.0;
            int j;
            if (b_jcontig) {
                j = e & 63;
                l = e >> 6;
            } else {
                l = e & 15;
                j = e >> 4;
            }
            const int64_t gj = j0 + j, gl2 = l0 + l;
            Bs[l][j] = (gj < g.N && gl2 < kend) ? ld_elem<BF32>(g.B, gl2 * g.sbl + gj * g.sbj) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < GK; ++l) {
            double av[4], bv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) av[r] = As[l][ty * 4 + r];
#pragma unroll
            for (int c = 0; c < 4; ++c) bv[c] = Bs[l][tx * 4 + c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = fma(av[r], bv[c], acc[r][c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + ty * 4 + r;
        if (gi >= g.M) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t gj = j0 + tx * 4 + c;
            if (gj >= g.N) continue;
            if (g.part) {
                g.part[((int64_t)blockIdx.z * g.M + gi) * g.N + gj] = acc[r][c];
                continue;
            }
            double* cp = g.C + gi * g.ldc + gj;
            const double v = g.alpha * acc[r][c];
            *cp = g.beta == 0.0 ? v : fma(g.beta, *cp, v);
        }
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

// Unblocked upper Cholesky of the nb x nb diagonal block at (k0, k0).
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* G, int64_t ld, int64_t k0, int nb,
                                                         DenseStatus* st) {
    __shared__ double T[CB][CB + 1];
    __shared__ double piv_sh;
    const int tid = threadIdx.x;
    double min_piv = 0.0, min_d = 0.0, max_d = 0.0;
    int first_fail = 0;
    if (tid == 0) {
        min_piv = st->min_pivot;
        min_d = st->min_diag;
        max_d = st->max_diag;
        first_fail = st->fail;
    }
    for (int e = tid; e < nb * nb; e += 256) {
        const int i = e / nb, j = e - i * nb;
        T[i][j] = (j >= i) ? G[(k0 + i) * ld + k0 + j] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (tid == 0) {
            double piv = T[j][j];
            min_piv = piv < min_piv ? piv : min_piv;
            if (!(piv > 0.0) || !__builtin_isfinite(piv)) {
                if (first_fail == 0) first_fail = (int)(k0 + j) + 1;
                piv = 1.0;
            }
            const double u = sqrt(piv);
            T[j][j] = u;
            min_d = u < min_d ? u : min_d;
            max_d = u > max_d ? u : max_d;
            piv_sh = u;
        }
        __syncthreads();
        const double u = piv_sh;
        for (int l = j + 1 + tid; l < nb; l += 256) T[j][l] /= u;
        __syncthreads();
        const int rem = nb - j - 1;
        for (int e = tid; e < rem * rem; e += 256) {
            const int i = j + 1 + e / rem, l = j + 1 + e % rem;
            if (l >= i) T[i][l] = fma(-T[j][i], T[j][l], T[i][l]);
        }
        __syncthreads();
    }
    for (int e = tid; e < nb * nb; e += 256) {
        const int i = e / nb, j = e - i * nb;
        G[(k0 + i) * ld + k0 + j] = (j >= i) ? T[i][j] : 0.0;
    }
    if (tid == 0) {
        st->min_pivot = min_piv;
        st->min_diag = min_d;
        st->max_diag = max_d;
        st->fail = first_fail;
    }
}

// Row panel of the Cholesky: G[k0:k0+nb, c] <- U_kk^{-T} G[k0:k0+nb, c] for
// every column c >= k0 + nb (one thread per column).
__global__ __launch_bounds__(64) void chol_panel_kernel(double* G, int64_t ld, int64_t k0, int nb,
                                                        int64_t d) {
    __shared__ double U[CB][CB + 1];
    __shared__ double Y[CB][64];
    const int tid = threadIdx.x;
    for (int e = tid; e < nb * nb; e += 64) {
        const int i = e / nb, j = e - i * nb;
        U[i][j] = G[(k0 + i) * ld + k0 + j];
    }
    __syncthreads();
    const int64_t c = k0 + nb + (int64_t)blockIdx.x * 64 + tid;
    const bool ok = c < d;
    for (int i = 0; i < nb; ++i) Y[i][tid] = ok ? G[(k0 + i) * ld + c] : 0.0;
    if (!ok) return;
    for (int i = 0; i < nb; ++i) {
        double v = Y[i][tid];
        for (int l = 0; l < i; ++l) v = fma(-U[l][i], Y[l][tid], v);
        Y[i][tid] = v / U[i][i];
    }
    for (int i = 0; i < nb; ++i) G[(k0 + i) * ld + c] = Y[i][tid];
}

// A[i, k0:k0+nb] <- A[i, k0:k0+nb] U_kk^{-1} (one thread per row).
__global__ __launch_bounds__(64) void trsm_rows_kernel(double* A, int64_t n, int64_t lda,
                                                       const double* U, int64_t ldu, int64_t k0,
                                                       int nb) {
    __shared__ double Us[CB][CB + 1];
    __shared__ double Q[CB][64];
    const int tid = threadIdx.x;
    for (int e = tid; e < nb * nb; e += 64) {
        const int i = e / nb, j = e - i * nb;
        Us[i][j] = U[(k0 + i) * ldu + k0 + j];
    }
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    for (int e = tid; e < 64 * nb; e += 64) {
        const int rr = e / nb, j = e - rr * nb;
        Q[j][rr] = (i0 + rr < n) ? A[(i0 + rr) * lda + k0 + j] : 0.0;
    }
    __syncthreads();
    if (i0 + tid < n) {
        for (int j = 0; j < nb; ++j) {
            double v = Q[j][tid];
            for (int l = 0; l < j; ++l) v = fma(-Q[l][tid], Us[l][j], v);
            Q[j][tid] = v / Us[j][j];
        }
    }
    __syncthreads();
    for (int e = tid; e < 64 * nb; e += 64) {
        const int rr = e / nb, j = e - rr * nb;
        if (i0 + rr < n) A[(i0 + rr) * lda + k0 + j] = Q[j][rr];
    }
}

__global__ void zero_lower_kernel(double* G, int64_t d, int64_t ld) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= d * d) return;
    const int64_t i = e / d, j = e - i * d;
    if (j < i) G[i * ld + j] = 0.0;
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

hipError_t gemm_f64(hipStream_t st, int64_t M, int64_t N, int64_t K, double alpha, const void* A,
                    int a_f32, int64_t sai, int64_t sal, const void* B, int b_f32, int64_t sbl,
                    int64_t sbj, double beta, double* C, int64_t ldc, int upper, double* work,
                    int64_t work_elems) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int64_t ti = ceil_div(M, GT), tj = ceil_div(N, GT);
    const int64_t tiles = upper ? (ti * (ti + 1)) / 2 : ti * tj;
    // split K until there are about 512 blocks, keeping >= 128 per chunk
    int64_t nz = 1;
    while (work && tiles * nz * 2 <= 512 && K / (nz * 2) >= 128 && (nz * 2) * M * N <= work_elems) nz *= 2;
    const int64_t kchunk = round_up(ceil_div(K, nz), GK);
    nz = ceil_div(K, kchunk);
    if (nz < 1) nz = 1;
    GemmArgs g{M, N, K, alpha, beta, A, sai, sal, B, sbl, sbj, C, ldc, upper,
               kchunk, nz > 1 ? work : nullptr};
    dim3 grid((unsigned)tj, (unsigned)ti, (unsigned)nz), block(256);
    if (a_f32 && b_f32)
        gemm_kernel<true, true><<<grid, block, 0, st>>>(g);
    else if (a_f32)
        gemm_kernel<true, false><<<grid, block, 0, st>>>(g);
    else if (b_f32)
        gemm_kernel<false, true><<<grid, block, 0, st>>>(g);
    else
        gemm_kernel<false, false><<<grid, block, 0, st>>>(g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nz == 1) return e;
    splitk_reduce_kernel<<<(unsigned)ceil_div(M * N, 256), 256, 0, st>>>(work, (int)nz, M, N, alpha,
                                                                         beta, C, ldc, upper);
    return hipGetLastError();
}

hipError_t cholesky_upper(hipStream_t st, double* G, int64_t d, int64_t ld, DenseStatus* status) {
    hipError_t e;
    for (int64_t k0 = 0; k0 < d; k0 += CB) {
        const int nb = (int)std::min<int64_t>(CB, d - k0);
        potrf_diag_kernel<<<1, 256, 0, st>>>(G, ld, k0, nb, status);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int64_t rem = d - k0 - nb;
        if (rem > 0) {
            chol_panel_kernel<<<(unsigned)ceil_div(rem, 64), 64, 0, st>>>(G, ld, k0, nb, d);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            double* P = G + k0 * ld + k0 + nb;
            e = gemm_f64(st, rem, rem, nb, -1.0, P, 0, 1, ld, P, 0, ld, 1, 1.0,
                         G + (k0 + nb) * ld + k0 + nb, ld, 1, nullptr, 0);
            if (e != hipSuccess) return e;
        }
    }
    zero_lower_kernel<<<(unsigned)ceil_div(d * d, 256), 256, 0, st>>>(G, d, ld);
    return hipGetLastError();
}

hipError_t trsm_right_upper(hipStream_t st, double* A, int64_t n, int64_t d, int64_t lda,
                            const double* U, int64_t ldu, double* work, int64_t work_elems) {
    hipError_t e;
    for (int64_t k0 = 0; k0 < d; k0 += CB) {
        const int nb = (int)std::min<int64_t>(CB, d - k0);
        if (k0 > 0) {
            e = gemm_f64(st, n, nb, k0, -1.0, A, 0, lda, 1, U + k0, 0, ldu, 1, 1.0, A + k0, lda, 0,
                         work, work_elems);
            if (e != hipSuccess) return e;
        }
        trsm_rows_kernel<<<(unsigned)ceil_div(n, 64), 64, 0, st>>>(A, n, lda, U, ldu, k0, nb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
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
