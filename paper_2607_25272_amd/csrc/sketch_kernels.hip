// Nested SRHT on gfx950: randomness tables and the multi-pass
// Walsh-Hadamard transform with the row gather (P, D) fused into the first
// pass and the nested row selection (I_K, I_hat) fused into the last one.
//
// Z = H_un D P X-tilde (Sec. 2.1 SRHT, Sec. 2.2 one transform for all
// nested sketches).  Stage s of the transform (s = 0 first) pairs rows k and
// k + 2^s and maps (a, b) -> (a + b, a - b).  The L stages are split into
// passes of at most NB_MAX consecutive bits; a pass over bits [lo, lo + nb)
// loads tiles of 2^nb rows (stride 2^lo) x CW columns into LDS and runs its
// stages in order, so every element goes through the same additions in the
// same order as a stage-by-stage transform.
#include "common.hpp"
#include "internal.hpp"
#include "rng.hpp"

namespace spcg {

namespace {

constexpr int NB_MAX = 11;       // bits per pass: 2^11 rows x 64 B = 128 KB of LDS
constexpr int FWHT_THREADS = 1024;

__global__ void tables_kernel(uint64_t seed, int L, int64_t np, int64_t mK, int64_t r,
                              int32_t* perm_sign, int32_t* inv_slot, int32_t* inv_hat) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    uint64_t uk = (uint64_t)k;
    uint32_t pk = (uint32_t)feistel_fwd(uk, L, seed, STREAM_P);
    uint32_t sb = sign_bit(seed, uk);
    perm_sign[k] = (int32_t)(pk | (sb << 31));
    if (inv_slot) {
        int64_t t = (int64_t)feistel_inv(uk, L, seed, STREAM_PI);
        inv_slot[k] = t < mK ? (int32_t)t : -1;
    }
    if (inv_hat) {
        int64_t t = (int64_t)feistel_inv(uk, L, seed, STREAM_PIHAT);
        inv_hat[k] = t < r ? (int32_t)t : -1;
    }
}

__global__ void export_kernel(uint64_t seed, int L, int64_t np, int64_t mK, int64_t r,
                              int32_t* slot_rows, int32_t* hat_rows, int32_t* input_perm,
                              uint8_t* sign_bits) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot_rows && i < mK) slot_rows[i] = (int32_t)feistel_fwd((uint64_t)i, L, seed, STREAM_PI);
    if (hat_rows && i < r) hat_rows[i] = (int32_t)feistel_fwd((uint64_t)i, L, seed, STREAM_PIHAT);
    if (input_perm && i < np) input_perm[i] = (int32_t)feistel_fwd((uint64_t)i, L, seed, STREAM_P);
    if (sign_bits && i < np / 8) {
        uint32_t byte = 0;
        for (int b = 0; b < 8; ++b) byte |= sign_bit(seed, (uint64_t)(i * 8 + b)) << b;
        sign_bits[i] = (uint8_t)byte;
    }
}

template <typename TIN>
struct InLoad;
template <>
struct InLoad<double> {
    __device__ static double get(const void* x, int64_t idx, const float*, int64_t) {
        return static_cast<const double*>(x)[idx];
    }
};
template <>
struct InLoad<float> {
    __device__ static float get(const void* x, int64_t idx, const float*, int64_t) {
        return static_cast<const float*>(x)[idx];
    }
};
template <>
struct InLoad<bf16_t> {
    __device__ static float get(const void* x, int64_t idx, const float*, int64_t) {
        return bf16_bits_to_f32(static_cast<const uint16_t*>(x)[idx]);
    }
};
template <>
struct InLoad<fp8_t> {
    __device__ static float get(const void* x, int64_t idx, const float* scale, int64_t col) {
        uint32_t v = static_cast<const uint8_t*>(x)[idx];
        // hardware OCP e4m3 -> f32 conversion of the low byte
        float f = __builtin_amdgcn_cvt_f32_fp8((int)v, 0);
        return f * scale[col];
    }
};

struct PassArgs {
    const void* x;
    int64_t ldx;
    const float* col_scale;
    int64_t N, d;
    const void* zin;
    void* zout;
    int64_t ldz;
    const int32_t* perm_sign;
    const int32_t* inv_slot;
    const int32_t* inv_hat;
    void* B;
    int64_t ldb;
    void* Bh;
    int64_t ldbh;
    int lo, nb;
    int64_t nchunks, ntiles;
};

// One block = one tile of 2^nb rows x CW columns.
template <typename TIN, typename TZ, int CW, bool FIRST, bool LAST>
__global__ __launch_bounds__(FWHT_THREADS) void fwht_pass_kernel(PassArgs a) {
    __shared__ TZ tile[(1 << NB_MAX) * CW];
    // Blocks are dispatched round-robin over the 8 XCDs; hand each XCD a
    // contiguous range of tiles so that the column chunks of one row group
    // (which share cache lines) meet in the same L2.
    int64_t bid = blockIdx.x, nblk = gridDim.x, tid;
    if ((nblk & 7) == 0) {
        tid = (bid & 7) * (nblk >> 3) + (bid >> 3);
    } else {
        tid = bid;
    }
    const int64_t o = tid / a.nchunks;
    const int64_t cc = tid - o * a.nchunks;
    const int nb = a.nb, lo = a.lo;
    const int64_t rows = 1ll << nb;
    const int64_t olo = o & ((1ll << lo) - 1);
    const int64_t ohi = o >> lo;
    const int64_t col0 = cc * CW;
    const int64_t nelem = rows * CW;

    // load
    for (int64_t e = threadIdx.x; e < nelem; e += FWHT_THREADS) {
        int64_t j = e / CW;
        int c = (int)(e - j * CW);
        int64_t k = (ohi << (lo + nb)) | (j << lo) | olo;
        int64_t col = col0 + c;
        TZ v = TZ(0);
        if (FIRST) {
            int32_t ps = a.perm_sign[k];
            int64_t src = (int64_t)(ps & 0x7fffffff);
            if (src < a.N && col < a.d) {
                v = (TZ)InLoad<TIN>::get(a.x, src * a.ldx + col, a.col_scale, col);
                if (ps < 0) v = -v;
            }
        } else {
            v = static_cast<const TZ*>(a.zin)[k * a.ldz + col];
        }
        tile[e] = v;
    }
    __syncthreads();
    // stages lo .. lo+nb-1 (local bit t)
    const int64_t npairs = (rows >> 1) * CW;
    for (int t = 0; t < nb; ++t) {
        const int64_t h = 1ll << t;
        for (int64_t e = threadIdx.x; e < npairs; e += FWHT_THREADS) {
            int64_t q = e / CW;
            int c = (int)(e - q * CW);
            int64_t j = ((q >> t) << (t + 1)) | (q & (h - 1));
            TZ u = tile[j * CW + c];
            TZ w = tile[(j + h) * CW + c];
            tile[j * CW + c] = u + w;
            tile[(j + h) * CW + c] = u - w;
        }
        __syncthreads();
    }
    // store
    for (int64_t e = threadIdx.x; e < nelem; e += FWHT_THREADS) {
        int64_t j = e / CW;
        int c = (int)(e - j * CW);
        int64_t k = (ohi << (lo + nb)) | (j << lo) | olo;
        int64_t col = col0 + c;
        TZ v = tile[e];
        if (LAST) {
            if (a.inv_slot) {
                int32_t t = a.inv_slot[k];
                if (t >= 0 && col < a.ldb) static_cast<TZ*>(a.B)[(int64_t)t * a.ldb + col] = v;
            }
            if (a.inv_hat) {
                int32_t t = a.inv_hat[k];
                if (t >= 0 && col < a.ldbh) static_cast<TZ*>(a.Bh)[(int64_t)t * a.ldbh + col] = v;
            }
        } else {
            static_cast<TZ*>(a.zout)[k * a.ldz + col] = v;
        }
    }
}

template <typename TIN, typename TZ, int CW>
hipError_t run_passes(hipStream_t st, const FwhtJob& job) {
    const int L = job.L;
    const int passes = (L + NB_MAX - 1) / NB_MAX;
    PassArgs a{};
    a.x = job.x;
    a.ldx = job.ldx;
    a.col_scale = job.col_scale;
    a.N = job.N;
    a.d = job.d;
    a.ldz = job.ldz;
    a.perm_sign = job.perm_sign;
    a.inv_slot = job.inv_slot;
    a.inv_hat = job.inv_hat;
    a.B = job.B;
    a.ldb = job.ldb;
    a.Bh = job.Bh;
    a.ldbh = job.ldbh;
    a.nchunks = job.ldz / CW;
    int lo = 0;
    for (int pi = 0; pi < passes; ++pi) {
        int nb = L / passes + (pi < L % passes ? 1 : 0);
        a.lo = lo;
        a.nb = nb;
        a.ntiles = (1ll << (L - nb)) * a.nchunks;
        a.zin = job.zbuf;
        a.zout = job.zbuf;
        bool first = pi == 0, last = pi == passes - 1;
        dim3 grid((unsigned)a.ntiles), block(FWHT_THREADS);
        if (first && last)
            fwht_pass_kernel<TIN, TZ, CW, true, true><<<grid, block, 0, st>>>(a);
        else if (first)
            fwht_pass_kernel<TIN, TZ, CW, true, false><<<grid, block, 0, st>>>(a);
        else if (last)
            fwht_pass_kernel<TIN, TZ, CW, false, true><<<grid, block, 0, st>>>(a);
        else
            fwht_pass_kernel<TIN, TZ, CW, false, false><<<grid, block, 0, st>>>(a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        lo += nb;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_sketch_tables(hipStream_t st, uint64_t seed, int L, int64_t mK, int64_t r,
                                int32_t* perm_sign, int32_t* inv_slot, int32_t* inv_hat) {
    int64_t np = 1ll << L;
    tables_kernel<<<(unsigned)ceil_div(np, 256), 256, 0, st>>>(seed, L, np, mK, r, perm_sign,
                                                                inv_slot, inv_hat);
    return hipGetLastError();
}

hipError_t launch_sketch_export(hipStream_t st, uint64_t seed, int L, int64_t mK, int64_t r,
                                int32_t* slot_rows, int32_t* hat_rows, int32_t* input_perm,
                                uint8_t* sign_bits) {
    int64_t np = 1ll << L;
    int64_t n = np;
    if (mK > n) n = mK;
    if (r > n) n = r;
    export_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(seed, L, np, mK, r, slot_rows,
                                                              hat_rows, input_perm, sign_bits);
    return hipGetLastError();
}

hipError_t run_fwht(hipStream_t st, const FwhtJob& job) {
    const int cw = fwht_chunk_cols(job.in_dtype, job.narrow);
    if (job.ldz % cw != 0 || (job.B && job.ldb != job.ldz) || (job.Bh && job.ldbh != job.ldz) ||
        job.ldz < job.d || job.L < 1 || job.L > 30)
        return hipErrorInvalidValue;
    if (job.narrow) {
        if (job.in_dtype != DT_F64 || job.d != 1) return hipErrorInvalidValue;
        return run_passes<double, double, 1>(st, job);
    }
    switch (job.in_dtype) {
        case DT_F64: return run_passes<double, double, 8>(st, job);
        case DT_F32: return run_passes<float, float, 16>(st, job);
        case DT_BF16: return run_passes<bf16_t, float, 16>(st, job);
        case DT_FP8: return run_passes<fp8_t, float, 16>(st, job);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace spcg
