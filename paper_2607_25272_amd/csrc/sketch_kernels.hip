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
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"
#include "rng.hpp"

namespace spcg {

namespace {

constexpr int NB_MAX = 11;       // bits per transform pass

// Round-function tables of n <= 3 Feistel streams (see feistel_table_entry),
// table i at rt + i feistel_table_size(L).
__global__ void feistel_table_kernel(uint64_t seed, int L, int n, uint64_t s0, uint64_t s1, uint64_t s2,
                                     uint32_t* rt) {
    const int64_t ts = feistel_table_size(L);
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * ts) return;
    const int i = (int)(e / ts);
    const uint64_t stream = i == 0 ? s0 : (i == 1 ? s1 : s2);
    rt[e] = feistel_table_entry(e - i * ts, L, seed, stream);
}

// 256 threads per block: the block's rows k share k >> 8, so one Philox call
// of the sign stream (thread 0, through LDS) gives all their signs.
__global__ __launch_bounds__(256) void tables_kernel(uint64_t seed, int L, int64_t np, int64_t mK, int64_t r,
                                                     int32_t* perm_sign, int32_t* inv_slot, int32_t* inv_hat,
                                                     const uint32_t* rt_p, const uint32_t* rt_pi,
                                                     const uint32_t* rt_pihat, int2* pair_t, int plo,
                                                     uint32_t* row_masks, int64_t N) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool in = k < np;
    if (perm_sign) {
        __shared__ uint64_t sw[4];
        if (threadIdx.x == 0) {
            const Philox4 w = philox4x64_10((uint64_t)blockIdx.x, 0, 0, 0, seed, STREAM_SIGN);
#pragma unroll
            for (int i = 0; i < 4; ++i) sw[i] = w.v[i];
        }
        __syncthreads();
        uint32_t sb = 0, pk = 0;
        if (in) {
            const uint32_t b = (uint32_t)(k & 255);
            sb = (uint32_t)((sw[b >> 6] >> (b & 63)) & 1ull);
            pk = feistel_fwd_tab((uint32_t)k, L, rt_p);
            perm_sign[k] = (int32_t)(pk | (sb << 31));
        }
        if (row_masks) {
            // 16-row groups are 16-lane groups of the wave (np >= 16 rows)
            const uint64_t sbits = __ballot(in && sb);
            const uint64_t vbits = __ballot(in && (int64_t)pk < N);
            const int g = (threadIdx.x & 63) >> 4;
            if (in && (threadIdx.x & 15) == 0)
                row_masks[k >> 4] = (uint32_t)((sbits >> (16 * g)) & 0xffffu) |
                                    ((uint32_t)((vbits >> (16 * g)) & 0xffffu) << 16);
        }
    }
    if (!in) return;
    int32_t s_slot = -1, s_hat = -1;
    if (inv_slot) {
        const int64_t t = feistel_inv_tab((uint32_t)k, L, rt_pi);
        s_slot = t < mK ? (int32_t)t : -1;
        inv_slot[k] = s_slot;
    }
    if (inv_hat) {
        const int64_t t = feistel_inv_tab((uint32_t)k, L, rt_pihat);
        s_hat = t < r ? (int32_t)t : -1;
        inv_hat[k] = s_hat;
    }
    if (pair_t) pair_t[((k & ((1ll << plo) - 1)) << (L - plo)) | (k >> plo)] = make_int2(s_slot, s_hat);
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

// Widening loads of the stored input: VL consecutive elements of one row.
template <typename TIN, typename TZ, int VL>
struct InVec;
template <int VL>
struct InVec<double, double, VL> {
    __device__ static void scalar(const void* x, int64_t idx, const float*, int64_t, double* o) {
        o[0] = static_cast<const double*>(x)[idx];
    }
    __device__ static void vec(const void* x, int64_t idx, const float*, int64_t, double* o) {
        const double2 v = *reinterpret_cast<const double2*>(static_cast<const double*>(x) + idx);
        o[0] = v.x;
        o[1] = v.y;
    }
};
template <int VL>
struct InVec<float, float, VL> {
    __device__ static void scalar(const void* x, int64_t idx, const float*, int64_t, float* o) {
        o[0] = static_cast<const float*>(x)[idx];
    }
    __device__ static void vec(const void* x, int64_t idx, const float*, int64_t, float* o) {
        const float4 v = *reinterpret_cast<const float4*>(static_cast<const float*>(x) + idx);
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
};
template <int VL>
struct InVec<bf16_t, float, VL> {
    __device__ static void scalar(const void* x, int64_t idx, const float*, int64_t, float* o) {
        o[0] = bf16_bits_to_f32(static_cast<const uint16_t*>(x)[idx]);
    }
    __device__ static void vec(const void* x, int64_t idx, const float*, int64_t, float* o) {
        const uint2 v = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(x) + idx);
        o[0] = __uint_as_float(v.x << 16);
        o[1] = __uint_as_float(v.x & 0xffff0000u);
        o[2] = __uint_as_float(v.y << 16);
        o[3] = __uint_as_float(v.y & 0xffff0000u);
    }
};
typedef float fwht_v2f __attribute__((ext_vector_type(2)));
template <int VL>
struct InVec<fp8_t, float, VL> {
    __device__ static void scalar(const void* x, int64_t idx, const float* sc, int64_t col, float* o) {
        const uint32_t v = static_cast<const uint8_t*>(x)[idx];
        o[0] = __builtin_amdgcn_cvt_f32_fp8((int)v, 0) * sc[col];
    }
    __device__ static void vec(const void* x, int64_t idx, const float* sc, int64_t col, float* o) {
        const int w = (int)*reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(x) + idx);
        const fwht_v2f lo = __builtin_amdgcn_cvt_pk_f32_fp8(w, false);
        const fwht_v2f hi = __builtin_amdgcn_cvt_pk_f32_fp8(w, true);
        o[0] = lo.x * sc[col];
        o[1] = lo.y * sc[col + 1];
        o[2] = hi.x * sc[col + 2];
        o[3] = hi.y * sc[col + 3];
    }
};

// Four floats rounded to nearest even bfloat16, one 8-byte store.
__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ void bf16_store4(uint16_t* p, const float* o) {
    const uint32_t w0 = f32_to_bf16_rne(o[0]) | (f32_to_bf16_rne(o[1]) << 16);
    const uint32_t w1 = f32_to_bf16_rne(o[2]) | (f32_to_bf16_rne(o[3]) << 16);
    *reinterpret_cast<uint2*>(p) = make_uint2(w0, w1);
}

template <typename TZ>
struct ZVec;
template <>
struct ZVec<float> {
    static constexpr int VL = 4;
    __device__ static void ld(const float* p, float* o) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
    __device__ static void st(float* p, const float* o) {
        *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
    }
};
template <>
struct ZVec<double> {
    static constexpr int VL = 2;
    __device__ static void ld(const double* p, double* o) {
        const double2 v = *reinterpret_cast<const double2*>(p);
        o[0] = v.x;
        o[1] = v.y;
    }
    __device__ static void st(double* p, const double* o) {
        *reinterpret_cast<double2*>(p) = make_double2(o[0], o[1]);
    }
};

struct PassArgs {
    const void* x;
    int64_t ldx;
    const void* x_last;   // first pass, 16-byte loads of rows only 4-byte aligned: padded copy of row N - 1
    const float* col_scale;
    int64_t N, d;
    int xvec;          // X rows allow aligned VL-element loads
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
    int b_bf16;        // store B rows as BF16
    const int2* slot_pairs;   // split last pass: (inv_slot, inv_hat) per row, tile-contiguous
    const uint32_t* row_masks;   // split first pass: sign / validity bits of 16 rows per word
    int lo, nb, q;
    int64_t nchunks, ntiles;
    // chunk-major Z of a two-pass streaming transform (zt_hibits > 0): the
    // element (k, col) sits at ((chunk << lobits | k_lo) << hibits | k_hi) * CW
    // + col mod CW with k = k_hi 2^lobits + k_lo, so that a last-pass tile
    // (fixed k_lo and chunk) is one contiguous block
    int zt_lobits, zt_hibits;
};

// One block = one tile of 2^nb rows x CW columns.
//
// Lane layout: LPR = CW / VL lanes cover one tile row with VL-element
// (16-byte) vectors; each thread holds R = 2^q tile rows of its VL columns
// in registers: the rows that differ only in a q-bit window of the row
// index.  The bits of the pass are processed in groups of at most q bits,
// low group first; inside a group the butterflies run in registers in
// ascending bit order, and between groups the tile goes once through LDS
// (one vector element at a time) to re-slice it along the next group's
// bits.  For the last, narrower group the window is widened downwards with
// already-finished bits so that every thread always holds R rows.
template <typename TIN, typename TZ, int CW, bool FIRST, bool LAST, int QMAX>
__global__ __launch_bounds__(QMAX == 5 ? 512 : 1024) void fwht_pass_kernel(PassArgs a) {
    constexpr int VL = CW == 1 ? 1 : ZVec<TZ>::VL;
    constexpr int LPR = CW / VL;
    constexpr int LPRP = LPR == 1 ? 1 : LPR + 1;   // padded LDS row (bank spreading)
    constexpr int RMAX = 1 << QMAX;
    extern __shared__ __align__(16) unsigned char fwht_lds[];
    TZ* lds = reinterpret_cast<TZ*>(fwht_lds);
    // Blocks are dispatched round-robin over the 8 XCDs; hand each XCD a
    // contiguous range of tiles so that the column chunks of one row group
    // (which share DRAM pages) are fetched by the same L2 close in time.
    int64_t bid = blockIdx.x, nblk = gridDim.x, tid;
    if ((nblk & 7) == 0) {
        tid = (bid & 7) * (nblk >> 3) + (bid >> 3);
    } else {
        tid = bid;
    }
    const int64_t o = tid / a.nchunks;
    const int64_t cc = tid - o * a.nchunks;
    const int nb = a.nb, lo = a.lo, q = a.q;
    const int R = 1 << q;
    const int64_t olo = o & ((1ll << lo) - 1);
    const int64_t ohi = o >> lo;
    const int lr = threadIdx.x % LPR;
    const int bidx = threadIdx.x / LPR;
    const int64_t col0 = cc * CW + lr * VL;

    auto tile_row = [&](int s0, int t) -> int {
        const int base = ((bidx >> s0) << (s0 + q)) | (bidx & ((1 << s0) - 1));
        return base | (t << s0);
    };
    auto global_row = [&](int j) -> int64_t { return (ohi << (lo + nb)) | ((int64_t)j << lo) | olo; };
    // element offset of Z(k, col) (row-major, or chunk-major as described
    // at PassArgs)
    auto zoff = [&](int64_t k, int64_t col) -> int64_t {
        if (a.zt_hibits == 0) return k * a.ldz + col;
        const int64_t klo = k & ((1ll << a.zt_lobits) - 1), khi = k >> a.zt_lobits;
        return ((((col / CW) << a.zt_lobits) | klo) << a.zt_hibits | khi) * CW + col % CW;
    };

    TZ v[RMAX][VL];
    // ---- load (window = bits [0, q))
    if (FIRST) {
        int32_t ps[RMAX];
#pragma unroll
        for (int t = 0; t < RMAX; ++t)
            if (t < R) ps[t] = a.perm_sign[global_row(tile_row(0, t))];
        const bool full = a.xvec && col0 + VL <= a.d;
#pragma unroll
        for (int t = 0; t < RMAX; ++t) {
            if (t < R) {
                const int64_t src = (int64_t)(ps[t] & 0x7fffffff);
#pragma unroll
                for (int e = 0; e < VL; ++e) v[t][e] = TZ(0);
                if (src < a.N) {
                    if (full) {
                        InVec<TIN, TZ, VL>::vec(a.x, src * a.ldx + col0, a.col_scale, col0, v[t]);
                    } else {
#pragma unroll
                        for (int e = 0; e < VL; ++e)
                            if (col0 + e < a.d)
                                InVec<TIN, TZ, VL>::scalar(a.x, src * a.ldx + col0 + e, a.col_scale,
                                                           col0 + e, &v[t][e]);
                    }
                    if (ps[t] < 0) {
#pragma unroll
                        for (int e = 0; e < VL; ++e) v[t][e] = -v[t][e];
                    }
                }
            }
        }
    } else {
#pragma unroll
        for (int t = 0; t < RMAX; ++t) {
            if (t < R) {
                const TZ* p = static_cast<const TZ*>(a.zin) + zoff(global_row(tile_row(0, t)), col0);
                if constexpr (VL == 1) {
                    v[t][0] = *p;
                } else {
                    ZVec<TZ>::ld(p, v[t]);
                }
            }
        }
    }
    int done = 0, s0 = 0;
    while (true) {
        const int w = min(q, nb - done);   // bits of this group
        const int e0 = q - w;              // finished bits below it in the window
        // butterflies on register-row bits [e0, e0 + w), ascending
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            if (b >= e0 && b < e0 + w && (1 << b) < R) {
#pragma unroll
                for (int t = 0; t < RMAX; ++t) {
                    if (t < R && !(t & (1 << b))) {
#pragma unroll
                        for (int e = 0; e < VL; ++e) {
                            const TZ x0 = v[t][e], x1 = v[t | (1 << b)][e];
                            v[t][e] = x0 + x1;
                            v[t | (1 << b)][e] = x0 - x1;
                        }
                    }
                }
            }
        }
        done += w;
        if (done >= nb) break;
        // re-slice through LDS for the next group, one vector element at a time
        const int wn = min(q, nb - done);
        const int s1 = done - (q - wn);
#pragma unroll
        for (int e = 0; e < VL; ++e) {
#pragma unroll
            for (int t = 0; t < RMAX; ++t)
                if (t < R) lds[tile_row(s0, t) * LPRP + lr] = v[t][e];
            __syncthreads();
#pragma unroll
            for (int t = 0; t < RMAX; ++t)
                if (t < R) v[t][e] = lds[tile_row(s1, t) * LPRP + lr];
            __syncthreads();
        }
        s0 = s1;
    }
    // ---- store
#pragma unroll
    for (int t = 0; t < RMAX; ++t) {
        if (t < R) {
            const int64_t k = global_row(tile_row(s0, t));
            if (LAST) {
                if (a.inv_slot) {
                    const int32_t sl = a.inv_slot[k];
                    if (sl >= 0) {
                        bool done_bf16 = false;
                        if constexpr (std::is_same<TZ, float>::value && VL == 4) {
                            if (a.b_bf16) {
                                bf16_store4(static_cast<uint16_t*>(a.B) + (int64_t)sl * a.ldb + col0, v[t]);
                                done_bf16 = true;
                            }
                        }
                        if (!done_bf16) {
                            TZ* p = static_cast<TZ*>(a.B) + (int64_t)sl * a.ldb + col0;
                            if constexpr (VL == 1) *p = v[t][0]; else ZVec<TZ>::st(p, v[t]);
                        }
                    }
                }
                if (a.inv_hat) {
                    const int32_t sl = a.inv_hat[k];
                    if (sl >= 0) {
                        TZ* p = static_cast<TZ*>(a.Bh) + (int64_t)sl * a.ldbh + col0;
                        if constexpr (VL == 1) *p = v[t][0]; else ZVec<TZ>::st(p, v[t]);
                    }
                }
            } else {
                TZ* p = static_cast<TZ*>(a.zout) + zoff(k, col0);
                if constexpr (VL == 1) *p = v[t][0]; else ZVec<TZ>::st(p, v[t]);
            }
        }
    }
}

// Streaming form of a pass at FP32 working precision (FP32, BF16 and FP8
// input).  A persistent block of 512 threads walks a fixed share of the
// tiles; the next tile streams from HBM into an LDS staging buffer through
// direct global->LDS loads while the current one goes through its
// butterflies, LDS exchanges and stores, so every CU keeps reads and writes
// in flight while it computes.  Tiles are 2^NB rows x CW columns with 16 rows
// per thread: CW = 32 gives NB = 10 (the shape the library launches; CW = 16
// would give NB = 11).  The butterflies
// run in the same order as in fwht_pass_kernel (stages in ascending bit
// order, each (a, b) -> (a + b, a - b)), so both kernels give bit-identical
// results.
//
// Per tile j: barrier (the staged tile j is complete in every wave); each
// thread reads its rows from the staging buffer; barrier (staging free);
// the loads of tile j + 1 into the staging buffer (and, first pass, the
// permutation entries of the tiles after it) are issued; butterflies and
// LDS re-slicing run; then one vmcnt(0) wait -- by then the staged loads,
// issued a whole tile of work earlier, have landed -- and the stores of
// tile j, which drain during the next tile.
//
// Staging layout: row-major, ROWB bytes per tile row, with the row index
// XOR-swizzled in its low bits by bits 4.. (so the 16-row groups that one
// wave reads at a time fall into different LDS banks).  A direct load
// writes 16 bytes per lane at consecutive LDS addresses, so each lane picks
// the (row, 16-byte piece) that lands at its address.  Exchange buffer: one
// FP32 element per (row, lane), rows swizzled the same way.
constexpr int STREAM_THREADS = 512;
constexpr int stream_vmcnt0() { return (0x7 << 4) | (0xf << 8); }   // s_waitcnt vmcnt(0)

__device__ __forceinline__ void stream_lds_load16(const void* src, void* lds) {
    __builtin_amdgcn_global_load_lds(const_cast<void*>(src), (__attribute__((address_space(3))) void*)(lds),
                                     16, 0, 0);
}

template <typename TI>
struct StageRead;   // 4 consecutive staged elements of one row -> FP32; scales of columns >= d read as 0
template <>
struct StageRead<float> {
    __device__ static void rd(const unsigned char* p, const float*, int64_t, int64_t, float* o) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
};
template <>
struct StageRead<bf16_t> {
    __device__ static void rd(const unsigned char* p, const float*, int64_t, int64_t, float* o) {
        const uint2 v = *reinterpret_cast<const uint2*>(p);
        o[0] = __uint_as_float(v.x << 16);
        o[1] = __uint_as_float(v.x & 0xffff0000u);
        o[2] = __uint_as_float(v.y << 16);
        o[3] = __uint_as_float(v.y & 0xffff0000u);
    }
};
template <>
struct StageRead<fp8_t> {
    __device__ static void rd(const unsigned char* p, const float* sc, int64_t col, int64_t d, float* o) {
        const int w = (int)*reinterpret_cast<const uint32_t*>(p);
        const fwht_v2f lo = __builtin_amdgcn_cvt_pk_f32_fp8(w, false);
        const fwht_v2f hi = __builtin_amdgcn_cvt_pk_f32_fp8(w, true);
        o[0] = lo.x * (col < d ? sc[col] : 0.f);
        o[1] = lo.y * (col + 1 < d ? sc[col + 1] : 0.f);
        o[2] = hi.x * (col + 2 < d ? sc[col + 2] : 0.f);
        o[3] = hi.y * (col + 3 < d ? sc[col + 3] : 0.f);
    }
};

// First pass: address of the staged piece of X row sr at column col.
// Rows past N and pieces past d read row 0 instead (the reader zeroes
// them).  XL: 16-byte loads of rows that are only 4-byte aligned; a piece
// may then reach up to 12 bytes into the next row, and row N - 1 is read
// from its copy x_last, which is padded so that no load leaves it.
template <int IB, bool XL>
__device__ __forceinline__ const unsigned char* x_piece(const PassArgs& a, int64_t sr, int64_t col) {
    const bool ok = sr < a.N && col < a.d;
    if constexpr (XL) {
        const bool last = sr == a.N - 1;
        const unsigned char* base = static_cast<const unsigned char*>(last ? a.x_last : a.x);
        return base + (ok ? (last ? col : sr * a.ldx + col) * IB : 0);
    } else {
        return static_cast<const unsigned char*>(a.x) + (ok ? (sr * a.ldx + col) * IB : 0);
    }
}

template <typename TIN, int CW, bool FIRST, bool LAST, bool XL = false>
__global__ __launch_bounds__(STREAM_THREADS) void fwht_stream_kernel(PassArgs a) {
    constexpr int VL = 4, Q = 4, R = 16, THREADS = STREAM_THREADS;
    constexpr int LPR = CW / VL;
    constexpr int ROWS = THREADS * R / LPR;
    constexpr int NB = __builtin_ctz(ROWS);      // bits of the pass: 9 or 10 (11 would fit too)
    constexpr int NG = (NB + Q - 1) / Q;        // register groups of the pass
    typedef typename std::conditional<FIRST, TIN, float>::type TI;   // staged element
    constexpr int IB = (int)sizeof(TI);
    constexpr int ROWB = CW * IB;               // staged bytes per tile row
    constexpr int STG = ROWS * ROWB;
    constexpr int NI = STG / (THREADS * 16);    // direct loads per thread per tile
    constexpr int SM = ROWB < 256 ? 256 / ROWB - 1 : 0;   // staging row swizzle
    constexpr int XM = 64 / LPR - 1;                       // exchange row swizzle
    static_assert(ROWS == (1 << NB) && !(FIRST && LAST), "stream tile shape");
    static_assert(ROWB >= 16 && NI >= 1 && NI * THREADS * 16 == STG && SM < 16 && XM < 16, "staging");
    // two separate LDS objects: the compiler then knows that exchange
    // traffic does not touch the buffer the direct loads are filling
    __shared__ __align__(16) unsigned char stg[STG];
    __shared__ __align__(16) float exb[ROWS * LPR];

    // This block's tiles are first + j * stride, j < count.  Blocks are
    // dispatched round-robin over the 8 XCDs; XCD x takes the x-th eighth of
    // the tiles, so the column chunks of one row group (which share DRAM
    // pages) are fetched through the same L2 close in time.
    const int64_t T = a.ntiles;
    const int64_t G = gridDim.x;
    int64_t first, stride, count;
    if ((G & 7) == 0 && (T & 7) == 0) {
        const int64_t per = T >> 3, M = G >> 3, m = blockIdx.x >> 3;
        first = (int64_t)(blockIdx.x & 7) * per + m;
        stride = M;
        count = m < per ? (per - m + M - 1) / M : 0;
    } else {
        first = blockIdx.x;
        stride = G;
        count = (int64_t)blockIdx.x < T ? (T - blockIdx.x + G - 1) / G : 0;
    }
    if (count == 0) return;   // uniform over the block

    const int lo = a.lo;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lr = threadIdx.x % LPR;
    const int bidx = threadIdx.x / LPR;
    // bx: this thread's row-group index (bidx), passed in so that the loop
    // can hand over a copy the compiler may not hoist: LDS addresses are then
    // recomputed per tile instead of occupying registers for the whole loop
    auto tile_row = [](int bx, int s0, int t) -> int {
        const int base = ((bx >> s0) << (s0 + Q)) | (bx & ((1 << s0) - 1));
        return base | (t << s0);
    };
    auto srow = [](int row) -> int { return row ^ ((row >> 4) & SM); };   // an involution
    auto xrow = [](int row) -> int { return row ^ ((row >> 4) & XM); };
    struct Tile {
        int64_t rowbase;   // global row of tile row 0
        int64_t cbase;     // first column of the tile
    };
    auto tile_of = [&](int64_t j) -> Tile {
        const int64_t tix = first + j * stride;
        const int64_t o = tix / a.nchunks;
        const int64_t cc = tix - o * a.nchunks;
        const int64_t olo = o & ((1ll << lo) - 1);
        const int64_t ohi = o >> lo;
        return Tile{(ohi << (lo + NB)) | olo, cc * CW};
    };
    auto grow = [&](const Tile& tl, int r) -> int64_t { return tl.rowbase | ((int64_t)r << lo); };
    // element offset of Z(k, col)
    auto zoff = [&](int64_t k, int64_t col) -> int64_t {
        if (a.zt_hibits == 0) return k * a.ldz + col;
        const int64_t klo = k & ((1ll << a.zt_lobits) - 1), khi = k >> a.zt_lobits;
        return ((((col / CW) << a.zt_lobits) | klo) << a.zt_hibits | khi) * CW + col % CW;
    };
    // tile row and 16-byte piece that direct load i of this lane fetches
    auto dma_slot = [&](int i, int& row, int& piece) {
        const int P = ((wave * NI + i) * 64 + lane) * 16;
        row = srow(P / ROWB);
        piece = (P % ROWB) / 16;
    };

    int32_t dp[NI];   // first pass: permutation entries of the rows this lane stages next
    int32_t cp[R];    // first pass: permutation entries of this thread's rows
    auto load_dperm = [&](int64_t j) __attribute__((always_inline)) {
        const Tile tl = tile_of(j);
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            int row, piece;
            dma_slot(i, row, piece);
            dp[i] = a.perm_sign[grow(tl, row)];
        }
    };
    auto load_cperm = [&](int64_t j) __attribute__((always_inline)) {
        const Tile tl = tile_of(j);
#pragma unroll
        for (int t = 0; t < R; ++t) cp[t] = a.perm_sign[grow(tl, tile_row(bidx, 0, t))];
    };
    auto issue_stage = [&](int64_t j) __attribute__((always_inline)) {
        const Tile tl = tile_of(j);
        unsigned char* dst = stg + wave * NI * 1024;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            int row, piece;
            dma_slot(i, row, piece);
            const int64_t col = tl.cbase + piece * (16 / IB);
            const unsigned char* src;
            if constexpr (FIRST) {
                src = x_piece<IB, XL>(a, (int64_t)(dp[i] & 0x7fffffff), col);
            } else {
                src = static_cast<const unsigned char*>(a.zin) + zoff(grow(tl, row), col) * 4;
            }
            stream_lds_load16(src, dst + i * 1024);
        }
    };

    float v[R][VL];
    int32_t sl[R], sh[R];
    // prologue: stage tile 0
    if constexpr (FIRST) {
        load_dperm(0);
        load_cperm(0);
    }
    issue_stage(0);
    if constexpr (FIRST) {
        if (count > 1) load_dperm(1);
    }
    __builtin_amdgcn_s_waitcnt(stream_vmcnt0());

    for (int64_t j = 0; j < count; ++j) {
        const Tile tl = tile_of(j);
        int bx = bidx, lx = lr;
        asm volatile("" : "+v"(bx), "+v"(lx));
        __syncthreads();   // every wave has waited for its part of tile j
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int row = tile_row(bx, 0, t);
            const int64_t col0 = tl.cbase + lr * VL;
            float x[VL];
            StageRead<TI>::rd(stg + srow(row) * ROWB + lx * VL * IB, a.col_scale, col0, a.d, x);
            if constexpr (FIRST) {
                const bool valid = (int64_t)(cp[t] & 0x7fffffff) < a.N;
#pragma unroll
                for (int e = 0; e < VL; ++e) {
                    float y = col0 + e < a.d ? x[e] : 0.f;
                    if (cp[t] < 0) y = -y;
                    v[t][e] = valid ? y : 0.f;
                }
            } else {
#pragma unroll
                for (int e = 0; e < VL; ++e) v[t][e] = x[e];
            }
        }
        __syncthreads();   // staging buffer free
        if (j + 1 < count) issue_stage(j + 1);
        if constexpr (FIRST) {
            if (j + 1 < count) load_cperm(j + 1);
            if (j + 2 < count) load_dperm(j + 2);
        }
        if constexpr (LAST) {
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const int64_t k = grow(tl, tile_row(bidx, NB - Q, t));
                sl[t] = a.inv_slot ? a.inv_slot[k] : -1;
                sh[t] = a.inv_hat ? a.inv_hat[k] : -1;
            }
        }
        int done = 0, s0 = 0;
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            const int w = NB - done < Q ? NB - done : Q;
            const int e0 = Q - w;
#pragma unroll
            for (int b = 0; b < Q; ++b) {
                if (b >= e0 && b < e0 + w) {
#pragma unroll
                    for (int t = 0; t < R; ++t) {
                        if (!(t & (1 << b))) {
#pragma unroll
                            for (int e = 0; e < VL; ++e) {
                                const float x0 = v[t][e], x1 = v[t | (1 << b)][e];
                                v[t][e] = x0 + x1;
                                v[t | (1 << b)][e] = x0 - x1;
                            }
                        }
                    }
                }
            }
            done += w;
            if (gi + 1 < NG) {
                const int wn = NB - done < Q ? NB - done : Q;
                const int s1 = done - (Q - wn);
#pragma unroll
                for (int e = 0; e < VL; ++e) {
#pragma unroll
                    for (int t = 0; t < R; ++t) exb[xrow(tile_row(bx, s0, t)) * LPR + lx] = v[t][e];
                    __syncthreads();
#pragma unroll
                    for (int t = 0; t < R; ++t) v[t][e] = exb[xrow(tile_row(bx, s1, t)) * LPR + lx];
                    __syncthreads();
                }
                s0 = s1;
            }
        }
        // the staged loads of tile j + 1 (and the table loads) are complete
        // after this wait; the stores below drain during the next tile
        __builtin_amdgcn_s_waitcnt(stream_vmcnt0());
        const int64_t col0 = tl.cbase + lr * VL;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            if constexpr (LAST) {
                if (sl[t] >= 0) {
                    if (a.b_bf16) {
                        bf16_store4(static_cast<uint16_t*>(a.B) + (int64_t)sl[t] * a.ldb + col0, v[t]);
                    } else {
                        ZVec<float>::st(static_cast<float*>(a.B) + (int64_t)sl[t] * a.ldb + col0, v[t]);
                    }
                }
                if (sh[t] >= 0) ZVec<float>::st(static_cast<float*>(a.Bh) + (int64_t)sh[t] * a.ldbh + col0, v[t]);
            } else {
                ZVec<float>::st(static_cast<float*>(a.zout) + zoff(grow(tl, tile_row(bidx, NB - Q, t)), col0), v[t]);
            }
        }
    }
}

// 11-bit pass at FP32 working precision in persistent 1024-thread blocks
// (one per CU) with half-tile staging.  A tile is 2048 rows x 32 columns
// (128-byte row segments, 256 KB); it sits in registers (16 rows x 4
// columns per thread) while it is transformed, and LDS holds one half-tile
// of staged input (128 KB for FP32 rows) and a 32 KB exchange buffer.
//
// Row bits of a tile and where they live.  At load, thread (wave w, lane l)
// holds rows t | (l >> 3) << 4 | w << 7, t < 16 its register index, so
// stages 0..3 run on register bits, stages 4..6 on lane bits 3..5 and
// stages 7..10 on the wave index:
//   stage 4 (lane bit 3): the partner's value from a DPP row rotation by 8,
//            then fma(+-1, x, partner): x + p below, p - x above;
//   stage 5 (lane bit 4): v_permlane16_swap of registers t and t + 8 gives
//            both pairs' operands in place; their sum and difference are
//            the two results, which swaps row bit 5 into register bit 3 and
//            row bit 3 into lane bit 4;
//   stage 6 (lane bit 5): the same with v_permlane32_swap on registers t and
//            t + 4 (row bit 6 into register bit 2, row bit 2 into lane bit 5);
// then one exchange through LDS (per column element, two 32 KB rounds by
// row bit 2, which is lane bit 5 on both sides) brings row bits 7..10 into
// the registers, and stages 7..10 run there.  Every stage is the butterfly
// (a, b) -> (a + b, a - b) in ascending stage order, as in fwht_pass_kernel,
// so the output is bit-identical to it.
//
// Per tile j:
//   A  the first half (row bit 10 = 0, staged during tile j-1) goes to the
//      registers of waves 0..7; the direct loads of the second half are
//      issued into the freed staging buffer; waves 0..7 run stages 0..6;
//   B  once the second half has landed, waves 8..15 take it and run stages
//      0..6; the direct loads of the next tile's first half are issued;
//   C  the exchange, stages 7..10, one vmcnt(0) wait (the next first half
//      has landed), and the stores, which drain during the next A phase.
constexpr int SPLIT_THREADS = 1024;

template <typename TIN, bool FIRST, bool LAST, bool XL = false>
__global__ __launch_bounds__(SPLIT_THREADS) void fwht_split_kernel(PassArgs a) {
    constexpr int DW = 16;   // bytes per direct load
    constexpr int CW = 32, VL = 4, R = 16, THREADS = SPLIT_THREADS;
    constexpr int LPR = CW / VL;                 // 8 lanes per tile row
    constexpr int NB = 11, HALF = 1 << (NB - 1);
    typedef typename std::conditional<FIRST, TIN, float>::type TI;   // staged element
    constexpr int IB = (int)sizeof(TI);
    constexpr int ROWB = CW * IB;                // staged bytes per tile row
    constexpr int STG = HALF * ROWB;             // one half-tile
    constexpr int NI = STG / (THREADS * DW);     // direct loads of DW bytes per thread per half-tile
    constexpr int SM = ROWB < 256 ? 256 / ROWB - 1 : 0;
    static_assert(NI >= 1 && NI * THREADS * DW == STG && !(FIRST && LAST),
                  "split tile shape");
    __shared__ __align__(16) unsigned char stg[STG];
    __shared__ __align__(16) float exb[HALF * LPR];

    const int64_t T = a.ntiles;
    const int64_t G = gridDim.x;
    int64_t first, stride, count;
    if ((G & 7) == 0 && (T & 7) == 0) {
        const int64_t per = T >> 3, M = G >> 3, m = blockIdx.x >> 3;
        first = (int64_t)(blockIdx.x & 7) * per + m;
        stride = M;
        count = m < per ? (per - m + M - 1) / M : 0;
    } else {
        first = blockIdx.x;
        stride = G;
        count = (int64_t)blockIdx.x < T ? (T - blockIdx.x + G - 1) / G : 0;
    }
    if (count == 0) return;   // uniform over the block

    const int lo = a.lo;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int myhalf = wave >> 3;
    auto srow = [](int row) -> int { return row ^ ((row >> 4) & SM); };
    struct Tile {
        int64_t rowbase;
        int64_t cbase;
    };
    // tile index = o * nchunks + cc, walked incrementally (uniform scalars)
    auto tile_at = [&](int64_t o, int64_t cc) -> Tile {
        const int64_t olo = o & ((1ll << lo) - 1);
        const int64_t ohi = o >> lo;
        return Tile{(ohi << (lo + NB)) | olo, cc * CW};
    };
    const int64_t nch = a.nchunks;
    int64_t o_cur = first / nch, c_cur = first - (first / nch) * nch;
    auto advance = [&](int64_t& o, int64_t& c) {
        c += stride;
        while (c >= nch) {
            c -= nch;
            ++o;
        }
    };
    auto grow = [&](const Tile& tl, int r) -> int64_t { return tl.rowbase | ((int64_t)r << lo); };
    auto zoff = [&](int64_t k, int64_t col) -> int64_t {
        if (a.zt_hibits == 0) return k * a.ldz + col;
        const int64_t klo = k & ((1ll << a.zt_lobits) - 1), khi = k >> a.zt_lobits;
        return ((((col / CW) << a.zt_lobits) | klo) << a.zt_hibits | khi) * CW + col % CW;
    };
    // tile row of register t at load (stage bits 0..3 in registers); lx is
    // an opaque copy of the lane index (see the loop)
    auto load_row = [&](int t, int lx) -> int { return t | ((lx >> 3) << 4) | (wave << 7); };
    // tile row of register t after the exchange (stage bits 7..10 in registers)
    auto final_row = [&](int t, int lx) -> int {
        return (wave & 1) | ((wave >> 1) & 1) << 1 | (lx >> 5) << 2 | ((lx >> 4) & 1) << 3 | ((lx >> 3) & 1) << 4 |
               ((wave >> 2) & 1) << 5 | ((wave >> 3) & 1) << 6 | t << 7;
    };
    // half-tile row and DW-byte piece that direct load i of this lane fetches
    auto dma_slot = [&](int i, int lx, int& row, int& piece) {
        const int P = ((wave * NI + i) * 64 + lx) * DW;
        row = srow(P / ROWB);
        piece = (P % ROWB) / DW;
    };
    // first pass: the direct loads of wave w fetch the half-tile rows
    // [64 w, 64 w + 64); lane l loads the permutation entry of row 64 w + l
    // and each load's row entry comes from its lane by a cross-lane permute
    auto load_dperm = [&](const Tile& tl, int h, int lx) __attribute__((always_inline)) -> int32_t {
        return a.perm_sign[(uint32_t)grow(tl, h * HALF + wave * 64 + lx)];
    };
    // first pass: sign (bit t) and validity (bit 16 + t) of this thread's 16
    // consecutive rows, one word of the row-mask table
    auto load_cmask = [&](const Tile& tl, int lx) __attribute__((always_inline)) -> uint32_t {
        return a.row_masks[(uint32_t)grow(tl, load_row(0, lx)) >> 4];
    };
    auto issue_half = [&](const Tile& tl, int h, int32_t dp, int lx) __attribute__((always_inline)) {
        unsigned char* dst = stg + wave * NI * 64 * DW;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            int row, piece;
            dma_slot(i, lx, row, piece);
            const int64_t col = tl.cbase + piece * (DW / IB);
            const unsigned char* src;
            if constexpr (FIRST) {
                const int32_t pe = __builtin_amdgcn_ds_bpermute((row - wave * 64) << 2, dp);
                src = x_piece<IB, XL>(a, (int64_t)(pe & 0x7fffffff), col);
            } else {
                src = static_cast<const unsigned char*>(a.zin) + zoff(grow(tl, h * HALF + row), col) * 4;
            }
            stream_lds_load16(src, dst + i * 1024);
        }
    };

    float v[R][VL];
    // this thread's rows of its half from the staging buffer
    auto read_own = [&](const Tile& tl, uint32_t cm, int lx) __attribute__((always_inline)) {
        const int64_t col0 = tl.cbase + (lx & 7) * VL;
        const int base = (((wave & 7) << 3) | (lx >> 3)) << 4;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            float x[VL];
            StageRead<TI>::rd(stg + srow(base | t) * ROWB + (lx & 7) * VL * IB, a.col_scale, col0, a.d, x);
            if constexpr (FIRST) {
                const bool valid = (cm >> (16 + t)) & 1u;
                const bool neg = (cm >> t) & 1u;
#pragma unroll
                for (int e = 0; e < VL; ++e) {
                    float y = col0 + e < a.d ? x[e] : 0.f;
                    if (neg) y = -y;
                    v[t][e] = valid ? y : 0.f;
                }
            } else {
#pragma unroll
                for (int e = 0; e < VL; ++e) v[t][e] = x[e];
            }
        }
    };
    // stages on register bits [b0, b1), ascending
    auto bfly = [&](int b0, int b1) __attribute__((always_inline)) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (b >= b0 && b < b1) {
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    if (!(t & (1 << b))) {
#pragma unroll
                        for (int e = 0; e < VL; ++e) {
                            const float x0 = v[t][e], x1 = v[t | (1 << b)][e];
                            v[t][e] = x0 + x1;
                            v[t | (1 << b)][e] = x0 - x1;
                        }
                    }
                }
            }
        }
    };
    // stages 4..6 on the lane bits (see above)
    auto lane_stages = [&](int lx) __attribute__((always_inline)) {
        const float sg = (lx & 8) ? -1.f : 1.f;
#pragma unroll
        for (int t = 0; t < R; ++t) {
#pragma unroll
            for (int e = 0; e < VL; ++e) {
                const float p = __int_as_float(
                    __builtin_amdgcn_update_dpp(0, __float_as_int(v[t][e]), 0x128, 0xf, 0xf, false));
                v[t][e] = __builtin_fmaf(sg, v[t][e], p);
            }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
#pragma unroll
            for (int e = 0; e < VL; ++e) {
                const auto w = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[t][e]),
                                                                __float_as_uint(v[t + 8][e]), false, false);
                const float xn = __uint_as_float(w[0]), yn = __uint_as_float(w[1]);
                v[t][e] = xn + yn;
                v[t + 8][e] = xn - yn;
            }
        }
#pragma unroll
        for (int t = 0; t < R; ++t) {
            if (t & 4) continue;
#pragma unroll
            for (int e = 0; e < VL; ++e) {
                const auto w = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[t][e]),
                                                                __float_as_uint(v[t + 4][e]), false, false);
                const float xn = __uint_as_float(w[0]), yn = __uint_as_float(w[1]);
                v[t][e] = xn + yn;
                v[t + 4][e] = xn - yn;
            }
        }
    };
    // row bits 7..10 into the registers: per column element, two rounds by
    // row bit 2 (lane bit 5 before and after); exchange index of a row:
    // r3 | r4 << 1 | r0 << 2 | r1 << 3 | r5 << 4 | r6 << 5 | r7..r10 << 6
    auto exchange = [&](int lx) __attribute__((always_inline)) {
        const int lrx = lx & 7, x3 = (lx >> 3) & 1, x4 = (lx >> 4) & 1, x5 = lx >> 5;
        const int wbase = ((x4 | x3 << 1 | wave << 6) << 3) + lrx;
        const int rbase = ((x4 | x3 << 1 | wave << 2) << 3) + lrx;
#pragma unroll
        for (int e = 0; e < VL; ++e) {
#pragma unroll
            for (int rho = 0; rho < 2; ++rho) {
                const bool active = x5 == rho;
                if (active) {
#pragma unroll
                    for (int t = 0; t < R; ++t) {
                        const int off = ((t & 1) << 2 | ((t >> 1) & 1) << 3 | ((t >> 3) & 1) << 4 | ((t >> 2) & 1) << 5) << 3;
                        exb[wbase + off] = v[t][e];
                    }
                }
                __syncthreads();
                if (active) {
#pragma unroll
                    for (int t = 0; t < R; ++t) v[t][e] = exb[rbase + (t << 9)];
                }
                __syncthreads();
            }
        }
    };

    // completes every pending butterfly before this point (the scheduler
    // would otherwise sink the last stages into the store loop and keep
    // their partial sums live)
    auto settle = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int e = 0; e < VL; ++e)
            asm volatile("" : "+v"(v[0][e]), "+v"(v[1][e]), "+v"(v[2][e]), "+v"(v[3][e]), "+v"(v[4][e]),
                         "+v"(v[5][e]), "+v"(v[6][e]), "+v"(v[7][e]), "+v"(v[8][e]), "+v"(v[9][e]),
                         "+v"(v[10][e]), "+v"(v[11][e]), "+v"(v[12][e]), "+v"(v[13][e]), "+v"(v[14][e]),
                         "+v"(v[15][e]));
    };

    int32_t dpa = 0, dpb = 0;   // first pass: this lane's entry for the next first / second half-tile
    uint32_t cm = 0;            // first pass: sign and validity of this thread's rows
    {
        const Tile t0 = tile_at(o_cur, c_cur);
        if constexpr (FIRST) {
            dpa = load_dperm(t0, 0, lane);
            __builtin_amdgcn_s_waitcnt(stream_vmcnt0());
        }
        issue_half(t0, 0, dpa, lane);
        if constexpr (FIRST) {
            cm = load_cmask(t0, lane);
            dpb = load_dperm(t0, 1, lane);
        }
    }
    __builtin_amdgcn_s_waitcnt(stream_vmcnt0());

    for (int64_t j = 0; j < count; ++j) {
        const Tile tl = tile_at(o_cur, c_cur);
        int64_t o_nx = o_cur, c_nx = c_cur;
        advance(o_nx, c_nx);
        const Tile tn = tile_at(o_nx, c_nx);
        // an opaque copy of the lane index, renewed per phase: lane-dependent
        // addresses are recomputed where they are used instead of being
        // hoisted out of the loop into registers
        int lx = lane;
        asm volatile("" : "+v"(lx));
        // ---- A: first half
        __syncthreads();   // every wave has waited for its loads of the first half
        if (myhalf == 0) read_own(tl, cm, lx);
        __syncthreads();   // staging free
        asm volatile("" : "+v"(lx));
        issue_half(tl, 1, dpb, lx);
        if constexpr (FIRST) {
            if (j + 1 < count) dpa = load_dperm(tn, 0, lx);
        }
        if (myhalf == 0) {
            bfly(0, 4);
            asm volatile("" : "+v"(lx));
            lane_stages(lx);
        }
        __builtin_amdgcn_s_waitcnt(stream_vmcnt0());
        // ---- B: second half
        __syncthreads();   // the second half is complete in every wave
        asm volatile("" : "+v"(lx));
        if (myhalf == 1) read_own(tl, cm, lx);
        __syncthreads();   // staging free
        asm volatile("" : "+v"(lx));
        if (j + 1 < count) {
            issue_half(tn, 0, dpa, lx);
            if constexpr (FIRST) {
                cm = load_cmask(tn, lx);
                dpb = load_dperm(tn, 1, lx);
            }
        }
        if (myhalf == 1) {
            bfly(0, 4);
            asm volatile("" : "+v"(lx));
            lane_stages(lx);
        }
        // ---- C: stages 7..10 and the stores
        asm volatile("" : "+v"(lx));
        exchange(lx);
        if constexpr (LAST) {
            // the output slots of this tile's rows (contiguous in slot_pairs)
            // into the free exchange buffer
            asm volatile("" : "+v"(lx));
            const int2* src = a.slot_pairs + ((tl.rowbase & ((1ll << lo) - 1)) << NB) + (wave * 64 + lx) * 2;
            stream_lds_load16(src, reinterpret_cast<unsigned char*>(exb) + wave * 1024);
        }
        bfly(0, 4);
        settle();
        // the next first half (and the table loads) are complete after this
        // wait; the stores below drain during the next tile
        __builtin_amdgcn_s_waitcnt(stream_vmcnt0());
        if constexpr (LAST) __syncthreads();   // the slot pairs are visible
        // the sixteen slot pairs are read together (one LDS round trip, not
        // one per row), then one row at a time: the opaque lane copy keeps
        // the compiler from computing all sixteen 64-bit store addresses up
        // front
        if constexpr (LAST) {
            int2 prs[R];
#pragma unroll
            for (int t = 0; t < R; ++t) prs[t] = reinterpret_cast<const int2*>(exb)[final_row(t, lx)];
#pragma unroll
            for (int t = 0; t < R; ++t) asm volatile("" : "+v"(prs[t].x), "+v"(prs[t].y));
#pragma unroll
            for (int t = 0; t < R; ++t) {
                asm volatile("" : "+v"(lx));
                const int2 pr = prs[t];
                const int64_t col0 = tl.cbase + (lx & 7) * VL;
                if (pr.x >= 0) {
                    if (a.b_bf16) {
                        bf16_store4(static_cast<uint16_t*>(a.B) + (int64_t)pr.x * a.ldb + col0, v[t]);
                    } else {
                        ZVec<float>::st(static_cast<float*>(a.B) + (int64_t)pr.x * a.ldb + col0, v[t]);
                    }
                }
                if (pr.y >= 0) ZVec<float>::st(static_cast<float*>(a.Bh) + (int64_t)pr.y * a.ldbh + col0, v[t]);
            }
        } else {
            // Z offsets are linear in the register index (row step 128)
            asm volatile("" : "+v"(lx));
            const int64_t col0 = tl.cbase + (lx & 7) * VL;
            const int64_t z0 = zoff(grow(tl, final_row(0, lx)), col0);
            const int64_t zs = zoff(grow(tl, final_row(1, lx)), col0) - z0;
            float* p = static_cast<float*>(a.zout) + z0;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                ZVec<float>::st(p, v[t]);
                p += zs;
                asm volatile("" : "+v"(p));
            }
        }
        o_cur = o_nx;
        c_cur = c_nx;
    }
}

// The 11-bit pass of fwht_split_kernel with quarter-tile staging: two 64 KB
// quarter buffers (FP32 rows) instead of one half-tile, so the loads of the
// quarter two ahead are in flight while a quarter goes to the registers and
// through stages 0..6, and no phase waits for the loads it has just issued
// (same register layout, butterflies, exchange and stores; bit-identical).
// Its waits are explicit vmcnt(NIQ) counts and its barriers wait for LDS
// only, so the compiler adds no vmcnt(0) in the loop (but one before the
// last pass's exchange): the quarter buffers are separate LDS objects,
// table entries and column scales are loaded a phase ahead before a
// quarter's direct loads, and the stores are global, not flat.  The last
// pass issues the next tile's quarter 1 after its exchange, which then
// runs through that free 64 KB quarter buffer in four rounds with every
// lane (eight rounds of half the lanes through the 32 KB buffer
// otherwise).
template <typename TIN, bool FIRST, bool LAST, bool XL = false>
__global__ __launch_bounds__(SPLIT_THREADS) void fwht_ring_kernel(PassArgs a) {
    constexpr int DW = 16;   // bytes per direct load
    constexpr int CW = 32, VL = 4, R = 16, THREADS = SPLIT_THREADS;
    constexpr int LPR = CW / VL;                 // 8 lanes per tile row
    constexpr int NB = 11, HALF = 1 << (NB - 1), QR = HALF / 2;   // 512 rows per quarter
    typedef typename std::conditional<FIRST, TIN, float>::type TI;   // staged element
    constexpr int IB = (int)sizeof(TI);
    constexpr int ROWB = CW * IB;                // staged bytes per tile row
    constexpr int QS = QR * ROWB;                // one quarter-tile
    constexpr int NIQ = QS / (THREADS * DW);     // direct loads of DW bytes per thread per quarter
    constexpr int SM = ROWB < 256 ? 256 / ROWB - 1 : 0;
    static_assert(NIQ >= 1 && NIQ * THREADS * DW == QS && !(FIRST && LAST),
                  "ring tile shape");
    static_assert(!LAST || QS >= (HALF * 2) * LPR * 4, "the last pass exchanges through a quarter buffer");
    // s_waitcnt vmcnt(n): all but the last n vector-memory loads have completed
    constexpr int VM_NIQ = (NIQ & 0xf) | (((NIQ >> 4) & 3) << 14) | (0x7 << 4) | (0xf << 8);
    // two quarter buffers, separate LDS objects (the compiler's waits for
    // the direct loads into one do not hold back reads of the other)
    __shared__ __align__(16) unsigned char stg0[QS];
    __shared__ __align__(16) unsigned char stg1[QS];
    // s_waitcnt lgkmcnt(0) alone, then a bare barrier: the direct loads in
    // flight are not waited for (a block barrier with its fence would add
    // vmcnt(0))
    constexpr int LGKM0 = 0xf | (3 << 14) | (0x7 << 4);
    auto lds_barrier = [&]() __attribute__((always_inline)) {
        __builtin_amdgcn_s_waitcnt(LGKM0);
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    };
    __shared__ __align__(16) float exb[HALF * LPR];

    const int64_t T = a.ntiles;
    const int64_t G = gridDim.x;
    int64_t first, stride, count;
    if ((G & 7) == 0 && (T & 7) == 0) {
        const int64_t per = T >> 3, M = G >> 3, m = blockIdx.x >> 3;
        first = (int64_t)(blockIdx.x & 7) * per + m;
        stride = M;
        count = m < per ? (per - m + M - 1) / M : 0;
    } else {
        first = blockIdx.x;
        stride = G;
        count = (int64_t)blockIdx.x < T ? (T - blockIdx.x + G - 1) / G : 0;
    }
    if (count == 0) return;   // uniform over the block

    const int lo = a.lo;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int myq = wave >> 2;   // the quarter whose rows this wave holds
    auto srow = [](int row) -> int { return row ^ ((row >> 4) & SM); };
    struct Tile {
        int64_t rowbase;
        int64_t cbase;
    };
    // tile index = o * nchunks + cc, walked incrementally (uniform scalars)
    auto tile_at = [&](int64_t o, int64_t cc) -> Tile {
        const int64_t olo = o & ((1ll << lo) - 1);
        const int64_t ohi = o >> lo;
        return Tile{(ohi << (lo + NB)) | olo, cc * CW};
    };
    const int64_t nch = a.nchunks;
    int64_t o_cur = first / nch, c_cur = first - (first / nch) * nch;
    auto advance = [&](int64_t& o, int64_t& c) {
        c += stride;
        while (c >= nch) {
            c -= nch;
            ++o;
        }
    };
    auto grow = [&](const Tile& tl, int r) -> int64_t { return tl.rowbase | ((int64_t)r << lo); };
    auto zoff = [&](int64_t k, int64_t col) -> int64_t {
        if (a.zt_hibits == 0) return k * a.ldz + col;
        const int64_t klo = k & ((1ll << a.zt_lobits) - 1), khi = k >> a.zt_lobits;
        return ((((col / CW) << a.zt_lobits) | klo) << a.zt_hibits | khi) * CW + col % CW;
    };
    // tile row of register t at load (stage bits 0..3 in registers); lx is
    // an opaque copy of the lane index (see the loop)
    auto load_row = [&](int t, int lx) -> int { return t | ((lx >> 3) << 4) | (wave << 7); };
    // tile row of register t after the exchange (stage bits 7..10 in registers)
    auto final_row = [&](int t, int lx) -> int {
        return (wave & 1) | ((wave >> 1) & 1) << 1 | (lx >> 5) << 2 | ((lx >> 4) & 1) << 3 | ((lx >> 3) & 1) << 4 |
               ((wave >> 2) & 1) << 5 | ((wave >> 3) & 1) << 6 | t << 7;
    };
    // quarter row and DW-byte piece that direct load i of this lane fetches
    auto dma_slot = [&](int i, int lx, int& row, int& piece) {
        const int P = ((wave * NIQ + i) * 64 + lx) * DW;
        row = srow(P / ROWB);
        piece = (P % ROWB) / DW;
    };
    // first pass: the direct loads of wave w fetch the quarter rows
    // [32 w, 32 w + 32); lane l < 32 loads the permutation entry of row
    // 32 w + l and each load's row entry comes from its lane by a cross-lane
    // permute
    auto load_dperm = [&](const Tile& tl, int q, int lx) __attribute__((always_inline)) -> int32_t {
        return a.perm_sign[(uint32_t)grow(tl, q * QR + wave * 32 + (lx & 31))];
    };
    // first pass: sign (bit t) and validity (bit 16 + t) of this thread's 16
    // consecutive rows, one word of the row-mask table
    auto load_cmask = [&](const Tile& tl, int lx) __attribute__((always_inline)) -> uint32_t {
        return a.row_masks[(uint32_t)grow(tl, load_row(0, lx)) >> 4];
    };
    auto issue_quarter = [&](const Tile& tl, int q, unsigned char* qbuf, int32_t dp, int lx)
                             __attribute__((always_inline)) {
        unsigned char* dst = qbuf + wave * NIQ * 64 * DW;
#pragma unroll
        for (int i = 0; i < NIQ; ++i) {
            int row, piece;
            dma_slot(i, lx, row, piece);
            const int64_t col = tl.cbase + piece * (DW / IB);
            const unsigned char* src;
            if constexpr (FIRST) {
                const int32_t pe = __builtin_amdgcn_ds_bpermute((row - wave * 32) << 2, dp);
                src = x_piece<IB, XL>(a, (int64_t)(pe & 0x7fffffff), col);
            } else {
                src = static_cast<const unsigned char*>(a.zin) + zoff(grow(tl, q * QR + row), col) * 4;
            }
            stream_lds_load16(src, dst + i * 1024);
        }
    };

    float v[R][VL];
    // first pass over FP8: the column scales of this lane's 4 columns, per
    // tile in registers (loaded a tile ahead, before a quarter's direct
    // loads, so the waits that cover those cover them)
    constexpr bool SCALED = FIRST && std::is_same<TIN, fp8_t>::value;
    float scl[VL], scn[VL];
#pragma unroll
    for (int e = 0; e < VL; ++e) scl[e] = scn[e] = 0.f;
    auto load_scale = [&](const Tile& tl, int lx, float* o) __attribute__((always_inline)) {
        const int64_t c = tl.cbase + (lx & 7) * VL;
#pragma unroll
        for (int e = 0; e < VL; ++e) o[e] = c + e < a.d ? a.col_scale[c + e] : 0.f;
    };
    // this thread's rows of its quarter from quarter buffer qb
    auto read_own = [&](const Tile& tl, const unsigned char* qb, uint32_t cm, int lx) __attribute__((always_inline)) {
        const int64_t col0 = tl.cbase + (lx & 7) * VL;
        const int base = (((wave & 3) << 3) | (lx >> 3)) << 4;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            float x[VL];
            StageRead<TI>::rd(qb + srow(base | t) * ROWB + (lx & 7) * VL * IB, scl, 0, VL, x);
            if constexpr (FIRST) {
                const bool valid = (cm >> (16 + t)) & 1u;
                const bool neg = (cm >> t) & 1u;
#pragma unroll
                for (int e = 0; e < VL; ++e) {
                    float y = col0 + e < a.d ? x[e] : 0.f;
                    if (neg) y = -y;
                    v[t][e] = valid ? y : 0.f;
                }
            } else {
#pragma unroll
                for (int e = 0; e < VL; ++e) v[t][e] = x[e];
            }
        }
    };
    // stages on register bits [b0, b1), ascending
    auto bfly = [&](int b0, int b1) __attribute__((always_inline)) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (b >= b0 && b < b1) {
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    if (!(t & (1 << b))) {
#pragma unroll
                        for (int e = 0; e < VL; ++e) {
                            const float x0 = v[t][e], x1 = v[t | (1 << b)][e];
                            v[t][e] = x0 + x1;
                            v[t | (1 << b)][e] = x0 - x1;
                        }
                    }
                }
            }
        }
    };
    // stages 4..6 on the lane bits (see above)
    auto lane_stages = [&](int lx) __attribute__((always_inline)) {
        const float sg = (lx & 8) ? -1.f : 1.f;
#pragma unroll
        for (int t = 0; t < R; ++t) {
#pragma unroll
            for (int e = 0; e < VL; ++e) {
                const float p = __int_as_float(
                    __builtin_amdgcn_update_dpp(0, __float_as_int(v[t][e]), 0x128, 0xf, 0xf, false));
                v[t][e] = __builtin_fmaf(sg, v[t][e], p);
            }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
#pragma unroll
            for (int e = 0; e < VL; ++e) {
                const auto w = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[t][e]),
                                                                __float_as_uint(v[t + 8][e]), false, false);
                const float xn = __uint_as_float(w[0]), yn = __uint_as_float(w[1]);
                v[t][e] = xn + yn;
                v[t + 8][e] = xn - yn;
            }
        }
#pragma unroll
        for (int t = 0; t < R; ++t) {
            if (t & 4) continue;
#pragma unroll
            for (int e = 0; e < VL; ++e) {
                const auto w = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[t][e]),
                                                                __float_as_uint(v[t + 4][e]), false, false);
                const float xn = __uint_as_float(w[0]), yn = __uint_as_float(w[1]);
                v[t][e] = xn + yn;
                v[t + 4][e] = xn - yn;
            }
        }
    };
    // row bits 7..10 into the registers: per column element, two rounds by
    // row bit 2 (lane bit 5 before and after); exchange index of a row:
    // r3 | r4 << 1 | r0 << 2 | r1 << 3 | r5 << 4 | r6 << 5 | r7..r10 << 6
    auto exchange = [&](int lx) __attribute__((always_inline)) {
        const int lrx = lx & 7, x3 = (lx >> 3) & 1, x4 = (lx >> 4) & 1, x5 = lx >> 5;
        const int wbase = ((x4 | x3 << 1 | wave << 6) << 3) + lrx;
        const int rbase = ((x4 | x3 << 1 | wave << 2) << 3) + lrx;
#pragma unroll
        for (int e = 0; e < VL; ++e) {
#pragma unroll
            for (int rho = 0; rho < 2; ++rho) {
                const bool active = x5 == rho;
                if (active) {
#pragma unroll
                    for (int t = 0; t < R; ++t) {
                        const int off = ((t & 1) << 2 | ((t >> 1) & 1) << 3 | ((t >> 3) & 1) << 4 | ((t >> 2) & 1) << 5) << 3;
                        exb[wbase + off] = v[t][e];
                    }
                }
                lds_barrier();
                if (active) {
#pragma unroll
                    for (int t = 0; t < R; ++t) v[t][e] = exb[rbase + (t << 9)];
                }
                lds_barrier();
            }
        }
    };
    // the same exchange through a 64 KB buffer (a free quarter buffer of
    // FP32 rows): row bit 2 (lane bit 5) picks its half, so every lane takes
    // part in each of four rounds instead of half the lanes in eight
    auto exchange_wide = [&](int lx, float* xb) __attribute__((always_inline)) {
        const int lrx = lx & 7, x3 = (lx >> 3) & 1, x4 = (lx >> 4) & 1, x5 = lx >> 5;
        const int wbase = ((x4 | x3 << 1 | wave << 6) << 3) + lrx + (x5 << 13);
        const int rbase = ((x4 | x3 << 1 | wave << 2) << 3) + lrx + (x5 << 13);
#pragma unroll
        for (int e = 0; e < VL; ++e) {
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const int off = ((t & 1) << 2 | ((t >> 1) & 1) << 3 | ((t >> 3) & 1) << 4 | ((t >> 2) & 1) << 5) << 3;
                xb[wbase + off] = v[t][e];
            }
            lds_barrier();
#pragma unroll
            for (int t = 0; t < R; ++t) v[t][e] = xb[rbase + (t << 9)];
            lds_barrier();
        }
    };

    // completes every pending butterfly before this point (the scheduler
    // would otherwise sink the last stages into the store loop and keep
    // their partial sums live)
    auto settle = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int e = 0; e < VL; ++e)
            asm volatile("" : "+v"(v[0][e]), "+v"(v[1][e]), "+v"(v[2][e]), "+v"(v[3][e]), "+v"(v[4][e]),
                         "+v"(v[5][e]), "+v"(v[6][e]), "+v"(v[7][e]), "+v"(v[8][e]), "+v"(v[9][e]),
                         "+v"(v[10][e]), "+v"(v[11][e]), "+v"(v[12][e]), "+v"(v[13][e]), "+v"(v[14][e]),
                         "+v"(v[15][e]));
    };

    int32_t dpn = 0;     // first pass: this lane's entry for the quarter issued next
    uint32_t cm = 0;     // first pass: sign and validity of this thread's rows
    uint32_t cmn = 0;    // first pass: the same for the next tile
    {
        const Tile t0 = tile_at(o_cur, c_cur);
        if constexpr (FIRST) {
            dpn = load_dperm(t0, 0, lane);
            cm = load_cmask(t0, lane);
            if constexpr (SCALED) load_scale(t0, lane, scl);
            __builtin_amdgcn_s_waitcnt(stream_vmcnt0());
        }
        issue_quarter(t0, 0, stg0, dpn, lane);
        int32_t dp1 = 0;
        if constexpr (FIRST) {
            dp1 = load_dperm(t0, 1, lane);
            __builtin_amdgcn_s_waitcnt(stream_vmcnt0());
            // before the direct loads, so that the wait below covers it
            dpn = load_dperm(t0, 2, lane);
        }
        issue_quarter(t0, 1, stg1, dp1, lane);
    }
    __builtin_amdgcn_s_waitcnt(VM_NIQ);   // quarter 0 has landed

    for (int64_t j = 0; j < count; ++j) {
        const Tile tl = tile_at(o_cur, c_cur);
        int64_t o_nx = o_cur, c_nx = c_cur;
        advance(o_nx, c_nx);
        const Tile tn = tile_at(o_nx, c_nx);
        const bool has_next = j + 1 < count;
        if constexpr (FIRST) cm = j > 0 ? cmn : cm;
        if constexpr (SCALED) {
            if (j > 0) {
#pragma unroll
                for (int e = 0; e < VL; ++e) scl[e] = scn[e];
            }
        }
        // an opaque copy of the lane index, renewed per phase: lane-dependent
        // addresses are recomputed where they are used instead of being
        // hoisted out of the loop into registers
        int lx = lane;
        // phases 0..3: quarter q (landed and, after the first barrier,
        // visible) goes to the registers of waves 4q..4q+3; once its buffer
        // is free, the quarter two ahead is issued into it (quarters 2, 3 of
        // this tile, then 0, 1 of the next); waves 4q..4q+3 run stages 0..6;
        // one wait then covers quarter q + 1 and leaves the new loads in
        // flight.  Per phase the loads go in the order: table entries for
        // the next phase, then the quarter's direct loads, so vmcnt(NIQ)
        // covers everything but those.  Every phase issues a quarter: on a
        // block's last tile, phases 2 and 3 reload quarters of this tile
        // (in bounds, never read), which keeps every wait the same
        // unconditional vmcnt(NIQ).
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned char* const qbuf = (q & 1) ? stg1 : stg0;
            lds_barrier();   // quarter q is complete in every wave
            asm volatile("" : "+v"(lx));
            if (myq == q) read_own(tl, qbuf, cm, lx);
            lds_barrier();   // buffer q & 1 is free
            asm volatile("" : "+v"(lx));
            const int32_t dpi = dpn;
            if constexpr (FIRST) {
                // the quarter issued in the next phase: (q + 3) & 3 of this
                // tile (q = 0) or of the next
                if (q == 0) dpn = load_dperm(tl, 3, lx);
                else if (has_next) dpn = load_dperm(tn, (q + 3) & 3, lx);
                if (q == 3 && has_next) {
                    cmn = load_cmask(tn, lx);
                    if constexpr (SCALED) load_scale(tn, lx, scn);
                }
            }
            // (the last pass issues quarter 1 of the next tile in phase C,
            // after the exchange through its buffer)
            if (!(LAST && q == 3)) issue_quarter(q < 2 || !has_next ? tl : tn, (q + 2) & 3, qbuf, dpi, lx);
            if (myq == q) {
                bfly(0, 4);
                asm volatile("" : "+v"(lx));
                lane_stages(lx);
            }
            if (q < 3) __builtin_amdgcn_s_waitcnt(VM_NIQ);   // quarter q + 1 has landed
        }
        // ---- C: stages 7..10 and the stores
        asm volatile("" : "+v"(lx));
        if constexpr (LAST) {
            // quarter buffer 1 is free here (quarter 1 of the next tile is
            // issued after the exchange): four rounds through it; then the
            // output slots of this tile's rows (contiguous in slot_pairs)
            // into the exchange buffer, and quarter 1, so that one
            // vmcnt(NIQ) below covers the slot pairs and leaves that quarter
            // in flight
            exchange_wide(lx, reinterpret_cast<float*>(stg1));
            asm volatile("" : "+v"(lx));
            const int2* src = a.slot_pairs + ((tl.rowbase & ((1ll << lo) - 1)) << NB) + (wave * 64 + lx) * 2;
            stream_lds_load16(src, reinterpret_cast<unsigned char*>(exb) + wave * 1024);
            asm volatile("" : "+v"(lx));
            issue_quarter(has_next ? tn : tl, 1, stg1, 0, lx);
        } else {
            exchange(lx);
        }
        bfly(0, 4);
        settle();
        // the next tile's quarter 0 (and, last pass, the slot pairs) has
        // landed; quarter 1 stays in flight, and the stores below drain
        // during the next tile
        __builtin_amdgcn_s_waitcnt(VM_NIQ);
        if constexpr (LAST) lds_barrier();   // the slot pairs are visible
        // the sixteen slot pairs are read together (one LDS round trip, not
        // one per row), then one row at a time: the opaque lane copy keeps
        // the compiler from computing all sixteen 64-bit store addresses up
        // front
        if constexpr (LAST) {
            int2 prs[R];
#pragma unroll
            for (int t = 0; t < R; ++t) prs[t] = reinterpret_cast<const int2*>(exb)[final_row(t, lx)];
#pragma unroll
            for (int t = 0; t < R; ++t) asm volatile("" : "+v"(prs[t].x), "+v"(prs[t].y));
#pragma unroll
            for (int t = 0; t < R; ++t) {
                asm volatile("" : "+v"(lx));
                const int2 pr = prs[t];
                const int64_t col0 = tl.cbase + (lx & 7) * VL;
                if (pr.x >= 0) {
                    if (a.b_bf16) {
                        bf16_store4(static_cast<uint16_t*>(a.B) + (int64_t)pr.x * a.ldb + col0, v[t]);
                    } else {
                        ZVec<float>::st(static_cast<float*>(a.B) + (int64_t)pr.x * a.ldb + col0, v[t]);
                    }
                }
                if (pr.y >= 0) ZVec<float>::st(static_cast<float*>(a.Bh) + (int64_t)pr.y * a.ldbh + col0, v[t]);
            }
        } else {
            // Z offsets are linear in the register index (row step 128)
            asm volatile("" : "+v"(lx));
            const int64_t col0 = tl.cbase + (lx & 7) * VL;
            const int64_t z0 = zoff(grow(tl, final_row(0, lx)), col0);
            const int64_t zs = zoff(grow(tl, final_row(1, lx)), col0) - z0;
            // global (not flat) stores: a flat store may address LDS, and
            // the compiler would wait for the direct loads in flight first
            typedef float f4v __attribute__((ext_vector_type(4)));
            typedef __attribute__((address_space(1))) f4v gf4v;
            gf4v* p = reinterpret_cast<gf4v*>(reinterpret_cast<uintptr_t>(static_cast<float*>(a.zout) + z0));
            const int64_t zs4 = zs / VL;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                *p = f4v{v[t][0], v[t][1], v[t][2], v[t][3]};
                p += zs4;
                asm volatile("" : "+v"(p));
            }
        }
        o_cur = o_nx;
        c_cur = c_nx;
    }
    // the reloads of the last tile land before the block's LDS is released
    __builtin_amdgcn_s_waitcnt(stream_vmcnt0());
}

// Threads per block and register window for a pass of nb bits.
template <typename TZ, int CW>
inline int pass_q(int nb) {
    constexpr int VL = CW == 1 ? 1 : ZVec<TZ>::VL;
    int q = nb < 4 ? nb : 4;
    while (((int64_t)(CW / VL) << (nb - q)) > 1024) ++q;
    return q;
}

template <typename TIN, typename TZ, int CW, bool FIRST, bool LAST, int QMAX>
hipError_t launch_pass_q(hipStream_t st, const PassArgs& a) {
    constexpr int VL = CW == 1 ? 1 : ZVec<TZ>::VL;
    constexpr int LPR = CW / VL;
    constexpr int LPRP = LPR == 1 ? 1 : LPR + 1;
    const size_t lds = (size_t)(1 << a.nb) * LPRP * sizeof(TZ);
    auto fn = fwht_pass_kernel<TIN, TZ, CW, FIRST, LAST, QMAX>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int threads = (int)(((int64_t)LPR << a.nb) >> a.q);
    if (threads > (QMAX == 5 ? 512 : 1024)) return hipErrorInvalidValue;
    fn<<<dim3((unsigned)a.ntiles), dim3(threads), lds, st>>>(a);
    return hipGetLastError();
}

// register window: exactly q = QMAX bits for passes of >= 4 bits, the whole
// pass for the tiny ones
template <typename TIN, typename TZ, int CW, bool FIRST, bool LAST>
hipError_t launch_pass(hipStream_t st, const PassArgs& a) {
    if (a.q == 5) return launch_pass_q<TIN, TZ, CW, FIRST, LAST, 5>(st, a);
    if (a.q == 4) return launch_pass_q<TIN, TZ, CW, FIRST, LAST, 4>(st, a);
    if (a.q <= 3 && a.q == a.nb) return launch_pass_q<TIN, TZ, CW, FIRST, LAST, 3>(st, a);
    return hipErrorInvalidValue;
}

template <typename TIN, typename TZ, int CW>
hipError_t launch_any(hipStream_t st, const PassArgs& a, bool first, bool last) {
    if (first && last) return launch_pass<TIN, TZ, CW, true, true>(st, a);
    if (first) return launch_pass<TIN, TZ, CW, true, false>(st, a);
    if (last) return launch_pass<TIN, TZ, CW, false, true>(st, a);
    return launch_pass<TIN, TZ, CW, false, false>(st, a);
}

template <typename TIN, int CW, bool FIRST, bool LAST, bool XL = false>
hipError_t launch_stream_one(hipStream_t st, const PassArgs& a, int64_t grid) {
    auto fn = fwht_stream_kernel<TIN, CW, FIRST, LAST, XL>;
    fn<<<dim3((unsigned)grid), dim3(STREAM_THREADS), 0, st>>>(a);
    return hipGetLastError();
}

// How a first pass stages the rows of X: 16-byte direct loads of rows that
// are 16-byte aligned, or of rows that are only 4-byte aligned with row
// N - 1 read from its padded copy; XS_NONE: no staged first pass (such rows
// take the tiled kernel).
enum XStage : int { XS_16 = 0, XS_NONE = 1, XS_16L = 2 };

template <typename TIN>
hipError_t launch_split(hipStream_t st, const PassArgs& a, int64_t grid, bool first, bool last, int xs) {
    const dim3 g((unsigned)grid), b(SPLIT_THREADS);
    if (first && last) return hipErrorInvalidValue;
    if (first && xs == XS_NONE) {
        return hipErrorInvalidValue;
    } else if (first && xs == XS_16L) {
        fwht_split_kernel<TIN, true, false, true><<<g, b, 0, st>>>(a);
    } else if (first) {
        fwht_split_kernel<TIN, true, false><<<g, b, 0, st>>>(a);
    } else if (last) {
        fwht_split_kernel<TIN, false, true><<<g, b, 0, st>>>(a);
    } else {
        fwht_split_kernel<TIN, false, false><<<g, b, 0, st>>>(a);
    }
    return hipGetLastError();
}

template <typename TIN>
hipError_t launch_ring(hipStream_t st, const PassArgs& a, int64_t grid, bool first, bool last, int xs) {
    const dim3 g((unsigned)grid), b(SPLIT_THREADS);
    if (first && last) return hipErrorInvalidValue;
    if (first && xs == XS_NONE) {
        return hipErrorInvalidValue;
    } else if (first && xs == XS_16L) {
        fwht_ring_kernel<TIN, true, false, true><<<g, b, 0, st>>>(a);
    } else if (first) {
        fwht_ring_kernel<TIN, true, false><<<g, b, 0, st>>>(a);
    } else if (last) {
        fwht_ring_kernel<TIN, false, true><<<g, b, 0, st>>>(a);
    } else {
        fwht_ring_kernel<TIN, false, false><<<g, b, 0, st>>>(a);
    }
    return hipGetLastError();
}

template <typename TIN, int CW>
hipError_t launch_stream(hipStream_t st, const PassArgs& a, int64_t grid, bool first, bool last, int xs) {
    if (first && last) return hipErrorInvalidValue;
    if (first && xs == XS_NONE) return hipErrorInvalidValue;
    if (first && xs == XS_16L) return launch_stream_one<TIN, CW, true, false, true>(st, a, grid);
    if (first) return launch_stream_one<TIN, CW, true, false>(st, a, grid);
    if (last) return launch_stream_one<TIN, CW, false, true>(st, a, grid);
    return launch_stream_one<TIN, CW, false, false>(st, a, grid);
}

// Passes of at most NB_MAX bits; each pass uses 256-byte row segments, or
// 128-byte ones for 11-bit passes (whose 256-byte tile would not fit).
// 10-bit passes at FP32 working precision of a multi-pass transform use the
// streaming kernel unless the job asks for one tile per block.
template <typename TIN, typename TZ>
hipError_t run_passes(hipStream_t st, const FwhtJob& job) {
    const int L = job.L;
    constexpr int E = sizeof(TZ);
    constexpr int CW_WIDE = 256 / E, CW_NARROW = 128 / E, CW_TINY = 64 / E;
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
    a.b_bf16 = job.b_bf16;
    a.slot_pairs = job.slot_pairs;
    a.row_masks = job.row_masks;
    constexpr int VL = ZVec<TZ>::VL;
    a.xvec = (job.ldx % VL == 0) && ((uintptr_t)job.x % (VL * sizeof(TIN)) == 0);
    // the first pass stages rows of X with 16-byte direct loads: rows
    // 16-byte aligned, or only 4-byte aligned when the job brings a padded
    // copy of row N - 1 (the last piece of a row may reach into the next)
    const bool x16 = (uintptr_t)job.x % 16 == 0 && (job.ldx * (int64_t)sizeof(TIN)) % 16 == 0;
    const bool x4 = (uintptr_t)job.x % 4 == 0 && (job.ldx * (int64_t)sizeof(TIN)) % 4 == 0;
    const bool x16l = !x16 && x4 && job.x_last != nullptr && job.N >= 2;
    const bool xdma = x16 || x16l;
    // staging of the first pass when it runs on a staged kernel (other rows
    // take the tiled kernel)
    const int xs = x16 ? XS_16 : x16l ? XS_16L : XS_NONE;
    a.x_last = x16l ? job.x_last : nullptr;
    const int split = fwht_split_tables(job.in_dtype, L, job.ldz, job.seg_bytes);
    // column width of the streaming kernel for a pass (0: one tile per block).
    // 11-bit passes would need 64-byte rows (CW = 16); with chunk-major Z the
    // tiled kernel's 128-byte rows measured faster there (2.71 against
    // 2.88 ms at N = 2e6, d = 256), so only passes of 9 and 10 bits stream
    auto stream_cw = [&](int nb, bool first) -> int {
        if (!std::is_same<TZ, float>::value) return 0;
        // 1024 x 128 B or 512 x 256 B tiles (128 KB each); 256 x 512 B tiles
        // for 8 bits would spill registers in the first pass
        const int scw = nb == 10 ? 32 : nb == 9 ? 64 : 0;
        if (!job.stream || job.num_cu <= 0 || !scw || passes < 2 || job.seg_bytes > 0 || job.ldz % scw != 0 ||
            (first && !xdma))
            return 0;
        return scw;
    };
    // column width of the one-tile-per-block kernel: the widest segment
    // whose tile fits the registers (256 B up to 10-bit passes, 128 B for 11
    // bits), unless the job asks for a narrower one
    auto tiled_cw = [&](int nb) -> int {
        int seg = nb <= 10 ? 256 : 128;
        if (job.seg_bytes > 0 && job.seg_bytes < seg) seg = job.seg_bytes;
        return seg / E;
    };
    auto pass_cw = [&](int nb, bool first) -> int {
        const int scw = stream_cw(nb, first);
        return scw ? scw : tiled_cw(nb);
    };
    // two passes with one column width keep Z chunk-major (last-pass tiles
    // then read contiguous blocks)
    const int nb0 = L / passes + (0 < L % passes ? 1 : 0);
    const bool ztrans = passes == 2 && pass_cw(nb0, true) == pass_cw(L - nb0, false);
    int lo = 0;
    for (int pi = 0; pi < passes; ++pi) {
        const int nb = L / passes + (pi < L % passes ? 1 : 0);
        const bool first = pi == 0, last = pi == passes - 1;
        a.zt_lobits = ztrans ? nb0 : 0;
        a.zt_hibits = ztrans ? L - nb0 : 0;
        if (last && job.wait_before_last) {
            const hipError_t e = hipStreamWaitEvent(st, job.wait_before_last, 0);
            if (e != hipSuccess) return e;
        }
        hipEvent_t ev0 = pi < 3 ? job.pass_ev[2 * pi] : nullptr, ev1 = pi < 3 ? job.pass_ev[2 * pi + 1] : nullptr;
        if (ev0) {
            const hipError_t e = hipEventRecord(ev0, st);
            if (e != hipSuccess) return e;
        }
        if constexpr (std::is_same<TZ, float>::value) {
            // 11-bit passes of 128-byte row segments stage quarter tiles in
            // a ring (seg_bytes -64: half tiles)
            if (nb == NB_MAX && job.stream && job.num_cu > 0 &&
                (first ? (split & 1) && xdma && job.row_masks : (split & 2) && job.slot_pairs)) {
                a.lo = lo;
                a.nb = nb;
                a.q = 4;
                a.nchunks = job.ldz / 32;
                a.ntiles = (1ll << (L - nb)) * a.nchunks;
                a.zin = job.zbuf;
                a.zout = job.zbuf;
                const int64_t grid = std::min<int64_t>(job.num_cu, a.ntiles);
                const bool ring = job.seg_bytes != -64;
                const hipError_t e = ring ? launch_ring<TIN>(st, a, grid, first, last, xs)
                                          : launch_split<TIN>(st, a, grid, first, last, xs);
                if (e != hipSuccess) return e;
                if (ev1) {
                    const hipError_t e1 = hipEventRecord(ev1, st);
                    if (e1 != hipSuccess) return e1;
                }
                lo += nb;
                continue;
            }
            const int scw = stream_cw(nb, first);
            if (scw) {
                a.lo = lo;
                a.nb = nb;
                a.q = 4;
                a.nchunks = job.ldz / scw;
                a.ntiles = (1ll << (L - nb)) * a.nchunks;
                a.zin = job.zbuf;
                a.zout = job.zbuf;
                const int64_t grid = std::min<int64_t>(job.num_cu, a.ntiles);
                const hipError_t e = scw == 32 ? launch_stream<TIN, 32>(st, a, grid, first, last, xs)
                                               : launch_stream<TIN, 64>(st, a, grid, first, last, xs);
                if (e != hipSuccess) return e;
                if (ev1) {
                    const hipError_t e1 = hipEventRecord(ev1, st);
                    if (e1 != hipSuccess) return e1;
                }
                lo += nb;
                continue;
            }
        }
        const int cw = tiled_cw(nb);
        a.lo = lo;
        a.nb = nb;
        a.q = cw == CW_WIDE ? pass_q<TZ, CW_WIDE>(nb) : cw == CW_NARROW ? pass_q<TZ, CW_NARROW>(nb)
                                                                     : pass_q<TZ, CW_TINY>(nb);
        if (a.q > 5) return hipErrorInvalidValue;
        a.nchunks = job.ldz / cw;
        a.ntiles = (1ll << (L - nb)) * a.nchunks;
        a.zin = job.zbuf;
        a.zout = job.zbuf;
        const hipError_t e = cw == CW_WIDE     ? launch_any<TIN, TZ, CW_WIDE>(st, a, first, last)
                             : cw == CW_NARROW ? launch_any<TIN, TZ, CW_NARROW>(st, a, first, last)
                                               : launch_any<TIN, TZ, CW_TINY>(st, a, first, last);
        if (e != hipSuccess) return e;
        if (ev1) {
            const hipError_t e1 = hipEventRecord(ev1, st);
            if (e1 != hipSuccess) return e1;
        }
        lo += nb;
    }
    return hipSuccess;
}

// Single-column FP64 transform (the response vector): 16 rows per thread.
hipError_t run_passes_narrow(hipStream_t st, const FwhtJob& job) {
    const int L = job.L;
    const int passes = (L + NB_MAX - 1) / NB_MAX;
    PassArgs a{};
    a.x = job.x;
    a.ldx = job.ldx;
    a.N = job.N;
    a.d = job.d;
    a.ldz = job.ldz;
    a.perm_sign = job.perm_sign;
    a.inv_slot = job.inv_slot;
    a.B = job.B;
    a.ldb = job.ldb;
    a.xvec = 0;
    a.nchunks = 1;
    int lo = 0;
    for (int pi = 0; pi < passes; ++pi) {
        const int nb = L / passes + (pi < L % passes ? 1 : 0);
        a.lo = lo;
        a.nb = nb;
        a.q = pass_q<double, 1>(nb);
        a.ntiles = 1ll << (L - nb);
        a.zin = job.zbuf;
        a.zout = job.zbuf;
        const hipError_t e = launch_any<double, double, 1>(st, a, pi == 0, pi == passes - 1);
        if (e != hipSuccess) return e;
        lo += nb;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_feistel_tables(hipStream_t st, uint64_t seed, int L, int n, const uint64_t* streams, uint32_t* rt) {
    if (L < 1 || L > 30 || n < 1 || n > 3) return hipErrorInvalidValue;
    const int64_t total = n * feistel_table_size(L);
    feistel_table_kernel<<<(unsigned)ceil_div(total, 256), 256, 0, st>>>(seed, L, n, streams[0], n > 1 ? streams[1] : 0,
                                                                         n > 2 ? streams[2] : 0, rt);
    return hipGetLastError();
}

hipError_t launch_sketch_round_tables(hipStream_t st, uint64_t seed, int L, uint32_t* rt) {
    const uint64_t streams[3] = {STREAM_P, STREAM_PI, STREAM_PIHAT};
    return launch_feistel_tables(st, seed, L, 3, streams, rt);
}

hipError_t launch_sketch_tables(hipStream_t st, uint64_t seed, int L, int64_t mK, int64_t r,
                                int32_t* perm_sign, int32_t* inv_slot, int32_t* inv_hat, const uint32_t* rt,
                                int2* pair_t, int plo, uint32_t* row_masks, int64_t N) {
    if (pair_t && (plo < 1 || plo >= L)) return hipErrorInvalidValue;
    if (row_masks && (L < 4 || !perm_sign)) return hipErrorInvalidValue;
    if (L < 1 || L > 30 || !rt) return hipErrorInvalidValue;
    const int64_t np = 1ll << L, ts = feistel_table_size(L);
    tables_kernel<<<(unsigned)ceil_div(np, 256), 256, 0, st>>>(seed, L, np, mK, r, perm_sign, inv_slot, inv_hat,
                                                                rt, rt + ts, rt + 2 * ts, pair_t, plo, row_masks,
                                                                N);
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

int fwht_passes(int L) { return (L + NB_MAX - 1) / NB_MAX; }

int fwht_split_tables(int in_dtype, int L, int64_t ldz, int seg_bytes) {
    if (in_dtype == DT_F64 || ldz % 32 != 0 || seg_bytes > 0) return 0;
    if (L == 2 * NB_MAX) return 3;
    if (L == 2 * NB_MAX - 1) return 1;
    return 0;
}

hipError_t run_fwht(hipStream_t st, const FwhtJob& job) {
    // a row segment narrower than the default chunk (seg_bytes > 0) only
    // needs rows that are a multiple of it
    int cw = fwht_chunk_cols(job.in_dtype, job.narrow);
    if (!job.narrow && job.seg_bytes > 0) cw = std::min(cw, job.seg_bytes / (job.in_dtype == DT_F64 ? 8 : 4));
    if (cw < 1 || job.ldz % cw != 0 || (job.B && job.ldb != job.ldz) || (job.Bh && job.ldbh != job.ldz) ||
        job.ldz < job.d || job.L < 1 || job.L > 30)
        return hipErrorInvalidValue;
    if (job.narrow) {
        if (job.in_dtype != DT_F64 || job.d != 1) return hipErrorInvalidValue;
        return run_passes_narrow(st, job);
    }
    switch (job.in_dtype) {
        case DT_F64: return run_passes<double, double>(st, job);
        case DT_F32: return run_passes<float, float>(st, job);
        case DT_BF16: return run_passes<bf16_t, float>(st, job);
        case DT_FP8: return run_passes<fp8_t, float>(st, job);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace spcg
