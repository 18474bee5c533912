// PCG products on gfx950: one HBM pass over a row-major m x d matrix A.
//
// The two tall-skinny products of a PCG iteration (Sec. 2.2: 4 m d of the
// (4m + 13) d + 2 d^2 flops) are fused into one read of A:
//
//   S  mode: s = A^T (A p)                      (the CG product)
//   G  mode: g = A^T (b - A x), ||b - A x||^2, ||A x||^2   (stage start)
//   SG mode: both in the same pass              (full-data refinement)
//
// Layout: each row is covered by LPR lanes (a power of two <= 64) that
// load VEC-element 16-byte vectors, NSLOT per lane; 64 / LPR rows share a
// wavefront.  For each row the lanes form the dot product(s) with a group
// shuffle reduction and then accumulate w * a_row into per-lane column
// accumulators held in registers, so A is read exactly once and never
// staged.  Each block owns a contiguous range of rows and writes one FP64
// partial per column; the partials are summed in a fixed order by the
// d-space kernel (deterministic results).
//
// Accumulation: the p-product uses float for FP32/BF16/FP8 storage and
// double for FP64 storage; everything involving x and b (the residual and
// the gradient) accumulates in double, with the stored values widened
// exactly.  FP8 per-column scales are folded into p and x on entry and
// into the partial columns on exit.
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace spcg {

namespace {

constexpr int NW = 8;        // waves per block (one block per CU, 2 waves per SIMD)
constexpr int DMAX_LDS = 4096;

typedef float v2f __attribute__((ext_vector_type(2)));

template <int BYTES>
struct RawVec;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <>
struct RawVec<16> {
    typedef u32x4 T;
};
template <>
struct RawVec<8> {
    typedef u32x2 T;
};
template <>
struct RawVec<4> {
    typedef uint32_t T;
};
template <>
struct RawVec<2> {
    typedef uint16_t T;
};
template <>
struct RawVec<1> {
    typedef uint8_t T;
};

template <typename TS>
struct Store;
template <>
struct Store<double> {
    typedef double CT;
    static constexpr int BYTES = 8;
    static constexpr int VMAX = 2;
};
template <>
struct Store<float> {
    typedef float CT;
    static constexpr int BYTES = 4;
    static constexpr int VMAX = 4;
};
template <>
struct Store<bf16_t> {
    typedef float CT;
    static constexpr int BYTES = 2;
    static constexpr int VMAX = 8;
};
template <>
struct Store<fp8_t> {
    typedef float CT;
    static constexpr int BYTES = 1;
    static constexpr int VMAX = 16;
};

__device__ __forceinline__ uint32_t word_of(const u32x4& v, int i) { return v[i]; }
__device__ __forceinline__ uint32_t word_of(const u32x2& v, int i) { return v[i]; }
__device__ __forceinline__ uint32_t word_of(const uint32_t& v, int) { return v; }
__device__ __forceinline__ uint32_t word_of(const uint16_t& v, int) { return v; }
__device__ __forceinline__ uint32_t word_of(const uint8_t& v, int) { return v; }

// Widen the VEC elements of a raw vector into out[0..VEC).
template <typename TS, int VEC, typename R>
struct Widen;

template <int VEC, typename R>
struct Widen<double, VEC, R> {
    __device__ static void run(const R& raw, double* out) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            uint32_t lo = word_of(raw, 2 * e), hi = word_of(raw, 2 * e + 1);
            out[e] = __hiloint2double((int)hi, (int)lo);
        }
    }
};
template <int VEC, typename R>
struct Widen<float, VEC, R> {
    __device__ static void run(const R& raw, float* out) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) out[e] = __uint_as_float(word_of(raw, e));
    }
};
template <int VEC, typename R>
struct Widen<bf16_t, VEC, R> {
    __device__ static void run(const R& raw, float* out) {
        if constexpr (VEC == 1) {
            out[0] = __uint_as_float((uint32_t)raw << 16);
        } else {
#pragma unroll
            for (int e = 0; e < VEC; e += 2) {
                uint32_t w = word_of(raw, e / 2);
                out[e] = __uint_as_float(w << 16);
                out[e + 1] = __uint_as_float(w & 0xffff0000u);
            }
        }
    }
};
template <int VEC, typename R>
struct Widen<fp8_t, VEC, R> {
    __device__ static void run(const R& raw, float* out) {
        if constexpr (VEC == 1) {
            out[0] = __builtin_amdgcn_cvt_f32_fp8((int)(uint32_t)raw, 0);
        } else {
#pragma unroll
            for (int e = 0; e < VEC; e += 4) {
                int w = (int)word_of(raw, e / 4);
                v2f lo = __builtin_amdgcn_cvt_pk_f32_fp8(w, false);
                v2f hi = __builtin_amdgcn_cvt_pk_f32_fp8(w, true);
                out[e] = lo.x;
                out[e + 1] = lo.y;
                out[e + 2] = hi.x;
                out[e + 3] = hi.y;
            }
        }
    }
};

struct ProdArgs {
    const void* A;
    int64_t m, lda, rpb;
    int d, nvec;
    const float* col_scale;
    const double* b;
    int64_t ldbv;
    const double* x;
    const double* p;
    double* part_s;
    double* part_g;
    double* part_scal;
    int64_t dpad;
    const int32_t* gate;   // optional: return at once unless *gate >= gmin
    int32_t gmin;
    int32_t lshift;        // 16-byte loads of rows only 4-byte aligned: the last row's loads start this many bytes early
};

// a launch switched off by a device-side decision (uniform over the grid)
__device__ __forceinline__ bool gated_off(const ProdArgs& a) { return a.gate && *a.gate < a.gmin; }

template <typename TS, int VEC, int LPR, int NSLOT, int MODE, int U>
__global__ __launch_bounds__(64 * NW) void product_kernel(ProdArgs a) {
    if (gated_off(a)) return;
    typedef typename Store<TS>::CT CT;
    typedef typename RawVec<VEC * Store<TS>::BYTES>::T Raw;
    constexpr bool DO_S = MODE != PM_G;
    constexpr bool DO_G = MODE != PM_S;
    constexpr bool FP8 = std::is_same<TS, fp8_t>::value;
    constexpr int RPW = 64 / LPR;
    constexpr int NC = NSLOT * VEC;
    constexpr int DCOLS = NSLOT * VEC * LPR;
    __shared__ double red_s[DO_S ? DCOLS : 1];
    __shared__ double red_g[DO_G ? DCOLS : 1];
    __shared__ double red_scal[2 * NW];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lir = lane & (LPR - 1), rs = lane / LPR;
    const int d = a.d;

    CT preg[NC];
    double xreg[NC];
    CT sacc[NC];
    double gacc[NC];
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const int i = s * VEC + e;
            const int col = (lir + s * LPR) * VEC + e;
            // unconditional (clamped) loads: issued together, one wait
            const int cc = min(col, d - 1);
            const bool ok = col < d;
            const double sc = FP8 ? (double)a.col_scale[cc] : 1.0;
            const double pv = DO_S ? a.p[cc] * sc : 0.0;
            const double xv = DO_G ? a.x[cc] * sc : 0.0;
            preg[i] = ok ? (CT)pv : CT(0);
            xreg[i] = ok ? xv : 0.0;
            sacc[i] = CT(0);
            gacc[i] = 0.0;
        }
    }
    double r2 = 0.0, ax2 = 0.0;

    const int64_t r0 = (int64_t)blockIdx.x * a.rpb;
    const int64_t r1 = min(a.m, r0 + a.rpb);
    const char* Abase = static_cast<const char*>(a.A);
    const int64_t row_bytes = a.lda * Store<TS>::BYTES;

    // Rolling prefetch: slot u of `raw` holds row (base + u * RPW) of the
    // current sweep; right after a row is consumed its slot is refilled with
    // the same row of the next sweep, so U rows stay in flight per wave while
    // only one row is widened at a time.
    const int64_t sweep = (int64_t)NW * U * RPW;
    auto load_row = [&](int64_t row, Raw* dst) {
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            const int vi = lir + s * LPR;
            if (row < r1 && vi < a.nvec) {
                dst[s] = __builtin_nontemporal_load(reinterpret_cast<const Raw*>(
                    Abase + row * row_bytes + (int64_t)vi * (VEC * Store<TS>::BYTES)));
            } else {
                dst[s] = Raw{};
            }
        }
    };
    Raw raw[U][NSLOT];
    const int64_t first = r0 + (int64_t)wave * (U * RPW) + rs;
#pragma unroll
    for (int u = 0; u < U; ++u) load_row(first + u * RPW, raw[u]);
    for (int64_t base = first; base - rs < r1; base += sweep) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = base + u * RPW;
            const bool valid = row < r1;
            CT v[NC];
#pragma unroll
            for (int s = 0; s < NSLOT; ++s) Widen<TS, VEC, Raw>::run(raw[u][s], v + s * VEC);
            load_row(row + sweep, raw[u]);
            CT dp = CT(0);
            double dx = 0.0;
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                if (DO_S) dp = fma(v[i], preg[i], dp);
                if (DO_G) dx = fma((double)v[i], xreg[i], dx);
            }
            if constexpr (DO_S) {
                if constexpr (LPR == 64) dp = wave_sum(dp); else dp = group_sum<LPR>(dp);
            }
            double w = 0.0;
            if (DO_G) {
                if constexpr (LPR == 64) dx = wave_sum(dx); else dx = group_sum<LPR>(dx);
                const double bb = valid ? a.b[row * a.ldbv] : 0.0;
                w = valid ? bb - dx : 0.0;
                if (lir == 0 && valid) {
                    r2 = fma(w, w, r2);
                    ax2 = fma(dx, dx, ax2);
                }
            }
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                if (DO_S) sacc[i] = fma(dp, v[i], sacc[i]);
                if (DO_G) gacc[i] = fma(w, (double)v[i], gacc[i]);
            }
        }
    }

    // lanes with the same lir in different row slots hold the same columns
#pragma unroll
    for (int o = LPR; o < 64; o <<= 1) {
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            if (DO_S) sacc[i] += __shfl_xor(sacc[i], o);
            if (DO_G) gacc[i] += __shfl_xor(gacc[i], o);
        }
    }
    // fixed wave order into LDS
    for (int wv = 0; wv < NW; ++wv) {
        if (wave == wv && rs == 0) {
#pragma unroll
            for (int s = 0; s < NSLOT; ++s) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int col = (lir + s * LPR) * VEC + e;
                    if (col < d) {
                        const int i = s * VEC + e;
                        if (DO_S) red_s[col] = (wv == 0 ? 0.0 : red_s[col]) + (double)sacc[i];
                        if (DO_G) red_g[col] = (wv == 0 ? 0.0 : red_g[col]) + gacc[i];
                    }
                }
            }
        }
        __syncthreads();
    }
    if (DO_G) {
        r2 = group_sum<64>(r2);
        ax2 = group_sum<64>(ax2);
        if (lane == 0) {
            red_scal[2 * wave] = r2;
            red_scal[2 * wave + 1] = ax2;
        }
    }
    __syncthreads();
    const int64_t prow = (int64_t)blockIdx.x * a.dpad;
    for (int col = threadIdx.x; col < d; col += 64 * NW) {
        const double sc = FP8 ? (double)a.col_scale[col] : 1.0;
        if (DO_S) a.part_s[prow + col] = red_s[col] * sc;
        if (DO_G) a.part_g[prow + col] = red_g[col] * sc;
    }
    if (DO_G && threadIdx.x == 0) {
        double t0 = 0.0, t1 = 0.0;
        for (int wv = 0; wv < NW; ++wv) {
            t0 += red_scal[2 * wv];
            t1 += red_scal[2 * wv + 1];
        }
        a.part_scal[2 * blockIdx.x] = t0;
        a.part_scal[2 * blockIdx.x + 1] = t1;
    }
}

// ---- LDS-staged variant for rows of more than 32 vectors ------------------
//
// Rows stream through a ring of RING LDS tiles that direct global->LDS
// loads (global_load_lds_dword / _dwordx4) fill; a tile holds NW rows, one
// per wave.  While a wave works on tile t, the loads of tiles t+1 .. t+RING-1
// are in flight without occupying registers, so about (RING-1) * NW rows per
// CU are outstanding (registers only hold the column accumulators).  The
// ring is as deep as the LDS allows (ring_depth): 4 slots of 4 KB rows, 8
// of 2 KB rows and 12 of 1 KB rows, so narrow rows (BF16, FP8) keep as
// many bytes in flight as wide ones.  Every wave issues the same loads per tile (rows
// past the block's range and vectors past the row are clamped to valid
// addresses and ignored), so an explicit vmcnt wait covers exactly the
// loads of the tile about to be read, and the s_barrier that follows makes
// the whole tile visible and frees the slot refilled next.  Each ring slot
// is a separate LDS object, so the compiler's own waits for the loads into
// one slot do not hold back reads of another.  In G/SG mode the FP64 b of
// each row rides along as a 4-byte-per-lane load.
constexpr int RING_LDS = 150 * 1024;   // LDS bytes the ring may take
constexpr int ring_depth(int slot) {
    return slot * 12 <= RING_LDS ? 12 : slot * 8 <= RING_LDS ? 8 : slot * 6 <= RING_LDS ? 6 : 4;
}
constexpr int vmcnt_imm(int n) { return (n & 0xf) | (((n >> 4) & 3) << 14) | (0x7 << 4) | (0xf << 8); }

template <int DMAB>
__device__ __forceinline__ void lds_load(const void* src, void* lds) {
    void* g = const_cast<void*>(src);
    auto* l = (__attribute__((address_space(3))) void*)(lds);
    if constexpr (DMAB == 16) {
        __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
    } else {
        static_assert(DMAB == 4, "4- or 16-byte loads");
        __builtin_amdgcn_global_load_lds(g, l, 4, 0, 0);
    }
}

template <typename TS, int DMAB, int NSLOT, int MODE>
__global__ __launch_bounds__(64 * NW) void product_ring_kernel(ProdArgs a) {
    if (gated_off(a)) return;
    typedef typename Store<TS>::CT CT;
    typedef typename RawVec<DMAB>::T Raw;
    constexpr int VEC = DMAB / Store<TS>::BYTES;
    constexpr bool DO_S = MODE != PM_G;
    constexpr bool DO_G = MODE != PM_S;
    constexpr bool FP8 = std::is_same<TS, fp8_t>::value;
    constexpr int NC = NSLOT * VEC;
    constexpr int DCOLS = NC * 64;
    constexpr int RW = NSLOT * 64 * DMAB;            // staged bytes of one row
    // rows per wave and tile.  Two rows per wave (overlapping their
    // dot-product and reduction chains) measured no faster for 1 KB FP8 or
    // 2 KB BF16 rows of the SG mode: the VALU work per row (FP64 residual
    // and gradient accumulation, 16 columns per lane) bounds them, not the
    // per-row latency.
    constexpr int RPW = 1;
    constexpr int NOPS = RPW * (NSLOT + (DO_G ? 1 : 0));   // loads per wave per tile
    // one slot: RPW x NW staged rows, then (G/SG) 256 bytes per row for b
    constexpr int SLOT = RPW * NW * RW + (DO_G ? RPW * NW * 256 : 0);
    constexpr int RING = ring_depth(SLOT);
    static_assert(DCOLS * 8 <= NW * RW, "reduction buffers alias the ring");
    static_assert((RING - 2) * NOPS < 64, "vmcnt range");
    // one LDS object per slot (slots past RING are 16-byte placeholders),
    // each after a 16-byte guard: the loads of a shifted last row (see
    // issue) begin up to 12 bytes before its staging row
    __shared__ __align__(16) unsigned char t0_[SLOT + 16];
    __shared__ __align__(16) unsigned char t1_[SLOT + 16];
    __shared__ __align__(16) unsigned char t2_[SLOT + 16];
    __shared__ __align__(16) unsigned char t3_[SLOT + 16];
    __shared__ __align__(16) unsigned char t4_[RING > 4 ? SLOT + 16 : 32];
    __shared__ __align__(16) unsigned char t5_[RING > 5 ? SLOT + 16 : 32];
    __shared__ __align__(16) unsigned char t6_[RING > 6 ? SLOT + 16 : 32];
    __shared__ __align__(16) unsigned char t7_[RING > 7 ? SLOT + 16 : 32];
    __shared__ __align__(16) unsigned char t8_[RING > 8 ? SLOT + 16 : 32];
    __shared__ __align__(16) unsigned char t9_[RING > 9 ? SLOT + 16 : 32];
    __shared__ __align__(16) unsigned char t10_[RING > 10 ? SLOT + 16 : 32];
    __shared__ __align__(16) unsigned char t11_[RING > 11 ? SLOT + 16 : 32];
    unsigned char* const t0 = t0_ + 16;
    unsigned char* const t1 = t1_ + 16;
    unsigned char* const t2 = t2_ + 16;
    unsigned char* const t3 = t3_ + 16;
    unsigned char* const t4 = t4_ + 16;
    unsigned char* const t5 = t5_ + 16;
    unsigned char* const t6 = t6_ + 16;
    unsigned char* const t7 = t7_ + 16;
    unsigned char* const t8 = t8_ + 16;
    unsigned char* const t9 = t9_ + 16;
    unsigned char* const t10 = t10_ + 16;
    unsigned char* const t11 = t11_ + 16;
    __shared__ double red_scal[2 * NW];
    auto slot = [&](auto kc) -> unsigned char* {
        constexpr int k = decltype(kc)::value;
        if constexpr (k == 0) return t0;
        else if constexpr (k == 1) return t1;
        else if constexpr (k == 2) return t2;
        else if constexpr (k == 3) return t3;
        else if constexpr (k == 4) return t4;
        else if constexpr (k == 5) return t5;
        else if constexpr (k == 6) return t6;
        else if constexpr (k == 7) return t7;
        else if constexpr (k == 8) return t8;
        else if constexpr (k == 9) return t9;
        else if constexpr (k == 10) return t10;
        else return t11;
    };

    // wave index as a wave-uniform (scalar) value: row offsets stay in SGPRs
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int d = a.d;
    CT preg[NC];
    double xreg[NC];
    CT sacc[NC];
    double gacc[NC];
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const int i = s * VEC + e;
            const int col = (lane + s * 64) * VEC + e;
            const int cc = min(col, d - 1);
            const bool ok = col < d;
            const double sc = FP8 ? (double)a.col_scale[cc] : 1.0;
            const double pv = DO_S ? a.p[cc] * sc : 0.0;
            const double xv = DO_G ? a.x[cc] * sc : 0.0;
            preg[i] = ok ? (CT)pv : CT(0);
            xreg[i] = ok ? xv : 0.0;
            sacc[i] = CT(0);
            gacc[i] = 0.0;
        }
    }
    double r2 = 0.0, ax2 = 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * a.rpb;
    const int64_t r1 = min(a.m, r0 + a.rpb);
    const int64_t rlast = r1 - 1;   // >= 0: a.m >= 1 and r1 = a.m for blocks past the end
    const int64_t ntile = r1 > r0 ? (r1 - r0 + NW * RPW - 1) / (NW * RPW) : 0;
    const char* Abase = static_cast<const char*>(a.A);
    const int64_t row_bytes = a.lda * Store<TS>::BYTES;
    const int64_t vlast = a.nvec - 1;
    // Rows only 4-byte aligned (16-byte loads, lshift > 0): a row's last
    // vector reaches up to 12 bytes into the next row, except for the
    // matrix's last row (in the last block), whose vectors start lshift
    // bytes early (in the previous row) and land lshift bytes early in LDS,
    // so that its data sits where the reader expects it.  The last lshift
    // bytes of its staging row are then not loaded; they are read as
    // columns past d (times zero), so every staging row's last 16 bytes
    // start at zero here, before any load.
    const bool shifted = DMAB == 16 && a.lshift > 0 && r1 == a.m;
    if (shifted) {
        for (int e = threadIdx.x; e < RING * RPW * NW; e += 64 * NW) {
            const int sidx = e / (RPW * NW), rowi = e % (RPW * NW);
            unsigned char* sb = sidx == 0 ? t0 : sidx == 1 ? t1 : sidx == 2 ? t2 : sidx == 3 ? t3 : sidx == 4 ? t4
                              : sidx == 5 ? t5 : sidx == 6 ? t6 : sidx == 7 ? t7 : sidx == 8 ? t8 : sidx == 9 ? t9
                              : sidx == 10 ? t10 : t11;
            *reinterpret_cast<uint4*>(sb + rowi * RW + RW - 16) = make_uint4(0u, 0u, 0u, 0u);
        }
        __syncthreads();
    }

    // row rr of this wave in tile `tile` (rows of a wave stay in order)
    auto row_of = [&](int64_t tile, int rr) -> int64_t { return r0 + (tile * RPW + rr) * NW + wave; };
    auto issue = [&](int64_t tile, unsigned char* T) {
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) {
            const int64_t row = min(row_of(tile, rr), rlast);
            const int sh = (shifted && row == a.m - 1) ? a.lshift : 0;
            const char* src = Abase + row * row_bytes - sh;
            unsigned char* dst = T + (rr * NW + wave) * RW - sh;
#pragma unroll
            for (int s = 0; s < NSLOT; ++s) {
                const int64_t vi = min<int64_t>(s * 64 + lane, vlast);
                lds_load<DMAB>(src + vi * DMAB, dst + s * 64 * DMAB);
            }
            if constexpr (DO_G) {
                lds_load<4>(reinterpret_cast<const char*>(a.b + row * a.ldbv) + 4 * (lane & 1),
                            T + RPW * NW * RW + (rr * NW + wave) * 256);
            }
        }
    };
    auto consume = [&](int64_t tile, const unsigned char* T) {
        if (row_of(tile, 0) >= r1) return;
        CT v[RPW][NC];
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) {
#pragma unroll
            for (int s = 0; s < NSLOT; ++s) {
                const Raw raw = *reinterpret_cast<const Raw*>(T + (rr * NW + wave) * RW + (s * 64 + lane) * DMAB);
                Widen<TS, VEC, Raw>::run(raw, v[rr] + s * VEC);
            }
        }
        // two partial sums per dot product (even / odd columns of the lane)
        CT dp[RPW][2];
        double dx[RPW][2];
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) {
            dp[rr][0] = dp[rr][1] = CT(0);
            dx[rr][0] = dx[rr][1] = 0.0;
        }
#pragma unroll
        for (int i = 0; i < NC; ++i) {
#pragma unroll
            for (int rr = 0; rr < RPW; ++rr) {
                if (DO_S) dp[rr][i & 1] = fma(v[rr][i], preg[i], dp[rr][i & 1]);
                if (DO_G) dx[rr][i & 1] = fma((double)v[rr][i], xreg[i], dx[rr][i & 1]);
            }
        }
        CT ps[RPW];
        double w[RPW];
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) {
            // a row past the range (its loads were clamped to a valid row)
            // contributes nothing
            const bool live = row_of(tile, rr) < r1;
            ps[rr] = CT(0);
            w[rr] = 0.0;
            if (DO_S) {
                const CT t = wave_sum(dp[rr][0] + dp[rr][1]);
                ps[rr] = live ? t : CT(0);
            }
            if constexpr (DO_G) {
                const double ax = wave_sum(dx[rr][0] + dx[rr][1]);
                const double bb = *reinterpret_cast<const double*>(T + RPW * NW * RW + (rr * NW + wave) * 256);
                const double ww = bb - ax;
                w[rr] = live ? ww : 0.0;
                if (lane == 0 && live) {
                    r2 = fma(ww, ww, r2);
                    ax2 = fma(ax, ax, ax2);
                }
            }
        }
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) {
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                if (DO_S) sacc[i] = fma(ps[rr], v[rr][i], sacc[i]);
                if (DO_G) gacc[i] = fma(w[rr], (double)v[rr][i], gacc[i]);
            }
        }
    };

    static_for<0, RING - 1>([&](auto kc) { issue(decltype(kc)::value, slot(kc)); });
    for (int64_t t = 0; t < ntile; t += RING) {
        // step k: wait for tile t + k (slot k), refill slot k - 1 (read
        // at step k - 1, freed by this barrier) with tile t + k + RING - 1
        static_for<0, RING>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            __builtin_amdgcn_s_waitcnt(vmcnt_imm((RING - 2) * NOPS));
            __builtin_amdgcn_s_barrier();
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            issue(t + k + RING - 1, slot(std::integral_constant<int, (k + RING - 1) % RING>{}));
            consume(t + k, slot(kc));
        });
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // cross-lane, then fixed wave order into LDS (the ring is free now)
    double* red_s = reinterpret_cast<double*>(t0);
    double* red_g = reinterpret_cast<double*>(t1);
    for (int wv = 0; wv < NW; ++wv) {
        if (wave == wv) {
#pragma unroll
            for (int s = 0; s < NSLOT; ++s) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int col = (lane + s * 64) * VEC + e;
                    if (col < d) {
                        const int i = s * VEC + e;
                        if (DO_S) red_s[col] = (wv == 0 ? 0.0 : red_s[col]) + (double)sacc[i];
                        if (DO_G) red_g[col] = (wv == 0 ? 0.0 : red_g[col]) + gacc[i];
                    }
                }
            }
        }
        __syncthreads();
    }
    if (DO_G) {
        if (lane == 0) {
            red_scal[2 * wave] = r2;
            red_scal[2 * wave + 1] = ax2;
        }
    }
    __syncthreads();
    const int64_t prow = (int64_t)blockIdx.x * a.dpad;
    for (int col = threadIdx.x; col < d; col += 64 * NW) {
        const double sc = FP8 ? (double)a.col_scale[col] : 1.0;
        if (DO_S) a.part_s[prow + col] = red_s[col] * sc;
        if (DO_G) a.part_g[prow + col] = red_g[col] * sc;
    }
    if (DO_G && threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int wv = 0; wv < NW; ++wv) {
            s0 += red_scal[2 * wv];
            s1 += red_scal[2 * wv + 1];
        }
        a.part_scal[2 * blockIdx.x] = s0;
        a.part_scal[2 * blockIdx.x + 1] = s1;
    }
}

template <typename TS, int DMAB, int NSLOT>
hipError_t launch_ring(hipStream_t st, const ProdArgs& a, int mode, int nblocks) {
    dim3 grid(nblocks), block(64 * NW);
    switch (mode) {
        case PM_S: product_ring_kernel<TS, DMAB, NSLOT, PM_S><<<grid, block, 0, st>>>(a); break;
        case PM_G: product_ring_kernel<TS, DMAB, NSLOT, PM_G><<<grid, block, 0, st>>>(a); break;
        default: product_ring_kernel<TS, DMAB, NSLOT, PM_SG><<<grid, block, 0, st>>>(a); break;
    }
    return hipGetLastError();
}

// Ring shapes: 16-byte loads (VEC = 16 / element size) or 4-byte loads, at
// most 16 columns per lane (d <= 1024 with 16-byte loads).
template <typename TS>
hipError_t launch_ring_type(hipStream_t st, const ProdArgs& a, int mode, int nblocks, int dmab, int nslot) {
    constexpr int B = Store<TS>::BYTES;
    if (dmab == 16) {
        if (nslot == 1) return launch_ring<TS, 16, 1>(st, a, mode, nblocks);
        if constexpr (16 / B * 2 <= 16) {
            if (nslot == 2) return launch_ring<TS, 16, 2>(st, a, mode, nblocks);
        }
        if constexpr (16 / B * 4 <= 16) {
            if (nslot == 4) return launch_ring<TS, 16, 4>(st, a, mode, nblocks);
        }
    }
    if constexpr (B <= 4) {
        if (dmab == 4) {
            if (nslot == 1) return launch_ring<TS, 4, 1>(st, a, mode, nblocks);
            if (nslot == 2) return launch_ring<TS, 4, 2>(st, a, mode, nblocks);
            if (nslot == 4) return launch_ring<TS, 4, 4>(st, a, mode, nblocks);
        }
    }
    return hipErrorInvalidValue;
}

// rows in flight per wave: enough to keep ~64 KB of loads outstanding per
// CU with 16 resident waves, without spilling (the SG mode holds both
// products' operands and accumulators)
template <int NC, int MODE>
constexpr int unroll_rows() {
    return MODE == PM_S ? (NC <= 16 ? 4 : 2) : (NC <= 8 ? 4 : 2);
}

template <typename TS, int VEC, int LPR, int NSLOT>
hipError_t launch_shape(hipStream_t st, const ProdArgs& a, int mode, int nblocks) {
    dim3 grid(nblocks), block(64 * NW);
    switch (mode) {
        case PM_S:
            product_kernel<TS, VEC, LPR, NSLOT, PM_S, unroll_rows<NSLOT * VEC, PM_S>()><<<grid, block, 0, st>>>(a);
            break;
        case PM_G:
            product_kernel<TS, VEC, LPR, NSLOT, PM_G, unroll_rows<NSLOT * VEC, PM_G>()><<<grid, block, 0, st>>>(a);
            break;
        default:
            product_kernel<TS, VEC, LPR, NSLOT, PM_SG, unroll_rows<NSLOT * VEC, PM_SG>()><<<grid, block, 0, st>>>(a);
            break;
    }
    return hipGetLastError();
}

template <typename TS, int VEC>
hipError_t launch_vec(hipStream_t st, const ProdArgs& a, int mode, int nblocks, int lpr, int nslot) {
    if (lpr == 4) return launch_shape<TS, VEC, 4, 1>(st, a, mode, nblocks);
    if (lpr == 8) return launch_shape<TS, VEC, 8, 1>(st, a, mode, nblocks);
    if (lpr == 16) return launch_shape<TS, VEC, 16, 1>(st, a, mode, nblocks);
    if (lpr == 32) return launch_shape<TS, VEC, 32, 1>(st, a, mode, nblocks);
    if (nslot == 1) return launch_shape<TS, VEC, 64, 1>(st, a, mode, nblocks);
    if (nslot == 2) return launch_shape<TS, VEC, 64, 2>(st, a, mode, nblocks);
    if (nslot == 4) return launch_shape<TS, VEC, 64, 4>(st, a, mode, nblocks);
    if constexpr (VEC * 64 * 8 <= DMAX_LDS) {
        if (nslot == 8) return launch_shape<TS, VEC, 64, 8>(st, a, mode, nblocks);
    }
    if constexpr (VEC * 64 * 16 <= DMAX_LDS) {
        if (nslot == 16) return launch_shape<TS, VEC, 64, 16>(st, a, mode, nblocks);
    }
    return hipErrorInvalidValue;
}

template <typename TS>
hipError_t launch_type(hipStream_t st, const ProdArgs& a, int mode, int nblocks, int vec, int lpr,
                       int nslot) {
    if (vec == Store<TS>::VMAX) return launch_vec<TS, Store<TS>::VMAX>(st, a, mode, nblocks, lpr, nslot);
    if (vec == 1) return launch_vec<TS, 1>(st, a, mode, nblocks, lpr, nslot);
    return hipErrorInvalidValue;
}

}  // namespace

int64_t product_max_blocks(int num_cu) { return (int64_t)(num_cu > 0 ? num_cu : 256); }

int64_t product_max_d(int dtype) { return dtype == DT_F64 ? 2048 : 4096; }

hipError_t run_product(hipStream_t st, const ProdJob& j, int* nblocks_out) {
    *nblocks_out = 0;
    const int bytes = dtype_bytes(j.dtype);
    if (bytes == 0 || j.d < 1 || j.m < 0) return hipErrorInvalidValue;
    if (j.m == 0) return hipSuccess;
    // LDS-staged kernel for rows of more than 32 load vectors
    for (int dmab : {16, 4}) {
        if (dmab < bytes) continue;
        const int rv = dmab / bytes;
        const int64_t nv = ceil_div(j.d, rv);
        const bool mode_ok = j.mode == PM_S || j.ldbv >= 1;
        bool ok = (j.lda * bytes) % dmab == 0 && (uintptr_t)j.A % dmab == 0 && nv * rv <= j.dmem && mode_ok;
        int lshift = 0;
        if (!ok && dmab == 16 && mode_ok && (j.lda * bytes) % 4 == 0 && (uintptr_t)j.A % 4 == 0 && j.lda == j.dmem &&
            j.d * bytes >= 16 && j.m >= 2) {
            // rows only 4-byte aligned whose every stride byte is readable:
            // 16-byte loads reach into the next row, the last row is loaded
            // early (the kernel's shifted rows)
            ok = true;
            lshift = (int)(nv * 16 - j.d * bytes);
        }
        if (!ok) continue;
        if (nv <= 32 || nv > 256) break;
        int ns = 1;
        while (ns * 64 < nv) ns <<= 1;
        if (ns * rv > 16) break;
        int64_t nb = std::max<int64_t>(1, std::min<int64_t>(ceil_div(j.m, NW * 4), product_max_blocks(j.num_cu)));
        const int64_t rpb = ceil_div(j.m, nb);
        nb = ceil_div(j.m, rpb);
        ProdArgs a{};
        a.A = j.A;
        a.m = j.m;
        a.lda = j.lda;
        a.rpb = rpb;
        a.d = (int)j.d;
        a.nvec = (int)nv;
        a.col_scale = j.col_scale;
        a.b = j.b;
        a.ldbv = j.ldbv;
        a.x = j.x;
        a.p = j.p;
        a.part_s = j.part_s;
        a.part_g = j.part_g;
        a.part_scal = j.part_scal;
        a.dpad = j.dpad;
        a.gate = j.gate;
        a.gmin = j.gmin;
        a.lshift = lshift;
        hipError_t e;
        switch (j.dtype) {
            case DT_F64: e = launch_ring_type<double>(st, a, j.mode, (int)nb, dmab, ns); break;
            case DT_F32: e = launch_ring_type<float>(st, a, j.mode, (int)nb, dmab, ns); break;
            case DT_BF16: e = launch_ring_type<bf16_t>(st, a, j.mode, (int)nb, dmab, ns); break;
            case DT_FP8: e = launch_ring_type<fp8_t>(st, a, j.mode, (int)nb, dmab, ns); break;
            default: e = hipErrorInvalidValue;
        }
        if (e == hipSuccess) *nblocks_out = (int)nb;
        return e;
    }
    int vec = 16 / bytes;
    int64_t nvec = ceil_div(j.d, vec);
    const bool aligned = (j.lda % vec == 0) && ((uintptr_t)j.A % 16 == 0) && (nvec * vec <= j.dmem);
    if (!aligned) {
        vec = 1;
        nvec = j.d;
    }
    int lpr = 4;
    while (lpr < 64 && lpr < nvec) lpr <<= 1;
    int64_t ns = ceil_div(nvec, lpr);
    int nslot = 1;
    while (nslot < ns) nslot <<= 1;
    if (nslot > 16 || (int64_t)nslot * vec * lpr > DMAX_LDS) return hipErrorInvalidValue;
    const int64_t rows_per_sweep = (int64_t)NW * 4 * (64 / lpr);
    int64_t nb = ceil_div(j.m, rows_per_sweep * 2);
    nb = std::max<int64_t>(1, std::min<int64_t>(nb, product_max_blocks(j.num_cu)));
    int64_t rpb = ceil_div(j.m, nb);
    nb = ceil_div(j.m, rpb);
    ProdArgs a{};
    a.A = j.A;
    a.m = j.m;
    a.lda = j.lda;
    a.rpb = rpb;
    a.d = (int)j.d;
    a.nvec = (int)nvec;
    a.col_scale = j.col_scale;
    a.b = j.b;
    a.ldbv = j.ldbv;
    a.x = j.x;
    a.p = j.p;
    a.part_s = j.part_s;
    a.part_g = j.part_g;
    a.part_scal = j.part_scal;
    a.dpad = j.dpad;
    a.gate = j.gate;
    a.gmin = j.gmin;
    hipError_t e;
    switch (j.dtype) {
        case DT_F64: e = launch_type<double>(st, a, j.mode, (int)nb, vec, lpr, nslot); break;
        case DT_F32: e = launch_type<float>(st, a, j.mode, (int)nb, vec, lpr, nslot); break;
        case DT_BF16: e = launch_type<bf16_t>(st, a, j.mode, (int)nb, vec, lpr, nslot); break;
        case DT_FP8: e = launch_type<fp8_t>(st, a, j.mode, (int)nb, vec, lpr, nslot); break;
        default: e = hipErrorInvalidValue;
    }
    if (e == hipSuccess) *nblocks_out = (int)nb;
    return e;
}

}  // namespace spcg
