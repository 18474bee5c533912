// Nested CountSketch (the SPCG-CS variant of Sec. 4.3) on gfx950.
//
// A CountSketch with m buckets adds every row k of the data, times a random
// sign s(k), into bucket h(k): (S M)[b] = sum_{h(k) = b} s(k) M[k] (a sparse
// operator, Sec. 2.1; O(Nd) work, the remark after Theorem 3.4).  Buckets
// come from a keyed bijection q of the padded rows [0, N'): h(k) = q(k) mod m,
// so each bucket receives floor(N'/m) or ceil(N'/m) rows and nested sizes
// m_i | m_{i+1} give S_i M by folding S_{i+1} M (buckets b + t m_i added).
//
// The gather kernel inverts the map: a table lists, for every slot y, the
// row k with q(k) = y and its sign, and bucket b sums the rows of slots
// b, b + m, b + 2m, ... in that order (fixed order, no atomics).  A group
// of 16, 32 or 64 lanes (the narrowest that covers the row, 4 columns per
// lane) handles one (bucket, window) pair and keeps up to four row segments
// in flight; the rows are random, but each segment is contiguous (1 KB for a
// 256-column FP32 window).  Every row of X is read exactly once per sketch.
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"
#include "rng.hpp"

namespace spcg {

namespace {

constexpr int CS_WAVES = 4;     // waves per block
constexpr int CS_MU = 4;        // member rows in flight per wave

__global__ void cs_tables_kernel(uint64_t seed, int L, int64_t np, int32_t* tbl, int32_t* tbl_hat,
                                 const uint32_t* rt, const uint32_t* rt_hat) {
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= np) return;
    if (tbl) {
        const uint64_t k = feistel_inv_tab((uint32_t)y, L, rt);
        tbl[y] = (int32_t)((uint32_t)k | (sign_bit(seed, k) << 31));
    }
    if (tbl_hat) {
        const uint64_t k = feistel_inv_tab((uint32_t)y, L, rt_hat);
        tbl_hat[y] = (int32_t)((uint32_t)k | (sign_bit_stream(seed, k, STREAM_CS_HAT_SIGN) << 31));
    }
}

// Four consecutive elements of row `row` from column c, widened; zeros
// beyond d.
template <typename TIN, typename TZ>
struct Load4;
template <>
struct Load4<double, double> {
    __device__ static void run(const void* x, int64_t row, int64_t ldx, int64_t c, int64_t d, bool vec, const float*,
                               double* o) {
        const double* p = static_cast<const double*>(x) + row * ldx + c;
        if (vec && c + 4 <= d) {
            const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
            o[0] = a.x;
            o[1] = a.y;
            o[2] = b.x;
            o[3] = b.y;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = c + e < d ? p[e] : 0.0;
        }
    }
};
template <>
struct Load4<float, float> {
    __device__ static void run(const void* x, int64_t row, int64_t ldx, int64_t c, int64_t d, bool vec, const float*,
                               float* o) {
        const float* p = static_cast<const float*>(x) + row * ldx + c;
        if (vec && c + 4 <= d) {
            const float4 a = *reinterpret_cast<const float4*>(p);
            o[0] = a.x;
            o[1] = a.y;
            o[2] = a.z;
            o[3] = a.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = c + e < d ? p[e] : 0.f;
        }
    }
};
template <>
struct Load4<bf16_t, float> {
    __device__ static void run(const void* x, int64_t row, int64_t ldx, int64_t c, int64_t d, bool vec, const float*,
                               float* o) {
        const uint16_t* p = static_cast<const uint16_t*>(x) + row * ldx + c;
        if (vec && c + 4 <= d) {
            const uint2 a = *reinterpret_cast<const uint2*>(p);
            o[0] = __uint_as_float(a.x << 16);
            o[1] = __uint_as_float(a.x & 0xffff0000u);
            o[2] = __uint_as_float(a.y << 16);
            o[3] = __uint_as_float(a.y & 0xffff0000u);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = c + e < d ? bf16_bits_to_f32(p[e]) : 0.f;
        }
    }
};
template <>
struct Load4<fp8_t, float> {
    __device__ static void run(const void* x, int64_t row, int64_t ldx, int64_t c, int64_t d, bool vec,
                               const float* sc, float* o) {
        const uint8_t* p = static_cast<const uint8_t*>(x) + row * ldx + c;
        if (vec && c + 4 <= d) {
            const uint32_t a = *reinterpret_cast<const uint32_t*>(p);
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = fp8e4m3_bits_to_f32((a >> (8 * e)) & 0xffu) * sc[c + e];
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = c + e < d ? fp8e4m3_bits_to_f32(p[e]) * sc[c + e] : 0.f;
        }
    }
};

__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

template <typename TZ>
__device__ __forceinline__ void store4(void* out, int out_dtype, int64_t idx, const TZ* v) {
    if constexpr (std::is_same<TZ, double>::value) {
        double2* p = reinterpret_cast<double2*>(static_cast<double*>(out) + idx);
        p[0] = make_double2(v[0], v[1]);
        p[1] = make_double2(v[2], v[3]);
    } else {
        if (out_dtype == DT_BF16) {
            const uint32_t w0 = f32_to_bf16_rne(v[0]) | (f32_to_bf16_rne(v[1]) << 16);
            const uint32_t w1 = f32_to_bf16_rne(v[2]) | (f32_to_bf16_rne(v[3]) << 16);
            *reinterpret_cast<uint2*>(static_cast<uint16_t*>(out) + idx) = make_uint2(w0, w1);
        } else {
            *reinterpret_cast<float4*>(static_cast<float*>(out) + idx) = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
}

// C consecutive elements of one row, as raw 32-bit words (loaded first,
// widened later, so that many rows' loads are in flight at once).
template <typename TIN, int C>
struct Piece {
    static constexpr int EB = (int)sizeof(TIN);
    static constexpr int NW = (C * EB + 3) / 4;
    uint32_t w[NW];
};

// the row's elements col .. col + C - 1 (zeros past d); one vector load
// when the piece lies inside the row and vec is set
template <typename TIN, int C>
__device__ __forceinline__ void load_piece(Piece<TIN, C>& pc, const void* x, int64_t row, int64_t ldx, int64_t col,
                                           int64_t d, bool vec) {
    constexpr int EB = (int)sizeof(TIN), BYTES = C * EB;
    const unsigned char* p = static_cast<const unsigned char*>(x) + (row * ldx + col) * EB;
    if (vec && col + C <= d) {
        if constexpr (BYTES == 8) {
            const uint2 v = *reinterpret_cast<const uint2*>(p);
            pc.w[0] = v.x;
            pc.w[1] = v.y;
        } else {
            static_assert(BYTES % 16 == 0, "8-, 16- or 32-byte pieces");
#pragma unroll
            for (int h = 0; h < BYTES / 16; ++h) {
                const uint4 v = reinterpret_cast<const uint4*>(p)[h];
                pc.w[4 * h] = v.x;
                pc.w[4 * h + 1] = v.y;
                pc.w[4 * h + 2] = v.z;
                pc.w[4 * h + 3] = v.w;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < Piece<TIN, C>::NW; ++i) pc.w[i] = 0u;
#pragma unroll
        for (int e = 0; e < C; ++e) {
            if (col + e < d) {
                if constexpr (EB == 1) {
                    pc.w[e / 4] |= (uint32_t)p[e] << (8 * (e % 4));
                } else if constexpr (EB == 2) {
                    pc.w[e / 2] |= (uint32_t)reinterpret_cast<const uint16_t*>(p)[e] << (16 * (e % 2));
                } else if constexpr (EB == 4) {
                    pc.w[e] = reinterpret_cast<const uint32_t*>(p)[e];
                } else {
                    pc.w[2 * e] = reinterpret_cast<const uint32_t*>(p)[2 * e];
                    pc.w[2 * e + 1] = reinterpret_cast<const uint32_t*>(p)[2 * e + 1];
                }
            }
        }
    }
}

// exact widening of a piece (FP8 without its column scale)
template <typename TIN, typename TZ, int C>
__device__ __forceinline__ void widen_piece(const Piece<TIN, C>& pc, TZ* o) {
    if constexpr (std::is_same<TIN, double>::value) {
#pragma unroll
        for (int e = 0; e < C; ++e) o[e] = __hiloint2double((int)pc.w[2 * e + 1], (int)pc.w[2 * e]);
    } else if constexpr (std::is_same<TIN, float>::value) {
#pragma unroll
        for (int e = 0; e < C; ++e) o[e] = __uint_as_float(pc.w[e]);
    } else if constexpr (std::is_same<TIN, bf16_t>::value) {
#pragma unroll
        for (int e = 0; e < C; e += 2) {
            o[e] = __uint_as_float(pc.w[e / 2] << 16);
            o[e + 1] = __uint_as_float(pc.w[e / 2] & 0xffff0000u);
        }
    } else {
        typedef float v2f_t __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int e = 0; e < C; e += 4) {
            const v2f_t lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)pc.w[e / 4], false);
            const v2f_t hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)pc.w[e / 4], true);
            o[e] = lo.x;
            o[e + 1] = lo.y;
            o[e + 2] = hi.x;
            o[e + 3] = hi.y;
        }
    }
}

// C columns per lane: 16-byte pieces (8-byte for FP8, two 16-byte loads for
// FP64); a lane group of LPB lanes covers a C LPB-column window.
template <typename TIN>
constexpr int tree_cols() {
    return std::is_same<TIN, bf16_t>::value || std::is_same<TIN, fp8_t>::value ? 8 : 4;
}
struct GatherArgs {
    CsJob j;
    int nwin;      // column windows per row
    int xvec;      // rows allow aligned 4-element loads
    int nseg;      // segments per bucket (slots t = seg, seg + nseg, ...)
    void* seg_out; // nseg > 1: partial sums [seg][bucket][ld] in the sum type
};

// LPB lanes take one (bucket, C LPB-column window) pair (C = tree_cols:
// 8 for BF16 / FP8, 4 otherwise), so a wave holds 64 / LPB buckets at once
// when the rows are short.
template <typename TIN, typename TZ, int LPB>
__global__ __launch_bounds__(64 * CS_WAVES) void cs_gather_kernel(GatherArgs a) {
    constexpr int NG = 64 / LPB;
    constexpr int C = tree_cols<TIN>();
    constexpr bool FP8 = std::is_same<TIN, fp8_t>::value;
    const CsJob& j = a.j;
    const int lane = threadIdx.x & 63, gi = lane / LPB, sl = lane % LPB;
    const int64_t wave0 = (int64_t)blockIdx.x * CS_WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t nwaves = (int64_t)gridDim.x * CS_WAVES;
    const int64_t ntask = j.nbk * a.nwin * a.nseg;
    const int64_t step = (int64_t)a.nseg * j.nbk;    // between a segment's slots
    const bool vec = a.xvec != 0;
    for (int64_t t0 = wave0 * NG; t0 < ntask; t0 += nwaves * NG) {
        const int64_t task = t0 + gi;
        if (task >= ntask) continue;
        const int64_t rest = task / a.nseg;
        const int sg = (int)(task - rest * a.nseg);
        const int64_t b = rest / a.nwin;
        const int w = (int)(rest - b * a.nwin);
        const int64_t c = (int64_t)w * C * LPB + C * sl;
        const bool do_y = j.outy && w == 0;
        TZ acc[C];
#pragma unroll
        for (int q = 0; q < C; ++q) acc[q] = TZ(0);
        double yacc = 0.0;
        for (int64_t y0 = b + sg * j.nbk; y0 < j.Np; y0 += CS_MU * step) {
            int32_t e[CS_MU];
#pragma unroll
            for (int u = 0; u < CS_MU; ++u) {
                const int64_t yv = y0 + (int64_t)u * step;
                e[u] = yv < j.Np ? j.tbl[yv] : 0x7fffffff;   // past the end: no row
            }
            Piece<TIN, C> pc[CS_MU];
            double yv_[CS_MU];
#pragma unroll
            for (int u = 0; u < CS_MU; ++u) {
                const int64_t k = e[u] & 0x7fffffff;
                yv_[u] = 0.0;
                if (k < j.N) {
                    load_piece<TIN, C>(pc[u], j.x, k, j.ldx, c, j.d, vec);
                    if (do_y && sl < j.k) yv_[u] = j.y[k * j.ldy_in + sl];
                } else {
#pragma unroll
                    for (int i = 0; i < Piece<TIN, C>::NW; ++i) pc[u].w[i] = 0u;
                }
            }
#pragma unroll
            for (int u = 0; u < CS_MU; ++u) {
                TZ v[C];
                widen_piece<TIN, TZ, C>(pc[u], v);
                const bool neg = e[u] < 0;
#pragma unroll
                for (int q = 0; q < C; ++q) acc[q] += neg ? -v[q] : v[q];
                yacc += neg ? -yv_[u] : yv_[u];
            }
        }
        // FP8: the power-of-two column scales, applied to the sums (exact)
        if constexpr (FP8) {
#pragma unroll
            for (int q = 0; q < C; ++q) acc[q] *= c + q < j.d ? j.col_scale[c + q] : 0.f;
        }
        constexpr int SUM_DT = std::is_same<TZ, double>::value ? DT_F64 : DT_F32;
        if (c < j.ld) {
#pragma unroll
            for (int q = 0; q < C; q += 4) {
                if (a.nseg > 1) {
                    store4<TZ>(a.seg_out, SUM_DT, ((int64_t)sg * j.nbk + b) * j.ld + c + q, acc + q);
                } else {
                    store4<TZ>(j.out, j.out_dtype, b * j.ld + c + q, acc + q);
                    if (j.work) store4<TZ>(j.work, SUM_DT, b * j.ld + c + q, acc + q);
                }
            }
        }
        if (do_y && sl < j.ldoy) j.outy[b * j.ldoy + sl] = sl < j.k ? yacc : 0.0;
    }
}

// Bucket rows from segment partials: sum over segments in ascending order.
template <typename TZ>
__global__ __launch_bounds__(256) void cs_seg_reduce_kernel(const TZ* part, int nseg, int64_t nbk, int64_t ld, void* out,
                                                            int out_dtype) {
    const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (e >= nbk * ld) return;
    TZ v[4] = {TZ(0), TZ(0), TZ(0), TZ(0)};
    for (int sg = 0; sg < nseg; ++sg) {
        const TZ* p = part + (int64_t)sg * nbk * ld + e;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += p[q];
    }
    store4<TZ>(out, out_dtype, e, v);
}

template <typename TZ>
__global__ __launch_bounds__(256) void cs_fold_kernel(const TZ* src, TZ* work, void* dst, int out_dtype, int64_t ld,
                                                      int64_t mc, int g) {
    const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;   // first of 4 columns
    if (e >= mc * ld) return;
    const int64_t b = e / ld, c = e - b * ld;
    TZ v[4] = {TZ(0), TZ(0), TZ(0), TZ(0)};
    for (int t = 0; t < g; ++t) {
        const TZ* p = src + (b + (int64_t)t * mc) * ld + c;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += p[q];
    }
    if (work) {
#pragma unroll
        for (int q = 0; q < 4; ++q) work[b * ld + c + q] = v[q];
    }
    store4<TZ>(dst, out_dtype, b * ld + c, v);
}

__global__ __launch_bounds__(256) void cs_fold_y_kernel(const double* src, double* dst, int64_t ldy, int64_t mc, int g) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= mc * ldy) return;
    const int64_t b = e / ldy, c = e - b * ldy;
    double v = 0.0;
    for (int t = 0; t < g; ++t) v += src[(b + (int64_t)t * mc) * ldy + c];
    dst[e] = v;
}


struct TreeArgs {
    CsJob j;                 // j.nbk: finest bucket count
    int nwin, xvec;
    void* out[4];
    double* outy[4];
    int64_t m[4];
    void* work;
};

constexpr int ipow(int g, int j) { return j == 0 ? 1 : g * ipow(g, j - 1); }

constexpr int TREE_MU = 2;      // slots per finest bucket loaded together

// BF16 / FP8 input: 8 columns per lane (16- or 8-byte pieces) and every
// finest bucket's TREE_MU next rows loaded together (the 4-column kernel
// left these narrow rows latency-bound: 6.6-7.4 ms whatever the element
// size at N = 4e6, d = 1000)
template <typename TIN, typename TZ, int G, int J, int LPB>
__global__ __launch_bounds__(64 * CS_WAVES) void cs_gather_tree_kernel(TreeArgs a) {
    static_assert(tree_cols<TIN>() == 8, "narrow input only");
    constexpr int NF = ipow(G, J);   // finest buckets per coarse bucket
    constexpr int NG = 64 / LPB;     // coarse buckets per wave (short rows)
    constexpr int C = tree_cols<TIN>();
    constexpr bool FP8 = std::is_same<TIN, fp8_t>::value;
    const CsJob& j = a.j;
    const int lane = threadIdx.x & 63, gi = lane / LPB, sl = lane % LPB;
    const int64_t wave0 = (int64_t)blockIdx.x * CS_WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t nwaves = (int64_t)gridDim.x * CS_WAVES;
    const int64_t mc = a.m[J];
    const int64_t ntask = mc * a.nwin;
    const bool vec = a.xvec != 0;
    for (int64_t t0 = wave0 * NG; t0 < ntask; t0 += nwaves * NG) {
        const int64_t task = t0 + gi;
        if (task >= ntask) continue;
        const int64_t c = task / a.nwin;
        const int w = (int)(task - c * a.nwin);
        const int64_t col = (int64_t)w * C * LPB + C * sl;
        const bool do_y = j.outy && w == 0;
        TZ acc[NF][C];
        double yacc[NF];
#pragma unroll
        for (int t = 0; t < NF; ++t) {
#pragma unroll
            for (int q = 0; q < C; ++q) acc[t][q] = TZ(0);
            yacc[t] = 0.0;
        }
        // the slots of finest bucket c + t mc are c + t mc + s nbk, s =
        // 0, 1, ...; TREE_MU slots of every finest bucket per round, all
        // rows' loads issued before any is added, each bucket's rows added
        // in ascending slot order
        for (int64_t s0 = 0; c + s0 * j.nbk < j.Np; s0 += TREE_MU) {
            int32_t e[NF][TREE_MU];
#pragma unroll
            for (int t = 0; t < NF; ++t) {
#pragma unroll
                for (int u = 0; u < TREE_MU; ++u) {
                    const int64_t yv = c + t * mc + (s0 + u) * j.nbk;
                    e[t][u] = yv < j.Np ? j.tbl[yv] : 0x7fffffff;   // past the end: no row
                }
            }
            Piece<TIN, C> pc[NF][TREE_MU];
            double yv_[NF][TREE_MU];
#pragma unroll
            for (int t = 0; t < NF; ++t) {
#pragma unroll
                for (int u = 0; u < TREE_MU; ++u) {
                    const int64_t k = e[t][u] & 0x7fffffff;
                    yv_[t][u] = 0.0;
                    if (k < j.N) {
                        load_piece<TIN, C>(pc[t][u], j.x, k, j.ldx, col, j.d, vec);
                        if (do_y && sl < j.k) yv_[t][u] = j.y[k * j.ldy_in + sl];
                    } else {
#pragma unroll
                        for (int i = 0; i < Piece<TIN, C>::NW; ++i) pc[t][u].w[i] = 0u;
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < NF; ++t) {
#pragma unroll
                for (int u = 0; u < TREE_MU; ++u) {
                    TZ v[C];
                    widen_piece<TIN, TZ, C>(pc[t][u], v);
                    const bool neg = e[t][u] < 0;
#pragma unroll
                    for (int q = 0; q < C; ++q) acc[t][q] += neg ? -v[q] : v[q];
                    yacc[t] += neg ? -yv_[t][u] : yv_[t][u];
                }
            }
        }
        // FP8: the power-of-two column scales, applied to the sums (exact:
        // scaling by 2^e commutes with FP32 rounding in the normal range)
        if constexpr (FP8) {
#pragma unroll
            for (int q = 0; q < C; ++q) {
                const float sc = col + q < j.d ? j.col_scale[col + q] : 0.f;
#pragma unroll
                for (int t = 0; t < NF; ++t) acc[t][q] *= sc;
            }
        }
        auto put = [&](void* out, int dt, int64_t row, const TZ* v) __attribute__((always_inline)) {
#pragma unroll
            for (int q = 0; q < C; q += 4) store4<TZ>(out, dt, row * j.ld + col + q, v + q);
        };
#pragma unroll
        for (int t = 0; t < NF; ++t) {
            if (col < j.ld) put(a.out[0], j.out_dtype, c + t * mc, acc[t]);
            if (do_y && sl < j.ldoy) a.outy[0][(c + t * mc) * j.ldoy + sl] = sl < j.k ? yacc[t] : 0.0;
        }
        // coarser levels: bucket s of level l adds buckets s + r G^(J-l) of
        // level l - 1 in ascending r (the folding order)
#pragma unroll
        for (int l = 1; l <= J; ++l) {
            const int nb = ipow(G, J - l);
#pragma unroll
            for (int s2 = 0; s2 < NF; ++s2) {
                if (s2 >= nb) continue;
#pragma unroll
                for (int r = 1; r < G; ++r) {
#pragma unroll
                    for (int q = 0; q < C; ++q) acc[s2][q] += acc[s2 + r * nb][q];
                    yacc[s2] += yacc[s2 + r * nb];
                }
                if (col < j.ld) put(a.out[l], j.out_dtype, c + s2 * mc, acc[s2]);
                if (do_y && sl < j.ldoy) a.outy[l][(c + s2 * mc) * j.ldoy + sl] = sl < j.k ? yacc[s2] : 0.0;
            }
        }
        if (a.work && col < j.ld) put(a.work, std::is_same<TZ, double>::value ? DT_F64 : DT_F32, c, acc[0]);
    }
}

// FP32 / FP64 input: 4 columns per lane, each finest bucket's rows walked
// in turn (CS_MU at a time); at high occupancy this keeps the FP32 pass
// near the mixed read/write ceiling, where loading every finest bucket's
// rows together (cs_gather_tree_kernel) measured slower (9.9 against
// 11.6 ms for the sketch phase at N = 4e6, d = 1000)
template <typename TIN, typename TZ, int G, int J, int LPB>
__global__ __launch_bounds__(64 * CS_WAVES) void cs_gather_tree4_kernel(TreeArgs a) {
    constexpr int NF = ipow(G, J);   // finest buckets per coarse bucket
    constexpr int NG = 64 / LPB;     // coarse buckets per wave (short rows)
    const CsJob& j = a.j;
    const int lane = threadIdx.x & 63, gi = lane / LPB, sl = lane % LPB;
    const int64_t wave0 = (int64_t)blockIdx.x * CS_WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t nwaves = (int64_t)gridDim.x * CS_WAVES;
    const int64_t mc = a.m[J];
    const int64_t ntask = mc * a.nwin;
    const bool vec = a.xvec != 0;
    for (int64_t t0 = wave0 * NG; t0 < ntask; t0 += nwaves * NG) {
        const int64_t task = t0 + gi;
        if (task >= ntask) continue;
        const int64_t c = task / a.nwin;
        const int w = (int)(task - c * a.nwin);
        const int64_t col = (int64_t)w * 4 * LPB + 4 * sl;
        const bool do_y = j.outy && w == 0;
        TZ acc[NF][4];
        double yacc[NF];
#pragma unroll
        for (int t = 0; t < NF; ++t) {
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[t][q] = TZ(0);
            yacc[t] = 0.0;
            // finest bucket c + t mc: its slots in ascending order
            for (int64_t y0 = c + t * mc; y0 < j.Np; y0 += CS_MU * j.nbk) {
                int32_t e[CS_MU];
#pragma unroll
                for (int u = 0; u < CS_MU; ++u) {
                    const int64_t yv = y0 + (int64_t)u * j.nbk;
                    e[u] = yv < j.Np ? j.tbl[yv] : 0x7fffffff;
                }
                TZ v[CS_MU][4];
                double yv_[CS_MU];
#pragma unroll
                for (int u = 0; u < CS_MU; ++u) {
                    const int64_t k = e[u] & 0x7fffffff;
                    yv_[u] = 0.0;
                    if (k < j.N) {
                        Load4<TIN, TZ>::run(j.x, k, j.ldx, col, j.d, vec, j.col_scale, v[u]);
                        if (do_y && sl < j.k) yv_[u] = j.y[k * j.ldy_in + sl];
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) v[u][q] = TZ(0);
                    }
                }
#pragma unroll
                for (int u = 0; u < CS_MU; ++u) {
                    const bool neg = e[u] < 0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[t][q] += neg ? -v[u][q] : v[u][q];
                    yacc[t] += neg ? -yv_[u] : yv_[u];
                }
            }
            if (col < j.ld) store4<TZ>(a.out[0], j.out_dtype, (c + t * mc) * j.ld + col, acc[t]);
            if (do_y && sl < j.ldoy) a.outy[0][(c + t * mc) * j.ldoy + sl] = sl < j.k ? yacc[t] : 0.0;
        }
        // coarser levels: bucket s of level l adds buckets s + r G^(J-l) of
        // level l - 1 in ascending r (the folding order)
#pragma unroll
        for (int l = 1; l <= J; ++l) {
            const int nb = ipow(G, J - l);
#pragma unroll
            for (int s2 = 0; s2 < NF; ++s2) {
                if (s2 >= nb) continue;
#pragma unroll
                for (int r = 1; r < G; ++r) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[s2][q] += acc[s2 + r * nb][q];
                    yacc[s2] += yacc[s2 + r * nb];
                }
                if (col < j.ld) store4<TZ>(a.out[l], j.out_dtype, (c + s2 * mc) * j.ld + col, acc[s2]);
                if (do_y && sl < j.ldoy) a.outy[l][(c + s2 * mc) * j.ldoy + sl] = sl < j.k ? yacc[s2] : 0.0;
            }
        }
        if (a.work && col < j.ld)
            store4<TZ>(a.work, std::is_same<TZ, double>::value ? DT_F64 : DT_F32, c * j.ld + col, acc[0]);
    }
}

template <typename TIN, typename TZ, int G, int J, int LPB>
hipError_t tree_launch(hipStream_t st, const TreeArgs& a) {
    const int64_t ntask = a.m[J] * a.nwin;
    const int64_t blocks = std::min<int64_t>(ceil_div(ntask, CS_WAVES * (64 / LPB)), 65536);
    if constexpr (tree_cols<TIN>() == 4)
        cs_gather_tree4_kernel<TIN, TZ, G, J, LPB><<<dim3((unsigned)blocks), dim3(64 * CS_WAVES), 0, st>>>(a);
    else
        cs_gather_tree_kernel<TIN, TZ, G, J, LPB><<<dim3((unsigned)blocks), dim3(64 * CS_WAVES), 0, st>>>(a);
    return hipGetLastError();
}

template <typename TIN, typename TZ, int LPB>
hipError_t tree_dispatch_l(hipStream_t st, const TreeArgs& a, int g, int levels) {
    if (levels == 0) return tree_launch<TIN, TZ, 2, 0, LPB>(st, a);
    if (g == 2) {
        if (levels == 1) return tree_launch<TIN, TZ, 2, 1, LPB>(st, a);
        if (levels == 2) return tree_launch<TIN, TZ, 2, 2, LPB>(st, a);
        if (levels == 3) return tree_launch<TIN, TZ, 2, 3, LPB>(st, a);
    }
    if (g == 4 && levels == 1) return tree_launch<TIN, TZ, 4, 1, LPB>(st, a);
    return hipErrorInvalidValue;
}

template <typename TIN, typename TZ>
hipError_t tree_dispatch(hipStream_t st, const TreeArgs& a, int g, int levels, int lpb) {
    if (lpb == 16) return tree_dispatch_l<TIN, TZ, 16>(st, a, g, levels);
    if (lpb == 32) return tree_dispatch_l<TIN, TZ, 32>(st, a, g, levels);
    return tree_dispatch_l<TIN, TZ, 64>(st, a, g, levels);
}

template <typename TIN, typename TZ, int LPB>
hipError_t gather_launch_l(hipStream_t st, const GatherArgs& a) {
    const int64_t ntask = a.j.nbk * a.nwin * a.nseg;
    const int64_t blocks = std::min<int64_t>(ceil_div(ntask, CS_WAVES * (64 / LPB)), 65536);
    cs_gather_kernel<TIN, TZ, LPB><<<dim3((unsigned)blocks), dim3(64 * CS_WAVES), 0, st>>>(a);
    return hipGetLastError();
}

template <typename TIN, typename TZ>
hipError_t gather_launch(hipStream_t st, const GatherArgs& a, int lpb) {
    if (lpb == 16) return gather_launch_l<TIN, TZ, 16>(st, a);
    if (lpb == 32) return gather_launch_l<TIN, TZ, 32>(st, a);
    return gather_launch_l<TIN, TZ, 64>(st, a);
}

// Lanes per (bucket, window): the narrowest power of two >= 16 that covers
// the row with `cols` columns per lane (and the responses, one per lane).
int lanes_per_bucket(int64_t ld, int64_t k, int cols = 4) {
    int lpb = 16;
    while (lpb < 64 && (cols * lpb < ld || lpb < k)) lpb *= 2;
    return lpb;
}

}  // namespace

hipError_t launch_cs_tables(hipStream_t st, uint64_t seed, int L, int32_t* tbl, int32_t* tbl_hat, uint32_t* rt) {
    if (L < 1 || L > 30 || !rt) return hipErrorInvalidValue;
    const int64_t np = 1ll << L, ts = feistel_table_size(L);
    const uint64_t streams[2] = {STREAM_CS, STREAM_CS_HAT};
    const hipError_t e = launch_feistel_tables(st, seed, L, 2, streams, rt);
    if (e != hipSuccess) return e;
    cs_tables_kernel<<<(unsigned)ceil_div(np, 256), 256, 0, st>>>(seed, L, np, tbl, tbl_hat, rt, rt + ts);
    return hipGetLastError();
}

hipError_t run_cs_gather(hipStream_t st, const CsJob& j) {
    const bool f64 = j.in_dtype == DT_F64;
    if (j.nbk <= 0 || j.ld < j.d || j.ld % 4 != 0 || j.Np >= (1ll << 31) || j.N > j.Np) return hipErrorInvalidValue;
    if (f64 != (j.out_dtype == DT_F64)) return hipErrorInvalidValue;
    if (j.outy && (j.k < 1 || j.k > 64 || j.ldoy < j.k || j.ldoy > 64)) return hipErrorInvalidValue;
    GatherArgs a{};
    a.j = j;
    const int C = (j.in_dtype == DT_BF16 || j.in_dtype == DT_FP8) ? 8 : 4;   // tree_cols
    const int lpb = lanes_per_bucket(j.ld, j.outy ? std::max<int64_t>(j.k, j.ldoy) : 1, C);
    a.nwin = (int)ceil_div(j.ld, (int64_t)C * lpb);
    // few, long buckets (the preconditioner sketch at small d): split each
    // bucket's slots over segments so that enough lane groups stream rows
    a.nseg = 1;
    const int64_t groups = j.nbk * a.nwin, members = ceil_div(j.Np, j.nbk);
    const size_t sum_es = (j.in_dtype == DT_F64) ? 8 : 4;
    if (!j.outy && !j.work && j.scratch && groups < 16384 && members > 64) {
        int64_t ns = std::min<int64_t>(ceil_div(16384, groups), members / 16);
        ns = std::min<int64_t>(ns, (int64_t)(j.scratch_bytes / ((size_t)j.nbk * j.ld * sum_es)));
        if (ns > 1) {
            a.nseg = (int)ns;
            a.seg_out = j.scratch;
        }
    }
    const int es = dtype_bytes(j.in_dtype);
    const int64_t align = std::min<int64_t>(16, (int64_t)C * es);
    a.xvec = (j.ldx * es) % align == 0 && (uintptr_t)j.x % align == 0;
    hipError_t e;
    switch (j.in_dtype) {
        case DT_F64: e = gather_launch<double, double>(st, a, lpb); break;
        case DT_F32: e = gather_launch<float, float>(st, a, lpb); break;
        case DT_BF16: e = gather_launch<bf16_t, float>(st, a, lpb); break;
        case DT_FP8: e = gather_launch<fp8_t, float>(st, a, lpb); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || a.nseg == 1) return e;
    const unsigned blocks = (unsigned)ceil_div(j.nbk * j.ld / 4, 256);
    if (f64)
        cs_seg_reduce_kernel<double><<<blocks, 256, 0, st>>>(static_cast<const double*>(a.seg_out), a.nseg, j.nbk,
                                                             j.ld, j.out, j.out_dtype);
    else
        cs_seg_reduce_kernel<float><<<blocks, 256, 0, st>>>(static_cast<const float*>(a.seg_out), a.nseg, j.nbk, j.ld,
                                                            j.out, j.out_dtype);
    return hipGetLastError();
}

hipError_t run_cs_gather_tree(hipStream_t st, const CsTreeJob& t) {
    const CsJob& j = t.base;
    const bool f64 = j.in_dtype == DT_F64;
    if (t.levels < 0 || t.levels > 3 || j.nbk != t.m[0] || j.ld < j.d || j.ld % 4 != 0 || j.Np >= (1ll << 31) ||
        j.N > j.Np)
        return hipErrorInvalidValue;
    for (int l = 1; l <= t.levels; ++l)
        if (t.m[l] <= 0 || t.m[l - 1] != t.m[l] * t.growth) return hipErrorInvalidValue;
    if (f64 != (j.out_dtype == DT_F64)) return hipErrorInvalidValue;
    if (j.outy && (j.k < 1 || j.k > 64 || j.ldoy < j.k || j.ldoy > 64)) return hipErrorInvalidValue;
    TreeArgs a{};
    a.j = j;
    a.j.outy = nullptr;
    // C columns per lane (tree_cols): 8 for BF16 / FP8, 4 otherwise
    const int C = (j.in_dtype == DT_BF16 || j.in_dtype == DT_FP8) ? 8 : 4;
    const int lpb = lanes_per_bucket(j.ld, t.outy[0] ? std::max<int64_t>(j.k, j.ldoy) : 1, C);
    a.nwin = (int)ceil_div(j.ld, (int64_t)C * lpb);
    const int es = dtype_bytes(j.in_dtype);
    const int64_t align = std::min<int64_t>(16, (int64_t)C * es);
    a.xvec = (j.ldx * es) % align == 0 && (uintptr_t)j.x % align == 0;
    for (int l = 0; l <= t.levels; ++l) {
        a.out[l] = t.out[l];
        a.outy[l] = t.outy[l];
        a.m[l] = t.m[l];
    }
    a.j.outy = t.outy[0];
    a.work = t.work;
    switch (j.in_dtype) {
        case DT_F64: return tree_dispatch<double, double>(st, a, t.growth, t.levels, lpb);
        case DT_F32: return tree_dispatch<float, float>(st, a, t.growth, t.levels, lpb);
        case DT_BF16: return tree_dispatch<bf16_t, float>(st, a, t.growth, t.levels, lpb);
        case DT_FP8: return tree_dispatch<fp8_t, float>(st, a, t.growth, t.levels, lpb);
        default: return hipErrorInvalidValue;
    }
}

hipError_t run_cs_fold(hipStream_t st, bool f64, const void* src, void* work, void* dst, int out_dtype, int64_t ld,
                       int64_t mc, int g, const double* ysrc, double* ydst, int64_t ldy, int64_t k) {
    if (mc <= 0 || g < 1 || ld % 4 != 0) return hipErrorInvalidValue;
    const int64_t n4 = mc * ld / 4;
    const unsigned blocks = (unsigned)ceil_div(n4, 256);
    if (f64) {
        cs_fold_kernel<double><<<blocks, 256, 0, st>>>(static_cast<const double*>(src), static_cast<double*>(work),
                                                       dst, out_dtype, ld, mc, g);
    } else {
        cs_fold_kernel<float><<<blocks, 256, 0, st>>>(static_cast<const float*>(src), static_cast<float*>(work), dst,
                                                      out_dtype, ld, mc, g);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ysrc) return e;
    (void)k;
    cs_fold_y_kernel<<<(unsigned)ceil_div(mc * ldy, 256), 256, 0, st>>>(ysrc, ydst, ldy, mc, g);
    return hipGetLastError();
}

}  // namespace spcg
