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
// Work is a list of tasks (problem, first row, last row); one launch per
// row-width class covers every task of that class in a batch of
// independent problems.  A task's block streams 16-row tiles of its A
// through a ring of LDS slots filled by direct global->LDS loads (the same
// scheme as the single-RHS product: equal load counts per wave and tile,
// explicit vmcnt waits, bare barriers, one LDS object per slot), so the
// next tiles are in flight while the matrix cores work on the current one.
// The constant B operands of the first GEMM (P and x split hi + lo) stay in
// registers for the whole task: wave w owns the 16-column K groups w, w + 8,
// ..., with the K order inside a group permuted so that each lane's four A
// values are one LDS read.  The 8 waves' 16 x 16 partials of W are combined
// through LDS (each wave sums two rows and forms their residual once), and
// each wave then owns every 8th 16-column output tile of the second GEMM,
// whose K (row) order is permuted to make its LDS reads conflict-free, with
// the accumulators in registers.  The residual is formed in FP64 as
// (b - A x_hi) - A x_lo.  The task writes one FP32 partial d x 16 block per
// output; the per-problem d-space kernel sums the partials of its tasks in
// a fixed order.
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace spcg {

namespace {

constexpr int MT = 16;          // rows per tile (MFMA M)
constexpr int KP = 16;          // right-hand sides per MFMA (N)
constexpr int MR_DMAX = 512;    // columns supported
constexpr int MRW = 8;          // waves per block

typedef float mv4f __attribute__((ext_vector_type(4)));

constexpr int mr_vmcnt_imm(int n) { return (n & 0xf) | (((n >> 4) & 3) << 14) | (0x7 << 4) | (0xf << 8); }
// wait for LDS (lgkm) only: vmcnt and expcnt at their maxima
constexpr int MR_LGKM0 = 0xf | (3 << 14) | (0x7 << 4);

template <int DMAB>
__device__ __forceinline__ void mr_lds_load(const void* src, void* lds) {
    void* g = const_cast<void*>(src);
    auto* l = (__attribute__((address_space(3))) void*)(lds);
    if constexpr (DMAB == 16) {
        __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
    } else {
        static_assert(DMAB == 4, "4- or 16-byte loads");
        __builtin_amdgcn_global_load_lds(g, l, 4, 0, 0);
    }
}

template <typename TS>
__device__ __forceinline__ float lds_elem(const unsigned char* row, int col);
template <>
__device__ __forceinline__ float lds_elem<float>(const unsigned char* row, int col) {
    return reinterpret_cast<const float*>(row)[col];
}
template <>
__device__ __forceinline__ float lds_elem<bf16_t>(const unsigned char* row, int col) {
    return bf16_bits_to_f32(reinterpret_cast<const uint16_t*>(row)[col]);
}

// Four consecutive elements of an LDS row (16-byte aligned for FP32, 8 for
// BF16), widened: one LDS read.
template <typename TS>
__device__ __forceinline__ void lds_elem4(const unsigned char* row, int col, float* o);
template <>
__device__ __forceinline__ void lds_elem4<float>(const unsigned char* row, int col, float* o) {
    const float4 v = *reinterpret_cast<const float4*>(row + 4 * col);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
}
template <>
__device__ __forceinline__ void lds_elem4<bf16_t>(const unsigned char* row, int col, float* o) {
    const uint2 v = *reinterpret_cast<const uint2*>(row + 2 * col);
    o[0] = __uint_as_float(v.x << 16);
    o[1] = __uint_as_float(v.x & 0xffff0000u);
    o[2] = __uint_as_float(v.y << 16);
    o[3] = __uint_as_float(v.y & 0xffff0000u);
}

// PIPE = false: per tile, GEMM1, the W partials, a barrier, the reduction,
// a barrier and GEMM2 (three barriers per 16-row tile).  PIPE = true:
// software-pipelined over two tiles with two barriers per tile: the
// reduction of tile u (lanes < 32, vector ALU and LDS) runs beside GEMM1 of
// tile u + 1 on the matrix cores, then GEMM2 of tile u.  RING LDS slots hold
// the tiles being read and the tiles in flight (PIPE reads two at a time).
template <typename TS, int MODE, int DMAB, int NIR, bool PIPE, int RING, int NW>
__global__ __launch_bounds__(64 * NW) void mrhs_product_kernel(const MrhsTask* __restrict__ tasks, int task0,
                                                                const MrhsProblem* __restrict__ probs,
                                                                float* part_s, float* part_g, float* part_scal) {
    constexpr bool DO_S = MODE != PM_G;
    constexpr bool DO_G = MODE != PM_S;
    constexpr int ES = std::is_same<TS, float>::value ? 4 : 2;
    constexpr int RB = NIR * 64 * DMAB;              // staged bytes per row
    constexpr int PITCH = RB + 16;                   // 16-byte pad: row starts hit different banks
    constexpr int YB = DO_G ? 256 : 0;               // staged b bytes per row (k FP64 values)
    constexpr int SLOT = MT * PITCH + MT * YB;
    constexpr int AJOBS = MT * NIR;                  // A loads per tile
    constexpr int OPS = AJOBS / NW + (DO_G ? MT / NW : 0);   // loads per wave per tile
    static_assert(AJOBS % NW == 0 && MT % NW == 0, "even split of the loads");
    constexpr int RPW = MT / NW;   // tile rows whose W reduction a wave takes
    // widest row of the class: the register arrays below are sized for it
    constexpr int DCLS = NIR * 64 * DMAB / ES < MR_DMAX ? NIR * 64 * DMAB / ES : MR_DMAX;
    constexpr int KG = (DCLS / 16 + NW - 1) / NW;     // 16-column K groups per wave (first GEMM)
    constexpr int MAXT = (DCLS / 16 + NW - 1) / NW;   // second-GEMM output tiles per wave
    static_assert(RING >= (PIPE ? 3 : 2) && RING <= 4 && (RING - 2) * OPS < 64, "ring shape");
    // each slot starts with a 16-byte guard: the loads of a shifted last
    // row (see issue) begin up to 12 bytes before its staging row
    __shared__ __align__(16) unsigned char sl0_[SLOT + 16];
    __shared__ __align__(16) unsigned char sl1_[SLOT + 16];
    __shared__ __align__(16) unsigned char sl2_[RING > 2 ? SLOT + 16 : 32];
    __shared__ __align__(16) unsigned char sl3_[RING > 3 ? SLOT + 16 : 32];
    unsigned char* const sl0 = sl0_ + 16;
    unsigned char* const sl1 = sl1_ + 16;
    unsigned char* const sl2 = sl2_ + 16;
    unsigned char* const sl3 = sl3_ + 16;
    // Column packing: the first GEMM's B operand is [P | x_hi | x_lo] (the
    // matrices this mode needs, k columns each) laid side by side over
    // NS1 = ceil(NM1 k / 16) 16-column slabs, and the second GEMM's is
    // [W_p | g] over NS2 = ceil(NM2 k / 16) slabs, so small k runs fewer
    // MFMAs.  Packed column q is matrix q / k, right-hand side q mod k.
    constexpr int NM1 = (DO_S ? 1 : 0) + (DO_G ? 2 : 0);
    constexpr int NM2 = (DO_S ? 1 : 0) + (DO_G ? 1 : 0);
    // per-wave partials of W per slab; row pitch 20 keeps the MFMA-layout
    // stores (rows 4 lg + v, column li) conflict-free
    __shared__ float W1[NM1][NW][MT][KP + 4];
    // the second GEMM's packed B operand (pitch 36: its reads are conflict-free)
    __shared__ float W2[MT][2 * KP + 4];
    __shared__ float nrm[2][NW][32];

    const MrhsTask task = tasks[blockIdx.x];
    const int64_t gtask = (int64_t)task0 + blockIdx.x;
    const MrhsProblem pb = probs[task.prob];
    const int d = pb.d, k = pb.k;
    const int dt = (d + 15) / 16;          // 16-column tiles of d
    const int ns1 = (NM1 * k + 15) / 16, ns2 = (NM2 * k + 15) / 16;
    // wave index as a wave-uniform (scalar) value: row offsets stay in SGPRs
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int li = lane & 15, lg = lane >> 4;
    const int nvec = (d * ES + DMAB - 1) / DMAB;    // load vectors holding the row's data
    const char* Abase = static_cast<const char*>(pb.A);
    const int64_t rowb = pb.lda * ES;
    const int64_t rlast = task.r1 - 1;
    for (int e = threadIdx.x; e < MT * (2 * KP + 4); e += 64 * NW) (&W2[0][0])[e] = 0.f;
    // Rows whose start is only 4-byte aligned (16-byte loads, lshift > 0):
    // the last 16-byte vector of a row reaches up to 12 bytes into the next
    // row, except for the matrix's last row (a task of its own), whose
    // vectors start lshift bytes earlier (in the previous row) and land
    // lshift bytes earlier in LDS, so that its data sits where the readers
    // expect it.  Its last lshift staged bytes are then not written; they
    // are read as columns past d (times zero), so they start at zero here,
    // before any load.
    const bool shifted_last = DMAB == 16 && pb.lshift > 0 && task.r0 == pb.m - 1;
    const int sh = shifted_last ? pb.lshift : 0;
    const char* const Abase_s = Abase - sh;
    if (shifted_last) {
        for (int e = threadIdx.x; e < RING * MT; e += 64 * NW) {
            const int sidx = e / MT;
            unsigned char* sb = sidx == 0 ? sl0 : sidx == 1 ? sl1 : sidx == 2 ? sl2 : sl3;
            *reinterpret_cast<uint4*>(sb + (e % MT) * PITCH + RB - 16) = make_uint4(0u, 0u, 0u, 0u);
        }
        __syncthreads();
    }

    // constant B operands of the first GEMM: P and x = hi + lo (~48 bits),
    // zero outside d x k.  A x = A x_hi + A x_lo: the high product only
    // changes when x_hi does, so steps far below FP32 resolution of x still
    // move the residual through the low product.
    // The K order inside each 16-column group q is permuted: at step u lane
    // group lg takes column 16 q + 4 lg + u, so a lane's four A values of a
    // group are contiguous (one LDS read) and the B constants follow.
    float b1[NM1][KG][4];
#pragma unroll
    for (int sl = 0; sl < NM1; ++sl) {
        const int qc = 16 * sl + li;           // packed column of this lane
        const int mi = qc / k, c = qc - mi * k;
        // matrix mi: P (when DO_S) first, then x_hi, then x_lo
        const int src = DO_S ? mi : mi + 1;    // 0 P, 1 x_hi, 2 x_lo
        // one load per value, no branch; the vectors live in global memory
        typedef const __attribute__((address_space(1))) double gdouble;
        gdouble* base = (gdouble*)(src == 0 ? pb.P : pb.X);
#pragma unroll
        for (int g = 0; g < KG; ++g) {
            const int q = wave + NW * g;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int row = 16 * q + 4 * lg + u;
                const bool ok = row < d && mi < NM1;
                const double xv = base[(int64_t)(ok ? c : 0) * pb.ldv + (ok ? row : 0)];
                const float hi = (float)xv, lo = (float)(xv - (double)hi);
                // a 0/1 weight rather than a select keeps the load unconditional
                // (all loads of the slab in flight at once; the values are finite)
                b1[sl][g][u] = (src == 2 ? lo : hi) * (ok ? 1.f : 0.f);
            }
        }
        // bound the loads in flight (registers) to one slab
        __builtin_amdgcn_sched_barrier(0);
    }
    mv4f acc[2][MAXT];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        acc[0][t] = mv4f{0.f, 0.f, 0.f, 0.f};
        acc[1][t] = mv4f{0.f, 0.f, 0.f, 0.f};
    }
    float r2 = 0.f, ax2 = 0.f;   // per lane l < 32: column l mod 16, rows 2 wave + l / 16
    const int64_t ntile = (task.r1 - task.r0 + MT - 1) / MT;

    auto issue = [&](int64_t tl, unsigned char* T) __attribute__((always_inline)) {
        // (a shifted last-row task: every load is of that row, sh bytes early)
        unsigned char* Ts = T - sh;
#pragma unroll
        for (int q = 0; q < AJOBS / NW; ++q) {
            const int job = wave + NW * q;
            const int r = job / NIR, c = job % NIR;
            const int64_t grow = min(task.r0 + tl * MT + r, rlast);
            const int vi = min(c * 64 + lane, nvec - 1);
            mr_lds_load<DMAB>(Abase_s + grow * rowb + (int64_t)vi * DMAB, Ts + r * PITCH + c * 64 * DMAB);
            // keep each address computation next to its load (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (DO_G) {
#pragma unroll
            for (int q = 0; q < MT / NW; ++q) {
                const int r = wave + NW * q;
                const int64_t grow = min(task.r0 + tl * MT + r, rlast);
                const int w = min(lane, 2 * k - 1);
                mr_lds_load<4>(reinterpret_cast<const char*>(pb.b + grow * pb.ldb) + 4 * w,
                               T + MT * PITCH + r * 256);
            }
        }
    };
    // first GEMM: this wave's K groups of W = A_t [P | x_hi | x_lo] (packed)
    auto gemm1 = [&](const unsigned char* T, mv4f* w1) __attribute__((always_inline)) {
#pragma unroll
        for (int sl = 0; sl < NM1; ++sl) w1[sl] = mv4f{0.f, 0.f, 0.f, 0.f};
        const unsigned char* arow = T + li * PITCH;
        // the slab count is uniform per task: one loop body per count, so
        // the MFMA chains carry no per-instruction conditions
        // every K group's A values first (their LDS reads in flight together;
        // groups past d read group 0 and are not used), then the MFMA chains
        float a4[KG][4];
#pragma unroll
        for (int g = 0; g < KG; ++g) {
            const int q = wave + NW * g;
            lds_elem4<TS>(arow, 16 * (q < dt ? q : 0) + 4 * lg, a4[g]);
        }
        auto run = [&](auto ns_c) __attribute__((always_inline)) {
            constexpr int NS = decltype(ns_c)::value;
#pragma unroll
            for (int g = 0; g < KG; ++g) {
                const int q = wave + NW * g;
                if (q < dt) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
#pragma unroll
                        for (int sl = 0; sl < NS; ++sl)
                            w1[sl] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[g][u], b1[sl][g][u], w1[sl], 0, 0, 0);
                    }
                }
            }
        };
        if constexpr (NM1 >= 3) {
            if (ns1 >= 3) run(std::integral_constant<int, 3>{});
            else if (ns1 == 2) run(std::integral_constant<int, 2>{});
            else run(std::integral_constant<int, 1>{});
        } else if constexpr (NM1 == 2) {
            if (ns1 == 2) run(std::integral_constant<int, 2>{});
            else run(std::integral_constant<int, 1>{});
        } else {
            run(std::integral_constant<int, 1>{});
        }
    };
    // this wave's partials of W into LDS (unused slabs store their zeros)
    auto store_w1 = [&](const mv4f* w1) __attribute__((always_inline)) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
#pragma unroll
            for (int sl = 0; sl < NM1; ++sl) W1[sl][wave][4 * lg + v][li] = w1[sl][v];
        }
    };
    // reduce-scatter: wave w sums the NW partials of its RPW rows (lane
    // l < 16 RPW: row RPW w + l / 16, right-hand side l mod 16) in a fixed
    // order, forms the residual there once, and publishes the second GEMM's
    // packed B operand
    // Every partial is loaded before the sums (the LDS reads in flight
    // together); lanes with cc >= k read valid LDS (packed columns < NM1 16)
    // and write nothing.
    auto reduce = [&](int64_t tl, const unsigned char* T) __attribute__((always_inline)) {
        if (lane < 16 * RPW) {
            const int rr = RPW * wave + (lane >> 4), cc = lane & 15;
            const bool act = cc < k;
            const bool ok = task.r0 + tl * MT + rr < task.r1;
            if constexpr (DO_S) {
                float pp[NW];
#pragma unroll
                for (int w = 0; w < NW; ++w) pp[w] = W1[0][w][rr][cc];
                // every partial is in a register before the first add (the
                // scheduler would otherwise wait out each read before the next)
#pragma unroll
                for (int w = 0; w < NW; ++w) asm volatile("" : "+v"(pp[w]));
                float t0 = 0.f;
#pragma unroll
                for (int w = 0; w < NW; ++w) t0 += pp[w];
                if (act) W2[rr][cc] = ok ? t0 : 0.f;
            }
            if constexpr (DO_G) {
                const int qh = (DO_S ? k : 0) + cc, ql = qh + k;
                float ph[NW], pl[NW];
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    ph[w] = W1[qh >> 4][w][rr][qh & 15];
                    pl[w] = W1[ql >> 4][w][rr][ql & 15];
                }
                const double bv = reinterpret_cast<const double*>(T + MT * PITCH + rr * 256)[cc];
#pragma unroll
                for (int w = 0; w < NW; ++w) asm volatile("" : "+v"(ph[w]), "+v"(pl[w]));
                float t1 = 0.f, tlo = 0.f;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    t1 += ph[w];
                    tlo += pl[w];
                }
                const double res = ok ? (bv - (double)t1) - (double)tlo : 0.0;
                if (act) {
                    W2[rr][(DO_S ? k : 0) + cc] = (float)res;
                    if (ok) {
                        r2 = fmaf((float)res, (float)res, r2);
                        ax2 = fmaf(t1, t1, ax2);
                    }
                }
            }
        }
    };
    // second GEMM: [S | G][:, tile mt] += A_t^T [W_p | g], with the rows of
    // the tile permuted: at step u lane group lg takes row 4 lg + u
    // (conflict-free LDS reads of A_t^T)
    auto gemm2 = [&](const unsigned char* T) __attribute__((always_inline)) {
        float b2[2][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            b2[0][u] = W2[4 * lg + u][li];
            b2[1][u] = NM2 > 1 ? W2[4 * lg + u][16 + li] : 0.f;
        }
        // the A^T values of every output tile first (tiles past d read tile
        // 0 and are not used), then the MFMA chains
        float av[MAXT][4];
#pragma unroll
        for (int t = 0; t < MAXT; ++t) {
            const int mt = wave + NW * t;
#pragma unroll
            for (int u = 0; u < 4; ++u) av[t][u] = lds_elem<TS>(T + (4 * lg + u) * PITCH, 16 * (mt < dt ? mt : 0) + li);
        }
        auto run = [&](auto ns_c) __attribute__((always_inline)) {
            constexpr int NS = decltype(ns_c)::value;
#pragma unroll
            for (int t = 0; t < MAXT; ++t) {
                const int mt = wave + NW * t;
                if (mt < dt) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
#pragma unroll
                        for (int sl = 0; sl < NS; ++sl)
                            acc[sl][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t][u], b2[sl][u], acc[sl][t], 0, 0, 0);
                    }
                }
            }
        };
        if constexpr (NM2 > 1) {
            if (ns2 > 1) run(std::integral_constant<int, 2>{});
            else run(std::integral_constant<int, 1>{});
        } else {
            run(std::integral_constant<int, 1>{});
        }
    };
    auto lds_barrier = [&]() __attribute__((always_inline)) {
        __builtin_amdgcn_s_waitcnt(MR_LGKM0);
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    };
    // one LDS object per slot: the slot of a step is known at compile time
    auto slot = [&](auto i_c) __attribute__((always_inline)) -> unsigned char* {
        constexpr int i = decltype(i_c)::value % RING;
        if constexpr (i == 0) return sl0;
        else if constexpr (i == 1) return sl1;
        else if constexpr (i == 2) return sl2;
        else return sl3;
    };

    // tiles 0 .. RING - 2 in flight; the loop issues one tile per step.
    // The work of steps past the last tile is skipped (uniform over the
    // block); their waits, barriers and loads (clamped rows, ignored) stay,
    // so that every path through a step has the same loads in flight.
    static_for<0, RING - 1>([&](auto kc) { issue(decltype(kc)::value, slot(kc)); });
    if constexpr (!PIPE) {
        for (int64_t t = 0; t < ntile; t += RING) {
            // step k: wait for tile t + k (tiles up to t + k + RING - 2 are
            // issued), refill the slot read at step k - 1
            static_for<0, RING>([&](auto kc) {
                constexpr int kk = decltype(kc)::value;
                __builtin_amdgcn_s_waitcnt(mr_vmcnt_imm((RING - 2) * OPS));
                __builtin_amdgcn_s_barrier();
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                issue(t + kk + RING - 1, slot(std::integral_constant<int, kk + RING - 1>{}));
                if (t + kk < ntile) {
                    mv4f w1[NM1];
                    gemm1(slot(kc), w1);
                    store_w1(w1);
                    lds_barrier();
                    reduce(t + kk, slot(kc));
                    lds_barrier();
                    gemm2(slot(kc));
                }
            });
        }
    } else {
        // GEMM1 of tile 0 before the loop; step u then runs the reduction
        // of tile u beside GEMM1 of tile u + 1, and after the second
        // barrier GEMM2 of tile u and the W partials of tile u + 1
        __builtin_amdgcn_s_waitcnt(mr_vmcnt_imm((RING - 2) * OPS));
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        {
            mv4f w1[NM1];
            gemm1(sl0, w1);
            store_w1(w1);
        }
        for (int64_t t = 0; t < ntile; t += RING) {
            static_for<0, RING>([&](auto kc) {
                constexpr int kk = decltype(kc)::value;
                // tile u + 1 has landed (tiles up to u + RING - 2 are
                // issued); the barrier also publishes the W partials of tile
                // u and frees the slot GEMM2 read at step u - 1
                __builtin_amdgcn_s_waitcnt(mr_vmcnt_imm((RING - 3) * OPS));
                __builtin_amdgcn_s_barrier();
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                issue(t + kk + RING - 1, slot(std::integral_constant<int, kk + RING - 1>{}));
                if (t + kk < ntile) {
                    mv4f w1n[NM1];
                    reduce(t + kk, slot(kc));
                    gemm1(slot(std::integral_constant<int, kk + 1>{}), w1n);
                    lds_barrier();   // W2 of tile u is visible; the partials of tile u are read
                    store_w1(w1n);
                    gemm2(slot(kc));
                }
            });
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // partial outputs: part[task][col][c] (c < 16), unpacked from the slabs
    const int64_t base = gtask * MR_DMAX * KP;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
        const int q2 = 16 * sl + li;
        const int mi = q2 / k, c = q2 - mi * k;
        if (mi >= NM2) continue;
        float* out = (DO_S && mi == 0) ? part_s : part_g;
#pragma unroll
        for (int t = 0; t < MAXT; ++t) {
            const int mt = wave + NW * t;
            if (mt < dt) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int col = 16 * mt + 4 * lg + v;
                    out[base + (int64_t)col * KP + c] = acc[sl][t][v];
                }
            }
        }
    }
    if (DO_G) {
        // per-column norms: every wave's row lanes, in a fixed order
        if (lane < 16 * RPW) {
            nrm[0][wave][lane] = r2;
            nrm[1][wave][lane] = ax2;
        }
        __syncthreads();
        if (threadIdx.x < KP) {
            const int c = threadIdx.x;
            float a0 = 0.f, a1 = 0.f;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
#pragma unroll
                for (int h = 0; h < RPW; ++h) {
                    a0 += nrm[0][w][c + 16 * h];
                    a1 += nrm[1][w][c + 16 * h];
                }
            }
            part_scal[gtask * 2 * KP + c] = a0;
            part_scal[gtask * 2 * KP + KP + c] = a1;
        }
    }
}

// ---- register-staged fallback for row layouts the load-to-LDS path cannot
// read (rows whose byte stride is not a multiple of 4): 16-row tiles are
// widened element by element into LDS, one tile at a time.
constexpr int MRG_WAVES = 4;
constexpr int MRG_LD = MR_DMAX + 4;

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
__global__ __launch_bounds__(64 * MRG_WAVES) void mrhs_product_reg_kernel(const MrhsTask* __restrict__ tasks, int task0,
                                                                     const MrhsProblem* __restrict__ probs,
                                                                     float* part_s, float* part_g,
                                                                     float* part_scal) {
    constexpr bool DO_S = MODE != PM_G;
    constexpr bool DO_G = MODE != PM_S;
    __shared__ float At[MT][MRG_LD];
    __shared__ float Ps[DO_S ? MR_DMAX : 1][KP];
    __shared__ float Xs[DO_G ? MR_DMAX : 1][KP];    // x rounded to FP32
    __shared__ float Xl[DO_G ? MR_DMAX : 1][KP];    // x - Xs, the low part
    __shared__ float Wp[MRG_WAVES][MT][KP + 1];
    __shared__ float Wgp[DO_G ? MRG_WAVES : 1][MT][KP + 1];
    __shared__ float Wlp[DO_G ? MRG_WAVES : 1][MT][KP + 1];

    const MrhsTask task = tasks[blockIdx.x];
    const int64_t gtask = (int64_t)task0 + blockIdx.x;
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
    for (int e = threadIdx.x; e < MR_DMAX * KP; e += 64 * MRG_WAVES) {
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
    constexpr int MAXT = MR_DMAX / 16 / MRG_WAVES;
    mv4f accS[MAXT], accG[MAXT];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        accS[t] = mv4f{0.f, 0.f, 0.f, 0.f};
        accG[t] = mv4f{0.f, 0.f, 0.f, 0.f};
    }
    float r2 = 0.f, ax2 = 0.f;   // per lane: column li, rows of its groups
    // first-GEMM K range of this wave
    const int kq = (d4 + MRG_WAVES - 1) / MRG_WAVES;
    const int ks0 = wave * kq, ks1 = min(d4, ks0 + kq);

    for (int64_t row0 = task.r0; row0 < task.r1; row0 += MT) {
        __syncthreads();   // previous tile fully consumed
        for (int e = threadIdx.x; e < MT * MR_DMAX; e += 64 * MRG_WAVES) {
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
            for (int w = 0; w < MRG_WAVES; ++w) {
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
            const int mt = wave + MRG_WAVES * t;
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
    const int64_t base = gtask * MR_DMAX * KP;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        const int mt = wave + MRG_WAVES * t;
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
            part_scal[gtask * 2 * KP + c] = ((nrm[0][0][c] + nrm[0][1][c]) + nrm[0][2][c]) + nrm[0][3][c];
            part_scal[gtask * 2 * KP + KP + c] =
                ((nrm[1][0][c] + nrm[1][1][c]) + nrm[1][2][c]) + nrm[1][3][c];
        }
    }
}


template <typename TS, int DMAB, int NIR, bool PIPE, int RING, int NW = MRW>
hipError_t mr_launch_shape(hipStream_t st, int mode, const MrhsTask* tasks, int task0, int ntasks,
                           const MrhsProblem* probs, float* ps, float* pg, float* pscal) {
    dim3 grid(ntasks), block(64 * NW);
    switch (mode) {
        case PM_S:
            mrhs_product_kernel<TS, PM_S, DMAB, NIR, PIPE, RING, NW><<<grid, block, 0, st>>>(tasks, task0, probs, ps,
                                                                                             pg, pscal);
            break;
        case PM_G:
            mrhs_product_kernel<TS, PM_G, DMAB, NIR, PIPE, RING, NW><<<grid, block, 0, st>>>(tasks, task0, probs, ps,
                                                                                             pg, pscal);
            break;
        default:
            mrhs_product_kernel<TS, PM_SG, DMAB, NIR, PIPE, RING, NW><<<grid, block, 0, st>>>(tasks, task0, probs,
                                                                                              ps, pg, pscal);
            break;
    }
    return hipGetLastError();
}

// 4 slots fit the LDS for rows of at most 1 KB
constexpr bool mr_pipe4(int dmab, int nir) { return nir * 64 * dmab <= 1024; }

template <typename TS, int DMAB, int NIR>
hipError_t mr_launch(hipStream_t st, int mode, int shape, const MrhsTask* tasks, int task0, int ntasks,
                     const MrhsProblem* probs, float* ps, float* pg, float* pscal) {
    if (shape == MR_SHAPE_PLAIN)
        return mr_launch_shape<TS, DMAB, NIR, false, 3>(st, mode, tasks, task0, ntasks, probs, ps, pg, pscal);
    if constexpr (mr_pipe4(DMAB, NIR)) {
        if (shape == MR_SHAPE_PIPE4)
            return mr_launch_shape<TS, DMAB, NIR, true, 4>(st, mode, tasks, task0, ntasks, probs, ps, pg, pscal);
    }
    return mr_launch_shape<TS, DMAB, NIR, true, 3>(st, mode, tasks, task0, ntasks, probs, ps, pg, pscal);
}

template <typename TS>
hipError_t mr_launch_class(hipStream_t st, int mode, int cls, int shape, const MrhsTask* tasks, int task0,
                           int ntasks, const MrhsProblem* probs, float* ps, float* pg, float* pscal) {
    switch (cls) {
        case MR_CLASS_16x1: return mr_launch<TS, 16, 1>(st, mode, shape, tasks, task0, ntasks, probs, ps, pg, pscal);
        case MR_CLASS_16x2: return mr_launch<TS, 16, 2>(st, mode, shape, tasks, task0, ntasks, probs, ps, pg, pscal);
        case MR_CLASS_4x1: return mr_launch<TS, 4, 1>(st, mode, shape, tasks, task0, ntasks, probs, ps, pg, pscal);
        case MR_CLASS_4x2: return mr_launch<TS, 4, 2>(st, mode, shape, tasks, task0, ntasks, probs, ps, pg, pscal);
        case MR_CLASS_4x4: return mr_launch<TS, 4, 4>(st, mode, shape, tasks, task0, ntasks, probs, ps, pg, pscal);
        case MR_CLASS_4x8: return mr_launch<TS, 4, 8>(st, mode, shape, tasks, task0, ntasks, probs, ps, pg, pscal);
        default: break;
    }
    if (cls == MR_CLASS_GENERIC) {
        dim3 grid(ntasks), block(64 * MRG_WAVES);
        switch (mode) {
            case PM_S: mrhs_product_reg_kernel<TS, PM_S><<<grid, block, 0, st>>>(tasks, task0, probs, ps, pg, pscal); break;
            case PM_G: mrhs_product_reg_kernel<TS, PM_G><<<grid, block, 0, st>>>(tasks, task0, probs, ps, pg, pscal); break;
            default: mrhs_product_reg_kernel<TS, PM_SG><<<grid, block, 0, st>>>(tasks, task0, probs, ps, pg, pscal); break;
        }
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

}  // namespace

int mrhs_max_d() { return MR_DMAX; }
int mrhs_max_k() { return KP; }

// 16-byte loads from rows that are only 4-byte aligned: every byte of the
// row stride is readable (lda == dmem), a row holds at least 16 bytes and
// there are at least two rows.  The last vector of row r < m - 1 then ends
// inside row r + 1; the matrix's last row is loaded lshift bytes earlier.
int mrhs_row_shift(int dtype, const void* A, int64_t m, int64_t lda, int64_t dmem, int d) {
    const int es = dtype == DT_F32 ? 4 : 2;
    const int64_t nv = ((int64_t)d * es + 15) / 16;
    const bool aligned = (lda * es) % 16 == 0 && (uintptr_t)A % 16 == 0 && nv * 16 <= dmem * es;
    if (aligned) return 0;
    const bool ok = (lda * es) % 4 == 0 && (uintptr_t)A % 4 == 0 && lda == dmem && (int64_t)d * es >= 16 && m >= 2 &&
                    lda >= d;
    return ok ? (int)(nv * 16 - (int64_t)d * es) : -1;
}

int mrhs_class(int dtype, const void* A, int64_t m, int64_t lda, int64_t dmem, int d) {
    const int es = dtype == DT_F32 ? 4 : 2;
    for (int dmab : {16, 4}) {
        const int64_t nv = ((int64_t)d * es + dmab - 1) / dmab;
        const bool ok = dmab == 16 ? mrhs_row_shift(dtype, A, m, lda, dmem, d) >= 0
                                   : (lda * es) % dmab == 0 && (uintptr_t)A % dmab == 0 && nv * dmab <= dmem * es;
        if (!ok) continue;
        const int64_t ni = (nv + 63) / 64;
        if (dmab == 16) {
            if (ni <= 1) return MR_CLASS_16x1;
            if (ni <= 2) return MR_CLASS_16x2;
            continue;
        }
        if (ni <= 1) return MR_CLASS_4x1;
        if (ni <= 2) return MR_CLASS_4x2;
        if (ni <= 4) return MR_CLASS_4x4;
        if (ni <= 8) return MR_CLASS_4x8;
    }
    return MR_CLASS_GENERIC;
}

bool mrhs_shape_native(int cls, int shape) {
    if (shape == MR_SHAPE_PIPE4)
        return cls == MR_CLASS_16x1 || cls == MR_CLASS_4x1 || cls == MR_CLASS_4x2 || cls == MR_CLASS_4x4;
    if (shape == MR_SHAPE_PIPE3) return cls != MR_CLASS_GENERIC;
    return shape == MR_SHAPE_PLAIN;
}

hipError_t run_mrhs_product(hipStream_t st, int dtype, int mode, int cls, int shape, const MrhsTask* tasks,
                            int task0, int ntasks, const MrhsProblem* probs, float* part_s, float* part_g,
                            float* part_scal) {
    if (ntasks <= 0) return hipSuccess;
    if (dtype == DT_F32)
        return mr_launch_class<float>(st, mode, cls, shape, tasks + task0, task0, ntasks, probs, part_s, part_g,
                                      part_scal);
    if (dtype == DT_BF16)
        return mr_launch_class<bf16_t>(st, mode, cls, shape, tasks + task0, task0, ntasks, probs, part_s, part_g,
                                       part_scal);
    return hipErrorInvalidValue;
}

}  // namespace spcg

namespace spcg {

namespace {

constexpr int DS_THREADS = 512;

__device__ __forceinline__ bool dfinite(double v) { return __builtin_isfinite(v); }

// Column sums over j of a[j][c] * b[j][c] for every c < 16, fixed order.
__device__ void colwise_dot(const double* a, const double* b, int64_t ldv, int d, int k, double* out,
                            double (*red)[KP + 1]) {
    const int c = threadIdx.x % KP, q = threadIdx.x / KP;   // 16 lanes per column
    double t = 0.0;
    if (c < k) {
#pragma unroll 8
        for (int j = q; j < d; j += DS_THREADS / KP) t = fma(a[(int64_t)c * ldv + j], b[(int64_t)c * ldv + j], t);
    }
    red[q][c] = t;
    __syncthreads();
    if (threadIdx.x < KP) {
        double s = 0.0;
        for (int w = 0; w < DS_THREADS / KP; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Step 1 of the d-space update: the task partials of every element summed
// in task order, one thread per element of the d x 16 block and RS_SLICES
// blocks per problem (a problem can have thousands of tasks when few
// problems are active; one block per problem then waited out their loads
// one after another).  Per element the order is the tasks' order, so the
// sums do not depend on the launch shape.  Writes G (starts), S and Gt.
constexpr int RS_SLICES = MR_DMAX * KP / DS_THREADS;
__global__ __launch_bounds__(DS_THREADS) void mrhs_reduce_kernel(int variant, const MrhsProblem* __restrict__ probs,
                                                                  const float* __restrict__ part_s,
                                                                  const float* __restrict__ part_g) {
    const MrhsProblem pb = probs[blockIdx.y];
    if (!pb.active) return;
    const int d = pb.d, k = pb.k;
    const int e = blockIdx.x * DS_THREADS + threadIdx.x;   // element j KP + c
    const int j = e / KP, c = e % KP;
    if (j >= d || c >= k) return;
    const bool start = variant == PA_START || variant == PA_START_NESTED;
    const bool want_s = !start, want_g = variant != PA_STEP;
    constexpr int U = 8;   // tasks whose loads are in flight together
    double ss = 0.0, gg = 0.0;
    int t = pb.t0;
    for (; t + U <= pb.t1; t += U) {
        float vs[U], vg[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t o = (int64_t)(t + u) * MR_DMAX * KP + e;
            vs[u] = want_s ? part_s[o] : 0.f;
            vg[u] = want_g ? part_g[o] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ss += (double)vs[u];
            gg += (double)vg[u];
        }
    }
    for (; t < pb.t1; ++t) {
        const int64_t o = (int64_t)t * MR_DMAX * KP + e;
        if (want_s) ss += (double)part_s[o];
        if (want_g) gg += (double)part_g[o];
    }
    const int64_t o = c * pb.ldv + j;
    if (start) {
        pb.G[o] = variant == PA_START_NESTED && pb.gscale != 0.0 ? fma(pb.gscale, pb.G[o], gg * pb.c2) : gg * pb.c2;
    } else {
        pb.S[o] = ss * pb.c2;
        if (variant == PA_REFRESH) pb.Gt[o] = gg * pb.c2;
    }
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
    // PA_START_NESTED starts like PA_START, from g = gscale g + c2 (partials)
    const bool start = variant == PA_START || variant == PA_START_NESTED;
    const bool want_g = variant != PA_STEP;
    // 1. the element sums are mrhs_reduce_kernel's (launched before); the
    //    residual and fit norms of each column: 32 groups of threads take
    //    every 32nd task in order, then the groups add in group order
    if (want_g) {
        constexpr int NG = DS_THREADS / KP;   // 32 groups of 16 columns
        const int c = threadIdx.x % KP, g = threadIdx.x / KP;
        double r2 = 0.0, ax2 = 0.0;
        for (int t = pb.t0 + g; t < pb.t1; t += NG) {
            r2 += (double)part_scal[(int64_t)t * 2 * KP + c];
            ax2 += (double)part_scal[(int64_t)t * 2 * KP + KP + c];
        }
        red[g][c] = r2;
        __syncthreads();
        if (threadIdx.x < KP) {
            double v = 0.0;
            for (int q = 0; q < NG; ++q) v += red[q][c];
            colv[c] = v * pb.c2;
        }
        __syncthreads();
        red[g][c] = ax2;
        __syncthreads();
        if (threadIdx.x < KP) {
            double v = 0.0;
            for (int q = 0; q < NG; ++q) v += red[q][c];
            colw[c] = v * pb.c2;
        }
    }
    __syncthreads();
    if (want_g && threadIdx.x < k) {
        pb.sc[threadIdx.x].resid2 = colv[threadIdx.x];
        pb.sc[threadIdx.x].ax2 = colw[threadIdx.x];
    }
    // 2. step: alpha = rho / p^T s; x += alpha p; g = (g or g_true) - alpha s
    if (!start) {
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
#pragma unroll 8
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
}

// z = M g for rows [ZR s, ZR s + ZR) of one problem (block (s, p)), all k
// columns.  M = W W^T is symmetric, so row i is read as column i: the lanes
// of a wave take consecutive i and each load of M is one contiguous row
// segment.  The j range is split into four quarters (thread t: row t mod
// ZR, quarter t / ZR), whose partial sums are added in quarter order; the
// slice's share of g^T z goes to rho_part, summed over the slices in slice
// order by the next kernel.
constexpr int ZR = 128;
constexpr int ZQ = DS_THREADS / ZR;
constexpr int ZSL = MR_DMAX / ZR;
static_assert(ZQ * ZR == DS_THREADS && ZSL * ZR == MR_DMAX && ZSL == MR_ZSLICES, "z slices");

__global__ __launch_bounds__(DS_THREADS) void mrhs_dspace_z_kernel(const MrhsProblem* __restrict__ probs) {
    __shared__ double gs[MR_DMAX][KP];   // g, then the quarter partials of z
    const MrhsProblem pb = probs[blockIdx.y];
    const int s = blockIdx.x;
    if (!pb.active || s * ZR >= pb.d) return;   // uniform over the block
    const int d = pb.d, k = pb.k;
    const int64_t ldv = pb.ldv;
#pragma unroll 8
    for (int e = threadIdx.x; e < d * KP; e += DS_THREADS) {
        const int j = e / KP, c = e % KP;
        gs[j][c] = c < k ? pb.G[c * ldv + j] : 0.0;
    }
    __syncthreads();
    const int r = threadIdx.x % ZR, q = threadIdx.x / ZR;
    const int i = s * ZR + r;
    const bool h = i < d;
    const int dq = (d + ZQ - 1) / ZQ;
    const int j0 = q * dq, j1 = min(d, j0 + dq);
    double a0[KP];
#pragma unroll
    for (int c = 0; c < KP; ++c) a0[c] = 0.0;
    // every column, without branches (g is zero past k): straight-line code
    // lets the loads of later j issue before these FMAs
#pragma unroll 4
    for (int j = j0; j < j1; ++j) {
        const double m0 = h ? pb.Minv[(int64_t)j * d + i] : 0.0;
#pragma unroll
        for (int c = 0; c < KP; ++c) a0[c] = fma(m0, gs[j][c], a0[c]);
    }
    __syncthreads();   // gs is free: it takes the quarter partials
    double (*zp)[ZR][KP] = reinterpret_cast<double (*)[ZR][KP]>(&gs[0][0]);
    static_assert(ZQ * ZR <= MR_DMAX, "partials fit");
#pragma unroll
    for (int c = 0; c < KP; ++c) zp[q][r][c] = a0[c];
    __syncthreads();
    double gz[KP];
    if (q == 0) {
#pragma unroll
        for (int c = 0; c < KP; ++c) {
            double z = zp[0][r][c];
#pragma unroll
            for (int w = 1; w < ZQ; ++w) z += zp[w][r][c];
            gz[c] = 0.0;
            if (c < k && h) {
                pb.Z[c * ldv + i] = z;
                gz[c] = pb.G[c * ldv + i] * z;
            }
        }
    }
    __syncthreads();   // the partials are read: zp[1] takes the g z terms
    if (q == 0) {
#pragma unroll
        for (int c = 0; c < KP; ++c) zp[1][r][c] = gz[c];
    }
    __syncthreads();
    if (threadIdx.x < KP) {
        const int c = threadIdx.x;
        double t = 0.0;
        for (int w = 0; w < ZR; ++w) t += zp[1][w][c];
        pb.rho_part[s * KP + c] = t;
    }
}

// rho' = g^T z (the slices' shares in slice order); p = z (start) or
// z + (rho'/rho) p
__global__ __launch_bounds__(DS_THREADS) void mrhs_dspace_p_kernel(int variant, const MrhsProblem* __restrict__ probs) {
    __shared__ double gamma_sh[KP];
    __shared__ int step_sh[KP];
    const MrhsProblem pb = probs[blockIdx.x];
    if (!pb.active) return;
    const int d = pb.d, k = pb.k;
    const int64_t ldv = pb.ldv;
    const int nsl = (d + ZR - 1) / ZR;
    if (threadIdx.x < KP) {
        const int c = threadIdx.x;
        int mode = 0;
        double gm = 0.0;
        if (c < k) {
            double rn = 0.0;
            for (int sl = 0; sl < nsl; ++sl) rn += pb.rho_part[sl * KP + c];
            MrhsScalars& sc = pb.sc[c];
            const bool start = variant == PA_START || variant == PA_START_NESTED;
            const bool skip = sc.breakdown || (!start && sc.exact);
            if (!skip) {
                if (!dfinite(rn)) {
                    sc.breakdown = 1;
                } else if (start) {
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
#pragma unroll 8
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
    mrhs_reduce_kernel<<<dim3(RS_SLICES, nprob), DS_THREADS, 0, st>>>(variant, probs, part_s, part_g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    mrhs_dspace_kernel<<<nprob, DS_THREADS, 0, st>>>(variant, probs, part_s, part_g, part_scal);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    mrhs_dspace_z_kernel<<<dim3(ZSL, nprob), DS_THREADS, 0, st>>>(probs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    mrhs_dspace_p_kernel<<<nprob, DS_THREADS, 0, st>>>(variant, probs);
    return hipGetLastError();
}

}  // namespace spcg
