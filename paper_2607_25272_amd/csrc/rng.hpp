// Counter-based randomness of the SRHT (host and device).
//
// The SRHT S = sqrt(N/m) (H D P)_{I,:} needs random signs (D), a random
// permutation (P) and uniformly sampled rows (I); the nested construction
// needs I_1 c ... c I_K.  Everything is a pure function of (seed, index):
//
//  * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of
//    (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
//    with the key bumped by the Weyl constants between rounds.
//  * Sign of row k: bit (k mod 256) of the 256-bit block at counter
//    (k / 256, 0, 0, 0) under key (seed, STREAM_SIGN); a set bit means -1.
//  * Permutations of [0, 2^L): an alternating Feistel network of 6 rounds.
//    x splits into a high part of ceil(L/2) bits and a low part of the
//    rest; each round maps (l, r) -> (r, l ^ F(r)) with F = word 0 of
//    Philox((r, round, L, 0), (seed, stream)) masked to the width of l, and
//    the two widths swap.  pi(t) for t < m gives nested row sets.
#pragma once
#include <stdint.h>

#ifndef SPCG_HD
#if defined(__HIPCC__)
#define SPCG_HD __host__ __device__
#else
#define SPCG_HD
#endif
#endif

namespace spcg {

enum : uint64_t {
    STREAM_SIGN = 1,
    STREAM_P = 2,
    STREAM_PI = 3,
    STREAM_PIHAT = 4,
    // CountSketch: bucket bijection of the stage sketches, and the
    // preconditioner sketch's own bijection and signs
    STREAM_CS = 5,
    STREAM_CS_HAT = 6,
    STREAM_CS_HAT_SIGN = 7
};
constexpr int FEISTEL_ROUNDS = 6;

SPCG_HD inline void mul_hilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
#if defined(__HIP_DEVICE_COMPILE__)
    hi = __umul64hi(a, b);
    lo = a * b;
#else
    unsigned __int128 p = (unsigned __int128)a * b;
    hi = (uint64_t)(p >> 64);
    lo = (uint64_t)p;
#endif
}

struct Philox4 {
    uint64_t v[4];
};

SPCG_HD inline Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                     uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        if (rnd > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mul_hilo64(M0, c0, hi0, lo0);
        mul_hilo64(M1, c2, hi1, lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    Philox4 out;
    out.v[0] = c0;
    out.v[1] = c1;
    out.v[2] = c2;
    out.v[3] = c3;
    return out;
}

// 1 when the sign of row k in the given stream is -1 (D_kk for STREAM_SIGN).
SPCG_HD inline uint32_t sign_bit_stream(uint64_t seed, uint64_t k, uint64_t stream) {
    Philox4 w = philox4x64_10(k >> 8, 0, 0, 0, seed, stream);
    uint32_t b = (uint32_t)(k & 255);
    return (uint32_t)((w.v[b >> 6] >> (b & 63)) & 1ull);
}

// 1 when D_kk = -1.
SPCG_HD inline uint32_t sign_bit(uint64_t seed, uint64_t k) { return sign_bit_stream(seed, k, STREAM_SIGN); }

SPCG_HD inline uint64_t feistel_round(uint64_t half, int rnd, int L, uint64_t seed, uint64_t stream) {
    return philox4x64_10(half, (uint64_t)rnd, (uint64_t)L, 0, seed, stream).v[0];
}

SPCG_HD inline uint64_t low_mask(int bits) { return bits >= 64 ? ~0ull : ((1ull << bits) - 1ull); }

// pi(x) on [0, 2^L)
SPCG_HD inline uint64_t feistel_fwd(uint64_t x, int L, uint64_t seed, uint64_t stream) {
    const int a = (L + 1) / 2, b = L - a;
    uint64_t l = x >> b, r = x & low_mask(b);
    int wl = a, wr = b;
#pragma unroll
    for (int j = 0; j < FEISTEL_ROUNDS; ++j) {
        uint64_t f = feistel_round(r, j, L, seed, stream) & low_mask(wl);
        uint64_t nl = r, nr = l ^ f;
        l = nl;
        r = nr;
        int t = wl;
        wl = wr;
        wr = t;
    }
    return (l << b) | r;
}

// pi^{-1}(y) on [0, 2^L)
SPCG_HD inline uint64_t feistel_inv(uint64_t y, int L, uint64_t seed, uint64_t stream) {
    const int a = (L + 1) / 2, b = L - a;
    uint64_t l = y >> b, r = y & low_mask(b);
    int wl = a, wr = b;  // widths after the last round
#pragma unroll
    for (int j = FEISTEL_ROUNDS - 1; j >= 0; --j) {
        // after round j: l = r_prev, r = l_prev ^ F(r_prev) masked to width(l_prev) = wr
        uint64_t f = feistel_round(l, j, L, seed, stream) & low_mask(wr);
        uint64_t pl = r ^ f, pr = l;
        l = pl;
        r = pr;
        int t = wl;
        wl = wr;
        wr = t;
    }
    return (l << b) | r;
}

// Table form of the same network.  Round j only ever sees one half of the
// word, a value below 2^ceil(L/2), so its round function can be tabulated:
// entry (j, h) = F_j(h) masked to round j's output width (ceil(L/2) bits for
// even j, floor(L/2) for odd j; the mask both directions apply).  With the
// table, pi and pi^{-1} cost six lookups instead of six Philox calls.
SPCG_HD inline int64_t feistel_table_size(int L) { return (int64_t)FEISTEL_ROUNDS << ((L + 1) / 2); }

SPCG_HD inline uint32_t feistel_table_entry(int64_t e, int L, uint64_t seed, uint64_t stream) {
    const int a = (L + 1) / 2, b = L - a;
    const int j = (int)(e >> a);
    const uint64_t h = (uint64_t)e & low_mask(a);
    return (uint32_t)(feistel_round(h, j, L, seed, stream) & low_mask((j & 1) ? b : a));
}

// pi(x) on [0, 2^L), L <= 30, from the stream's round table
SPCG_HD inline uint32_t feistel_fwd_tab(uint32_t x, int L, const uint32_t* rt) {
    const int a = (L + 1) / 2, b = L - a;
    uint32_t l = x >> b, r = x & (uint32_t)low_mask(b);
#pragma unroll
    for (int j = 0; j < FEISTEL_ROUNDS; ++j) {
        const uint32_t nr = l ^ rt[((int64_t)j << a) + r];
        l = r;
        r = nr;
    }
    return (l << b) | r;
}

// pi^{-1}(y) on [0, 2^L), L <= 30, from the stream's round table
SPCG_HD inline uint32_t feistel_inv_tab(uint32_t y, int L, const uint32_t* rt) {
    const int a = (L + 1) / 2, b = L - a;
    uint32_t l = y >> b, r = y & (uint32_t)low_mask(b);
#pragma unroll
    for (int j = FEISTEL_ROUNDS - 1; j >= 0; --j) {
        const uint32_t pl = r ^ rt[((int64_t)j << a) + l];
        r = l;
        l = pl;
    }
    return (l << b) | r;
}

}  // namespace spcg
