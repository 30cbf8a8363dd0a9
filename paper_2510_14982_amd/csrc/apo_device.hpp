// apo_device.hpp -- device-side primitives of the APO step for gfx950:
// the counter-based draw stream, the keyed subset permutation behind
// "randperm", the fitness order used by the rank sort, and wavefront
// reductions.  Header-only, included by the kernels only.
#pragma once

#ifndef APO_HOST_SHIM   // defined only by the CPU test harness of these primitives
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>

namespace apok {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Ten rounds of two
// 32x32 -> 64-bit products; the key advances by the Weyl constants between
// rounds.  The counter is (purpose << 24 | block, index, iteration, run) and
// the key is the 64-bit seed.
// ---------------------------------------------------------------------------
struct Words {
    uint32_t w[4];
};

__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // one 32 x 32 -> 64-bit product each (v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Words r;
    r.w[0] = c0; r.w[1] = c1; r.w[2] = c2; r.w[3] = c3;
    return r;
}

enum : uint32_t { TAG_INIT = 1, TAG_ITER = 2, TAG_RANK = 3, TAG_ELEM = 4 };

struct Stream {
    uint32_t k0, k1, run;
    __device__ __forceinline__ Words block(uint32_t tag, uint32_t blk, uint32_t index,
                                           uint32_t iter) const {
        return philox4x32_10((tag << 24) | blk, index, iter, run, k0, k1);
    }
};

// "rand" in (0, 1): (k + 1/2) 2^-23 with k the top 23 bits of the word.  The
// value has 24 significant bits, so binary32 and binary64 hold it exactly.
template <typename T>
__device__ __forceinline__ T uniform(uint32_t w) {
    return (T(w >> 9) + T(0.5)) * T(1.1920928955078125e-07);  // 2^-23
}

// Uniform integer in [0, n): floor(w n / 2^32).
__device__ __forceinline__ uint32_t bounded(uint32_t w, uint32_t n) {
    return __umulhi(w, n);
}

// ---------------------------------------------------------------------------
// Exact m-subsets of [0, n) from a keyed alternating Feistel network over
// b = max(2, ceil(log2 n)) bits.  The set Dr of ranks is {x : pi(x) < m}
// with pi the network cycle-walked back into [0, n), so a rank is tested
// on its own with O(1) work; a coordinate mask is the first m values below
// n along the network's order of [0, 2^b) (subset_mask_group).  Round
// counts grow as the domain shrinks (24, 20, 16, 12, 8 for b <= 4, 5-6, 7,
// 8-9, >= 10); for b <= 6 the round function is a table held in the round
// key, above it is the top bits of a 24 x 24-bit product.  Round keys
// 8 .. rounds - 1 are derived from keys 0..7.
// ---------------------------------------------------------------------------
struct Subset {
    uint32_t k[24];
    uint32_t n;        // domain size
    uint32_t rounds;   // even
    uint32_t a0, c0;   // initial widths of the left / right halves
    uint32_t walk;     // 2^b: no cycle of the pass is longer
    bool table;
};

// Domain-dependent parameters (everything except the keys).
__device__ __forceinline__ void subset_shape(Subset &s, uint32_t n) {
    // b = max(2, ceil(log2 n))
    uint32_t bits = n <= 1 ? 0u : 32u - (uint32_t)__builtin_clz(n - 1u);
    bits = bits < 2 ? 2 : bits;
    s.n = n;
    s.rounds = bits <= 4 ? 24u : bits <= 6 ? 20u : bits <= 7 ? 16u : bits <= 9 ? 12u : 8u;
    s.table = bits <= 6;
    s.a0 = bits - bits / 2;
    s.c0 = bits / 2;
    s.walk = bits >= 32 ? 0xFFFFFFFFu : (1u << bits);
}

__device__ __forceinline__ void subset_init(Subset &s, const uint32_t *keys8, uint32_t n) {
    subset_shape(s, n);
#pragma unroll
    for (int i = 0; i < 8; ++i) s.k[i] = keys8[i];
#pragma unroll
    for (int i = 8; i < 24; ++i) {
        uint32_t x = s.k[i - 8] ^ (s.k[i - 7] >> 16) ^ (uint32_t)i;
        x = x * 0x7FEB352Du;
        // only the keys of the rounds in use (the rest stay zero)
        s.k[i] = i < (int)s.rounds ? x ^ (x >> 15) : 0u;
    }
}

// One round's function of the right half R (width c) into a bits.
template <bool TABLE>
__device__ __forceinline__ uint32_t feistel_f(uint32_t k, uint32_t R, uint32_t a, uint32_t c) {
    if (TABLE) return (k >> (uint32_t)__umul24(a, R)) & ((1u << a) - 1u);   // a R < 32
    // HIP's __umul24 returns int: shift the product as unsigned
    return (uint32_t)__umul24((R << (24u - c)) ^ (k >> 8), (k & 0xFFFFFFu) | 1u) >> (32u - a);
}

// A pass with a compile-time round count and round function, so the rounds
// unroll without per-round branches.
template <int ROUNDS, bool TABLE>
__device__ __forceinline__ uint32_t feistel_fwd(const uint32_t *k, uint32_t a0, uint32_t c0,
                                                uint32_t x) {
    uint32_t L = x >> c0;
    uint32_t R = x & ((1u << c0) - 1u);
#pragma unroll
    for (int i = 0; i < ROUNDS; ++i) {
        const uint32_t a = (i & 1) ? c0 : a0;   // current left width
        const uint32_t c = (i & 1) ? a0 : c0;   // current right width
        const uint32_t f = feistel_f<TABLE>(k[i], R, a, c);
        const uint32_t nl = R;
        R = L ^ f;
        L = nl;
    }
    return (L << c0) | R;   // an even number of rounds restores the widths
}

// Round counts: 24 and 20 use the table function, 16, 12 and 8 the product.
__device__ __forceinline__ uint32_t subset_pass(const Subset &s, uint32_t x) {
    switch (s.rounds) {
    case 24: return feistel_fwd<24, true>(s.k, s.a0, s.c0, x);
    case 20: return feistel_fwd<20, true>(s.k, s.a0, s.c0, x);
    case 16: return feistel_fwd<16, false>(s.k, s.a0, s.c0, x);
    case 12: return feistel_fwd<12, false>(s.k, s.a0, s.c0, x);
    default: return feistel_fwd<8, false>(s.k, s.a0, s.c0, x);
    }
}

// Cycle walking: the pass permutes [0, 2^b), so the orbit of x < n comes
// back below n within 2^b passes; the count bounds the loop regardless.
__device__ __forceinline__ uint32_t subset_pi(const Subset &s, uint32_t x) {
    uint32_t y = x;
    uint32_t steps = 0;
    do {
        y = subset_pass(s, y);
    } while (y >= s.n && ++steps < s.walk);
    return y;
}

// The coordinate-mask m-subset as a bitmask in LDS: the first m values
// below n along the pass order p(0), p(1), ..., p(2^b - 1) (one pass, no
// cycle walking).  Built by the G lanes of one group (lanes lane0 ..
// lane0 + G - 1 of one wavefront, all active): each round the lanes take
// U G consecutive positions (lane l holds positions base + j G + l, j < U,
// whose U passes are independent chains evaluated together), and, position
// block by block in order, a ballot gives each valid lane the number of
// valid values before it, so the first m are kept without any lane waiting
// on another.  For m > n / 2 the last n - m values (scanning from the end)
// are cleared from an all-ones mask instead.  U = 4 (`ilp`) shortens the
// chain where many rounds are needed or latency alone counts; U = 1 spends
// no passes past the last one needed, the choice where issue slots count.
template <int G, int U, int ROUNDS, bool TABLE>
__device__ __forceinline__ void subset_mask_scan(const Subset &s, uint32_t cnt, bool comp,
                                                 uint32_t *words, int lane, int lane0) {
    const uint32_t n = s.n, dom = s.walk;
    const uint64_t group = (G >= 64 ? ~0ull : ((1ull << G) - 1ull)) << lane0;
    const uint64_t below = (1ull << (lane0 + lane)) - 1ull;   // lanes before this one
    uint32_t taken = 0;
    for (uint32_t base = 0; taken < cnt && base < dom; base += U * G) {
        uint32_t y[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t pos = base + (uint32_t)(j * G + lane);
            const uint32_t x = pos < dom ? (comp ? dom - 1u - pos : pos) : 0u;
            y[j] = feistel_fwd<ROUNDS, TABLE>(s.k, s.a0, s.c0, x);
            if (pos >= dom) y[j] = 0xFFFFFFFFu;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const bool valid = y[j] < n;
            const uint64_t vb = __ballot(valid) & group;
            const uint32_t before = (uint32_t)__popcll(vb & below);
            if (valid && taken + before < cnt) {
                if (comp)
                    atomicAnd(&words[y[j] >> 5], ~(1u << (y[j] & 31)));
                else
                    atomicOr(&words[y[j] >> 5], 1u << (y[j] & 31));
            }
            taken += (uint32_t)__popcll(vb);
        }
    }
}

template <int G, int U>
__device__ __forceinline__ void subset_mask_rounds(const Subset &s, uint32_t cnt, bool comp,
                                                   uint32_t *words, int lane, int lane0) {
    switch (s.rounds) {
    case 24: subset_mask_scan<G, U, 24, true>(s, cnt, comp, words, lane, lane0); break;
    case 20: subset_mask_scan<G, U, 20, true>(s, cnt, comp, words, lane, lane0); break;
    case 16: subset_mask_scan<G, U, 16, false>(s, cnt, comp, words, lane, lane0); break;
    case 12: subset_mask_scan<G, U, 12, false>(s, cnt, comp, words, lane, lane0); break;
    default: subset_mask_scan<G, U, 8, false>(s, cnt, comp, words, lane, lane0); break;
    }
}

template <int G>
__device__ __forceinline__ void subset_mask_group(const Subset &s, uint32_t m, uint32_t *words,
                                                  int nwords, int lane, int lane0,
                                                  bool ilp = false) {
    const uint32_t n = s.n;
    const bool comp = m > n - m;
    const uint32_t cnt = comp ? n - m : m;
    for (int w = lane; w < nwords; w += G) words[w] = comp ? 0xFFFFFFFFu : 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (ilp)
        subset_mask_rounds<G, 4>(s, cnt, comp, words, lane, lane0);
    else
        subset_mask_rounds<G, 1>(s, cnt, comp, words, lane, lane0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Membership in the m-subset; m >= n selects all, m == 0 none.
__device__ __forceinline__ bool subset_has(const Subset &s, uint32_t x, uint32_t m) {
    if (m >= s.n) return true;
    if (m == 0) return false;
    return subset_pi(s, x) < m;
}

// ---------------------------------------------------------------------------
// Fitness order: ascending, -0 == +0, every NaN after +inf, ties by id.
// The order-preserving unsigned image of a float/double; NaN maps to the
// all-ones pattern, both zeros to the image of +0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t order_key(float f) {
    if (f != f) return 0xFFFFFFFFu;
    if (f == 0.0f) f = 0.0f;
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ uint64_t order_key(double f) {
    if (f != f) return 0xFFFFFFFFFFFFFFFFull;
    if (f == 0.0) f = 0.0;
    const uint64_t b = (uint64_t)__double_as_longlong(f);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

// Strict "better than" used by the greedy selection: NaN never wins.
template <typename T>
__device__ __forceinline__ bool strictly_less(T a, T b) {
    return a < b;
}

// A lane exchange applied to every 32-bit word of a value: DPP controls
// within rows of 16 lanes, or a swizzle within 32.
template <typename T>
struct Words32 {
    static_assert(sizeof(T) % 4 == 0, "32-bit words");
    int w[sizeof(T) / 4];
};
template <int CTRL, typename T>
__device__ __forceinline__ T lane_dpp(T v) {
    Words32<T> a, b;
    __builtin_memcpy(&a, &v, sizeof(T));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i)
        b.w[i] = __builtin_amdgcn_update_dpp(0, a.w[i], CTRL, 0xF, 0xF, true);
    T r;
    __builtin_memcpy(&r, &b, sizeof(T));
    return r;
}
template <typename T>
__device__ __forceinline__ T lane_swap16(T v) {   // lane l <-> l ^ 16
    Words32<T> a, b;
    __builtin_memcpy(&a, &v, sizeof(T));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i)
        b.w[i] = __builtin_amdgcn_ds_swizzle(a.w[i], 0x401F);   // and 0x1F, xor 0x10
    T r;
    __builtin_memcpy(&r, &b, sizeof(T));
    return r;
}

// Sum over an aligned group of G lanes (all active).  Stage by stage each
// lane adds its value to that of a partner holding the same partial sum of
// the other half of its block (quad xor 1 and xor 2, then the mirrors of 8
// and 16 lanes, then xor 16 and xor 32), and the two lanes of a pair add
// the same two operands, so every lane of the group ends with a
// bit-identical total.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
    if (G >= 2) v += lane_dpp<0xB1>(v);     // quad_perm [1, 0, 3, 2]
    if (G >= 4) v += lane_dpp<0x4E>(v);     // quad_perm [2, 3, 0, 1]
    if (G >= 8) v += lane_dpp<0x141>(v);    // row_half_mirror
    if (G >= 16) v += lane_dpp<0x140>(v);   // row_mirror
    if (G >= 32) v += lane_swap16(v);
    if (G >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

}  // namespace apok
