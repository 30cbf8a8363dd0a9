// CPU harness for the device primitives of the HIP library
// (paper_2510_14982_amd/csrc/apo_device.hpp): the header is compiled for the
// host with stand-ins that keep HIP's exact signatures (in particular
// `int __umul24(unsigned, unsigned)`), and its draws, subset permutation and
// fitness order are printed for comparison with the oracle.
// Usage: device_primitives_host <mode> ; reads queries on stdin.
//   mode "pi":     lines "n x k0..k7"    -> pi(x)
//   mode "philox": lines "c0 c1 c2 c3 k0 k1" -> 4 words
//   mode "key32":  lines "<hex bits of a float>" -> order key
//   mode "mask":   lines "n m k0..k7"    -> the members of the coordinate-mask
//                  m-subset, ascending, space separated
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#define APO_HOST_SHIM 1
#define __device__
#define __forceinline__ inline
static inline int __umul24(unsigned int a, unsigned int b) {
    return (int)((a & 0xFFFFFFu) * (b & 0xFFFFFFu));
}
static inline unsigned int __umulhi(unsigned int a, unsigned int b) {
    return (unsigned int)(((uint64_t)a * b) >> 32);
}
static inline unsigned int __float_as_uint(float f) { unsigned int u; std::memcpy(&u, &f, 4); return u; }
static inline long long __double_as_longlong(double f) { long long u; std::memcpy(&u, &f, 8); return u; }
template <class T> static inline T __shfl_xor(T v, int, int) { return v; }
// one lane: the ballot is that lane's predicate in bit 0
static inline unsigned long long __ballot(int pred) { return pred ? 1ull : 0ull; }
static inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
// lane exchanges (unused with one lane)
#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) (src)
#define __builtin_amdgcn_ds_swizzle(src, pat) (src)
// one "lane" runs the whole group loop on the host (G = 1)
#define __builtin_amdgcn_fence(a, b) ((void)0)
#define __builtin_amdgcn_wave_barrier() ((void)0)
#define __ATOMIC_RELEASE 0
#define __ATOMIC_ACQUIRE 0
static inline unsigned atomicOr(unsigned *p, unsigned v) { unsigned o = *p; *p |= v; return o; }
static inline unsigned atomicAnd(unsigned *p, unsigned v) { unsigned o = *p; *p &= v; return o; }
#include "apo_device.hpp"

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    const char *mode = argv[1];
    if (!std::strcmp(mode, "pi")) {
        unsigned n, x, k[8];
        while (std::scanf("%u %u %u %u %u %u %u %u %u %u", &n, &x, &k[0], &k[1], &k[2], &k[3],
                          &k[4], &k[5], &k[6], &k[7]) == 10) {
            apok::Subset s;
            apok::subset_init(s, k, n);
            std::printf("%u\n", apok::subset_pi(s, x));
        }
    } else if (!std::strcmp(mode, "philox")) {
        unsigned c[4], k[2];
        while (std::scanf("%u %u %u %u %u %u", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
            apok::Words w = apok::philox4x32_10(c[0], c[1], c[2], c[3], k[0], k[1]);
            std::printf("%u %u %u %u\n", w.w[0], w.w[1], w.w[2], w.w[3]);
        }
    } else if (!std::strcmp(mode, "mask")) {
        unsigned n, m, k[8];
        static unsigned words[1 << 11];
        while (std::scanf("%u %u %u %u %u %u %u %u %u %u", &n, &m, &k[0], &k[1], &k[2], &k[3],
                          &k[4], &k[5], &k[6], &k[7]) == 10) {
            apok::Subset s;
            apok::subset_init(s, k, n);
            const int nw = (int)((n + 31) / 32);
            // both scan forms (one position a round, and four) give the same set
            static unsigned words4[1 << 11];
            apok::subset_mask_group<1>(s, m, words, nw, 0, 0, false);
            apok::subset_mask_group<1>(s, m, words4, nw, 0, 0, true);
            if (std::memcmp(words, words4, (size_t)nw * 4) != 0) {
                std::printf("scan forms differ\n");
                return 1;
            }
            for (unsigned x = 0; x < n; ++x)
                if ((words[x >> 5] >> (x & 31)) & 1u) std::printf("%u ", x);
            std::printf("\n");
        }
    } else if (!std::strcmp(mode, "key32")) {
        unsigned b;
        while (std::scanf("%x", &b) == 1) {
            float f;
            std::memcpy(&f, &b, 4);
            std::printf("%u\n", apok::order_key(f));
        }
    }
    return 0;
}
