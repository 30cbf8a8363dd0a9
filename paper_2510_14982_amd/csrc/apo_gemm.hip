// apo_gemm.hip -- the GEMM form of the step for rotated objectives of large
// dimension (binary32 state): per iteration
//   candidates  -> Yr [ps][Dp] (rank order) and A = bf16(y - o) [ps][Kp]
//   Z = A M^T on the matrix cores (binary32 or BF16 operands), with the
//                  objective's row sums fused into the epilogue (partials)
//   selection   -> strict greedy choice, rows written to the next buffer.
// With bfloat16 (BF16) operands the product is a cheap estimate: each
// candidate whose comparison with its parent the estimate cannot settle
// under a rigorous error bound -- and every certain acceptance -- is
// re-scored by the same binary32 product on the listed rows, so every stored
// fitness equals the binary32 form's.  The elite's final fitness is
// re-scored in binary64.
#include "apo_step.hpp"

namespace apok {

// Binary32 product: 128 x 64 output tile per workgroup, both operands staged
// through LDS in chunks of 32 K.
constexpr int kGM = 128, kGN = 64;       // output tile of a workgroup
static_assert(kGN == 64, "a workgroup sums one 64-column objective half");
constexpr int kGRowB = 128;              // bytes of K per row and chunk
constexpr int kGLds = kGRowB + 16;       // LDS row stride in bytes (9 x 16: rows of a
                                         // fragment read fall in distinct bank groups)
constexpr int kGQ = kGRowB / 32;         // 16-byte vectors of A per loader thread
constexpr int kGBT = 256 / kGN;          // loader threads per row of M
constexpr int kGQB = kGRowB / kGBT / 16; // 16-byte vectors of M per loader thread
constexpr size_t kGemmLds = (size_t)(kGM + kGN) * kGLds;   // dynamic LDS of the product

// BF16 product: 256 x 128 output tile per workgroup (8 wavefronts of 32 rows,
// two per SIMD), A straight from global memory into fragments, M's 128 rows
// through LDS in chunks of kBK K, two buffers.  Both BF16 operands are stored in MFMA
// fragment order: per 16-row group and 32-K chunk one 1 KiB block, lane l's
// 16 bytes holding row l % 16, K 8 (l / 16) .. + 7 of the chunk.
constexpr int kBM = 256, kBN = 128, kBK = 32;
constexpr int kBKS = kBK / 32;           // MFMA k-steps per chunk
static_assert(kBK == 32, "one fragment block of M per chunk");
constexpr int kBBlk = 1024;              // bytes of one fragment block
constexpr int kBThreads = 512;           // 8 wavefronts
constexpr int kBRT = kBM / 16 / (kBThreads / 64);   // row tiles of 16 per wavefront
constexpr int kBQ = (kBN / 16) * kBBlk / (16 * kBThreads);   // 16-byte units each thread
                                                             // stages per chunk
static_assert(kBRT == 2 && kBQ == 1, "one column group of M per wavefront and chunk");
constexpr size_t kBBuf = (size_t)(kBN / 16) * kBBlk;   // M of one chunk: 8 blocks
constexpr size_t kBLdsBytes = 2 * kBBuf;
// LDS reserved at launch: more than half of a CU's 160 KB, so that a CU
// holds one workgroup and a grid of one workgroup per CU spreads over all CUs.
constexpr size_t kBLdsLaunch = 96 * 1024;
static_assert(kBLdsBytes <= kBLdsLaunch, "BF16 product LDS");

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// One product launch: rows are list slots (list != nullptr: slot k is rank
// list[k], *count slots) or ranks (rows of them).
struct GemmRun {
    const uint16_t *Ab;   // BF16 A rows [pop][Kp], or nullptr: A = y - o from Yr
    const float *Yr;      // [pop][Dp]
    const float *o;       // [Dp]
    const void *B;        // M rows [Np][Kp] (BF16 or binary32)
    const int32_t *list;
    const int32_t *count;
    int rows, D, Dp, Kp, Np, kind;
    float *P1, *P2;       // [slot][Np / 64]
};

__device__ __forceinline__ uint16_t to_bf16(float x) {   // round to nearest even
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// Candidates of one iteration (or of the initial population), by rank.
// ---------------------------------------------------------------------------
template <int G, int NCH, int NPMAX, bool BF16>
__global__ __launch_bounds__(256) void gemm_cand(Params p, GemmBufs w, int init) {
    typedef float T;
    const int lane = threadIdx.x & (G - 1);
    const int item = (blockIdx.x * 256 + threadIdx.x) / G;
    if (!init && blockIdx.x == 0 && threadIdx.x == 0) *w.count = 0;   // rescore list
    if (item >= p.pop) return;
    const int D = p.dim, Dp = p.Dp;
    const Iter it = load_iter(p, init);
    const int t = it.t;
    const T *Xc = (const T *)p.X[(t + 1) & 1];
    constexpr int MW = (4 * G * NCH + 31) / 32;
    __shared__ uint32_t mwords[256 / G][MW];
    Plan<T, NPMAX> c;
    Rows<T, NCH> rw;
    if (init) {
        c.op = OP_DORMANCY; c.id = item; c.r = item; c.m = (uint32_t)D; c.fold = T(0);
    } else {
        Draws<T> d;
        plan_draws<T, NPMAX>(p, item, t, (threadIdx.x & 63) & ~(G - 1), lane, c, d);
        uniform_draws<G>(d);
        plan_decide<T, NPMAX>(p, item, it, d, c);
        plan_pick<T, NPMAX>(d, c);
        load_rows<T, NPMAX, NCH, G>(p, c, lane, Xc, rw);
        plan_mask<T, NPMAX, G>(p, c, mwords[threadIdx.x / G], lane);
        plan_pairs<T, NPMAX>(p, item, t, d, c);
    }
    const T *o = (const T *)p.shift;
    float *yrow = w.Yr + (size_t)item * Dp;
    // BF16 A in MFMA fragment order: block (item / 16, d / 32) holds 64 lanes
    // x 8 values, lane item % 16 + 16 ((d % 32) / 8) taking d % 8 = 0..7
    uint16_t *ablk = BF16 ? w.Ab + (size_t)(item >> 4) * (size_t)(w.Kp / 32) * 512 : nullptr;
    float ss = 0.f;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const int d0 = 4 * (lane + ch * G);
        if (d0 < D) {
            T y[4], ov[4];
            candidate4<T, NPMAX>(p, c, t, init != 0, d0, Xc, rw.x[ch], rw.xj[ch], rw.am[ch],
                                 rw.ap[ch], y);
            load4(o + d0, ov);
            store4(yrow + d0, y);
            uint32_t hb[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float a = d0 + e < D ? y[e] - ov[e] : 0.f;
                ss += a * a;
                hb[e] = BF16 ? to_bf16(a) : 0u;
            }
            if (BF16) {
                const int kk = d0 & 31, lf = (item & 15) + 16 * (kk >> 3);
                *(uint2 *)(ablk + ((size_t)(d0 >> 5) * 64 + lf) * 8 + (kk & 7)) =
                    make_uint2(hb[0] | (hb[1] << 16), hb[2] | (hb[3] << 16));
            }
        }
    }
    if (BF16) {
        ss = group_sum<G>(ss);
        if (lane == 0) w.anorm[item] = sqrtf(ss);
    }
    if (p.trace && !init && lane == 0) p.trOp[c.id] = c.op;
}

// One chunk (kGRowB bytes of K) of a loader thread's half rows of A and B
// into registers: B from the packed binary32 M rows, A = y - o computed from
// the binary32 candidates.
struct GemmChunk {
    uint4 a[kGQ], b[kGQB];
};

__device__ __forceinline__ GemmChunk gemm_fetch(const GemmRun &g, const unsigned char *Bp,
                                                int arow, bool live, int lh, int kc) {
    GemmChunk c;
    const uint4 *bp = (const uint4 *)(Bp + (size_t)kc * 4);
#pragma unroll
    for (int q = 0; q < kGQB; ++q) c.b[q] = bp[q];
    const int k0 = kc + lh * (kGRowB / 8);   // 4-byte elements of the half row
    const float *yr = g.Yr + (size_t)arow * g.Dp;
    if (live && k0 + 4 * kGQ <= g.D) {
#pragma unroll
        for (int q = 0; q < kGQ; ++q) {
            const float4 y4 = ((const float4 *)(yr + k0))[q];
            const float4 o4 = ((const float4 *)(g.o + k0))[q];
            c.a[q] = make_uint4(__float_as_uint(y4.x - o4.x), __float_as_uint(y4.y - o4.y),
                                __float_as_uint(y4.z - o4.z), __float_as_uint(y4.w - o4.w));
        }
    } else {
#pragma unroll
        for (int q = 0; q < kGQ; ++q) {
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = k0 + 4 * q + e;
                v[e] = (live && k < g.D) ? yr[k] - g.o[k] : 0.f;
            }
            c.a[q] = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]),
                                __float_as_uint(v[2]), __float_as_uint(v[3]));
        }
    }
    return c;
}

// Objective terms of one output element, added to the row's two partial sums
// (P1: the summed terms, or z^2 for Ackley; P2: cos 2 pi z for Ackley, z^2
// otherwise).  Columns past D (live false) add nothing.
template <int KIND>
__device__ __forceinline__ void obj_terms(float z, bool live, float &g1, float &g2) {
    const float zz = z * z;
    if constexpr (KIND == K_RASTRIGIN) {
        g1 += live ? zz - 10.f * cos2pi(z) + 10.f : 0.f;
        g2 += live ? zz : 0.f;
    } else if constexpr (KIND == K_ACKLEY) {
        g1 += live ? zz : 0.f;
        g2 += live ? cos2pi(z) : 0.f;
    } else {
        g1 += live ? zz : 0.f;
        g2 += live ? zz : 0.f;
    }
}

// ---------------------------------------------------------------------------
// Binary32 product Z = A M^T with the objective's per-row sums over each
// 64-column half tile fused into the epilogue.  Rows are list slots (the
// ranks of a re-score list) or ranks; A = y - o is computed from Yr while
// loading.  Workgroup: 128 rows x 64 columns (one objective half), 4
// wavefronts of 32 rows each (2 x 4 MFMA 16 x 16 x 4 tiles), so that a CU
// holds four workgroups; K in chunks of 128 bytes per row, the next chunk
// fetched into registers during the MFMA work.
// ---------------------------------------------------------------------------
template <int KIND>
__global__ __launch_bounds__(256) void gemm_obj_f32(GemmRun g) {
    constexpr int KC = kGRowB / 4;
    extern __shared__ __align__(16) unsigned char gsm[];
    unsigned char *sA = gsm, *sB = gsm + kGM * kGLds;
    const int nrows = g.list ? *g.count : g.rows;
    // the column blocks of a row block on one XCD (workgroup b runs on XCD
    // b mod 8), so the block's A rows are fetched from HBM once into its L2
    const int nM = (g.rows + kGM - 1) / kGM, nN = g.Np / kGN;
    const int b = blockIdx.x;
    int rb, nb;
    if ((nM & 7) == 0) {
        const int x = b & 7, idx = b >> 3;
        rb = (idx / nN) * 8 + x;
        nb = idx % nN;
    } else {
        rb = b / nN;
        nb = b % nN;
    }
    const int m0 = rb * kGM;
    if (m0 >= nrows) return;   // the whole workgroup: no barrier is skipped
    const int n0 = nb * kGN;
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
    const int lr = tid >> 1, lh = tid & 1;                  // A loader: row, half chunk
    const int br = tid / kGBT, bq = tid % kGBT;              // M loader: row, part
    const int slot = m0 + lr;
    const bool live = slot < nrows;
    const int arow = live ? (g.list ? g.list[slot] : slot) : 0;
    const unsigned char *Bp =
        (const unsigned char *)g.B + (size_t)(n0 + br) * g.Kp * 4 + bq * (kGQB * 16);
    f32x4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int wr = 32 * wave;
    GemmChunk ch = gemm_fetch(g, Bp, arow, live, lh, 0);
    for (int kc = 0; kc < g.Kp; kc += KC) {
        __syncthreads();   // the previous chunk's readers are done
        uint4 *da = (uint4 *)(sA + lr * kGLds + lh * (kGRowB / 2));
        uint4 *db = (uint4 *)(sB + br * kGLds + bq * (kGQB * 16));
#pragma unroll
        for (int q = 0; q < kGQ; ++q) da[q] = ch.a[q];
#pragma unroll
        for (int q = 0; q < kGQB; ++q) db[q] = ch.b[q];
        __syncthreads();
        if (kc + KC < g.Kp)   // in flight during the MFMA work
            ch = gemm_fetch(g, Bp, arow, live, lh, kc + KC);
#pragma unroll
        for (int ks = 0; ks < KC / 4; ++ks) {
            // 16 x 16 x 4 FP32: lane l holds A[l % 16][l / 16], B[l / 16][l % 16]
            const int kb = (ks * 4 + (l >> 4)) * 4;
            float a[2], b[4];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = *(const float *)(sA + (wr + 16 * i + (l & 15)) * kGLds + kb);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                b[j] = *(const float *)(sB + (16 * j + (l & 15)) * kGLds + kb);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    // epilogue: element v of lane l in tile (i, j) is Z[row 4 (l / 16) + v][col l % 16]
    const int half = n0 / 64, NH = g.Np / 64;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float g1 = 0.f, g2 = 0.f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int col = n0 + 16 * j + (l & 15);
                obj_terms<KIND>(acc[i][j][v], col < g.D, g1, g2);
            }
            g1 = group_sum<16>(g1);
            g2 = group_sum<16>(g2);
            const int srow = m0 + wr + 16 * i + 4 * (l >> 4) + v;
            if ((l & 15) == 0 && srow < nrows) {
                g.P1[(size_t)srow * NH + half] = g1;
                g.P2[(size_t)srow * NH + half] = g2;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// BF16 estimate product Z = bf16(y - o) bf16(M)^T with binary32 accumulation
// on the 16 x 16 x 32 BF16 matrix cores, the same epilogue partials as the
// binary32 product.  Workgroup tile 256 rows x 128 columns: wavefront w owns
// rows 32 w .. 32 w + 31 (2 x 8 MFMA tiles, 64 accumulators per lane; two
// wavefronts per SIMD, so one's loads overlap the other's matrix work) and
// reads its A rows from global memory straight into fragment registers,
// kBDA chunks ahead; the 128 rows of M the eight wavefronts share are staged
// through LDS in chunks of 32 K (two buffers, one barrier per chunk).  The
// tiles of a row block are placed on one XCD (workgroup b runs on XCD b mod
// 8), so the block's A rows are fetched from HBM once into that XCD's L2.
// ---------------------------------------------------------------------------
struct BChunkA {
    u32x4 v[kBRT][kBKS];   // [row tile][k-step]: 8 BF16 of K per lane and step
};

// A of chunk kc (K elements) for the lane's four row tiles: A is stored in
// fragment order (each 16-row x 32-K block is the 64 lanes' 16 bytes in lane
// order), so a wavefront's load of one tile is 1 KiB contiguous; aoff[i] is
// the lane's byte offset in its row group's first block.
__device__ __forceinline__ void bf16_load_a(const unsigned char *abase, const uint32_t (&aoff)[kBRT],
                                            int kc, BChunkA &a) {
    const unsigned char *b = abase + (size_t)kc * 32;   // 1 KiB per 32 K
#pragma unroll
    for (int i = 0; i < kBRT; ++i)
#pragma unroll
        for (int s = 0; s < kBKS; ++s) a.v[i][s] = *(const u32x4 *)(b + aoff[i] + 1024 * s);
}

// Prefetch depths of the BF16 product, in chunks: A rows come from HBM (or
// from the L2 after the first of a row block's workgroups), M's rows from
// the L2.
constexpr int kBDA = 3, kBDB = 2;

// One K chunk c of the BF16 product (A in a[c % 4], M in LDS buffer c & 1).
// Issued first: the A loads of chunk c + kBDA into a[(c + kBDA) % 4] and the
// M loads of chunk c + kBDB into bs[c % 2]; after the MFMA work, M of chunk
// c + 1 (loaded one chunk earlier, in bs[(c + 1) % 2]) goes to LDS buffer
// (c + 1) & 1.  Chunks past the end re-read the last one (unused).
template <int PH>
__device__ __forceinline__ void bf16_chunk(int c, int nc, const unsigned char *abase,
                                           const uint32_t (&aoff)[kBRT],
                                           const unsigned char *bsrc, size_t bstride,
                                           unsigned char *bdst, const unsigned char *bfr,
                                           BChunkA (&a)[4], u32x4 (&bs)[2][kBQ],
                                           f32x4 (&acc)[kBRT][8]) {
    {
        const size_t ob = (size_t)min(c + kBDB, nc - 1) * kBBlk;
#pragma unroll
        for (int q = 0; q < kBQ; ++q) bs[PH % 2][q] = *(const u32x4 *)(bsrc + q * bstride + ob);
        bf16_load_a(abase, aoff, min(c + kBDA, nc - 1) * kBK, a[(PH + kBDA) % 4]);
    }
    __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the MFMA work
    const BChunkA &cur = a[PH];
    const unsigned char *sb = bfr + (PH & 1) * kBBuf;
#pragma unroll
    for (int s = 0; s < kBKS; ++s) {
        // lane l: B[k = 8 (l / 16) .. + 7 of the chunk][column 16 j + l % 16]
        u32x4 bv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) bv[j] = *(const u32x4 *)(sb + j * kBBlk);
        __builtin_amdgcn_sched_barrier(0);   // all eight reads in flight before the MFMAs
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int i = 0; i < kBRT; ++i)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, cur.v[i][s]), __builtin_bit_cast(bf16x8, bv[j]),
                    acc[i][j], 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
    unsigned char *d = bdst + ((PH + 1) & 1) * kBBuf;
#pragma unroll
    for (int q = 0; q < kBQ; ++q)
        *(u32x4 *)(d + q * ((kBThreads / 64) * kBBlk)) = bs[(PH + 1) % 2][q];
    __syncthreads();
}

template <int KIND>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void gemm_obj_bf16(
    GemmRun g) {
    extern __shared__ __align__(16) unsigned char gsm[];
    const int nrows = g.rows;   // ranks (the BF16 product has no list form)
    const int nM = (g.rows + kBM - 1) / kBM, nN = g.Np / kBN;
    const int b = blockIdx.x;
    int rb, nb;
    if ((nM & 7) == 0) {
        const int x = b & 7, idx = b >> 3;
        rb = (idx / nN) * 8 + x;
        nb = idx % nN;
    } else {
        rb = b / nN;
        nb = b % nN;
    }
    const int m0 = rb * kBM, n0 = nb * kBN;
    if (m0 >= nrows) return;   // the whole workgroup: no barrier is skipped
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
    // lane l: row 16 i + l % 16 of the wavefront's rows, K offset 8 (l / 16),
    // in the row group's fragment-order blocks (A holds whole 256-row tiles;
    // rows past the end are zero and their sums are not stored).  The 32-bit
    // byte offsets hold: at most 65536 rows of 1024 BF16 values (128 MiB).
    const unsigned char *abase = (const unsigned char *)g.Ab;
    uint32_t aoff[kBRT];
#pragma unroll
    for (int i = 0; i < kBRT; ++i) {
        const uint32_t rg = (uint32_t)(m0 + 16 * kBRT * wave + 16 * i) >> 4;
        aoff[i] = (rg * (uint32_t)(g.Kp / 32) * 64u + (uint32_t)l) * 16u;
    }
    // M staging: thread tid moves lane tid % 64 of column group n0 / 16 +
    // tid / 64 (one fragment block per wavefront, contiguous), to the same
    // place of the chunk's LDS buffer (kBQ == 1: one 16-byte unit a thread)
    const size_t bstride = (size_t)(kBThreads / 64) * (g.Kp / 32) * kBBlk;   // next groups
    const unsigned char *bsrc = (const unsigned char *)g.B +
                                ((size_t)(n0 / 16 + (tid >> 6)) * (g.Kp / 32) * kBBlk) +
                                (size_t)(tid & 63) * 16;
    unsigned char *bdst = gsm + (tid >> 6) * kBBlk + (tid & 63) * 16;
    // fragment reads: lane l's 16 bytes of column group j's block
    const unsigned char *bfr = gsm + l * 16;
    f32x4 acc[kBRT][8];
#pragma unroll
    for (int i = 0; i < kBRT; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nc = g.Kp / kBK;   // a multiple of 4: Kp is a multiple of 128
    BChunkA a[4];
    u32x4 bs[2][kBQ];
    // prologue: A of chunks 0 .. kBDA - 1, M of chunk 0 into LDS buffer 0 and
    // M of chunk 1 into bs[1]
#pragma unroll
    for (int q = 0; q < kBQ; ++q) {
        bs[0][q] = *(const u32x4 *)(bsrc + q * bstride);
        bs[1][q] = *(const u32x4 *)(bsrc + q * bstride + kBBlk);
    }
#pragma unroll
    for (int c = 0; c < kBDA; ++c) bf16_load_a(abase, aoff, c * kBK, a[c]);
#pragma unroll
    for (int q = 0; q < kBQ; ++q) *(u32x4 *)(bdst + q * ((kBThreads / 64) * kBBlk)) = bs[0][q];
    __syncthreads();
    for (int c = 0; c < nc; c += 4) {
        bf16_chunk<0>(c, nc, abase, aoff, bsrc, bstride, bdst, bfr, a, bs, acc);
        bf16_chunk<1>(c + 1, nc, abase, aoff, bsrc, bstride, bdst, bfr, a, bs, acc);
        bf16_chunk<2>(c + 2, nc, abase, aoff, bsrc, bstride, bdst, bfr, a, bs, acc);
        bf16_chunk<3>(c + 3, nc, abase, aoff, bsrc, bstride, bdst, bfr, a, bs, acc);
    }
    // epilogue: element v of lane l in tile (i, j) is Z[row 4 (l / 16) + v][col l % 16];
    // columns 0..63 and 64..127 of the tile give two half partials
    const int NH = g.Np / 64;
#pragma unroll
    for (int i = 0; i < kBRT; ++i) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int srow = m0 + 16 * kBRT * wave + 16 * i + 4 * (l >> 4) + v;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float g1 = 0.f, g2 = 0.f;
#pragma unroll
                for (int j = 4 * h; j < 4 * h + 4; ++j) {
                    const int col = n0 + 16 * j + (l & 15);
                    obj_terms<KIND>(acc[i][j][v], col < g.D, g1, g2);
                }
                g1 = group_sum<16>(g1);
                g2 = group_sum<16>(g2);
                if ((l & 15) == 0 && srow < nrows) {
                    g.P1[(size_t)srow * NH + n0 / 64 + h] = g1;
                    g.P2[(size_t)srow * NH + n0 / 64 + h] = g2;
                }
            }
        }
    }
}

// Objective of a row from its partial sums (fixed order).
__device__ __forceinline__ void row_sums(const GemmRun &g, int slot, float &s1, float &s2) {
    const int NH = g.Np / 64;
    s1 = 0.f;
    s2 = 0.f;
    for (int h = 0; h < NH; ++h) {
        s1 += g.P1[(size_t)slot * NH + h];
        s2 += g.P2[(size_t)slot * NH + h];
    }
}

__device__ __forceinline__ float row_objective(int kind, int D, float s1, float s2) {
    if (kind == K_ACKLEY)
        return -20.f * expf(-0.2f * sqrtf(s1 / (float)D)) - expf(s2 / (float)D) + 20.f +
               (float)kE;
    return s1;
}

// Copies a row of D floats (one wavefront).
__device__ __forceinline__ void copy_row(float *dst, const float *src, int D, int l) {
    for (int d0 = 4 * l; d0 < D; d0 += 256) {
        if (d0 + 4 <= D) {
            *(float4 *)(dst + d0) = *(const float4 *)(src + d0);
        } else {
            for (int d = d0; d < D; ++d) dst[d] = src[d];
        }
    }
}

// Selection (one wavefront per rank).  mode 0: every rank's binary32
// fitness from the product's partials (slot = rank); mode 1 (BF16 form):
// ranks the classification settled as rejections carry the parent row over,
// the others take their binary32 fitness from the re-score product (slot =
// status[r]).  Writes the chosen row and fitness of the next buffer.
__global__ __launch_bounds__(256) void gemm_select(Params p, GemmRun g, GemmBufs w, int init,
                                                   int mode) {
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int t = init ? 0 : __hip_atomic_load(&p.ctrl->t_next, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (!init && blockIdx.x == 0 && threadIdx.x == 0) {
        p.ctrl->t = t;   // iteration closed
        if (mode == 1) *w.total += (unsigned long long)*w.count;
    }
    const int r = blockIdx.x * 4 + wave;
    if (r >= p.pop) return;
    const int id = init ? r : p.perm[r];
    const int slot = mode == 1 ? w.status[r] : r;
    const float fold = init ? 0.f : ((const float *)p.Fs)[r];
    float fnew;
    if (slot >= 0) {
        float s1, s2;
        row_sums(g, slot, s1, s2);
        fnew = row_objective(p.kind, p.dim, s1, s2);
    } else {
        fnew = w.anorm[r];   // the classification left the BF16 estimate here
    }
    const bool accept = init || (slot >= 0 && fnew < fold);
    const float *X0 = (const float *)p.X[(t + 1) & 1];
    float *X1 = (float *)p.X[t & 1];
    const float *y = w.Yr + (size_t)r * p.Dp;
    copy_row(X1 + (size_t)id * p.Dp, accept ? y : X0 + (size_t)id * p.Dp, p.dim, l);
    if (l == 0) ((float *)p.F)[id] = accept ? fnew : fold;
    if (p.trace && !init) {
        copy_row((float *)p.trY + (size_t)id * p.Dp, y, p.dim, l);
        if (l == 0) ((float *)p.trF)[id] = fnew;
    }
}

// BF16 classification (one thread per rank): from the estimate F^ and the
// bound B on |F^ - F32| (F32 = the binary32 form's value of the same
// candidate), a candidate with F^ - B >= F_old is certainly rejected
// (status -1); every other rank is appended to the re-score list (status =
// its slot), with one atomic per workgroup.  The estimate is left in
// anorm[r] for the trace.
__global__ __launch_bounds__(256) void gemm_classify(Params p, GemmRun g, GemmBufs w) {
    __shared__ int s_n[4], s_base;
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
    const int r = blockIdx.x * 256 + tid;
    const int D = p.dim;
    bool need = false;
    float fhat = 0.f;
    if (r < p.pop) {
        float s1, s2;
        row_sums(g, r, s1, s2);
        fhat = row_objective(p.kind, D, s1, s2);
        const float fold = ((const float *)p.Fs)[r];
        // Error of the estimate's coordinate vector against the binary32
        // form's, in the 2-norm (a = y - o in binary32, z = M a, M in binary32,
        // the estimate's operands a_b = bf16(a) and M_b = bf16(M)):
        //   operand rounding  M_b a_b - M a = M (a_b - a) + (M_b - M) a_b, with
        //     ||M||_2 <= 1.01 (orthogonal rows in binary32),
        //     ||a_b - a||_2 <= 2^-8 ||a||_2 and ||M_b - M||_2 <= nrm_dM;
        //   accumulation      the binary32 form's sums over D rounded products
        //     and the estimate's over D exact ones: |error_i| <= gam
        //     sum_j |M_ij| |a_j| with gam = gamma_(D+2) (times (1 + 2^-8)^2 for
        //     the rounded BF16 operands), whose 2-norm is <= gam || |M| ||_2
        //     ||a||_2, || |M| ||_2 <= nrm_absM.
        const float ub = 0.00390625f;                                  // 2^-8
        const float u32 = 5.9604645e-8f;                               // 2^-24
        const float gam = (float)(D + 2) * u32 / (1.f - (float)(D + 2) * u32);
        const float an = 1.001f * w.anorm[r];   // ||a||_2 as summed in binary32
        const float E = (1.01f * ub + w.nrm_dM * (1.f + ub) +
                         gam * (1.f + (1.f + ub) * (1.f + ub)) * w.nrm_absM) * an;
        const float sD = sqrtf((float)D);
        // sum_i |cos 2 pi a_i - cos 2 pi b_i| <= min(2 D, 2 pi ||a - b||_1),
        // ||.||_1 <= sqrt(D) ||.||_2
        const float dc = fminf(2.f * (float)D, 6.2831853f * sD * E);
        const float gD = 2.f * (float)D * u32;               // binary32 evaluation of sums
        float B;
        if (p.kind == K_ACKLEY) {
            // r = ||z||_2 / sqrt(D) moves by at most E / sqrt(D); 20 exp(-0.2 r) is
            // 4-Lipschitz in r; exp(S2 / D) <= e
            const float rr = sqrtf(s1 / (float)D);
            B = 4.f * E / sD + 2.7182818f * dc / (float)D + gD * (4.f * rr + 2.7182818f);
        } else {
            // | ||z^||^2 - ||z~||^2 | <= E (2 ||z^||_2 + E)
            const float zn = sqrtf(s2);                      // ||z^||_2
            B = E * (2.f * zn + E) + (p.kind == K_RASTRIGIN ? 10.f * dc : 0.f) +
                gD * (s2 + (p.kind == K_RASTRIGIN ? 20.f * (float)D : 0.f));
        }
        B = B * 1.05f + 1e-6f * (fabsf(fhat) + fabsf(fold));
        need = !(fhat - B >= fold);
    }
    const uint64_t bal = __ballot(need);
    const int before = (int)__popcll(bal & ((1ull << l) - 1ull));
    if (l == 0) s_n[wave] = (int)__popcll(bal);
    __syncthreads();
    if (tid == 0) s_base = atomicAdd(w.count, s_n[0] + s_n[1] + s_n[2] + s_n[3]);
    __syncthreads();
    int off = s_base + before;
    for (int q = 0; q < wave; ++q) off += s_n[q];
    if (r < p.pop) {
        w.status[r] = need ? off : -1;
        if (need) w.list[off] = r;
        w.anorm[r] = fhat;
    }
}

// Binary64 re-score of one row (the elite), in two launches.  elite_z: one
// wavefront per output n, lanes over k (rows of M read contiguously), the
// row summed by the fixed butterfly: z64[n] = (M (x - o))_n.
__global__ __launch_bounds__(64) void elite_z(Params p, GemmBufs w, const double *x) {
    const int D = p.dim, n = blockIdx.x, l = threadIdx.x;
    const double *m = w.Md + (size_t)n * D;
    double z = 0.0;
    for (int k = l; k < D; k += 64) z += m[k] * (x[k] - w.o64[k]);
    z = group_sum<64>(z);
    if (l == 0) w.z64[n] = z;
}

// elite_f: the objective from z64 (one workgroup of 1024 threads, thread i
// takes n = i, i + 1024, ...; per-wavefront butterflies, then the sixteen
// wavefront sums in order).  out[0] receives F.
__global__ __launch_bounds__(1024) void elite_f(Params p, GemmBufs w, double *out) {
    __shared__ double red[2][16];
    const int D = p.dim, wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    double s1 = 0.0, s2 = 0.0;
    for (int n = threadIdx.x; n < D; n += 1024) {
        const double z = w.z64[n];
        if (p.kind == K_RASTRIGIN) {
            s1 += z * z - 10.0 * cos(2.0 * kPi * z) + 10.0;
        } else if (p.kind == K_ACKLEY) {
            s1 += z * z;
            s2 += cos(2.0 * kPi * z);
        } else {
            s1 += z * z;
        }
    }
    s1 = group_sum<64>(s1);
    s2 = group_sum<64>(s2);
    if (l == 0) {
        red[0][wave] = s1;
        red[1][wave] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < 16; ++i) {
            a += red[0][i];
            b += red[1][i];
        }
        out[0] = p.kind == K_ACKLEY
                     ? -20.0 * exp(-0.2 * sqrt(a / (double)D)) - exp(b / (double)D) + 20.0 + kE
                     : a;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static GemmRun gemm_run(const Params &p, const GemmBufs &w, bool bf16, bool listed) {
    GemmRun g;
    g.Ab = bf16 ? w.Ab : nullptr;
    g.Yr = w.Yr;
    g.o = (const float *)p.shift;
    g.B = bf16 ? (const void *)w.Mb : (const void *)w.Mf;
    g.list = listed ? w.list : nullptr;
    g.count = w.count;
    g.rows = p.pop;
    g.D = p.dim;
    g.Dp = p.Dp;
    g.Kp = w.Kp;
    g.Np = w.Np;
    g.kind = p.kind;
    g.P1 = w.P1;
    g.P2 = w.P2;
    return g;
}

template <bool BF16>
static hipError_t launch_cand(const Params &p, const GemmBufs &w, int init, hipStream_t s) {
    const int G = lanes_for_dim(p.dim), NCH = chunks_for_dim(p.dim);
    const long long threads = (long long)p.pop * G;
    const dim3 grid((unsigned)((threads + 255) / 256)), block(256);
#define APO_CAND(GG, CC)                                                                     \
    if (G == GG && NCH == CC) {                                                              \
        if (p.np == 1)                                                                       \
            launch_k(p, gemm_cand<GG, CC, 1, BF16>, grid, block, 0, s, p, w, init);          \
        else                                                                                 \
            launch_k(p, gemm_cand<GG, CC, kMaxNp, BF16>, grid, block, 0, s, p, w, init);     \
        return hipGetLastError();                                                            \
    }
    APO_ELEM_SHAPES(APO_CAND)
#undef APO_CAND
    return hipErrorInvalidValue;
}

template <int KIND>
static hipError_t launch_gemm_t(const Params &p, const GemmRun &g, bool bf16, hipStream_t s) {
    if (bf16) {
        if (g.list) return hipErrorInvalidValue;
        const hipError_t ea = hipFuncSetAttribute((const void *)gemm_obj_bf16<KIND>,
                                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  (int)kBLdsLaunch);
        if (ea != hipSuccess) return ea;
        const int nM = (g.rows + kBM - 1) / kBM, nN = g.Np / kBN;
        launch_k(p, gemm_obj_bf16<KIND>, dim3((unsigned)(nM * nN)), dim3(kBThreads), kBLdsLaunch, s, g);
        return hipGetLastError();
    }
    const hipError_t ea = hipFuncSetAttribute((const void *)gemm_obj_f32<KIND>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize,
                                              (int)kGemmLds);
    if (ea != hipSuccess) return ea;
    const dim3 grid((unsigned)((g.Np / kGN) * ((g.rows + kGM - 1) / kGM))), block(256);
    launch_k(p, gemm_obj_f32<KIND>, grid, block, kGemmLds, s, g);
    return hipGetLastError();
}

static hipError_t launch_gemm(const Params &p, const GemmRun &g, bool bf16, hipStream_t s) {
    switch (g.kind) {
    case K_SPHERE: return launch_gemm_t<K_SPHERE>(p, g, bf16, s);
    case K_RASTRIGIN: return launch_gemm_t<K_RASTRIGIN>(p, g, bf16, s);
    case K_ACKLEY: return launch_gemm_t<K_ACKLEY>(p, g, bf16, s);
    default: return hipErrorInvalidValue;   // the GEMM form takes the rotated objectives above
    }
}

hipError_t launch_gemm_stage(const Params &p, const GemmBufs &w, int init, int stage,
                             hipStream_t s) {
    const bool bf16 = w.bf16 && !init;   // the initial fitness is taken in binary32
    const dim3 sgrid((unsigned)((p.pop + 3) / 4)), sblock(256);
    switch (stage) {
    case 0:
        return bf16 ? launch_cand<true>(p, w, init, s) : launch_cand<false>(p, w, init, s);
    case 1:
        return launch_gemm(p, gemm_run(p, w, bf16, false), bf16, s);
    case 2:
        if (!bf16) return hipSuccess;
        launch_k(p, gemm_classify, dim3((unsigned)((p.pop + 255) / 256)), sblock, 0, s, p,
                 gemm_run(p, w, true, false), w);
        return hipGetLastError();
    case 3:
        if (!bf16) return hipSuccess;
        return launch_gemm(p, gemm_run(p, w, false, true), false, s);
    case 4:
        launch_k(p, gemm_select, sgrid, sblock, 0, s, p, gemm_run(p, w, false, false), w, init,
                 bf16 ? 1 : 0);
        return hipGetLastError();
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_gemm_step(const Params &p, const GemmBufs &w, int init, hipStream_t s) {
    for (int stage = 0; stage < 5; ++stage) {
        const hipError_t e = launch_gemm_stage(p, w, init, stage, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_elite_f64(const Params &p, const GemmBufs &w, const double *x, double *out,
                            hipStream_t s) {
    hipLaunchKernelGGL(elite_z, dim3((unsigned)p.dim), dim3(64), 0, s, p, w, x);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(elite_f, dim3(1), dim3(1024), 0, s, p, w, out);
    return hipGetLastError();
}

}  // namespace apok
