// apo_kernels.hip -- gfx950 kernels of the APO population step.
//
//   rank_kernel   sort by fitness: each protozoan's rank is the number of
//                 protozoa before it in the fitness order (ties by id),
//                 counted in parallel over the whole population; then
//                 perm[rank] = id.  Also opens the iteration: draws pf
//                 (Eq. (11)) and the Dr subset keys (Algorithm 1) and
//                 flags the ranks in Dr.
//   (the step kernels themselves live in apo_step.hpp)
//   best_kernel   argmin in the fitness order and a copy of that row.
//   hist_count_kernel, hist_sum_kernel
//                 256-bin histogram of an 8-bit image (LDS copies per
//                 workgroup, then one workgroup adds the workgroups' rows).
#include "apo_step.hpp"

#include <mutex>

namespace apok {

// ---------------------------------------------------------------------------
// Rank sort.  rank(i) = #{j : (F_j, j) before (F_i, i)} in the fitness order,
// so perm[rank(i)] = i.  One workgroup of NT threads (512 for a single run,
// 256 in batches) ranks 8 protozoa.
// Each thread holds the order keys of its share of the population in
// registers (j = tid, tid + NT, ...), compares them against the 8 keys
// being ranked (read by LDS broadcast) and keeps 8 counters, which are
// summed over the workgroup by butterflies and LDS at the end.  No
// workgroup depends on another.  Each workgroup also opens the iteration
// (pf of Eq. (11), |Dr| and the Dr subset keys) and, for the ranks it
// finds, writes the fitness in rank order (Fs, which the step reads instead
// of F) and whether the rank is in Dr.  Workgroup 0 publishes the
// iteration in the control block.
// ---------------------------------------------------------------------------
constexpr int kRankPass = 4096;    // keys per pass (kRankPass / NT per thread)

template <typename T, int NT>
__device__ __forceinline__ void rank_body(const Params &p, int blk) {
    constexpr int kRankJ = kRankPass / NT, NW = NT / 64;
    __shared__ uint64_t s_ki[kRankPer];
    __shared__ int32_t part[NW][kRankPer];
    __shared__ uint32_t s_keys[24];
    __shared__ int32_t s_mdr;
    const T *F = (const T *)p.F;
    const int ps = p.pop;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int i0 = blk * kRankPer;
    // the iteration this sort opens (a vector load: the key loads below are
    // issued without waiting for it)
    const int t = __hip_atomic_load(&p.ctrl->t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;

    // The first pass's key loads and the ranked protozoa's own fitness are
    // all issued before the barrier, so the kernel waits for memory once
    // (an index past the end reads the last element and is then replaced by
    // the padding key).
    T fj[kRankJ];
#pragma unroll
    for (int u = 0; u < kRankJ; ++u) {
        const int j = NT * u + tid;
        fj[u] = F[j < ps ? j : ps - 1];
    }
    T fi = T(0);
    if (tid < kRankPer) {
        fi = F[i0 + tid < ps ? i0 + tid : ps - 1];
        const uint64_t k = RankKey<T>::make(fi, i0 + tid);
        s_ki[tid] = i0 + tid < ps ? k : ~0ull;
    }
    int32_t cnt[kRankPer];
#pragma unroll
    for (int q = 0; q < kRankPer; ++q) cnt[q] = 0;
    __syncthreads();
    uint64_t ki[kRankPer];
#pragma unroll
    for (int q = 0; q < kRankPer; ++q) ki[q] = s_ki[q];

    for (int base = 0; base < ps; base += kRankPass) {
        if (base > 0) {   // further passes (ps above 4096)
#pragma unroll
            for (int u = 0; u < kRankJ; ++u) {
                const int j = base + NT * u + tid;
                fj[u] = F[j < ps ? j : ps - 1];
            }
        }
        // the last wavefront opens the iteration while its loads are in flight
        if (base == 0 && wave == 3) open_iteration(p, t, s_keys, &s_mdr);
        uint64_t kj[kRankJ];
#pragma unroll
        for (int u = 0; u < kRankJ; ++u) {
            const int j = base + NT * u + tid;
            const uint64_t k = RankKey<T>::make(fj[u], j);
            kj[u] = j < ps ? k : ~0ull;   // ~0 sorts after all
        }
#pragma unroll
        for (int u = 0; u < kRankJ; ++u) {
            if (base + NT * u >= ps) break;   // the rest of the pass is padding
            const int j = base + NT * u + tid;
#pragma unroll
            for (int q = 0; q < kRankPer; ++q)
                cnt[q] += RankKey<T>::before(kj[u], j, ki[q], i0 + q) ? 1 : 0;
        }
    }
    // a padding key equals ~0 and never precedes a real key except another
    // padding key; real keys with id < ps are all below ~0, and the double
    // version's id tie-break only applies among equal real keys
#pragma unroll
    for (int q = 0; q < kRankPer; ++q) {
        const int32_t v = group_sum<64>(cnt[q]);
        if (lane == 0) part[wave][q] = v;
    }
    __syncthreads();
    if (tid < kRankPer && i0 + tid < ps) {
        int rank = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) rank += part[w][tid];
        p.perm[rank] = i0 + tid;
        ((T *)p.Fs)[rank] = fi;
        // Dr of Algorithm 1: rank r belongs iff pi(r) < |Dr|
        Subset drs;
        subset_shape(drs, (uint32_t)ps);
#pragma unroll
        for (int q = 0; q < 24; ++q) drs.k[q] = s_keys[q];
        p.drf[rank] = subset_has(drs, (uint32_t)rank, (uint32_t)s_mdr) ? 1 : 0;
    }
    if (blk == 0 && tid == 64) {   // publish the iteration for the step
        p.ctrl->m_dr = s_mdr;
        p.ctrl->p_ah = p.p_ah[t];
        p.ctrl->fscale = p.fscale[t];
        p.ctrl->cnear = p.cnear[t];
        p.ctrl->t_next = t;
    }
}

// The LDS form of the sort (rank_small_body) is in apo_step.hpp: the persistent
// form of small runs uses it too.

template <typename T, int NT>
__device__ __forceinline__ void rank_any(const Params &p, int blk) {
    if (p.rank_lds)
        rank_small_body<T>(p, blk);
    else
        rank_body<T, NT>(p, blk);
}

// A single run: 512 threads a workgroup (its LDS form, pop <= 256, ranks
// with the first 256).
template <typename T>
__global__ __launch_bounds__(512) void rank_kernel(Params p) {
    rank_any<T, 512>(p, (int)blockIdx.x);
}

// Several runs in one launch: workgroup b sorts block blocks[b].y of run
// blocks[b].x.
template <typename T>
__global__ __launch_bounds__(256) void rank_kernel_batch(const Params *runs, const int2 *blocks) {
    const int2 b = blocks[blockIdx.x];
    rank_any<T, 256>(runs[b.x], b.y);
}

// ---------------------------------------------------------------------------
// Best protozoan of buffer `cur`: one workgroup of 1024 threads.
// out_row[0] = fitness, out_row[1..dim] = position (as binary64).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void best_kernel(Params p, int cur, double *out_row) {
    __shared__ uint64_t sk[1024];
    __shared__ int32_t si[1024];
    const T *F = (const T *)p.F;
    uint64_t bk = ~0ull;
    int32_t bi = 0x7FFFFFFF;
    for (int i = threadIdx.x; i < p.pop; i += 1024) {
        const uint64_t k = (uint64_t)order_key(F[i]);
        if (k < bk || (k == bk && i < bi)) {
            bk = k;
            bi = i;
        }
    }
    sk[threadIdx.x] = bk;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const uint64_t k2 = sk[threadIdx.x + s];
            const int32_t i2 = si[threadIdx.x + s];
            if (k2 < sk[threadIdx.x] || (k2 == sk[threadIdx.x] && i2 < si[threadIdx.x])) {
                sk[threadIdx.x] = k2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    const int id = si[0];
    const T *row = (const T *)p.X[cur] + (size_t)id * p.Dp;
    for (int d = threadIdx.x; d < p.dim; d += 1024) out_row[1 + d] = (double)row[d];
    if (threadIdx.x == 0) {
        out_row[0] = (double)F[id];
        p.ctrl->best_id = id;
        p.ctrl->best_f = (double)F[id];
    }
}

// ---------------------------------------------------------------------------
// Histogram tables for the thresholding objectives (binary64, bins in
// order): P[g] = sum_{h<g} p_h, S[g] = sum_{h<g} p_h ln p_h,
// M1[g] = sum_{h<g} h p_h, with p_h = count_h / N.  One workgroup of 256
// threads: each loads one count and forms its bin's terms; N is the exact
// integer total; one thread then adds the terms in bin order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void hist_tables_kernel(const uint64_t *hist, double *tab) {
    __shared__ unsigned long long s_c[256];
    __shared__ double s_p[256], s_s[256], s_m[256];
    const int g = threadIdx.x;
    const unsigned long long c = hist[g];
    s_c[g] = c;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {   // exact: integers
        unsigned long long v = 0;
        if (g < h) v = s_c[g] + s_c[g + h];
        __syncthreads();
        if (g < h) s_c[g] = v;
        __syncthreads();
    }
    const double N = (double)s_c[0];
    const double pg = (double)c / N;
    s_p[g] = pg;
    s_s[g] = pg > 0.0 ? pg * log(pg) : 0.0;
    s_m[g] = (double)g * pg;
    __syncthreads();
    if (g == 0) {
        double *P = tab, *S = tab + 257, *M1 = tab + 514;
        double a = 0.0, b = 0.0, m = 0.0;
        P[0] = S[0] = M1[0] = 0.0;
        for (int q = 0; q < 256; ++q) {
            a = a + s_p[q];
            b = b + s_s[q];
            m = m + s_m[q];
            P[q + 1] = a;
            S[q + 1] = b;
            M1[q + 1] = m;
        }
    }
}

__global__ void zero_u32_kernel(uint32_t *a, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0u;
}

// 8-bit histogram, two kernels.  hist_count: each workgroup of 512 threads
// counts its share of the image into LDS: sixteen copies chosen by
// lane % 16, so lanes that meet the same grey level (frequent in images
// made of uniform regions) mostly hit different copies; copies are 257
// words apart so equal levels of different copies sit in different banks.
// Bytes before the first and after the last 16-byte boundary are counted
// one by one; the rest is read as 16-byte vectors, four per thread in
// flight.  The 256 counts go to the workgroup's row of the partial table.
// Workgroup 0 of the counting pass also clears the 64-bit output.
// hist_sum: workgroup j (of ceil(rows / 32)) adds rows j, j + grid, ...,
// one thread per bin with its 32 loads in flight together, and adds that
// to the output with one 64-bit atomic per bin.  The kernel boundary
// between the two publishes the rows and the cleared output:
// no workgroup of the counting pass waits on another or fences its writes
// (a device-scope release writes back the whole L2 of its XCD, and one per
// workgroup costs more than the counting).  Integer sums: exact in any
// order.
constexpr int kHistCopies = 16;
constexpr int kHistStride = 257;
constexpr int kHistThreads = 512;
constexpr int kHistUnroll = 4;
constexpr int kHistSumBatch = 32;   // rows per thread of the sum, loaded together

struct HistScratch {
    uint32_t *rows;                // [kHistBlocks][256]
    unsigned long long *out;       // [256]
};

__device__ __forceinline__ void hist_add16(uint32_t *mine, const uint4 &q) {
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int b = 0; b < 4; ++b) atomicAdd(&mine[(w[j] >> (8 * b)) & 0xFFu], 1u);
    }
}

__global__ __launch_bounds__(kHistThreads) void hist_count_kernel(const uint8_t *img, uint64_t n,
                                                                  uint32_t *rows,
                                                                  unsigned long long *out) {
    __shared__ uint32_t h[kHistCopies * kHistStride];
    if (blockIdx.x == 0 && threadIdx.x < 256) out[threadIdx.x] = 0ull;
    uint32_t *mine = h + (threadIdx.x & (kHistCopies - 1)) * kHistStride;
    for (int b = threadIdx.x; b < kHistCopies * kHistStride; b += kHistThreads) h[b] = 0u;
    __syncthreads();
    uint64_t head = (16u - ((uintptr_t)img & 15u)) & 15u;
    if (head > n) head = n;
    const uint64_t nvec = (n - head) / 16;
    const uint64_t tid = (uint64_t)blockIdx.x * kHistThreads + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * kHistThreads;
    if (tid < head) atomicAdd(&mine[img[tid]], 1u);
    const uint4 *v = (const uint4 *)(img + head);
    for (uint64_t i0 = tid; i0 < nvec; i0 += kHistUnroll * stride) {
        uint4 q[kHistUnroll];
#pragma unroll
        for (int u = 0; u < kHistUnroll; ++u) {
            const uint64_t i = i0 + (uint64_t)u * stride;
            q[u] = i < nvec ? v[i] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < kHistUnroll; ++u)
            if (i0 + (uint64_t)u * stride < nvec) hist_add16(mine, q[u]);
    }
    for (uint64_t i = head + nvec * 16 + tid; i < n; i += stride) atomicAdd(&mine[img[i]], 1u);
    __syncthreads();
    const int b = threadIdx.x;   // bins: the first 256 threads
    if (b < 256) {
        uint32_t s = 0;
#pragma unroll
        for (int c = 0; c < kHistCopies; ++c) s += h[c * kHistStride + b];
        rows[(size_t)blockIdx.x * 256 + b] = s;
    }
}

__global__ __launch_bounds__(256) void hist_sum_kernel(const uint32_t *rows, int nb,
                                                       unsigned long long *out) {
    const int bin = threadIdx.x;
    uint32_t v[kHistSumBatch];
#pragma unroll
    for (int u = 0; u < kHistSumBatch; ++u) {
        const int r = (int)blockIdx.x + (int)gridDim.x * u;
        v[u] = r < nb ? rows[(size_t)r * 256 + bin] : 0u;
    }
    unsigned long long t = 0;
#pragma unroll
    for (int u = 0; u < kHistSumBatch; ++u) t += v[u];
    atomicAdd(&out[bin], t);
}

// ---------------------------------------------------------------------------
// Host-side launch selection.
// ---------------------------------------------------------------------------

hipError_t launch_elem_f32(const Params &p, int init, hipStream_t s);
hipError_t launch_elem_f64(const Params &p, int init, hipStream_t s);
hipError_t launch_tile_f32(const Params &p, int init, hipStream_t s);
hipError_t launch_tile_f64(const Params &p, int init, hipStream_t s);
hipError_t launch_elem_batch_f32(const Params &proto, const BatchLaunch &b, hipStream_t s);
hipError_t launch_elem_batch_f64(const Params &proto, const BatchLaunch &b, hipStream_t s);
hipError_t launch_tile_batch_f32(const Params &proto, const BatchLaunch &b, hipStream_t s);
hipError_t launch_tile_batch_f64(const Params &proto, const BatchLaunch &b, hipStream_t s);

static hipError_t launch_step_any(const Params &p, bool fp64, int init, hipStream_t s) {
    if (p.gemm) return launch_gemm_step(p, p.gb, init, s);
    const bool tile = p.rotated || p.kind == K_KAPUR || p.kind == K_OTSU;
    if (tile) return fp64 ? launch_tile_f64(p, init, s) : launch_tile_f32(p, init, s);
    return fp64 ? launch_elem_f64(p, init, s) : launch_elem_f32(p, init, s);
}

hipError_t launch_persist_f32(const Params &p, int t0, int n, hipStream_t s);
hipError_t launch_persist_f64(const Params &p, int t0, int n, hipStream_t s);
hipError_t launch_tile_persist_f32(const Params &p, int t0, int n, hipStream_t s);
hipError_t launch_tile_persist_f64(const Params &p, int t0, int n, hipStream_t s);

hipError_t launch_persist(const Params &p, bool fp64, int t0, int n, hipStream_t s) {
    if (tile_form(p))
        return fp64 ? launch_tile_persist_f64(p, t0, n, s) : launch_tile_persist_f32(p, t0, n, s);
    return fp64 ? launch_persist_f64(p, t0, n, s) : launch_persist_f32(p, t0, n, s);
}

hipError_t launch_init(const Params &p, bool fp64, hipStream_t s) {
    return launch_step_any(p, fp64, 1, s);
}

hipError_t launch_step(const Params &p, bool fp64, hipStream_t s) {
    return launch_step_any(p, fp64, 0, s);
}

hipError_t launch_rank(const Params &p, bool fp64, hipStream_t s) {
    const dim3 grid((unsigned)rank_blocks(p)), block(512);
    if (fp64)
        launch_k(p, rank_kernel<double>, grid, block, 0, s, p);
    else
        launch_k(p, rank_kernel<float>, grid, block, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_rank_batch(const BatchLaunch &b, bool fp64, hipStream_t s) {
    const dim3 grid((unsigned)b.nblocks), block(256);
    if (fp64)
        hipLaunchKernelGGL(rank_kernel_batch<double>, grid, block, 0, s, b.runs, b.blocks);
    else
        hipLaunchKernelGGL(rank_kernel_batch<float>, grid, block, 0, s, b.runs, b.blocks);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *a, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, n);
    return hipGetLastError();
}


hipError_t launch_step_batch(const Params &proto, bool fp64, const BatchLaunch &b, hipStream_t s) {
    if (tile_form(proto))
        return fp64 ? launch_tile_batch_f64(proto, b, s) : launch_tile_batch_f32(proto, b, s);
    return fp64 ? launch_elem_batch_f64(proto, b, s) : launch_elem_batch_f32(proto, b, s);
}





hipError_t launch_best(const Params &p, bool fp64, int cur, double *out_row, hipStream_t s) {
    if (fp64)
        hipLaunchKernelGGL(best_kernel<double>, dim3(1), dim3(1024), 0, s, p, cur, out_row);
    else
        hipLaunchKernelGGL(best_kernel<float>, dim3(1), dim3(1024), 0, s, p, cur, out_row);
    return hipGetLastError();
}

hipError_t launch_hist_tables(const Params &p, const uint64_t *d_hist, hipStream_t s) {
    hipLaunchKernelGGL(hist_tables_kernel, dim3(1), dim3(256), 0, s, d_hist, (double *)p.htab);
    return hipGetLastError();
}

// Scratch layout: the partial rows, then the 256 uint64 counts.
static HistScratch hist_scratch(void *scratch) {
    HistScratch sc;
    sc.rows = (uint32_t *)scratch;
    sc.out = (unsigned long long *)((unsigned char *)scratch + histogram_out_offset());
    return sc;
}

size_t histogram_scratch_bytes() { return kHistScratchBytes; }

static int histogram_blocks(uint64_t n) {
    const uint64_t per = (uint64_t)kHistThreads * kHistUnroll * 16;   // bytes per workgroup pass
    uint64_t blocks = (n + per - 1) / per;
    if (blocks < 1) blocks = 1;
    if (blocks > (uint64_t)kHistBlocks) blocks = kHistBlocks;
    return (int)blocks;
}

static hipError_t launch_histogram_sc(const uint8_t *img, uint64_t n, const HistScratch &sc,
                                      hipStream_t s) {
    const int nb = histogram_blocks(n);
    hipLaunchKernelGGL(hist_count_kernel, dim3((unsigned)nb), dim3(kHistThreads), 0, s, img, n,
                       sc.rows, sc.out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int groups = (nb + kHistSumBatch - 1) / kHistSumBatch;
    hipLaunchKernelGGL(hist_sum_kernel, dim3((unsigned)groups), dim3(256), 0, s,
                       (const uint32_t *)sc.rows, nb, sc.out);
    return hipGetLastError();
}

hipError_t launch_histogram(const uint8_t *img, uint64_t n, void *scratch, hipStream_t s) {
    return launch_histogram_sc(img, n, hist_scratch(scratch), s);
}

// The histogram's scratch for callers that cannot allocate: one file-scope
// array per device, held until the process ends.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol): the device address of each GPU's copy is looked up once, with
// that GPU current, and kept per device.  Every call on a GPU uses that
// GPU's copy, so calls that overlap on one GPU race.
__device__ __align__(256) unsigned char scratch[kHistScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static hipError_t scratch_of_current_device(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_histogram_noalloc(const uint8_t *img, uint64_t n, unsigned long long *d_out,
                                    hipStream_t s) {
    void *ptr = nullptr;
    const hipError_t e = scratch_of_current_device(&ptr);
    if (e != hipSuccess) return e;
    HistScratch sc = hist_scratch(ptr);
    sc.out = d_out;   // the counts go straight to the caller's buffer
    return launch_histogram_sc(img, n, sc, s);
}

}  // namespace apok
