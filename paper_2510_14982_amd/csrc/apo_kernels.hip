// apo_kernels.hip -- gfx950 kernels of the APO population step.
//
//   rank_kernel   sort by fitness: each protozoan's rank is the number of
//                 protozoa before it in the fitness order (ties by id),
//                 counted in parallel over the whole population; then
//                 perm[rank] = id.  Also opens the iteration: draws pf
//                 (Eq. (11)) and the Dr subset keys (Algorithm 1).
//   (the step kernels themselves live in apo_step.hpp)
//   best_kernel   argmin in the fitness order and a copy of that row.
//   hist_kernel   256-bin histogram of an 8-bit image, per-wave LDS copies.
#include "apo_step.hpp"

namespace apok {

// ---------------------------------------------------------------------------
// Rank sort.  grid = ceil(pop / 64) workgroups of 1024 threads; each
// workgroup ranks 64 protozoa (one per lane) and its 16 wavefronts split
// the comparisons over the population.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool key_before(uint64_t kj, int j, uint64_t ki, int i) {
    return kj < ki || (kj == ki && j < i);
}

template <typename T>
__global__ __launch_bounds__(1024) void rank_kernel(Params p) {
    __shared__ int32_t cnt[16][64];
    const int tcur = p.ctrl->t;
    const T *F = (const T *)p.F[tcur & 1];
    const int ps = p.pop;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const Stream rng = stream_of(p);
        const int t = tcur + 1;
        const Words w0 = rng.block(TAG_ITER, 0, 0, (uint32_t)t);
        const double pf = p.pf_max * uniform<double>(w0.w[0]);            // Eq. (11)
        p.ctrl->m_dr = (int32_t)ceil((double)ps * pf);                    // |Dr|
        const Words b1 = rng.block(TAG_ITER, 1, 0, (uint32_t)t);
        const Words b2 = rng.block(TAG_ITER, 2, 0, (uint32_t)t);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            p.ctrl->dr_keys[i] = b1.w[i];
            p.ctrl->dr_keys[4 + i] = b2.w[i];
        }
        p.ctrl->t_next = t;
    }

    const int i = blockIdx.x * 64 + lane;
    const uint64_t ki = i < ps ? (uint64_t)order_key(F[i]) : ~0ull;
    int32_t c = 0;
    const int nblk = (ps + 63) / 64;
    for (int b = wave; b < nblk; b += 16) {
        const int jl = b * 64 + lane;
        const uint64_t kl = jl < ps ? (uint64_t)order_key(F[jl]) : ~0ull;
        const int jmax = ps - b * 64 < 64 ? ps - b * 64 : 64;
        const uint32_t klo = (uint32_t)kl, khi = (uint32_t)(kl >> 32);
        for (int s = 0; s < jmax; ++s) {
            const uint32_t lo = __builtin_amdgcn_readlane(klo, s);
            const uint32_t hi = __builtin_amdgcn_readlane(khi, s);
            const uint64_t kj = ((uint64_t)hi << 32) | lo;
            c += key_before(kj, b * 64 + s, ki, i) ? 1 : 0;
        }
    }
    cnt[wave][lane] = c;
    __syncthreads();
    if (wave == 0 && i < ps) {
        int32_t rank = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) rank += cnt[w][lane];
        p.perm[rank] = i;
    }
}

// ---------------------------------------------------------------------------
// Best protozoan of buffer `cur`: one workgroup of 1024 threads.
// out_row[0] = fitness, out_row[1..dim] = position (as binary64).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void best_kernel(Params p, int cur, double *out_row) {
    __shared__ uint64_t sk[1024];
    __shared__ int32_t si[1024];
    const T *F = (const T *)p.F[cur];
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
// Histogram tables for the thresholding objectives (one thread, binary64,
// bins in order): P[g] = sum_{h<g} p_h, S[g] = sum_{h<g} p_h ln p_h,
// M1[g] = sum_{h<g} h p_h, with p_h = count_h / N.
// ---------------------------------------------------------------------------
__global__ void hist_tables_kernel(const uint64_t *hist, double *tab) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double N = 0.0;
    for (int g = 0; g < 256; ++g) N += (double)hist[g];
    double *P = tab, *S = tab + 257, *M1 = tab + 514;
    P[0] = S[0] = M1[0] = 0.0;
    for (int g = 0; g < 256; ++g) {
        const double pg = (double)hist[g] / N;
        P[g + 1] = P[g] + pg;
        S[g + 1] = S[g] + (pg > 0.0 ? pg * log(pg) : 0.0);
        M1[g + 1] = M1[g] + (double)g * pg;
    }
}

__global__ void zero_u32_kernel(uint32_t *a, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0u;
}

// 8-bit histogram: per-wavefront LDS copies absorb runs of equal grey
// levels; each workgroup merges its copies into the output once.  The bytes
// before the first 16-byte boundary and after the last one are counted one
// by one; the rest is read as 16-byte vectors.
__global__ __launch_bounds__(256) void hist_kernel(const uint8_t *img, uint64_t n, uint32_t *hist) {
    __shared__ uint32_t h[4][256];
    const int wave = threadIdx.x >> 6;
    for (int b = threadIdx.x; b < 4 * 256; b += 256) (&h[0][0])[b] = 0u;
    __syncthreads();
    uint64_t head = (16u - ((uintptr_t)img & 15u)) & 15u;
    if (head > n) head = n;
    const uint64_t nvec = (n - head) / 16;
    const uint64_t tid = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    if (tid < head) atomicAdd(&h[wave][img[tid]], 1u);
    const uint4 *v = (const uint4 *)(img + head);
    for (uint64_t i = tid; i < nvec; i += stride) {
        const uint4 q = v[i];
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
            for (int b = 0; b < 4; ++b) atomicAdd(&h[wave][(w[j] >> (8 * b)) & 0xFFu], 1u);
        }
    }
    for (uint64_t i = head + nvec * 16 + tid; i < n; i += stride) atomicAdd(&h[wave][img[i]], 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < 256; b += 256) {
        const uint32_t s = h[0][b] + h[1][b] + h[2][b] + h[3][b];
        if (s) atomicAdd(&hist[b], s);
    }
}

// ---------------------------------------------------------------------------
// Host-side launch selection.
// ---------------------------------------------------------------------------
int lanes_for_dim(int dim) {
    const int need = (dim + 3) / 4;
    int g = 4;
    while (g < need && g < 64) g <<= 1;
    return g;
}

int chunks_for_dim(int dim) {
    const int g = lanes_for_dim(dim);
    const int c = (dim + 4 * g - 1) / (4 * g);
    return c <= 1 ? 1 : c <= 2 ? 2 : c <= 4 ? 4 : -1;
}

hipError_t launch_elem_f32(const Params &p, int init, hipStream_t s);
hipError_t launch_elem_f64(const Params &p, int init, hipStream_t s);
hipError_t launch_tile_f32(const Params &p, int init, hipStream_t s);
hipError_t launch_tile_f64(const Params &p, int init, hipStream_t s);

static hipError_t launch_step_any(const Params &p, bool fp64, int init, hipStream_t s) {
    const bool tile = p.rotated || p.kind == K_KAPUR || p.kind == K_OTSU;
    if (tile) return fp64 ? launch_tile_f64(p, init, s) : launch_tile_f32(p, init, s);
    return fp64 ? launch_elem_f64(p, init, s) : launch_elem_f32(p, init, s);
}

hipError_t launch_init(const Params &p, bool fp64, hipStream_t s) {
    return launch_step_any(p, fp64, 1, s);
}

hipError_t launch_step(const Params &p, bool fp64, hipStream_t s) {
    return launch_step_any(p, fp64, 0, s);
}

hipError_t launch_rank(const Params &p, bool fp64, hipStream_t s) {
    const dim3 grid((p.pop + 63) / 64), block(1024);
    if (fp64)
        hipLaunchKernelGGL(rank_kernel<double>, grid, block, 0, s, p);
    else
        hipLaunchKernelGGL(rank_kernel<float>, grid, block, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_best(const Params &p, bool fp64, int cur, double *out_row, hipStream_t s) {
    if (fp64)
        hipLaunchKernelGGL(best_kernel<double>, dim3(1), dim3(1024), 0, s, p, cur, out_row);
    else
        hipLaunchKernelGGL(best_kernel<float>, dim3(1), dim3(1024), 0, s, p, cur, out_row);
    return hipGetLastError();
}

hipError_t launch_hist_tables(const Params &p, const uint64_t *d_hist, hipStream_t s) {
    hipLaunchKernelGGL(hist_tables_kernel, dim3(1), dim3(64), 0, s, d_hist, (double *)p.htab);
    return hipGetLastError();
}

hipError_t launch_histogram(const uint8_t *img, uint64_t n, uint32_t *hist, hipStream_t s) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(256), 0, s, hist, 256);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n == 0) return e;
    uint64_t blocks = (n / 16 + 256 * 4 - 1) / (256 * 4);
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(hist_kernel, dim3((unsigned)blocks), dim3(256), 0, s, img, n, hist);
    return hipGetLastError();
}

}  // namespace apok
