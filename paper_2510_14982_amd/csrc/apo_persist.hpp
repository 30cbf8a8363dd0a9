// apo_persist.hpp -- the persistent form of a single run's iterations (tiled
// step): one cooperative launch runs n iterations of Algorithm 1's loop
// body.  Each iteration is a rank phase (every workgroup ranks its own
// block of protozoa by counting over the whole population and writes their
// places in the order), a grid barrier, the tiled step of the workgroup's
// ranks (candidates, clamp, objective on the matrix cores, selection) and a
// second grid barrier, so an iteration costs two barriers instead of two
// kernel launches and the step knows t without reading the control block.
// Results are those of the two-kernel form (same device code for the sort
// order, the draws and the step).
#pragma once
#include "apo_step.hpp"

namespace apok {

// Grid barrier number k (1, 2, ...) of a launch: every workgroup arrives
// once per barrier on a counter that is zero when the launch starts, and
// the barrier opens when the counter reaches k * gridDim.x.  The wait is
// bounded: after kSpinLimit polls (or once another workgroup has given up)
// the workgroup records the failure and returns false, and every workgroup
// leaves at its next barrier, so the launch always ends.
constexpr int kSpinLimit = 1 << 22;

__device__ __forceinline__ bool grid_sync(Ctrl *c, unsigned k) {
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();   // this workgroup's writes before its arrival
        __hip_atomic_fetch_add(&c->sync_count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned target = k * gridDim.x;
        int ok = 1, spins = 0;
        while (__hip_atomic_load(&c->sync_count, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) <
               target) {
            if (__hip_atomic_load(&c->sync_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                ++spins > kSpinLimit) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (!ok) __hip_atomic_store(&c->sync_err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();   // the other workgroups' writes before this one's reads
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Rank phase: workgroup blk ranks the protozoa with ids [blk TM, blk TM +
// TM) by counting the order keys of the whole population that precede each
// of them (ascending fitness, -0 equal to +0, NaN last, ties by id: the
// sort kernel's order), then writes perm[rank] = id, Fs[rank] = F[id] and
// whether the rank belongs to Dr of iteration t (pf of Eq. (11) and the Dr
// subset keys are drawn by the workgroup's last wavefront while the keys
// load).
template <typename T, int TM>
__device__ __forceinline__ void rank_ids_phase(const Params &p, int t, int blk) {
    constexpr int NT = 512, NW = NT / 64, J = 8;   // J keys per thread per pass
    __shared__ uint64_t s_ki[TM];
    __shared__ int32_t s_part[NW][TM];
    __shared__ uint32_t s_keys[24];
    __shared__ int32_t s_mdr;
    const T *F = (const T *)p.F;
    const int ps = p.pop, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int i0 = blk * TM;
    T fj[J];
#pragma unroll
    for (int u = 0; u < J; ++u) {
        const int j = NT * u + tid;
        fj[u] = F[j < ps ? j : ps - 1];
    }
    T fi = T(0);
    if (tid < TM) {
        const int i = i0 + tid;
        fi = F[i < ps ? i : ps - 1];
        s_ki[tid] = i < ps ? RankKey<T>::make(fi, i) : ~0ull;
    }
    if (wave == NW - 1) open_iteration(p, t, s_keys, &s_mdr);
    int32_t cnt[TM];
#pragma unroll
    for (int q = 0; q < TM; ++q) cnt[q] = 0;
    __syncthreads();
    uint64_t ki[TM];
#pragma unroll
    for (int q = 0; q < TM; ++q) ki[q] = s_ki[q];
    for (int base = 0; base < ps; base += NT * J) {
        if (base > 0) {   // further passes (ps above 4096)
#pragma unroll
            for (int u = 0; u < J; ++u) {
                const int j = base + NT * u + tid;
                fj[u] = F[j < ps ? j : ps - 1];
            }
        }
#pragma unroll
        for (int u = 0; u < J; ++u) {
            if (base + NT * u >= ps) break;   // the rest of the pass is padding
            const int j = base + NT * u + tid;
            const uint64_t kj = j < ps ? RankKey<T>::make(fj[u], j) : ~0ull;
#pragma unroll
            for (int q = 0; q < TM; ++q)
                cnt[q] += RankKey<T>::before(kj, j, ki[q], i0 + q) ? 1 : 0;
        }
    }
    // a padding key (~0) never precedes a real key; among real keys the
    // binary64 id tie-break applies to equal keys only
#pragma unroll
    for (int q = 0; q < TM; ++q) {
        const int32_t v = group_sum<64>(cnt[q]);
        if (lane == 0) s_part[wave][q] = v;
    }
    __syncthreads();
    if (tid < TM && i0 + tid < ps) {
        int rank = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) rank += s_part[w][tid];
        p.perm[rank] = i0 + tid;
        ((T *)p.Fs)[rank] = fi;
        Subset drs;   // Dr of Algorithm 1: rank r belongs iff pi(r) < |Dr|
        subset_shape(drs, (uint32_t)ps);
#pragma unroll
        for (int q = 0; q < 24; ++q) drs.k[q] = s_keys[q];
        p.drf[rank] = subset_has(drs, (uint32_t)rank, (uint32_t)s_mdr) ? 1 : 0;
    }
}

// Iterations t0 + 1 .. t0 + iters.  Needs every workgroup resident at once
// (a cooperative launch) and sync_count zero at launch.
template <typename T, int G, int NCH, int NPMAX, int TM>
__global__ __launch_bounds__(512) void step_tile_persist(Params p, int t0, int iters) {
    const int blk = (int)blockIdx.x;
    unsigned k = 0;
    bool ok = true;
    for (int n = 1; n <= iters; ++n) {
        const int t = t0 + n;
        Iter it;
        it.t = t;
        it.p_ah = p.p_ah[t];
        it.fscale = p.fscale[t];
        it.cnear = p.cnear[t];
        rank_ids_phase<T, TM>(p, t, blk);
        ok = grid_sync(p.ctrl, ++k);
        if (!ok) break;
        step_tile_body<T, G, NCH, NPMAX, TM>(p, 0, blk, &it);
        ok = grid_sync(p.ctrl, ++k);
        if (!ok) break;
    }
    if (ok && blk == 0 && threadIdx.x == 0) {   // every workgroup has passed the last barrier
        p.ctrl->t = t0 + iters;
        p.ctrl->t_next = t0 + iters;
    }
}

// One compiled shape of the persistent form.  Tiles of more than 32 rows
// (lane groups of 4 or 8 in very large populations) keep the graph form:
// the rank phase holds a counter and a key per row in registers.
template <typename T, int NPMAX, int GG, int CC, int TMM>
hipError_t persist_shape(const Params &p, int t0, int iters, hipStream_t s, bool launch,
                         int nblk, size_t lds) {
    if constexpr (TMM > 32) {
        return hipErrorInvalidValue;
    } else {
        const void *fn = (const void *)step_tile_persist<T, GG, CC, NPMAX, TMM>;
        if (lds > 65536) {
            const hipError_t ea =
                hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (ea != hipSuccess) return ea;
        }
        int dev = 0, cus = 0, per = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 512, lds);
        if (e != hipSuccess) return e;
        if ((long long)per * cus < nblk) return hipErrorCooperativeLaunchTooLarge;
        if (!launch) return hipSuccess;
        Params pa = p;
        int a_t0 = t0, a_it = iters;
        void *args[] = {(void *)&pa, (void *)&a_t0, (void *)&a_it};
        return hipLaunchCooperativeKernel(fn, dim3((unsigned)nblk), dim3(512), args, (unsigned)lds,
                                          s);
    }
}

// Launch (or, with launch == false, only check that every workgroup of the
// run fits on the device at once).  Returns hipErrorInvalidValue for a
// shape without a persistent kernel and hipErrorCooperativeLaunchTooLarge
// when the grid does not fit.
template <typename T, int NPMAX>
hipError_t launch_tile_persist_t(const Params &p, int t0, int iters, hipStream_t s, bool launch) {
    const int G = tile_lanes(p), NCH = tile_chunks(p), TMr = tile_rows(p);
    if (NCH < 0) return hipErrorInvalidValue;
    const int nblk = (p.pop + TMr - 1) / TMr;
    const size_t lds = tile_lds_bytes(p, sizeof(T) == 8);
#define APO_PERSIST(GG, CC, TMM)                                                     \
    if (G == GG && NCH == CC && TMr == TMM)                                          \
        return persist_shape<T, NPMAX, GG, CC, TMM>(p, t0, iters, s, launch, nblk, lds);
    APO_TILE_SHAPES(APO_PERSIST)
#undef APO_PERSIST
    return hipErrorInvalidValue;
}

}  // namespace apok
