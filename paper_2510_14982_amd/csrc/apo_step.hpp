// apo_step.hpp -- the fused step kernels (candidate construction, clamp,
// objective, greedy selection) as templates.  Instantiated per precision
// and kernel family in apo_step_*.hip so the builds run in parallel.
#pragma once
#include <math.h>

#include "apo_device.hpp"
#include "apo_internal.h"

namespace apok {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr double kPi = 3.14159265358979323846;
constexpr double kE = 2.71828182845904523536;
constexpr double kEps = 2.220446049250313e-16;   // 2^-52, the eps of Eqs. (7), (10)

template <typename T>
struct V4;
template <>
struct V4<float> {
    typedef float __attribute__((ext_vector_type(4))) type;
};
template <>
struct V4<double> {
    typedef double __attribute__((ext_vector_type(4))) type;
};

template <typename T>
__device__ __forceinline__ void load4(const T *p, T v[4]) {
    const typename V4<T>::type q = *reinterpret_cast<const typename V4<T>::type *>(p);
    v[0] = q[0]; v[1] = q[1]; v[2] = q[2]; v[3] = q[3];
}

template <typename T>
__device__ __forceinline__ void store4(T *p, const T v[4]) {
    typename V4<T>::type q;
    q[0] = v[0]; q[1] = v[1]; q[2] = v[2]; q[3] = v[3];
    *reinterpret_cast<typename V4<T>::type *>(p) = q;
}

// cos(2 pi z): binary64 follows the textbook expression; binary32 reduces z
// exactly to [-1/2, 1/2] and uses the hardware cosine, which takes its
// argument in revolutions (measured within 1.3e-7 of binary64 cos there).
__device__ __forceinline__ double cos2pi(double z) { return cos(2.0 * kPi * z); }
__device__ __forceinline__ float cos2pi(float z) {
    return __builtin_amdgcn_cosf(z - rintf(z));
}

__device__ __forceinline__ Stream stream_of(const Params &p) {
    Stream s;
    s.k0 = p.seed_lo;
    s.k1 = p.seed_hi;
    s.run = p.run;
    return s;
}

// The open iteration's number and schedule scalars (Eqs. (4), (9), (12)),
// published by the sort in the control block; read once at kernel entry
// with vector loads (relaxed atomics), whose in-order counters let the
// loads that do not depend on t issue before the first wait on t.
struct Iter {
    int t;
    double p_ah, fscale, cnear;
};

__device__ __forceinline__ Iter load_iter(const Params &p, int init) {
    Iter it;
    if (init) {
        it.t = 0;
        it.p_ah = it.fscale = it.cnear = 0.0;
    } else {
        Ctrl *c = p.ctrl;
        it.t = __hip_atomic_load(&c->t_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        it.p_ah = __hip_atomic_load(&c->p_ah, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        it.fscale = __hip_atomic_load(&c->fscale, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        it.cnear = __hip_atomic_load(&c->cnear, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return it;
}

// ---------------------------------------------------------------------------
// Order keys of the sort and the opening of an iteration (shared by the sort
// kernel and the step).
// ---------------------------------------------------------------------------
template <typename T>
struct RankKey;
template <>
struct RankKey<float> {   // 32-bit order key with the id below it: unique
    __device__ static uint64_t make(float f, int j) {
        return ((uint64_t)order_key(f) << 32) | (uint32_t)j;
    }
    __device__ static bool before(uint64_t kj, int, uint64_t ki, int) { return kj < ki; }
};
template <>
struct RankKey<double> {  // 64-bit order key; equal keys fall back to the ids
    __device__ static uint64_t make(double f, int) { return order_key(f); }
    __device__ static bool before(uint64_t kj, int j, uint64_t ki, int i) {
        return kj < ki || (kj == ki && j < i);
    }
};

// Opens iteration t (one wavefront, no memory reads): pf of Eq. (11), |Dr|
// and the Dr subset key schedule into LDS.  Lanes 0-2 draw the three Philox
// blocks; lane 0 finishes.
__device__ __forceinline__ void open_iteration(const Params &p, int t, uint32_t *s_keys,
                                               int32_t *s_mdr) {
    const int lane = threadIdx.x & 63;
    const Stream rng = stream_of(p);
    const Words w = rng.block(TAG_ITER, (uint32_t)(lane < 3 ? lane : 0), 0, (uint32_t)t);
    const uint32_t u_pf = __shfl(w.w[0], 0, 64);
    uint32_t k8[8];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        k8[e] = __shfl(w.w[e], 1, 64);
        k8[4 + e] = __shfl(w.w[e], 2, 64);
    }
    if (lane == 0) {
        const int ps = p.pop;
        const double pf = p.pf_max * uniform<double>(u_pf);             // Eq. (11)
        const int32_t m_dr = (int32_t)ceil((double)ps * pf);              // |Dr|
        Subset drs;
        subset_init(drs, k8, (uint32_t)ps);
#pragma unroll
        for (int q = 0; q < 24; ++q) s_keys[q] = drs.k[q];
        *s_mdr = m_dr;
    }
}

// LDS form (ps <= kRankLdsMax): the run's keys are staged in LDS and each
// of the workgroup's 256 threads counts, for one protozoan, the keys that
// precede its own (broadcast reads), so a workgroup ranks 256 protozoa.
// Fewest workgroups: the form of small runs and of batches; a single run
// of a few hundred or more protozoa prefers the register form's many
// workgroups (lower latency).
constexpr int kRankSmall = kRankLdsMax;

template <typename T>
__device__ __forceinline__ void rank_small_body(const Params &p, int blk, int t_open = 0,
                                                bool publish = true) {
    __shared__ uint64_t s_k[kRankSmall];
    __shared__ uint32_t s_keys[24];
    __shared__ int32_t s_mdr;
    const T *F = (const T *)p.F;
    const int ps = p.pop;
    const int tid = threadIdx.x, wave = tid >> 6;
    // the iteration this sort opens: the one after the last completed, or
    // t_open when the caller runs the iterations itself (persistent form)
    const int t = t_open > 0 ? t_open
                             : __hip_atomic_load(&p.ctrl->t, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT) + 1;
    T f[kRankSmall / 256];
#pragma unroll
    for (int u = 0; u < kRankSmall / 256; ++u) {
        const int j = tid + 256 * u;
        f[u] = F[j < ps ? j : ps - 1];
    }
    if (wave == 3) open_iteration(p, t, s_keys, &s_mdr);
#pragma unroll
    for (int u = 0; u < kRankSmall / 256; ++u) {
        const int j = tid + 256 * u;
        if (j < ps && tid < 256) s_k[j] = RankKey<T>::make(f[u], j);
    }
    __syncthreads();
    // threads past 256 (workgroups of 512) take no part in the ranking
    const int i = blk * 256 + tid;
    if (i < ps && tid < 256) {
        const uint64_t ki = s_k[i];
        int rank = 0;
        for (int j = 0; j < ps; ++j) rank += RankKey<T>::before(s_k[j], j, ki, i) ? 1 : 0;
        p.perm[rank] = i;
        ((T *)p.Fs)[rank] = F[i];
        Subset drs;
        subset_shape(drs, (uint32_t)ps);
#pragma unroll
        for (int q = 0; q < 24; ++q) drs.k[q] = s_keys[q];
        p.drf[rank] = subset_has(drs, (uint32_t)rank, (uint32_t)s_mdr) ? 1 : 0;
    }
    if (publish && blk == 0 && tid == 64) {   // publish the iteration for the step
        p.ctrl->m_dr = s_mdr;
        p.ctrl->p_ah = p.p_ah[t];
        p.ctrl->fscale = p.fscale[t];
        p.ctrl->cnear = p.cnear[t];
        p.ctrl->t_next = t;
    }
}

// ---------------------------------------------------------------------------
// Per-protozoan plan of one iteration: which operation, its mask, scalars
// and neighbours.  Every lane of the protozoan's group computes the same
// plan (the group shares a wavefront, so this costs no extra issue slots).
// ---------------------------------------------------------------------------
template <typename T, int NPMAX>
struct Plan {
    int32_t op, id, r;
    uint32_t m;        // mask size: ceil(D i / ps) (Eq. (5)), ceil(D rand) (Eq. (3)), D
    Subset mask;
    const uint32_t *mw;   // the group's LDS bitmask of the mask (M_f or M_r)
    T fac;             // f of Eq. (4)
    T srep;            // +-rand of Eq. (2)
    T sgn;             // +- of Eq. (9)
    T cn;              // 1 - iter / iter_max of Eq. (9)
    T fold;            // fitness of the row
    int32_t idj;       // X_j of Eq. (6)
    int32_t idm[NPMAX], idp[NPMAX];   // (k-, k+) of Eq. (6) or (i-k, i+k) of Eq. (8)
    T w[NPMAX];        // Eq. (7) / Eq. (10)
};

template <typename T>
__device__ __forceinline__ T weight(T fa, T fb) {
    return exp(-fabs(fa / (fb + T(kEps))));
}

// The protozoan's draws and every load that depends only on them, issued
// before the decisions so they overlap the decision arithmetic: its id and
// old fitness, and the ids / fitness of the first neighbour pair under both
// foraging modes (k-, k+ and j of Eq. (6); i-1, i+1 of Eq. (8)); only the
// decided mode's rows are loaded afterwards.
template <typename T>
struct Draws {
    Words s0, k1, k2, q3;
    double p_dr;
    bool in_dr;                    // rank in Dr (flagged by the sort)
    int32_t idj, ida[2], idb[2];   // [0] autotroph pair, [1] heterotroph pair
    T fa[2], fb[2];
};

// `lane0` is the wavefront lane of the group's first lane; the group has at
// least four lanes, and its lanes 0..3 each draw one of the rank's blocks
// 0..3, which are then exchanged across the group.
template <typename T, int NPMAX>
__device__ __forceinline__ void plan_draws(const Params &p, int r, int t, int lane0, int lane,
                                           Plan<T, NPMAX> &c, Draws<T> &d) {
    const Stream rng = stream_of(p);
    const int ps = p.pop;
    const T *Fs = (const T *)p.Fs;   // fitness by rank, written by the sort
    c.r = r;
    c.id = p.perm[r];
    c.fold = Fs[r];
    d.p_dr = p.p_dr[r];
    d.in_dr = p.drf[r] != 0;
    const Words mine = rng.block(TAG_RANK, (uint32_t)(lane & 3), (uint32_t)r, (uint32_t)t);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        d.s0.w[e] = __shfl(mine.w[e], lane0 + 0, 64);
        d.k1.w[e] = __shfl(mine.w[e], lane0 + 1, 64);
        d.k2.w[e] = __shfl(mine.w[e], lane0 + 2, 64);
        d.q3.w[e] = __shfl(mine.w[e], lane0 + 3, 64);
    }
    // words 1, 2, 3 of the sequence at block 3: j, k-_1, k+_1
    const int j = (int)bounded(d.q3.w[1], (uint32_t)ps);
    const int km = r == 0 ? r : (int)bounded(d.q3.w[2], (uint32_t)r);
    const int kp = r == ps - 1 ? r : r + 1 + (int)bounded(d.q3.w[3], (uint32_t)(ps - 1 - r));
    const int a = r - 1 < 0 ? 0 : r - 1;
    const int b = r + 1 > ps - 1 ? ps - 1 : r + 1;
    d.idj = p.perm[j];
    d.ida[0] = p.perm[km];
    d.idb[0] = p.perm[kp];
    d.ida[1] = p.perm[a];
    d.idb[1] = p.perm[b];
    d.fa[0] = Fs[km];
    d.fb[0] = Fs[kp];
    d.fa[1] = Fs[a];
    d.fb[1] = Fs[b];
}

// With one protozoan per wavefront its draws are wavefront-uniform: move
// them to scalar registers (frees vector registers for the rows in flight).
template <int G, typename T>
__device__ __forceinline__ void uniform_draws(Draws<T> &d) {
    if (G == 64) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            d.s0.w[e] = __builtin_amdgcn_readfirstlane(d.s0.w[e]);
            d.k1.w[e] = __builtin_amdgcn_readfirstlane(d.k1.w[e]);
            d.k2.w[e] = __builtin_amdgcn_readfirstlane(d.k2.w[e]);
            d.q3.w[e] = __builtin_amdgcn_readfirstlane(d.q3.w[e]);
        }
    }
}

// The decisions of Algorithm 1 for rank r that need only the draws: Dr
// membership, the operation (Eqs. (12), (13)), the mask size and keys and
// the scalars.  The neighbour pairs follow in plan_pairs, once the loaded
// ids and fitness have arrived.
template <typename T, int NPMAX>
__device__ __forceinline__ void plan_decide(const Params &p, int r, const Iter &it,
                                            const Draws<T> &d, Plan<T, NPMAX> &c) {
    const int ps = p.pop, D = p.dim;
    c.fac = T(0); c.srep = T(0); c.cn = T(it.cnear); c.idj = 0;
    const uint32_t keys[8] = {d.k1.w[0], d.k1.w[1], d.k1.w[2], d.k1.w[3],
                              d.k2.w[0], d.k2.w[1], d.k2.w[2], d.k2.w[3]};
    subset_init(c.mask, keys, (uint32_t)D);
    const double u_op = uniform<double>(d.s0.w[0]);
    const double u_f = uniform<double>(d.s0.w[1]);
    const double u_rep = uniform<double>(d.s0.w[2]);
    const double sgn = uniform<double>(d.s0.w[3]) < 0.5 ? 1.0 : -1.0;
    c.sgn = T(sgn);

#pragma unroll
    for (int k = 0; k < NPMAX; ++k) {
        c.idm[k] = c.idp[k] = 0;
        c.w[k] = T(0);
    }
    if (d.in_dr) {
        if (d.p_dr > u_op) {                          // Eq. (13) -> dormancy
            c.op = OP_DORMANCY;
            c.m = (uint32_t)D;
        } else {                                      // reproduction, |M_r| = ceil(D rand)
            c.op = OP_REPRODUCTION;
            const uint64_t k = d.q3.w[0] >> 9;
            c.m = (uint32_t)(((uint64_t)D * (2ull * k + 1ull) + (1ull << 24) - 1ull) >> 24);
            c.srep = T(sgn * u_rep);
        }
        return;
    }
    c.fac = T(u_f * it.fscale);
    // ceil(D (r + 1) / ps) in 32 bits: D <= 1024 and ps <= 65536
    c.m = ((uint32_t)D * (uint32_t)(r + 1) + (uint32_t)ps - 1u) / (uint32_t)ps;
    c.op = it.p_ah > u_op ? OP_AUTOTROPH : OP_HETEROTROPH;   // Eq. (12)
}

// The decided operation's first neighbour ids (no memory reads): X_j and the
// first pair of Eq. (6) for an autotroph, of Eq. (8) for a heterotroph.
template <typename T, int NPMAX>
__device__ __forceinline__ void plan_pick(const Draws<T> &d, Plan<T, NPMAX> &c) {
    if (c.op < OP_AUTOTROPH) return;
    const bool autotroph = c.op == OP_AUTOTROPH;
    c.idj = d.idj;
    c.idm[0] = autotroph ? d.ida[0] : d.ida[1];
    c.idp[0] = autotroph ? d.idb[0] : d.idb[1];
}

// Neighbour ids and weights of a foraging protozoan: X_j and the pairs of
// Eq. (6) (autotroph) or Eq. (8) (heterotroph), weights of Eqs. (7), (10).
template <typename T, int NPMAX>
__device__ __forceinline__ void plan_pairs(const Params &p, int r, int t, const Draws<T> &d,
                                           Plan<T, NPMAX> &c) {
    if (c.op < OP_AUTOTROPH) return;
    const Stream rng = stream_of(p);
    const int ps = p.pop;
    const T *Fs = (const T *)p.Fs;
    const bool autotroph = c.op == OP_AUTOTROPH;
    c.idj = d.idj;
    c.idm[0] = autotroph ? d.ida[0] : d.ida[1];
    c.idp[0] = autotroph ? d.idb[0] : d.idb[1];
    c.w[0] = weight<T>(autotroph ? d.fa[0] : d.fa[1],
                       autotroph ? d.fb[0] : d.fb[1]);  // Eq. (7) / Eq. (10)
#pragma unroll
    for (int k = 1; k < NPMAX; ++k) {
        if (k < p.np) {
            int ra, rb;
            if (autotroph) {
                // words 2k+2 (k-) and 2k+3 (k+) of the sequence starting at block 3
                const Words bw = rng.block(TAG_RANK, 3 + (uint32_t)(2 * k + 2) / 4, (uint32_t)r,
                                           (uint32_t)t);
                const uint32_t wm = bw.w[(2 * k + 2) & 3], wp = bw.w[(2 * k + 3) & 3];
                ra = r == 0 ? r : (int)bounded(wm, (uint32_t)r);
                rb = r == ps - 1 ? r : r + 1 + (int)bounded(wp, (uint32_t)(ps - 1 - r));
            } else {                                  // i - k and i + k held in [1, ps]
                ra = r - (k + 1) < 0 ? 0 : r - (k + 1);
                rb = r + (k + 1) > ps - 1 ? ps - 1 : r + (k + 1);
            }
            c.idm[k] = p.perm[ra];
            c.idp[k] = p.perm[rb];
            c.w[k] = weight<T>(Fs[ra], Fs[rb]);
        }
    }
}

// ALLOW_ILP false: one position a lane per round always (the same set; the
// four-position form is then not compiled in).
template <typename T, int NPMAX, int G, bool ALLOW_ILP = true>
__device__ __forceinline__ void plan_mask(const Params &p, Plan<T, NPMAX> &c, uint32_t *mwords,
                                          int lane) {
    c.mw = mwords;
    // four positions a lane per round where the scan spans eight or more
    // rounds of G positions, or where the run is one workgroup (latency only)
    const bool ilp = ALLOW_ILP && (c.mask.walk >= 8u * G || (long long)p.pop * G <= 256);
    if (c.op != OP_DORMANCY)
        subset_mask_group<G>(c.mask, c.m, mwords, (p.dim + 31) / 32, lane,
                             (int)(threadIdx.x & 63) & ~(G - 1), ilp);
}

// Rows a lane reads for its NCH chunks of 4 coordinates, loaded before the
// mask is built: its own row and the decided operation's first pair (with
// X_j for an autotroph).
template <typename T, int NCH>
struct Rows {
    typedef typename V4<T>::type v4;
    v4 x[NCH];            // own row
    v4 xj[NCH];           // X_j of Eq. (6)
    v4 am[NCH], ap[NCH];  // first pair: k-, k+ of Eq. (6) or i-1, i+1 of Eq. (8)
};

template <typename T>
__device__ __forceinline__ typename V4<T>::type load4v(const T *p) {
    return *reinterpret_cast<const typename V4<T>::type *>(p);
}

// The own row (c.id known) and the decided operation's neighbour rows
// (c.idj, c.idm[0], c.idp[0] picked); a dormant or reproducing protozoan
// reads none.  Lanes past D read nothing.
template <typename T, int NPMAX, int NCH, int G>
__device__ __forceinline__ void load_rows(const Params &p, const Plan<T, NPMAX> &c, int lane,
                                          const T *Xc, Rows<T, NCH> &rw) {
    const int D = p.dim, Dp = p.Dp;
    const typename V4<T>::type zero = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const int d0 = 4 * (lane + ch * G);
        const bool in = d0 < D;
        rw.x[ch] = in ? load4v(Xc + (size_t)c.id * Dp + d0) : zero;
        const bool fo = in && c.op >= OP_AUTOTROPH;
        rw.xj[ch] = (fo && c.op == OP_AUTOTROPH) ? load4v(Xc + (size_t)c.idj * Dp + d0) : zero;
        rw.am[ch] = fo ? load4v(Xc + (size_t)c.idm[0] * Dp + d0) : zero;
        rw.ap[ch] = fo ? load4v(Xc + (size_t)c.idp[0] * Dp + d0) : zero;
    }
}

// Candidate values of the four coordinates d0..d0+3 of one protozoan,
// clamped to the bounds, from the preloaded rows x (own), xj, xm, xp (first
// pair of the decided operation); further pairs are read here.  Coordinates at or beyond D are set
// to zero (the row padding), in x as well.
template <typename T, int NPMAX>
__device__ __forceinline__ void candidate4(const Params &p, const Plan<T, NPMAX> &c, int t,
                                           bool init, int d0, const T *Xc,
                                           typename V4<T>::type &x,
                                           const typename V4<T>::type &xj,
                                           const typename V4<T>::type &xm,
                                           const typename V4<T>::type &xp, T y[4]) {
    const int D = p.dim, Dp = p.Dp;
    T lb[4], ub[4];
    load4((const T *)p.lb + d0, lb);
    load4((const T *)p.ub + d0, ub);
    if (init) x = typename V4<T>::type{T(0), T(0), T(0), T(0)};
    const Stream rng = stream_of(p);
    T U[4] = {T(0), T(0), T(0), T(0)};
    if (init) {
        const Words u = rng.block(TAG_INIT, (uint32_t)(d0 >> 2), (uint32_t)c.id, 0u);
#pragma unroll
        for (int e = 0; e < 4; ++e) U[e] = uniform<T>(u.w[e]);
    } else if (c.op != OP_AUTOTROPH) {
        const Words u = rng.block(TAG_ELEM, (uint32_t)(d0 >> 2), (uint32_t)c.r, (uint32_t)t);
#pragma unroll
        for (int e = 0; e < 4; ++e) U[e] = uniform<T>(u.w[e]);
    }
    const uint32_t mb = (init || c.op == OP_DORMANCY) ? 0xFu : (c.mw[d0 >> 5] >> (d0 & 31)) & 0xFu;
    if (init || c.op == OP_DORMANCY) {
#pragma unroll
        for (int e = 0; e < 4; ++e) y[e] = lb[e] + U[e] * (ub[e] - lb[e]);   // Eq. (1)
    } else if (c.op == OP_REPRODUCTION) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            y[e] = x[e];
            if ((mb >> e) & 1u)
                y[e] = x[e] + c.srep * (lb[e] + U[e] * (ub[e] - lb[e]));        // Eq. (2)
        }
    } else {
        T acc[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = T(0) + c.w[0] * (xm[e] - xp[e]);
#pragma unroll
        for (int k = 1; k < NPMAX; ++k) {
            if (k < p.np) {
                T xmk[4], xpk[4];
                load4(Xc + (size_t)c.idm[k] * Dp + d0, xmk);
                load4(Xc + (size_t)c.idp[k] * Dp + d0, xpk);
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[e] = acc[e] + c.w[k] * (xmk[e] - xpk[e]);
            }
        }
        const T npd = T(p.np);
        if (p.np > 1) {   // acc / np; with one pair the quotient is acc itself
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] = acc[e] / npd;
        }
        if (c.op == OP_AUTOTROPH) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                y[e] = x[e];
                if ((mb >> e) & 1u)
                    y[e] = x[e] + c.fac * ((xj[e] - x[e]) + acc[e]);                // Eq. (6)
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                y[e] = x[e];
                if ((mb >> e) & 1u) {
                    const T xnear = (T(1) + (c.sgn * U[e]) * c.cn) * x[e];         // Eq. (9)
                    y[e] = x[e] + c.fac * ((xnear - x[e]) + acc[e]);                // Eq. (8)
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        y[e] = (d0 + e < D) ? fmin(fmax(y[e], lb[e]), ub[e]) : T(0);
        if (d0 + e >= D) x[e] = T(0);
    }
}

// ---------------------------------------------------------------------------
// Fused elementwise step.  G lanes per protozoan (a power of two <= 64, so a
// group never straddles a wavefront), NCH chunks of 4 coordinates per lane.
// ---------------------------------------------------------------------------
// `itp`: the iteration and its scalars when the caller knows them (the
// persistent form); nullptr reads them from the control block.
template <typename T, int G, int NCH, int NPMAX>
__device__ __forceinline__ void step_elem_body(const Params &p, int init, int blk,
                                               const Iter *itp = nullptr) {
    const int lane = threadIdx.x & (G - 1);
    const int item = (blk * 256 + threadIdx.x) / G;
    if (item >= p.pop) return;
    const int D = p.dim, Dp = p.Dp;
    const Iter it = itp ? *itp : load_iter(p, init);
    const int t = it.t;
    const int src = (t + 1) & 1, dst = t & 1;
    const T *Xc = (const T *)(src ? p.X[1] : p.X[0]);   // (no dynamic index: p may be a local)
    const T *Fc = (const T *)p.Fs;   // old fitness, in rank order
    T *Xn = (T *)(dst ? p.X[1] : p.X[0]);
    T *Fn = (T *)p.F;

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
        plan_decide<T, NPMAX>(p, item, it, d, c);   // while the ids load
        plan_pick<T, NPMAX>(d, c);
        load_rows<T, NPMAX, NCH, G>(p, c, lane, Xc, rw);
        plan_mask<T, NPMAX, G>(p, c, mwords[threadIdx.x / G], lane);   // while the rows load
        plan_pairs<T, NPMAX>(p, item, t, d, c);
    }
    (void)Fc;

    T xs[NCH][4], ys[NCH][4];
    const T *o = (const T *)p.shift;
    T s1 = T(0), s2 = T(0);
    const bool separable = p.kind != K_ROSENBROCK;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const int d0 = 4 * (lane + ch * G);
        if (d0 < D) {
            candidate4<T, NPMAX>(p, c, t, init != 0, d0, Xc, rw.x[ch], rw.xj[ch], rw.am[ch],
                                 rw.ap[ch], ys[ch]);
#pragma unroll
            for (int e = 0; e < 4; ++e) xs[ch][e] = rw.x[ch][e];
            if (separable) {   // objective terms of this chunk right away
                T ov[4];
                load4(o + d0, ov);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (d0 + e < D) {
                        const T z = ys[ch][e] - ov[e];
                        if (p.kind == K_RASTRIGIN) {
                            s1 += z * z - T(10) * cos2pi(z) + T(10);
                        } else {
                            s1 += z * z;
                            if (p.kind == K_ACKLEY) s2 += cos2pi(z);
                        }
                    }
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) xs[ch][e] = ys[ch][e] = T(0);
        }
    }
    if (!separable) {   // Rosenbrock couples each coordinate with the next
        T zfirst[NCH], zs[NCH][4];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int d0 = 4 * (lane + ch * G);
            T ov[4] = {T(0), T(0), T(0), T(0)};
            if (d0 < D) load4(o + d0, ov);
#pragma unroll
            for (int e = 0; e < 4; ++e) zs[ch][e] = d0 < D ? ys[ch][e] - ov[e] : T(0);
            zfirst[ch] = zs[ch][0];
        }
        const int wl = threadIdx.x & 63;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            // next coordinate after this lane's chunk: lane + 1, or lane 0 of the next chunk
            const T nb_same = __shfl(zfirst[ch], wl + 1 < 64 ? wl + 1 : wl, 64);
            const T nb_next = __shfl(zfirst[ch + 1 < NCH ? ch + 1 : ch], wl - (G - 1), 64);
            const T after = lane < G - 1 ? nb_same : nb_next;
            const int d0 = 4 * (lane + ch * G);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (d0 + e + 1 < D) {
                    const T a = zs[ch][e] + T(1);
                    const T b = (e < 3 ? zs[ch][e + 1] : after) + T(1);
                    s1 += T(100) * (b - a * a) * (b - a * a) + (a - T(1)) * (a - T(1));
                }
            }
        }
    }
    s1 = group_sum<G>(s1);
    T fnew;
    if (p.kind == K_ACKLEY) {
        s2 = group_sum<G>(s2);
        fnew = T(-20) * exp(T(-0.2) * sqrt(s1 / T(D))) - exp(s2 / T(D)) + T(20) + T(kE);
    } else {
        fnew = s1;
    }
    const bool accept = init || strictly_less(fnew, c.fold);
    T *row = Xn + (size_t)c.id * Dp;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const int d0 = 4 * (lane + ch * G);
        if (d0 < D) store4(row + d0, accept ? ys[ch] : xs[ch]);
    }
    if (lane == 0) Fn[c.id] = accept ? fnew : c.fold;
    if (!init && !itp && blk == 0 && threadIdx.x == 0) p.ctrl->t = t;   // iteration closed
    if (p.trace && !init) {
        T *ty = (T *)p.trY + (size_t)c.id * Dp;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int d0 = 4 * (lane + ch * G);
            if (d0 < D) store4(ty + d0, ys[ch]);
        }
        if (lane == 0) {
            ((T *)p.trF)[c.id] = fnew;
            p.trOp[c.id] = c.op;
        }
    }
}

// One handle's launch: workgroup b is the run's block b.  A batch launch
// covers several runs with the same kernel shape: workgroup b does block
// blocks[b].y of run blocks[b].x, whose parameters are runs[blocks[b].x].
template <typename T, int G, int NCH, int NPMAX>
__global__ __launch_bounds__(256) void step_elem(Params p, int init) {
    step_elem_body<T, G, NCH, NPMAX>(p, init, (int)blockIdx.x);
}
template <typename T, int G, int NCH, int NPMAX>
__global__ __launch_bounds__(256) void step_elem_batch(const Params *runs, const int2 *blocks,
                                                       int init) {
    const int2 b = blocks[blockIdx.x];
    step_elem_body<T, G, NCH, NPMAX>(runs[b.x], init, b.y);
}

// ---------------------------------------------------------------------------
// Persistent form (apo_run of a run that one workgroup holds): one workgroup
// runs n iterations, each the sort (LDS form, the whole population) and the
// step, separated by workgroup barriers only.  The run's state and the
// read-only tables its iterations read are copied into an LDS image at entry
// (PersistImage) and the parameters' pointers redirected there, so an
// iteration touches no global memory apart from the trace; the state is
// copied back at exit and the control block written as the last iteration's
// sort and step would leave it.  The device code of sort and step is the
// two-kernel iteration's, so the results are the same bit for bit.
// ---------------------------------------------------------------------------
template <typename U>
__device__ __forceinline__ void block_copy(U *dst, const U *src, size_t n) {
    for (size_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

template <typename T>
__device__ __forceinline__ Params persist_enter(const Params &p, unsigned char *img) {
    const bool hist = p.kind == K_KAPUR || p.kind == K_OTSU;
    const PersistImage m = persist_image(p.pop, p.Dp, (int)sizeof(T), hist);
    const size_t rows = (size_t)p.pop * p.Dp;
    Params q = p;
    q.X[0] = img + m.x0;
    q.X[1] = img + m.x1;
    q.F = img + m.f;
    q.Fs = img + m.fs;
    q.perm = (int32_t *)(img + m.perm);
    q.drf = img + m.drf;
    q.p_dr = (const double *)(img + m.pdr);
    q.lb = img + m.lb;
    q.ub = img + m.ub;
    q.shift = img + m.sh;
    block_copy((T *)(img + m.x0), (const T *)p.X[0], rows);
    block_copy((T *)(img + m.x1), (const T *)p.X[1], rows);
    block_copy((T *)(img + m.f), (const T *)p.F, (size_t)p.pop);
    block_copy((double *)(img + m.pdr), p.p_dr, (size_t)p.pop);
    block_copy((T *)(img + m.lb), (const T *)p.lb, (size_t)p.Dp);
    block_copy((T *)(img + m.ub), (const T *)p.ub, (size_t)p.Dp);
    block_copy((T *)(img + m.sh), (const T *)p.shift, (size_t)p.Dp);
    if (hist) {
        q.htab = (const double *)(img + m.htab);
        block_copy((double *)(img + m.htab), p.htab, (size_t)3 * 257);
    }
    return q;
}

template <typename T>
__device__ __forceinline__ void persist_leave(const Params &p, const Params &q) {
    const size_t rows = (size_t)p.pop * p.Dp;
    block_copy((T *)p.X[0], (const T *)q.X[0], rows);
    block_copy((T *)p.X[1], (const T *)q.X[1], rows);
    block_copy((T *)p.F, (const T *)q.F, (size_t)p.pop);
    block_copy((T *)p.Fs, (const T *)q.Fs, (size_t)p.pop);
    block_copy(p.perm, (const int32_t *)q.perm, (size_t)p.pop);
    block_copy(p.drf, (const uint8_t *)q.drf, (size_t)p.pop);
}

__device__ __forceinline__ Iter iter_at(const Params &p, int t) {
    Iter it;
    it.t = t;
    it.p_ah = p.p_ah[t];
    it.fscale = p.fscale[t];
    it.cnear = p.cnear[t];
    return it;
}

template <typename T, int G, int NCH, int NPMAX>
__global__ __launch_bounds__(256) void run_elem_persist(Params p, int t0, int n) {
    extern __shared__ __align__(16) unsigned char pdyn[];
    const Params q = persist_enter<T>(p, pdyn);
    Iter it = iter_at(p, t0 + 1);
    __syncthreads();
    for (int k = 1; k <= n; ++k) {
        const int t = t0 + k;
        const Iter cur = it;
        if (k < n) it = iter_at(p, t + 1);   // the next iteration's scalars, ahead
        rank_small_body<T>(q, 0, t, k == n);
        __syncthreads();
        step_elem_body<T, G, NCH, NPMAX>(q, 0, 0, &cur);
        __syncthreads();
    }
    persist_leave<T>(p, q);
    if (threadIdx.x == 0) p.ctrl->t = t0 + n;   // iterations closed
}

template <typename T, int NPMAX>
hipError_t launch_persist_t(const Params &p, int t0, int n, hipStream_t s) {
    const int G = lanes_for_dim(p.dim), NCH = chunks_for_dim(p.dim);
    const bool fp64 = sizeof(T) == 8;
    if (!persist_form(p, fp64) || n < 1) return hipErrorInvalidValue;
    const size_t lds = persist_lds_bytes(p, fp64);
#define APO_PERSIST(GG, CC)                                                                  \
    if (G == GG && NCH == CC) {                                                              \
        const void *fn = (const void *)run_elem_persist<T, GG, CC, NPMAX>;                   \
        if (lds > 65536) {                                                                   \
            const hipError_t ea =                                                            \
                hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
            if (ea != hipSuccess) return ea;                                                 \
        }                                                                                    \
        launch_k(p, run_elem_persist<T, GG, CC, NPMAX>, dim3(1), dim3(256), lds, s, p, t0, n); \
        return hipGetLastError();                                                            \
    }
    APO_ELEM_SHAPES(APO_PERSIST)
#undef APO_PERSIST
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Tiled step: TM = max(16, 512 / G) consecutive ranks per workgroup of 512
// threads (one lane group per row; TM / 16 MFMA row blocks).
// LDS: Ys, Xs, As [TM][LS] candidates, own rows and y - o; Zs [TM][LZ]
// transformed coordinates (Rosenbrock) or sorted thresholds (histogram
// objectives); per-(row, column tile) partial sums [TM][Nt] x 2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ f32x4 mfma16x16x4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16x16x4(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row of the 16 x 16 output held by element v of lane l (column l % 16).
// The f32 form keeps four consecutive rows per lane group (row 4 (l/16) + v);
// the f64 form interleaves them (row 4 v + l/16), as measured on gfx950.
template <typename T>
__device__ __forceinline__ int mfma_out_row(int l, int v);
template <>
__device__ __forceinline__ int mfma_out_row<float>(int l, int v) { return 4 * (l >> 4) + v; }
template <>
__device__ __forceinline__ int mfma_out_row<double>(int l, int v) { return 4 * v + (l >> 4); }

// Thresholding objectives (Kapur entropy, Otsu between-class variance) of
// one candidate, by a team of 32 lanes of one wavefront.  Thresholds are
// the coordinates rounded half to even; each is placed at its position in
// ascending order by counting (ties keep coordinate order), so class c is
// the grey levels [t_(c-1), t_c) with t_(-1) = 0 and t_k = 256.  Class
// weights and moments are differences of the binary64 prefix tables
// P (probability), S (p ln p) and M1 (level x probability); empty classes
// add nothing.  Each lane adds its classes; the team total is the same in
// every lane.  F is minus the criterion.
template <typename T, int TT>
__device__ __forceinline__ double threshold_objective_team(const Params &p, const T *yrow,
                                                           int *ts, int tl, bool live) {
    const int k = p.dim;
    if (live) {
        for (int c = tl; c < k; c += TT) {
            const int v = (int)rint((double)yrow[c]);
            int pos = 0;
            for (int q = 0; q < k; ++q) {
                const int u = (int)rint((double)yrow[q]);
                pos += (u < v || (u == v && q < c)) ? 1 : 0;
            }
            ts[pos] = v;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double *P = p.htab, *S = p.htab + 257, *M1 = p.htab + 514;
    const double muT = M1[256];
    double part = 0.0;
    if (live) {
        for (int c = tl; c <= k; c += TT) {
            const int a = c == 0 ? 0 : ts[c - 1];
            const int b = c < k ? ts[c] : 256;
            const double omega = P[b] - P[a];
            if (omega > 0.0) {
                if (p.kind == K_KAPUR) {
                    part += log(omega) - (S[b] - S[a]) / omega;
                } else {
                    const double mu = (M1[b] - M1[a]) / omega;
                    part += omega * (mu - muT) * (mu - muT);
                }
            }
        }
    }
    return -group_sum<TT>(part);
}

// The objective of the first nrows rows of a tile by teams of TT lanes
// (512 / TT teams, rows in turn).  With k + 1 <= TT every lane holds at most
// one class, and the team sum equals that of a wider team bit for bit (the
// added lanes hold exact zeros), so the team size is a choice of speed only.
template <typename T, int TT>
__device__ __forceinline__ void threshold_rows(const Params &p, const T *Ys, int LS, int *Zi,
                                               int nrows, const int32_t *s_id, T *s_fnew) {
    const int tl = threadIdx.x & (TT - 1);
    for (int row = threadIdx.x / TT; row < nrows; row += 512 / TT) {
        const bool live = s_id[row] >= 0;
        const double f =
            threshold_objective_team<T, TT>(p, Ys + row * LS, Zi + row * (p.dim + 1), tl, live);
        if (tl == 0 && live) s_fnew[row] = T(f);
    }
}

// LDS row stride (elements) of the tile's row buffers (tile_row_stride of
// apo_shape.hpp on the run's padded sizes).
__host__ __device__ inline int tile_row_stride(const Params &p, int es) {
    return tile_row_stride(p.Dp, p.Ks, es);
}


// `itp`: the iteration and its scalars when the caller knows them; nullptr
// reads them from the control block, and workgroup 0 then closes the
// iteration there.
// FORM: what the objective is known to be at compile time -- 0 any (read
// from p), 1 a thresholding one (no matrix phase compiled in), 2 a rotated
// separable one (Sphere, Rastrigin, Ackley: no Rosenbrock or thresholding
// phases compiled in).
template <typename T, int G, int NCH, int NPMAX, int TM, int FORM = 0>
__device__ __forceinline__ void step_tile_body(const Params &p, int init, int blk,
                                               const Iter *itp = nullptr) {
    constexpr bool THR = FORM == 1, SEP = FORM == 2;
    constexpr int NT = 512, GROUPS = NT / G, RB = TM / 16;
    static_assert(TM % 16 == 0 && TM % (NT / 32) == 0, "row blocks of 16; teams of 32 lanes");
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t s_id[TM], s_op[TM];
    __shared__ uint32_t s_mwords[GROUPS][(4 * G * NCH + 31) / 32];
    __shared__ T s_fold[TM], s_fnew[TM];
    const int D = p.dim, Dp = p.Dp;
    const int LS = tile_row_stride(p, (int)sizeof(T)), LZ = p.Nt * 16 + 1;
    T *Ys = (T *)smem;        // clamped candidates
    T *Xs = Ys + TM * LS;     // own rows
    T *As = Xs + TM * LS;     // y - o, the matrix-core A operand
    T *Zs = As + TM * LS;     // z = M (y - o) when a coordinate's neighbour is needed
    const int zwords = TM * LZ > TM * (D + 1) ? TM * LZ : TM * (D + 1);
    T *s_p1 = Zs + zwords;    // [TM][Nt] per column-tile partial sums
    T *s_p2 = s_p1 + TM * p.Nt;
    const Iter it = itp ? *itp : load_iter(p, init);
    const int t = it.t;
    const int src = (t + 1) & 1, dst = t & 1;
    const T *Xc = (const T *)(src ? p.X[1] : p.X[0]);   // (no dynamic index: p may be a local)
    const T *Fc = (const T *)p.Fs;   // old fitness, in rank order
    T *Xn = (T *)(dst ? p.X[1] : p.X[0]);
    T *Fn = (T *)p.F;
    const T *o = (const T *)p.shift;
    const int r0 = blk * TM;
    const int lane = threadIdx.x & (G - 1), grp = threadIdx.x / G;

    // The B fragments (packed M^T) of each wavefront's first output tile
    // are requested before phase 1 so the loads overlap the candidate work,
    // when the K range is exactly PRE steps (one straight MFMA run).
    constexpr int PRE = sizeof(T) == 4 ? 32 : 16;
    T bpre[PRE];
    {
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
        const T *B = (const T *)p.rotp;
        if ((SEP || (!THR && p.rotated)) && p.Ks == PRE && wave < RB * p.Nt) {
            const int nt0 = wave % p.Nt;
#pragma unroll
            for (int ks = 0; ks < PRE; ++ks) bpre[ks] = B[((size_t)ks * p.Nt + nt0) * 64 + l];
        } else {
#pragma unroll
            for (int ks = 0; ks < PRE; ++ks) bpre[ks] = T(0);
        }
    }

    // zero the padded k range of the A operand (each group its rows)
    for (int row = grp; row < TM; row += GROUPS)
        for (int col = D + lane; col < 4 * p.Ks; col += G) As[row * LS + col] = T(0);

    // phase 1: candidates into LDS
    for (int row = grp; row < TM; row += GROUPS) {
        const int item = r0 + row;
        if (item < p.pop) {
            Plan<T, NPMAX> c;
            Rows<T, NCH> rw;
            if (init) {
                c.op = OP_DORMANCY; c.id = item; c.r = item; c.m = (uint32_t)D; c.fold = T(0);
            } else {
                Draws<T> d;
                plan_draws<T, NPMAX>(p, item, t, (threadIdx.x & 63) & ~(G - 1), lane, c, d);
                plan_decide<T, NPMAX>(p, item, it, d, c);   // while the ids load
                plan_pick<T, NPMAX>(d, c);
                load_rows<T, NPMAX, NCH, G>(p, c, lane, Xc, rw);
                // (the separable form's shapes, one chunk of at most 128
                // coordinates in 16-row tiles, scan few rounds)
                plan_mask<T, NPMAX, G, !SEP>(p, c, s_mwords[grp], lane);   // while the rows load
                plan_pairs<T, NPMAX>(p, item, t, d, c);
            }
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int d0 = 4 * (lane + ch * G);
                if (d0 < D) {
                    T y[4];
                    candidate4<T, NPMAX>(p, c, t, init != 0, d0, Xc, rw.x[ch], rw.xj[ch],
                                         rw.am[ch], rw.ap[ch], y);
                    T ov[4], a[4], xo[4];
                    load4(o + d0, ov);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        a[e] = y[e] - ov[e];
                        xo[e] = rw.x[ch][e];
                    }
                    if (d0 + 4 <= D) {
                        store4(Ys + row * LS + d0, y);
                        store4(Xs + row * LS + d0, xo);
                        store4(As + row * LS + d0, a);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            if (d0 + e < D) {
                                Ys[row * LS + d0 + e] = y[e];
                                Xs[row * LS + d0 + e] = xo[e];
                                As[row * LS + d0 + e] = a[e];
                            }
                        }
                    }
                }
            }
            if (lane == 0) {
                s_id[row] = c.id;
                s_op[row] = c.op;
                s_fold[row] = c.fold;
            }
        } else {
            for (int d = lane; d < D; d += G) Ys[row * LS + d] = Xs[row * LS + d] = As[row * LS + d] = T(0);
            if (lane == 0) s_id[row] = -1;
        }
    }
    __syncthreads();

    const bool thresholds = THR || (!SEP && (p.kind == K_KAPUR || p.kind == K_OTSU));
    const bool rot = SEP || (!THR && p.rotated);
    // separable objectives of a rotated problem are summed from the matrix
    // core accumulators in phase 2
    const bool separable = SEP || (rot && !thresholds && p.kind != K_ROSENBROCK);
    if (rot) {
        // phase 2: Z = (Y - o) M^T on the matrix cores.  Fragment layout of
        // v_mfma 16x16x4: A[i][k] in lane i + 16k, B[k][j] in lane j + 16k;
        // the output row of (lane, element) is given by mfma_out_row.
        const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
        const typename V4<T>::type zero = {T(0), T(0), T(0), T(0)};
        const T *B = (const T *)p.rotp;
        const int i = l & 15;
        // output tile tau = (row block rb, column tile nt), wavefronts in turn;
        // the contraction index of step ks in lane l is k = Ks (l / 16) + ks
        // (the host packs B with the same order), so a lane's A values are
        // contiguous: A[16 rb + i][Ks (l / 16) + ks] at Arow[ks]
        for (int tau = wave; tau < RB * p.Nt; tau += NT / 64) {
            const int rb = tau / p.Nt, nt = tau % p.Nt;
            const T *Arow = As + (16 * rb + i) * LS + (l >> 4) * p.Ks;
            typename V4<T>::type acc = zero;
            if (tau == wave && p.Ks == PRE) {
                // fragments already in registers: one straight run
                T a[PRE];
#pragma unroll
                for (int q = 0; q < PRE / 4; ++q) load4(Arow + 4 * q, a + 4 * q);
#pragma unroll
                for (int ks = 0; ks < PRE; ++ks) acc = mfma16x16x4(a[ks], bpre[ks], acc);
            } else {
                for (int k0 = 0; k0 < p.Ks; k0 += 8) {
                    T a[8], b[8];
                    load4(Arow + k0, a);
                    load4(Arow + k0 + 4, a + 4);
#pragma unroll
                    for (int u = 0; u < 8; ++u) b[u] = B[((size_t)(k0 + u) * p.Nt + nt) * 64 + l];
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc = mfma16x16x4(a[u], b[u], acc);
                }
            }
            if (!SEP && p.kind == K_ROSENBROCK) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Zs[(16 * rb + mfma_out_row<T>(l, v)) * LZ + 16 * nt + (l & 15)] = acc[v];
            } else {
                // separable objectives straight from the accumulators: the
                // 16 columns of this tile summed per row (butterfly over the
                // 16 lanes of a row group), one partial per (row, tile)
                const bool valid = 16 * nt + (l & 15) < D;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const T z = acc[v];
                    T g1 = T(0), g2 = T(0);
                    if (valid) {
                        if (p.kind == K_RASTRIGIN) {
                            g1 = z * z - T(10) * cos2pi(z) + T(10);
                        } else {
                            g1 = z * z;
                            if (p.kind == K_ACKLEY) g2 = cos2pi(z);
                        }
                    }
                    g1 = group_sum<16>(g1);
                    if (p.kind == K_ACKLEY) g2 = group_sum<16>(g2);
                    if ((l & 15) == 0) {
                        const int row = 16 * rb + mfma_out_row<T>(l, v);
                        s_p1[row * p.Nt + nt] = g1;
                        s_p2[row * p.Nt + nt] = g2;
                    }
                }
            }
        }
        __syncthreads();
    }

    // phase 3: objective per protozoan
    if (thresholds) {
        // teams of the smallest power of two >= k + 1 lanes (at most 32),
        // over the rows that hold a protozoan
        const int nrows = p.pop - r0 < TM ? p.pop - r0 : TM;
        int *Zi = (int *)Zs;
        if (D + 1 <= 2)
            threshold_rows<T, 2>(p, Ys, LS, Zi, nrows, s_id, s_fnew);
        else if (D + 1 <= 4)
            threshold_rows<T, 4>(p, Ys, LS, Zi, nrows, s_id, s_fnew);
        else if (D + 1 <= 8)
            threshold_rows<T, 8>(p, Ys, LS, Zi, nrows, s_id, s_fnew);
        else if (D + 1 <= 16)
            threshold_rows<T, 16>(p, Ys, LS, Zi, nrows, s_id, s_fnew);
        else
            threshold_rows<T, 32>(p, Ys, LS, Zi, nrows, s_id, s_fnew);
    } else if (separable) {
        // the row sums of the column-tile partials are taken in phase 4 by
        // each row's own group (the partials are visible since phase 2)
    } else {
        for (int row = grp; row < TM; row += GROUPS) {
            T s1 = T(0), s2 = T(0);
            if (s_id[row] >= 0) {
                for (int d = lane; d < D; d += G) {
                    const T z = rot ? Zs[row * LZ + d] : As[row * LS + d];
                    if (p.kind == K_ROSENBROCK) {
                        if (d + 1 < D) {
                            const T zn = rot ? Zs[row * LZ + d + 1] : As[row * LS + d + 1];
                            const T a = z + T(1), b = zn + T(1);
                            s1 += T(100) * (b - a * a) * (b - a * a) + (a - T(1)) * (a - T(1));
                        }
                    } else if (p.kind == K_RASTRIGIN) {
                        s1 += z * z - T(10) * cos2pi(z) + T(10);
                    } else {
                        s1 += z * z;
                        if (p.kind == K_ACKLEY) s2 += cos2pi(z);
                    }
                }
            }
            s1 = group_sum<G>(s1);
            s2 = group_sum<G>(s2);
            if (lane == 0 && s_id[row] >= 0) {
                s_fnew[row] = p.kind == K_ACKLEY
                                  ? T(-20) * exp(T(-0.2) * sqrt(s1 / T(D))) - exp(s2 / T(D)) +
                                        T(20) + T(kE)
                                  : s1;
            }
        }
    }
    if (!separable) __syncthreads();

    // phase 4: greedy selection and the double-buffered write
    if (!init && !itp && blk == 0 && threadIdx.x == 0) p.ctrl->t = t;   // iteration closed
    for (int row = grp; row < TM; row += GROUPS) {
        const int id = s_id[row];
        if (id < 0) continue;
        T fnew;
        if (separable) {
            // the same sequential sum in every lane (broadcast LDS reads)
            T s1 = T(0), s2 = T(0);
            for (int nt = 0; nt < p.Nt; ++nt) s1 += s_p1[row * p.Nt + nt];
            if (p.kind == K_ACKLEY)
                for (int nt = 0; nt < p.Nt; ++nt) s2 += s_p2[row * p.Nt + nt];
            fnew = p.kind == K_ACKLEY
                       ? T(-20) * exp(T(-0.2) * sqrt(s1 / T(D))) - exp(s2 / T(D)) + T(20) + T(kE)
                       : s1;
        } else {
            fnew = s_fnew[row];
        }
        const bool accept = init || strictly_less(fnew, s_fold[row]);
        const T *srcrow = accept ? Ys + row * LS : Xs + row * LS;
        T *out = Xn + (size_t)id * Dp;
        for (int d0 = 4 * lane; d0 < D; d0 += 4 * G) {
            if (d0 + 4 <= D) {
                T v[4];
                load4(srcrow + d0, v);
                store4(out + d0, v);
            } else {
                for (int d = d0; d < D; ++d) out[d] = srcrow[d];
            }
        }
        if (lane == 0) Fn[id] = accept ? fnew : s_fold[row];
        if (p.trace && !init) {
            T *ty = (T *)p.trY + (size_t)id * Dp;
            for (int d = lane; d < D; d += G) ty[d] = Ys[row * LS + d];
            if (lane == 0) {
                ((T *)p.trF)[id] = fnew;
                p.trOp[id] = s_op[row];
            }
        }
    }
}

template <typename T, int G, int NCH, int NPMAX, int TM>
__global__ __launch_bounds__(512) void step_tile(Params p, int init) {
    step_tile_body<T, G, NCH, NPMAX, TM>(p, init, (int)blockIdx.x);
}
// The tiled step of a thresholding run (no matrix phase compiled in), and
// of a rotated separable one (no Rosenbrock or thresholding phases).
template <typename T, int G, int NCH, int NPMAX, int TM>
__global__ __launch_bounds__(512) void step_tile_thr(Params p, int init) {
    step_tile_body<T, G, NCH, NPMAX, TM, 1>(p, init, (int)blockIdx.x);
}
template <typename T, int G, int NCH, int NPMAX, int TM>
__global__ __launch_bounds__(512) void step_tile_sep(Params p, int init) {
    step_tile_body<T, G, NCH, NPMAX, TM, 2>(p, init, (int)blockIdx.x);
}
template <typename T, int G, int NCH, int NPMAX, int TM>
__global__ __launch_bounds__(512) void step_tile_batch(const Params *runs, const int2 *blocks,
                                                       int init) {
    const int2 b = blocks[blockIdx.x];
    step_tile_body<T, G, NCH, NPMAX, TM>(runs[b.x], init, b.y);
}

// Persistent form of a tiled run whose population one tile holds (ps <= TM,
// ps <= 256): one workgroup runs n iterations of the sort (LDS form; its
// threads past 256 take no part) and the tiled step, separated by workgroup
// barriers, on the run's global buffers (the step's own LDS leaves no room
// for the run's image; the global form measured faster here as well); the
// iterations are closed in the control block at the end.
template <typename T, int G, int NCH, int NPMAX, int TM, bool THR>
__global__ __launch_bounds__(512) void run_tile_persist(Params p, int t0, int n) {
    for (int k = 1; k <= n; ++k) {
        const int t = t0 + k;
        rank_small_body<T>(p, 0, t);
        __syncthreads();
        const Iter it = iter_at(p, t);
        step_tile_body<T, G, NCH, NPMAX, TM, THR ? 1 : 0>(p, 0, 0, &it);
        __syncthreads();
    }
    if (threadIdx.x == 0 && n > 0) p.ctrl->t = t0 + n;   // iterations closed
}

// The launch of one persistent shape: thresholding runs take the kernel
// without the matrix phase where their shapes are (one chunk, at most 16
// lanes: k <= 64 thresholds).
template <typename T, int GG, int CC, int NPMAX, int TMM, bool THR>
hipError_t launch_tile_persist_one(const Params &p, int t0, int n, size_t lds, hipStream_t s) {
    const void *fn = (const void *)run_tile_persist<T, GG, CC, NPMAX, TMM, THR>;
    if (lds > 65536) {
        const hipError_t ea =
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (ea != hipSuccess) return ea;
    }
    launch_k(p, run_tile_persist<T, GG, CC, NPMAX, TMM, THR>, dim3(1), dim3(512), lds, s, p, t0,
             n);
    return hipGetLastError();
}

template <typename T, int GG, int CC, int NPMAX, int TMM>
hipError_t launch_tile_persist_shape(const Params &p, int t0, int n, size_t lds, hipStream_t s) {
    if constexpr (CC == 1 && GG <= 16) {
        if (p.kind == K_KAPUR || p.kind == K_OTSU)
            return launch_tile_persist_one<T, GG, CC, NPMAX, TMM, true>(p, t0, n, lds, s);
    }
    return launch_tile_persist_one<T, GG, CC, NPMAX, TMM, false>(p, t0, n, lds, s);
}


// A thresholding run's step on the kernel without the matrix phase, where its
// shape has one (one chunk, at most 16 lanes); `done` false: not launched here.
template <typename T, int GG, int CC, int NPMAX, int TMM>
hipError_t launch_tile_thr(const Params &p, int init, dim3 grid, size_t lds, hipStream_t s,
                           bool &done) {
    done = false;
    if constexpr (CC == 1 && GG <= 16) {
        if (p.kind == K_KAPUR || p.kind == K_OTSU) {
            done = true;
            if (lds > 65536) {
                const hipError_t ea =
                    hipFuncSetAttribute((const void *)step_tile_thr<T, GG, CC, NPMAX, TMM>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                if (ea != hipSuccess) return ea;
            }
            launch_k(p, step_tile_thr<T, GG, CC, NPMAX, TMM>, grid, dim3(512), lds, s, p, init);
            return hipGetLastError();
        }
    }
    if constexpr (CC == 1 && TMM == 16) {
        if (p.rotated && (p.kind == K_SPHERE || p.kind == K_RASTRIGIN || p.kind == K_ACKLEY)) {
            done = true;
            if (lds > 65536) {
                const hipError_t ea =
                    hipFuncSetAttribute((const void *)step_tile_sep<T, GG, CC, NPMAX, TMM>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                if (ea != hipSuccess) return ea;
            }
            launch_k(p, step_tile_sep<T, GG, CC, NPMAX, TMM>, grid, dim3(512), lds, s, p, init);
            return hipGetLastError();
        }
    }
    return hipSuccess;
}

// A launch of one handle (b == nullptr: grid of the run's own blocks, lds
// from its shape) or of a batch (b: the runs of one kernel shape, `p` one
// of them, lds the largest of theirs).
template <typename T, int NPMAX>
hipError_t launch_tile_t(const Params &p, int init, hipStream_t s, const BatchLaunch *b = nullptr) {
    const int G = tile_lanes(p), NCH = tile_chunks(p);
    if (NCH < 0) return hipErrorInvalidValue;
    {
        const int TMr = tile_rows(p);
        const dim3 grid(b ? (unsigned)b->nblocks : (unsigned)((p.pop + TMr - 1) / TMr));
        const dim3 block(512);
        const size_t lds = b ? b->lds : tile_lds_bytes(p, sizeof(T) == 8);
#define APO_TILE(GG, CC, TMM)                                                                \
    if (G == GG && NCH == CC && TMr == TMM) {                                                \
        const void *fn = b ? (const void *)step_tile_batch<T, GG, CC, NPMAX, TMM>           \
                           : (const void *)step_tile<T, GG, CC, NPMAX, TMM>;                 \
        if (lds > 65536) {                                                                   \
            const hipError_t ea =                                                            \
                hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
            if (ea != hipSuccess) return ea;                                                 \
        }                                                                                    \
        if (b) {                                                                             \
            hipLaunchKernelGGL((step_tile_batch<T, GG, CC, NPMAX, TMM>), grid, block, lds, s, \
                               b->runs, b->blocks, init);                                    \
        } else {                                                                             \
            bool done;                                                                       \
            const hipError_t et =                                                            \
                launch_tile_thr<T, GG, CC, NPMAX, TMM>(p, init, grid, lds, s, done);         \
            if (done) return et;                                                             \
            launch_k(p, step_tile<T, GG, CC, NPMAX, TMM>, grid, block, lds, s, p, init);     \
        }                                                                                    \
        return hipGetLastError();                                                            \
    }
        APO_TILE_SHAPES(APO_TILE)
#undef APO_TILE
        return hipErrorInvalidValue;
    }
}

template <typename T, int NPMAX>
hipError_t launch_tile_persist_t(const Params &p, int t0, int n, hipStream_t s) {
    const int G = tile_lanes(p), NCH = tile_chunks(p), TMr = tile_rows(p);
    const bool fp64 = sizeof(T) == 8;
    if (!persist_form(p, fp64) || n < 1 || NCH < 0) return hipErrorInvalidValue;
    const size_t lds = tile_lds_bytes(p, fp64);
#define APO_TILE_PERSIST(GG, CC, TMM)                                                        \
    if (G == GG && NCH == CC && TMr == TMM)                                                  \
        return launch_tile_persist_shape<T, GG, CC, NPMAX, TMM>(p, t0, n, lds, s);
    APO_TILE_SHAPES(APO_TILE_PERSIST)
#undef APO_TILE_PERSIST
    return hipErrorInvalidValue;
}

template <typename T, int NPMAX>
hipError_t launch_elem_t(const Params &p, int init, hipStream_t s, const BatchLaunch *b = nullptr) {
    const int G = lanes_for_dim(p.dim), NCH = chunks_for_dim(p.dim);
    if (NCH < 0) return hipErrorInvalidValue;
    const long long threads = (long long)p.pop * G;
    const dim3 grid(b ? (unsigned)b->nblocks : (unsigned)((threads + 255) / 256)), block(256);
#define APO_ELEM(GG, CC)                                                                     \
    if (G == GG && NCH == CC) {                                                              \
        if (b)                                                                               \
            hipLaunchKernelGGL((step_elem_batch<T, GG, CC, NPMAX>), grid, block, 0, s,       \
                               b->runs, b->blocks, init);                                    \
        else                                                                                 \
            launch_k(p, step_elem<T, GG, CC, NPMAX>, grid, block, 0, s, p, init);            \
        return hipGetLastError();                                                            \
    }
    APO_ELEM_SHAPES(APO_ELEM)
#undef APO_ELEM
    return hipErrorInvalidValue;
}


}  // namespace apok
