// apo_internal.h -- state shared between the host runtime (apo_api.cpp) and
// the kernel launchers (apo_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "apo_shape.hpp"

namespace apok {

enum : int32_t { OP_DORMANCY = 0, OP_REPRODUCTION = 1, OP_AUTOTROPH = 2, OP_HETEROTROPH = 3 };
enum : int32_t { K_SPHERE = 0, K_RASTRIGIN = 1, K_ROSENBROCK = 2, K_ACKLEY = 3, K_KAPUR = 4,
                 K_OTSU = 5 };

constexpr int kMaxNp = 8;        // neighbour pairs supported

// Device-resident control block, one per handle.  The rank kernel opens
// iteration t_next = t + 1 and draws its scalars; the step kernel closes it.
struct Ctrl {
    int32_t t;            // completed iterations
    int32_t t_next;       // iteration being computed
    int32_t m_dr;         // |Dr| of iteration t_next
    int32_t best_id;      // written by the best kernel
    double best_f;
    double p_ah, fscale, cnear;   // Eqs. (12), (4), (9) at t_next
    int32_t pad[48];
};

// Buffers of the GEMM form (rotated objectives of large dimension, and the
// BF16 form): candidates by rank, the product's operands and partial sums,
// the rescore list and M in the operand precisions.
struct GemmBufs {
    float *Yr;            // [pop][Dp] candidates by rank
    uint16_t *Ab;         // BF16 y - o in MFMA fragment order (BF16 form): per 16-row
                          // group and 32-K chunk, 64 lanes x 8 values (pop padded to 256)
    float *anorm;         // [pop] ||y - o||_2 (BF16 form)
    float *P1, *P2;       // [pop][Np / 64] partial row sums
    int32_t *list;        // [pop] ranks to re-score in binary32
    int32_t *status;      // [pop] rank's slot in the list, or -1 (settled rejection)
    int32_t *count;       // its length
    unsigned long long *total;   // rows re-scored so far (BF16 form)
    const uint16_t *Mb;   // M in BF16, MFMA fragment order (1 KiB per 16 rows x 32 K)
    const float *Mf;      // [Np][Kp] M in binary32
    const double *Md;     // [dim][dim] M in binary64 (elite re-score)
    const double *o64;    // [dim] shift in binary64
    double *z64;          // [dim] z of the elite re-score
    int32_t Kp, Np;       // K and N padded to 128
    int32_t bf16;         // 1: BF16 estimate + binary32 re-score
    float nrm_dM;         // upper bound of ||bf16(M) - M||_2 (M in binary32), from its row
                          // and column sums (||A||_2 <= sqrt(||A||_1 ||A||_inf))
    float nrm_absM;       // upper bound of || |M| ||_2, the same way
};

// Everything a kernel needs, passed by value.  Element pointers are typed
// by the handle's precision (float or double).
struct Params {
    int32_t dim, pop, np, max_iter;
    int32_t Dp;           // row stride (elements) of X and Y
    int32_t kind;         // objective
    int32_t rotated;      // 1: z = M (x - o) through the packed matrix
    int32_t Nt, Ks;       // MFMA tiles: output column tiles of 16, k-steps of 4
    int32_t rows;         // ranks per workgroup of the tiled step: 16, or 512 / lanes
    int32_t rank_lds;     // 1: the sort stages the keys in LDS (pop <= 1024)
    int32_t lanes;        // lanes per protozoan of the tiled step (0: lanes_for_dim)
    int32_t gemm;         // 1: the GEMM form of the step (gb)
    GemmBufs gb;
                          // (Ks padded to 32 or a multiple of 8; A and B zero there)
    int32_t trace;        // 1: write candidates to the trace buffers
    uint32_t seed_lo, seed_hi, run;
    double pf_max;
    void *X[2];           // [pop][Dp] positions, indexed by t & 1
    void *F;              // [pop] fitness by id (old values are read through Fs)
    int32_t *perm;        // [pop] rank -> id
    void *Fs;             // [pop] fitness in rank order (written with perm)
    uint8_t *drf;         // [pop] 1 if rank r is in Dr this iteration (written with perm)
    Ctrl *ctrl;
    const double *p_ah;   // [max_iter + 1] Eq. (12)
    const double *fscale; // [max_iter + 1] 1 + cos(pi t / T) of Eq. (4)
    const double *cnear;  // [max_iter + 1] 1 - t / T of Eq. (9)
    const double *p_dr;   // [pop] Eq. (13) for rank r + 1
    const void *lb, *ub, *shift;   // [Dp]
    const void *rotp;     // packed MFMA B fragments of M^T
    const double *htab;   // histogram prefix tables (3 x 257: P, S, M1)
    void *trY;            // [pop][Dp]
    void *trF;            // [pop]
    int32_t *trOp;        // [pop]
    // Host side only: when set, the launch records these events itself at
    // the kernel's start and end (timing of the kernel's execution alone).
    hipEvent_t ev_start, ev_stop;
};

// Launch through the dispatch-timed path when p carries timing events.
template <typename F, typename... Args>
inline void launch_k(const Params &p, F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                     Args... args) {
    if (p.ev_start)
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, s, p.ev_start, p.ev_stop, 0,
                              args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

// A batched launch: workgroup b runs block blocks[b].y of run blocks[b].x,
// whose parameters are runs[blocks[b].x] (device arrays); lds is the
// dynamic LDS of the launch (the largest of its runs).
struct BatchLaunch {
    const Params *runs;
    const int2 *blocks;
    int nblocks;
    size_t lds;
};

// Launchers (apo_kernels.hip).  All asynchronous on `s`; they return the
// launch status.
hipError_t launch_init(const Params &p, bool fp64, hipStream_t s);
hipError_t launch_rank(const Params &p, bool fp64, hipStream_t s);
hipError_t launch_step(const Params &p, bool fp64, hipStream_t s);
// The persistent form: iterations t0 + 1 .. t0 + n of a run with
// persist_form(p), sort and step of each, in one single-workgroup launch.
hipError_t launch_persist(const Params &p, bool fp64, int t0, int n, hipStream_t s);
hipError_t launch_best(const Params &p, bool fp64, int cur, double *out_row, hipStream_t s);
hipError_t launch_hist_tables(const Params &p, const uint64_t *d_hist, hipStream_t s);
// 256-bin histogram of n bytes into scratch (histogram_scratch_bytes():
// per-workgroup partial rows, then the 256 uint64 counts at byte offset
// histogram_out_offset()).  Stream-ordered (two launches), no allocation.
constexpr int kHistBlocks = 512;   // workgroups of the image pass at most
constexpr size_t histogram_out_offset() { return (size_t)kHistBlocks * 256 * 4; }
constexpr size_t kHistScratchBytes = histogram_out_offset() + 256 * 8;
size_t histogram_scratch_bytes();

hipError_t launch_histogram(const uint8_t *img, uint64_t n, void *scratch, hipStream_t s);
// The same histogram with the device's file-scope scratch array instead of
// a caller buffer, the counts written to d_out (device [256] uint64).  No
// allocation; calls that overlap on one device race on the shared scratch.
hipError_t launch_histogram_noalloc(const uint8_t *img, uint64_t n, unsigned long long *d_out,
                                    hipStream_t s);

// The GEMM form of one step (or of the initial evaluation), and the binary64
// re-score of one row x (device, binary64) into out[0].
hipError_t launch_gemm_step(const Params &p, const GemmBufs &w, int init, hipStream_t s);

hipError_t launch_zero_u32(uint32_t *a, int n, hipStream_t s);
// One stage of it: 0 candidates, 1 product (BF16 estimate or binary32),
// 2 BF16 classification, 3 binary32 re-score product, 4 selection.
hipError_t launch_gemm_stage(const Params &p, const GemmBufs &w, int init, int stage,
                             hipStream_t s);
hipError_t launch_elite_f64(const Params &p, const GemmBufs &w, const double *x, double *out,
                            hipStream_t s);

// Batches: every run of a step launch has the same kernel shape
// (step_shape), one rank launch per precision.
hipError_t launch_rank_batch(const BatchLaunch &b, bool fp64, hipStream_t s);
hipError_t launch_step_batch(const Params &proto, bool fp64, const BatchLaunch &b, hipStream_t s);
// Launch geometry of a run (host side; shared by the runtime, the launchers
// and the CPU checks of the batch tables).

// The tiled step's lanes per protozoan and chunks per lane for a run (its
// own lane count when set, else the dimension's); -1 chunks if none fits.
inline int tile_lanes(const Params &p) { return p.lanes > 0 ? p.lanes : lanes_for_dim(p.dim); }
inline int tile_chunks(const Params &p) { return chunks_for(p.dim, tile_lanes(p)); }

// Rows (consecutive ranks) per workgroup of the tiled step: one MFMA row
// block of 16, or "wide" -- one row per lane group of the 512 threads --
// which fills every thread when the lane groups are small (fewer, fuller
// workgroups: the choice of batches and of very large populations).
inline int tile_rows(const Params &p) { return p.rows > 16 ? p.rows : 16; }

// The tiled step serves rotated objectives and the thresholding objectives.
inline bool tile_form(const Params &p) {
    return p.rotated || p.kind == K_KAPUR || p.kind == K_OTSU;
}

inline size_t tile_lds_bytes(const Params &p, bool fp64) {
    return tile_dynamic_lds(p.dim, tile_rows(p), fp64 ? 8 : 4);
}

// Protozoa ranked per workgroup of the register form of the sort.
constexpr int kRankPer = 8;

// Workgroups of a run's sort: 256 protozoa each in the LDS form, kRankPer
// in the register form.
inline int rank_blocks(const Params &p) {
    return p.rank_lds ? (p.pop + 255) / 256 : (p.pop + kRankPer - 1) / kRankPer;
}

// Workgroups of a run's step.
inline int step_blocks(const Params &p) {
    if (tile_form(p)) return (p.pop + tile_rows(p) - 1) / tile_rows(p);
    return (int)(((long long)p.pop * lanes_for_dim(p.dim) + 255) / 256);
}

// Dynamic LDS of a run's step launch.
inline size_t step_lds_bytes(const Params &p, bool fp64) {
    return tile_form(p) ? tile_lds_bytes(p, fp64) : 0;
}

// Dynamic LDS of the persistent elementwise launch: the run's LDS image.
inline size_t persist_lds_bytes(const Params &p, bool fp64) {
    return persist_image(p.pop, p.Dp, fp64 ? 8 : 4, p.kind == K_KAPUR || p.kind == K_OTSU).total;
}

// Whether a run takes the persistent form of apo_run (one workgroup running
// every iteration): the whole population in one workgroup of the step --
// the elementwise step's 256 threads, or one tile -- and a sort of one LDS
// workgroup; the elementwise form also holds the run's LDS image.
inline bool persist_form(const Params &p, bool fp64) {
    if (p.gemm || p.pop > 256) return false;
    if (tile_form(p)) return p.pop <= tile_rows(p);
    return (long long)p.pop * lanes_for_dim(p.dim) <= 256 &&
           persist_lds_bytes(p, fp64) + kPersistStaticLds <= kLdsLimit;
}

// Instantiation key: precision, form, lanes, chunks, rows and whether np > 1
// (equal keys: one kernel serves both runs).
inline int step_shape(const Params &p, bool fp64) {
    return tile_form(p) ? pack_shape(fp64, true, p.np > 1, tile_lanes(p), tile_chunks(p),
                                     tile_rows(p))
                        : pack_shape(fp64, false, p.np > 1, lanes_for_dim(p.dim),
                                     chunks_for_dim(p.dim), 0);
}

// Largest population the LDS form of the sort takes.
constexpr int kRankLdsMax = 1024;


}  // namespace apok
