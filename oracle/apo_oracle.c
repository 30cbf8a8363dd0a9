/*
 * apo_oracle.c -- plain, slow, single-threaded FP64 CPU oracle for the
 * Artificial Protozoa Optimizer (APO) population step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no source with the HIP path: it
 * has its own Philox, its own subset permutation, its own objectives and its
 * own sort.
 *
 * What it follows (paper: "cuAPO: A CUDA-based Parallelization of
 * Artificial Protozoa Optimizer"):
 *   - Section 3 (APO): Eqs. (1)-(13) for dormancy, reproduction, the two
 *     foraging modes, their weights, masks and the operation probabilities.
 *   - Algorithm 1 (Section 4): the per-iteration order sort -> pf -> Dr ->
 *     per-protozoan update -> evaluate -> greedy select.
 *   - Section 4.1 (worked example): bounds are enforced by saturation and
 *     the selection is greedy.
 * Where the paper is silent or garbled the reading taken is stated next to
 * the code that implements it (they are the same readings the GPU library
 * takes, listed in the design notes).
 *
 * Random draws: both implementations consume the same counter-based stream,
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11), addressed by (purpose, block, index, iteration,
 * run) with the seed as key.  Exact m-subsets ("randperm(n, m)" in Eqs. (3),
 * (5) and Algorithm 1) come from a keyed alternating Feistel network on
 * ceil(log2 n) bits.  The dormancy/reproduction set Dr holds the ranks x
 * with pi(x) < m, pi being the network cycle-walked onto [0, n) (Black &
 * Rogaway, "Ciphers with arbitrary finite domains", CT-RSA 2002), so one
 * rank is tested on its own.  A coordinate mask holds the first m values
 * below n met along the network's own order of the whole 2^b domain.
 *
 * Everything is IEEE binary64, evaluated in the order the formulas are
 * written; the file is compiled with -ffp-contract=off.
 *
 * Threads: the protozoa of one iteration are independent given the
 * population at the start of the iteration (the synchronous reading of
 * Algorithm 1's parallel loop), so the per-rank candidates and the
 * evaluations may be spread over OpenMP threads (oracle_set_threads); every
 * value is computed by the same code in the same order whatever the thread
 * count, so results are bit-identical.  The default is one thread.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------ */
/* Problem description (owned by the caller)                           */
/* ------------------------------------------------------------------ */
enum { OR_SPHERE = 0, OR_RASTRIGIN = 1, OR_ROSENBROCK = 2, OR_ACKLEY = 3,
       OR_KAPUR = 4, OR_OTSU = 5 };
enum { OR_DORMANCY = 0, OR_REPRODUCTION = 1, OR_AUTOTROPH = 2,
       OR_HETEROTROPH = 3 };

typedef struct {
    int32_t dim;            /* D                                  */
    int32_t pop;            /* ps                                 */
    int32_t np;             /* neighbour pairs                    */
    int32_t max_iter;       /* iter_max (T)                       */
    double pf_max;          /* Eq. (11)                           */
    uint64_t seed;          /* Philox key                         */
    uint32_t run;           /* Philox counter word 3              */
    int32_t kind;           /* objective                          */
    const double *lb, *ub;  /* [dim] X_min, X_max                 */
    const double *shift;    /* [dim] or NULL (o = 0)              */
    const double *rot;      /* [dim*dim] row-major or NULL        */
    const uint64_t *hist;   /* [256] for Kapur / Otsu             */
    int32_t pdr_plus;       /* 1: Eq. (13) with the opposite sign  */
} oracle_problem;

/* Optional per-step record, every array indexed by protozoan id except
 * perm (indexed by rank).  nb holds, per id, 1 + 2*np neighbour ranks:
 * autotroph [j, k-_1, k+_1, ...], heterotroph [-1, a_1, b_1, ...],
 * -1 where unused. */
typedef struct {
    double *Y;        /* [pop*dim] candidate after the bound clamp   */
    double *Fy;       /* [pop] objective of the candidate            */
    int32_t *op;      /* [pop] operation code                        */
    int32_t *perm;    /* [pop] rank -> id                            */
    int32_t *mcount;  /* [pop] size of the mask (M_f or M_r), D for dormancy */
    int32_t *nb;      /* [pop*(1+2np)]                               */
    uint8_t *accepted;/* [pop] 1 if the candidate replaced the row   */
    int32_t *dr_count;/* [1] |Dr|                                    */
} oracle_trace;

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11): 10 rounds of two 32x32->64 multiplies, the  */
/* key bumped by the Weyl constants between rounds.                   */
/* ------------------------------------------------------------------ */
OR_EXPORT void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                                    uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter layout: word0 = purpose << 24 | block, word1 = index (id or
 * rank), word2 = iteration, word3 = run. */
enum { TAG_INIT = 1, TAG_ITER = 2, TAG_RANK = 3, TAG_ELEM = 4 };

static void draw_block(const oracle_problem *p, uint32_t tag, uint32_t block,
                       uint32_t index, uint32_t iter, uint32_t out[4])
{
    uint32_t ctr[4] = { (tag << 24) | block, index, iter, p->run };
    uint32_t key[2] = { (uint32_t)(p->seed & 0xFFFFFFFFu), (uint32_t)(p->seed >> 32) };
    oracle_philox4x32_10(ctr, key, out);
}

/* One 32-bit word of a counter stream: word q of the sequence that starts
 * at block b0 (block b0 + q/4, word q%4). */
static uint32_t draw_word(const oracle_problem *p, uint32_t tag, uint32_t b0,
                          uint32_t q, uint32_t index, uint32_t iter)
{
    uint32_t w[4];
    draw_block(p, tag, b0 + q / 4, index, iter, w);
    return w[q % 4];
}

/* "rand": a uniform number on the open interval (0, 1) built from the top
 * 23 bits k of a word as (k + 1/2) / 2^23, i.e. (2k + 1) / 2^24: 24
 * significant bits, so exactly representable in binary32 and binary64. */
OR_EXPORT double oracle_uniform(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) / 8388608.0;
}

/* A uniform integer in [0, n): floor(w * n / 2^32). */
OR_EXPORT uint32_t oracle_bounded(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

/* ------------------------------------------------------------------ */
/* Keyed bijection of [0, n) (randperm in Eqs. (3), (5), Algorithm 1). */
/*                                                                      */
/* An alternating (unbalanced) Feistel network on b = max(2,            */
/* ceil(log2 n)) bits, cycle-walked onto [0, n).  x = L * 2^c + R with  */
/* L of a = b - floor(b/2) bits and R of c = floor(b/2) bits; a round   */
/* maps (L, R) to (R, L xor f_i(R)) and swaps the widths.  Small        */
/* domains need more rounds to mix, so the round count depends on b:    */
/* 24 (b <= 4), 20 (b = 5, 6), 16 (b = 7), 12 (b = 8, 9), 8 (b >= 10).  */
/* For b <= 6 the round function is a table read from the round key     */
/* (f_i(R) = bits [a R, a R + a) of k_i); above, it is the top a bits   */
/* of a 24 x 24-bit product.  Keys 0..7 come from two Philox blocks;    */
/* key i >= 8 is derived from keys i-8 and i-7.                          */
/* ------------------------------------------------------------------ */
static uint32_t feistel_rounds(uint32_t bits)
{
    if (bits <= 4) return 24;
    if (bits <= 6) return 20;
    if (bits <= 7) return 16;
    if (bits <= 9) return 12;
    return 8;
}

static void feistel_keys(const uint32_t keys8[8], uint32_t *k, uint32_t rounds)
{
    for (uint32_t i = 0; i < 8; ++i)
        k[i] = keys8[i];
    for (uint32_t i = 8; i < rounds; ++i) {
        uint32_t x = k[i - 8] ^ (k[i - 7] >> 16) ^ i;
        x = x * 0x7FEB352Du;
        x = x ^ (x >> 15);
        k[i] = x;
    }
}

static uint32_t feistel_once(uint32_t x, uint32_t bits, const uint32_t *k, uint32_t rounds)
{
    uint32_t a = bits - bits / 2;   /* width of the left half  */
    uint32_t c = bits / 2;          /* width of the right half */
    uint32_t L = x >> c;
    uint32_t R = x & ((1u << c) - 1u);
    for (uint32_t i = 0; i < rounds; ++i) {
        uint32_t f;
        if (bits <= 6) {
            f = (k[i] >> (a * R)) & ((1u << a) - 1u);
        } else {
            uint32_t spread = (R << (24u - c)) ^ (k[i] >> 8);      /* < 2^24 */
            uint32_t mult = (k[i] & 0xFFFFFFu) | 1u;               /* < 2^24 */
            f = (uint32_t)(spread * mult) >> (32u - a);            /* top a bits */
        }
        uint32_t newL = R;
        uint32_t newR = L ^ f;
        L = newL;
        R = newR;
        uint32_t tmp = a; a = c; c = tmp;                          /* widths swap */
    }
    return (L << c) | R;
}

OR_EXPORT uint32_t oracle_subset_pi(uint32_t x, uint32_t n, const uint32_t keys[8])
{
    uint32_t bits = 2;
    while (bits < 32 && (1ull << bits) < (uint64_t)n)
        ++bits;
    uint32_t rounds = feistel_rounds(bits);
    uint32_t k[24];
    feistel_keys(keys, k, rounds);
    uint32_t y = feistel_once(x, bits, k, rounds);
    while (y >= n)
        y = feistel_once(y, bits, k, rounds);
    return y;
}

/* Is element x of [0, n) in the m-subset keyed by keys? (the set Dr) */
static int in_subset(uint32_t x, uint32_t n, uint32_t m, const uint32_t keys[8])
{
    return oracle_subset_pi(x, n, keys) < m;
}

/* The m-subset of the coordinates [0, n) for a mask (M_r of Eq. (3), M_f
 * of Eq. (5)): walk v = 0, 1, ..., 2^b - 1, apply one pass of the network
 * (no cycle walking) and keep the first m results below n.  Exactly m
 * members; every m-subset is equally likely when the pass is a random
 * permutation of [0, 2^b).  member[x] = 1 for members, 0 otherwise. */
OR_EXPORT void oracle_subset_mask(uint32_t n, uint32_t m, const uint32_t keys[8],
                                  uint8_t *member)
{
    uint32_t bits = 2;
    while (bits < 32 && (1ull << bits) < (uint64_t)n)
        ++bits;
    uint32_t rounds = feistel_rounds(bits);
    uint32_t k[24];
    feistel_keys(keys, k, rounds);
    memset(member, 0, n);
    uint32_t taken = 0;
    for (uint64_t v = 0; v < (1ull << bits) && taken < m; ++v) {
        uint32_t y = feistel_once((uint32_t)v, bits, k, rounds);
        if (y < n) {
            member[y] = 1;
            ++taken;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Objectives                                                         */
/* ------------------------------------------------------------------ */

/* z = M (x - o), written out as a plain matrix-vector product; M is
 * row-major, so z_i = sum_j M[i][j] (x_j - o_j). */
static void transform(const oracle_problem *p, const double *x, double *z)
{
    int D = p->dim;
    double *v = (double *)malloc(sizeof(double) * (size_t)D);
    for (int j = 0; j < D; ++j)
        v[j] = x[j] - (p->shift ? p->shift[j] : 0.0);
    if (p->rot) {
        for (int i = 0; i < D; ++i) {
            double s = 0.0;
            for (int j = 0; j < D; ++j)
                s += p->rot[(size_t)i * D + j] * v[j];
            z[i] = s;
        }
    } else {
        for (int i = 0; i < D; ++i)
            z[i] = v[i];
    }
    free(v);
}

static const double OR_PI = 3.14159265358979323846;
static const double OR_E = 2.71828182845904523536;

/* Kapur's entropy criterion (Kapur, Sahoo, Wong 1985) for k thresholds,
 * negated so that minimisation maximises the summed class entropies.
 * Each candidate coordinate is rounded half-to-even to a grey level; the
 * sorted levels b_1..b_k cut [0, 256) into classes [b_c, b_{c+1}); a level
 * equal to a threshold belongs to the upper class; an empty class adds 0. */
static double kapur(const oracle_problem *p, const double *x)
{
    int k = p->dim;
    int *t = (int *)malloc(sizeof(int) * (size_t)(k + 2));
    t[0] = 0;
    for (int c = 0; c < k; ++c)
        t[c + 1] = (int)rint(x[c]);
    t[k + 1] = 256;
    /* plain insertion sort of the k thresholds */
    for (int i = 2; i <= k; ++i)
        for (int j = i; j > 1 && t[j - 1] > t[j]; --j) {
            int s = t[j - 1]; t[j - 1] = t[j]; t[j] = s;
        }
    double N = 0.0;
    for (int g = 0; g < 256; ++g)
        N += (double)p->hist[g];
    double total = 0.0;
    for (int c = 0; c <= k; ++c) {
        double omega = 0.0;
        for (int g = t[c]; g < t[c + 1]; ++g)
            omega += (double)p->hist[g] / N;
        double H = 0.0;
        if (omega > 0.0) {
            for (int g = t[c]; g < t[c + 1]; ++g) {
                double pg = (double)p->hist[g] / N;
                if (pg > 0.0) {
                    double q = pg / omega;
                    H -= q * log(q);
                }
            }
        }
        total += H;
    }
    free(t);
    return -total;
}

/* Otsu's between-class variance for k thresholds (same class convention),
 * negated for minimisation. */
static double otsu(const oracle_problem *p, const double *x)
{
    int k = p->dim;
    int *t = (int *)malloc(sizeof(int) * (size_t)(k + 2));
    t[0] = 0;
    for (int c = 0; c < k; ++c)
        t[c + 1] = (int)rint(x[c]);
    t[k + 1] = 256;
    for (int i = 2; i <= k; ++i)
        for (int j = i; j > 1 && t[j - 1] > t[j]; --j) {
            int s = t[j - 1]; t[j - 1] = t[j]; t[j] = s;
        }
    double N = 0.0;
    for (int g = 0; g < 256; ++g)
        N += (double)p->hist[g];
    double muT = 0.0;
    for (int g = 0; g < 256; ++g)
        muT += (double)g * ((double)p->hist[g] / N);
    double sigma = 0.0;
    for (int c = 0; c <= k; ++c) {
        double omega = 0.0, m1 = 0.0;
        for (int g = t[c]; g < t[c + 1]; ++g) {
            double pg = (double)p->hist[g] / N;
            omega += pg;
            m1 += (double)g * pg;
        }
        if (omega > 0.0) {
            double mu = m1 / omega;
            sigma += omega * (mu - muT) * (mu - muT);
        }
    }
    free(t);
    return -sigma;
}

OR_EXPORT double oracle_objective(const oracle_problem *p, const double *x)
{
    if (p->kind == OR_KAPUR)
        return kapur(p, x);
    if (p->kind == OR_OTSU)
        return otsu(p, x);
    int D = p->dim;
    double *z = (double *)malloc(sizeof(double) * (size_t)D);
    transform(p, x, z);
    double f = 0.0;
    if (p->kind == OR_SPHERE) {                        /* Eq. (14) */
        for (int d = 0; d < D; ++d)
            f += z[d] * z[d];
    } else if (p->kind == OR_RASTRIGIN) {
        for (int d = 0; d < D; ++d)
            f += z[d] * z[d] - 10.0 * cos(2.0 * OR_PI * z[d]) + 10.0;
    } else if (p->kind == OR_ROSENBROCK) {
        /* textbook form on z + 1, so the minimum sits at x = o */
        for (int d = 0; d + 1 < D; ++d) {
            double a = z[d] + 1.0, b = z[d + 1] + 1.0;
            f += 100.0 * (b - a * a) * (b - a * a) + (a - 1.0) * (a - 1.0);
        }
    } else if (p->kind == OR_ACKLEY) {
        double s2 = 0.0, sc = 0.0;
        for (int d = 0; d < D; ++d) {
            s2 += z[d] * z[d];
            sc += cos(2.0 * OR_PI * z[d]);
        }
        f = -20.0 * exp(-0.2 * sqrt(s2 / D)) - exp(sc / D) + 20.0 + OR_E;
    } else {
        f = NAN;
    }
    free(z);
    return f;
}

/* ------------------------------------------------------------------ */
/* Fitness order used by the sort: ascending, -0 equal to +0, NaN after */
/* everything, equal values ordered by id.                             */
/* ------------------------------------------------------------------ */
/* the array qsort's comparator reads; one per calling thread, so that
 * concurrent calls from several host threads do not see each other's */
static _Thread_local const double *g_sort_F;

static int fitness_less(double a, int ia, double b, int ib)
{
    int na = isnan(a), nb = isnan(b);
    if (na != nb)
        return nb;            /* the non-NaN one comes first */
    if (!na && a != b)        /* -0 == +0 under != */
        return a < b;
    return ia < ib;
}

static int cmp_ids(const void *pa, const void *pb)
{
    int ia = *(const int32_t *)pa, ib = *(const int32_t *)pb;
    if (fitness_less(g_sort_F[ia], ia, g_sort_F[ib], ib)) return -1;
    if (fitness_less(g_sort_F[ib], ib, g_sort_F[ia], ia)) return 1;
    return 0;
}

OR_EXPORT void oracle_rank_order(int32_t pop, const double *F, int32_t *perm)
{
    for (int i = 0; i < pop; ++i)
        perm[i] = i;
    g_sort_F = F;
    qsort(perm, (size_t)pop, sizeof(int32_t), cmp_ids);
    g_sort_F = NULL;
}

/* ------------------------------------------------------------------ */
/* Initial population (Section 3.4: random values in the bounds, the    */
/* same form as Eq. (1)) and its evaluation (worked example, Step 1).  */
/* ------------------------------------------------------------------ */
OR_EXPORT void oracle_init(const oracle_problem *p, double *X, double *F)
{
    int D = p->dim;
#pragma omp parallel for schedule(static)
    for (int id = 0; id < p->pop; ++id) {
        for (int d = 0; d < D; ++d) {
            uint32_t w = draw_word(p, TAG_INIT, 0, (uint32_t)d, (uint32_t)id, 0);
            double u = oracle_uniform(w);
            X[(size_t)id * D + d] = p->lb[d] + u * (p->ub[d] - p->lb[d]);
        }
        F[id] = oracle_objective(p, &X[(size_t)id * D]);
    }
}

/* ------------------------------------------------------------------ */
/* Step 4-6 of the worked example: clamp to the bounds, evaluate, keep  */
/* the better of old and new.  Y holds candidates by id and is clamped  */
/* in place.                                                            */
/* ------------------------------------------------------------------ */
OR_EXPORT void oracle_finish(const oracle_problem *p, double *X, double *F, double *Y,
                             double *Fy, uint8_t *accepted)
{
    int D = p->dim;
#pragma omp parallel for schedule(static)
    for (int id = 0; id < p->pop; ++id) {
        double *y = &Y[(size_t)id * D];
        for (int d = 0; d < D; ++d)        /* saturate: 13.53 -> 10 in the example */
            y[d] = fmin(fmax(y[d], p->lb[d]), p->ub[d]);
        Fy[id] = oracle_objective(p, y);
    }
    for (int id = 0; id < p->pop; ++id) {
        /* greedy: the new position wins only if strictly better */
        int acc = Fy[id] < F[id];
        if (acc) {
            memcpy(&X[(size_t)id * D], &Y[(size_t)id * D], sizeof(double) * (size_t)D);
            F[id] = Fy[id];
        }
        if (accepted)
            accepted[id] = (uint8_t)acc;
    }
}

/* ------------------------------------------------------------------ */
/* The random values one rank consumes in one iteration.  oracle_step   */
/* draws them from the Philox stream; oracle_step_scripted takes them   */
/* from the caller, so hand-worked cases can fix every draw and check   */
/* the update formulas value by value.                                  */
/* ------------------------------------------------------------------ */
#define OR_MAX_NP 8

typedef struct {
    int32_t in_dr;            /* the rank belongs to Dr (Algorithm 1)             */
    double u_op;              /* rand compared with p_dr (Eq. (13)) or p_ah (Eq. (12)) */
    double u_f;               /* rand of the foraging factor, Eq. (4)             */
    double u_rep;             /* rand of Eq. (2)                                  */
    double sgn;               /* the "+-" of Eqs. (2) and (9): +1 or -1           */
    int32_t j;                /* rank of X_j, Eq. (6)                             */
    int32_t km[OR_MAX_NP];    /* ranks k- of the pairs of Eq. (6)                 */
    int32_t kp[OR_MAX_NP];    /* ranks k+ of the pairs of Eq. (6)                 */
    const uint8_t *mask;      /* [dim] M_r of Eq. (3) or M_f of Eq. (5), 1 = in   */
    const double *U;          /* [dim] "Rand" of Eqs. (1), (2), (9)               */
} oracle_draws;

/* Which operation rank r (0-based; the paper's i = r + 1) performs in
 * iteration t: in Dr, dormancy when p_dr of Eq. (13) exceeds rand, else
 * reproduction; outside Dr, the autotrophic mode when p_ah of Eq. (12)
 * exceeds rand, else the heterotrophic mode. */
static int decide_op(const oracle_problem *p, int32_t t, int r, const oracle_draws *dw)
{
    const int ps = p->pop, i = r + 1, T = p->max_iter;
    if (dw->in_dr) {
        /* Eq. (13) as printed; the variant flips the sign in front of the
         * cosine (the reading that makes the worst ranks, not the best,
         * the likeliest to go dormant) */
        double c_dr = cos((1.0 - (double)i / (double)ps) * OR_PI);
        double p_dr = p->pdr_plus ? 0.5 * (1.0 + c_dr) : 0.5 * (1.0 - c_dr);
        return p_dr > dw->u_op ? OR_DORMANCY : OR_REPRODUCTION;
    }
    double p_ah = 0.5 * (1.0 + cos(((double)t / (double)T) * OR_PI));
    return p_ah > dw->u_op ? OR_AUTOTROPH : OR_HETEROTROPH;
}

/* The candidate of rank r for operation op (Eqs. (1), (2), (4), (6)-(10)),
 * before the bound clamp, from the population (X, F by id) as it stood
 * when the iteration began.  acc is [dim] scratch; nbrow (may be NULL)
 * receives the neighbour ranks. */
static void candidate(const oracle_problem *p, int32_t t, int r, int op, const int32_t *perm,
                      const double *X, const double *F, const oracle_draws *dw, double *acc,
                      double *y, int32_t *nbrow)
{
    const int D = p->dim, ps = p->pop, np = p->np, T = p->max_iter;
    const double eps = 2.220446049250313e-16;   /* 2^-52 */
    const double *xi = &X[(size_t)perm[r] * D];
    const double *U = dw->U;
    const uint8_t *mask = dw->mask;

    if (op == OR_DORMANCY) {
        /* Eq. (1): a fresh protozoan in the bounds */
        for (int d = 0; d < D; ++d)
            y[d] = p->lb[d] + U[d] * (p->ub[d] - p->lb[d]);
        return;
    }
    if (op == OR_REPRODUCTION) {
        /* Eq. (2): X_i +- rand (X_min + Rand (X_max - X_min)) on M_r */
        for (int d = 0; d < D; ++d) {
            if (mask[d]) {
                double R = p->lb[d] + U[d] * (p->ub[d] - p->lb[d]);
                y[d] = xi[d] + (dw->sgn * dw->u_rep) * R;
            } else {
                y[d] = xi[d];
            }
        }
        return;
    }
    /* foraging: the factor f of Eq. (4) */
    const double f_scale = 1.0 + cos(((double)t / (double)T) * OR_PI);
    const double fac = dw->u_f * f_scale;
    for (int d = 0; d < D; ++d)
        acc[d] = 0.0;
    if (op == OR_AUTOTROPH) {
        /* Eqs. (6), (7).  j is any rank; k- a strictly better rank (itself
         * for the best); k+ a strictly worse rank (itself for the worst). */
        if (nbrow)
            nbrow[0] = dw->j;
        for (int k = 1; k <= np; ++k) {
            const int km = dw->km[k - 1], kp = dw->kp[k - 1];
            if (nbrow) {
                nbrow[2 * k - 1] = km;
                nbrow[2 * k] = kp;
            }
            const int idm = perm[km], idp = perm[kp];
            double wa = exp(-fabs(F[idm] / (F[idp] + eps)));
            for (int d = 0; d < D; ++d)
                acc[d] = acc[d] + wa * (X[(size_t)idm * D + d] - X[(size_t)idp * D + d]);
        }
        const double *xj = &X[(size_t)perm[dw->j] * D];
        for (int d = 0; d < D; ++d) {
            if (mask[d])
                y[d] = xi[d] + fac * ((xj[d] - xi[d]) + acc[d] / (double)np);
            else
                y[d] = xi[d];
        }
        return;
    }
    /* heterotroph, Eqs. (8)-(10); ranks i-k and i+k are held inside
     * [1, ps] */
    const double near_scale = 1.0 - (double)t / (double)T;
    for (int k = 1; k <= np; ++k) {
        int a = r - k < 0 ? 0 : r - k;
        int b = r + k > ps - 1 ? ps - 1 : r + k;
        if (nbrow) {
            nbrow[2 * k - 1] = a;
            nbrow[2 * k] = b;
        }
        const int ida = perm[a], idb = perm[b];
        double wh = exp(-fabs(F[ida] / (F[idb] + eps)));
        for (int d = 0; d < D; ++d)
            acc[d] = acc[d] + wh * (X[(size_t)ida * D + d] - X[(size_t)idb * D + d]);
    }
    for (int d = 0; d < D; ++d) {
        if (mask[d]) {
            double xnear = (1.0 + (dw->sgn * U[d]) * near_scale) * xi[d];   /* Eq. (9) */
            y[d] = xi[d] + fac * ((xnear - xi[d]) + acc[d] / (double)np);
        } else {
            y[d] = xi[d];
        }
    }
}

/* Rank r's draws of iteration t from the Philox stream.  The scalars come
 * first, then the operation is decided, and only then the mask, whose
 * size depends on it: ceil(D rand) for reproduction (Eq. (3)), ceil(D i /
 * ps) for foraging (Eq. (5)).  mask and U are [dim] buffers owned by the
 * caller; returns the operation and the mask size. */
static int philox_draws(const oracle_problem *p, int32_t t, int r, int m_dr,
                        const uint32_t dr_keys[8], oracle_draws *dw, uint8_t *mask, double *U,
                        int *m_out)
{
    const int D = p->dim, ps = p->pop, np = p->np, i = r + 1;
    uint32_t s0[4], mkeys[8];
    draw_block(p, TAG_RANK, 0, (uint32_t)r, (uint32_t)t, s0);
    draw_block(p, TAG_RANK, 1, (uint32_t)r, (uint32_t)t, mkeys);
    draw_block(p, TAG_RANK, 2, (uint32_t)r, (uint32_t)t, mkeys + 4);
    memset(dw, 0, sizeof(*dw));
    dw->in_dr = in_subset((uint32_t)r, (uint32_t)ps, (uint32_t)m_dr, dr_keys);
    dw->u_op = oracle_uniform(s0[0]);
    dw->u_f = oracle_uniform(s0[1]);
    dw->u_rep = oracle_uniform(s0[2]);
    /* "+-": one fair sign per protozoan and use */
    dw->sgn = oracle_uniform(s0[3]) < 0.5 ? 1.0 : -1.0;
    dw->mask = mask;
    dw->U = U;
    const int op = decide_op(p, t, r, dw);

    int m = D;
    if (op == OR_REPRODUCTION) {
        double u_mr = oracle_uniform(draw_word(p, TAG_RANK, 3, 0, (uint32_t)r, (uint32_t)t));
        m = (int)ceil((double)D * u_mr);
    } else if (op != OR_DORMANCY) {
        m = (int)ceil((double)D * (double)i / (double)ps);
    }
    if (op != OR_DORMANCY)
        oracle_subset_mask((uint32_t)D, (uint32_t)m, mkeys, mask);
    if (op == OR_AUTOTROPH) {
        dw->j = (int)oracle_bounded(draw_word(p, TAG_RANK, 3, 1, (uint32_t)r, (uint32_t)t),
                                    (uint32_t)ps);
        for (int k = 1; k <= np; ++k) {
            uint32_t wm = draw_word(p, TAG_RANK, 3, (uint32_t)(2 * k), (uint32_t)r, (uint32_t)t);
            uint32_t wp = draw_word(p, TAG_RANK, 3, (uint32_t)(2 * k + 1), (uint32_t)r,
                                    (uint32_t)t);
            dw->km[k - 1] = (r == 0) ? r : (int)oracle_bounded(wm, (uint32_t)r);
            dw->kp[k - 1] = (r == ps - 1) ? r
                            : r + 1 + (int)oracle_bounded(wp, (uint32_t)(ps - 1 - r));
        }
    } else {
        /* Eqs. (1), (2), (9) read Rand on (a subset of) the coordinates */
        for (int d = 0; d < D; ++d)
            U[d] = oracle_uniform(draw_word(p, TAG_ELEM, 0, (uint32_t)d, (uint32_t)r,
                                            (uint32_t)t));
    }
    *m_out = m;
    return op;
}

/* ------------------------------------------------------------------ */
/* One iteration t (1-based) of Algorithm 1, synchronous: every         */
/* candidate is built from the population as it stood when the          */
/* iteration began.  script == NULL draws from the Philox stream;       */
/* otherwise script[r] holds rank r's draws (Dr membership included).   */
/* ------------------------------------------------------------------ */
static int step_impl(const oracle_problem *p, int32_t t, double *X, double *F,
                     const oracle_draws *script, oracle_trace *tr)
{
    const int D = p->dim, ps = p->pop, np = p->np, T = p->max_iter;
    if (t < 1 || t > T || np < 1 || np > OR_MAX_NP)
        return -1;

    /* Sort the protozoa by fitness (Algorithm 1).  perm[r] is the id of
     * rank r (0-based here; the paper's rank i is r + 1). */
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)ps);
    oracle_rank_order(ps, F, perm);

    /* pf = pf_max * rand (Eq. (11)); Dr = randperm(ps, ceil(ps * pf)). */
    uint32_t w_it[4], dr_keys[8];
    int m_dr = 0;
    if (!script) {
        draw_block(p, TAG_ITER, 0, 0, (uint32_t)t, w_it);
        draw_block(p, TAG_ITER, 1, 0, (uint32_t)t, dr_keys);
        draw_block(p, TAG_ITER, 2, 0, (uint32_t)t, dr_keys + 4);
        double pf = p->pf_max * oracle_uniform(w_it[0]);
        m_dr = (int)ceil((double)ps * pf);
    } else {
        for (int r = 0; r < ps; ++r)
            m_dr += script[r].in_dr ? 1 : 0;
    }
    if (tr && tr->dr_count)
        tr->dr_count[0] = m_dr;

    double *Y = (double *)malloc(sizeof(double) * (size_t)ps * D);

#pragma omp parallel
    {
        /* per-thread scratch: the pair sum, Rand and the mask of one rank */
        double *acc = (double *)malloc(sizeof(double) * (size_t)D);
        double *U = (double *)malloc(sizeof(double) * (size_t)D);
        uint8_t *mask = (uint8_t *)malloc((size_t)D);
#pragma omp for schedule(static)
        for (int r = 0; r < ps; ++r) {
            const int id = perm[r];
            int32_t *nbrow = tr && tr->nb ? &tr->nb[(size_t)id * (1 + 2 * np)] : NULL;
            if (nbrow)
                for (int q = 0; q < 1 + 2 * np; ++q)
                    nbrow[q] = -1;
            oracle_draws own;
            const oracle_draws *dw;
            int op, m;
            if (script) {
                dw = &script[r];
                op = decide_op(p, t, r, dw);
                m = D;
                if (op != OR_DORMANCY) {
                    m = 0;
                    for (int d = 0; d < D; ++d)
                        m += dw->mask[d] ? 1 : 0;
                }
            } else {
                op = philox_draws(p, t, r, m_dr, dr_keys, &own, mask, U, &m);
                dw = &own;
            }
            candidate(p, t, r, op, perm, X, F, dw, acc, &Y[(size_t)id * D], nbrow);
            if (tr && tr->op)
                tr->op[id] = op;
            if (tr && tr->mcount)
                tr->mcount[id] = m;
        }
        free(acc);
        free(U);
        free(mask);
    }

    double *Fy = (double *)malloc(sizeof(double) * (size_t)ps);
    oracle_finish(p, X, F, Y, Fy, tr ? tr->accepted : NULL);
    if (tr) {
        if (tr->Y)
            memcpy(tr->Y, Y, sizeof(double) * (size_t)ps * D);
        if (tr->Fy)
            memcpy(tr->Fy, Fy, sizeof(double) * (size_t)ps);
        if (tr->perm)
            memcpy(tr->perm, perm, sizeof(int32_t) * (size_t)ps);
    }
    free(Fy);
    free(Y);
    free(perm);
    return 0;
}

OR_EXPORT int oracle_step(const oracle_problem *p, int32_t t, double *X, double *F,
                          oracle_trace *tr)
{
    return step_impl(p, t, X, F, NULL, tr);
}

/* The same iteration with every draw supplied: script[r] (r = 0-based
 * rank after the sort) gives rank r's Dr membership, rands, sign,
 * neighbour ranks, mask and Rand vector.  Nothing is drawn. */
OR_EXPORT int oracle_step_scripted(const oracle_problem *p, int32_t t, double *X, double *F,
                                   const oracle_draws *script, oracle_trace *tr)
{
    if (!script)
        return -1;
    return step_impl(p, t, X, F, script, tr);
}

/* Threads the oracle's loops over protozoa use (n > 0 sets the count);
 * returns the count in effect (1 in a build without OpenMP). */
OR_EXPORT int32_t oracle_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
    return (int32_t)omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Best protozoan: the minimum in the sort order (lowest id on ties). */
OR_EXPORT int32_t oracle_best(int32_t pop, const double *F)
{
    int32_t best = 0;
    for (int32_t id = 1; id < pop; ++id)
        if (fitness_less(F[id], id, F[best], best))
            best = id;
    return best;
}

/* Iterations t0+1 .. t0+iters on (X, F); returns the last t. */
OR_EXPORT int32_t oracle_run(const oracle_problem *p, int32_t t0, int32_t iters, double *X,
                             double *F)
{
    int32_t t = t0;
    for (int32_t n = 0; n < iters && t < p->max_iter; ++n) {
        ++t;
        oracle_step(p, t, X, F, NULL);
    }
    return t;
}

/* 256-bin histogram of an 8-bit image. */
OR_EXPORT void oracle_histogram_u8(const uint8_t *img, uint64_t n, uint64_t hist[256])
{
    for (int g = 0; g < 256; ++g)
        hist[g] = 0;
    for (uint64_t i = 0; i < n; ++i)
        hist[img[i]] += 1;
}
