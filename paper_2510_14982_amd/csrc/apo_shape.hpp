// apo_shape.hpp -- launch shapes of the step kernels: which (lanes per
// protozoan, 4-coordinate chunks per lane, rows per workgroup) are compiled,
// how a run's dimension maps onto one, the row strides of the workspace and
// the LDS a tiled launch needs.  Plain C++ with no HIP types, so the host
// runtime, the kernels and a CPU check of every shape share one definition.
#pragma once
#include <stddef.h>

#if defined(__HIPCC__)
#define APO_HD __host__ __device__
#else
#define APO_HD
#endif

// Every compiled shape of the tiled step (G lanes, NCH chunks, TM rows) and
// of the elementwise step (G lanes, NCH chunks): the launchers instantiate
// exactly these, and a run whose shape is not listed is refused at creation.
#define APO_TILE_SHAPES(X)                                                                  \
    X(4, 1, 16) X(8, 1, 16) X(16, 1, 16) X(32, 1, 16) X(64, 1, 16) X(64, 2, 16)            \
    X(4, 1, 128) X(8, 1, 64) X(16, 1, 32) X(4, 2, 128) X(4, 4, 128) X(8, 4, 64)
#define APO_ELEM_SHAPES(X) X(4, 1) X(8, 1) X(16, 1) X(32, 1) X(64, 1) X(64, 2) X(64, 4)

namespace apok {

constexpr int kTileThreads = 512;          // threads of a tiled-step workgroup
constexpr size_t kLdsLimit = 163840;       // LDS one workgroup may hold on gfx950 (160 KiB)

// Lanes per protozoan for a dimension: a power of two from 4 to 64 covering
// ceil(D / 4) lanes of four coordinates, capped at one wavefront.
APO_HD inline int lanes_for_dim(int dim) {
    const int need = (dim + 3) / 4;
    int g = 4;
    while (g < need && g < 64) g <<= 1;
    return g;
}

// Chunks of four coordinates per lane for G lanes: 1, 2 or 4 (-1: none fits).
APO_HD inline int chunks_for(int dim, int G) {
    const int c = (dim + 4 * G - 1) / (4 * G);
    return c <= 1 ? 1 : c <= 2 ? 2 : c <= 4 ? 4 : -1;
}
APO_HD inline int chunks_for_dim(int dim) { return chunks_for(dim, lanes_for_dim(dim)); }

// Rows of a "wide" tile: one row per lane group of the 512 threads (at least
// one MFMA row block of 16).
constexpr int tile_rows_wide(int G) { return kTileThreads / G > 16 ? kTileThreads / G : 16; }

// Workspace row stride (elements: rows start on 64 bytes), output column
// tiles of 16 and k-steps of 4 padded to a multiple of 8 (the matrix-core
// loop runs unguarded in blocks of 8 over zero padding).
inline int row_stride(int dim, int es) { return (dim + 64 / es - 1) / (64 / es) * (64 / es); }
inline int col_tiles(int dim) { return (dim + 15) / 16; }
inline int k_steps(int dim) { return ((dim + 3) / 4 + 7) / 8 * 8; }

// LDS row stride (elements) of the tile's row buffers.  The matrix-core A
// operand is read as 16-byte vectors by 16 lanes of 16 different rows at a
// time; a stride of an odd number of 16-byte units puts those rows in 16
// distinct groups of four banks.  Rows are also written as 16-byte vectors.
APO_HD inline int tile_row_stride(int Dp, int Ks, int es) {
    const int w = Dp > 4 * Ks ? Dp : 4 * Ks;
    const int per = 16 / es;                      // elements per 16 bytes
    int q = (w + per - 1) / per;
    if ((q & 1) == 0) ++q;
    return q * per;
}

// Dynamic LDS of a tiled launch: candidates, own rows and A = y - o
// [TM][LS] each, Zs [TM][max(16 Nt + 1, D + 1)], two partial sums [TM][Nt].
inline size_t tile_dynamic_lds(int dim, int TM, int es) {
    const size_t LS = (size_t)tile_row_stride(row_stride(dim, es), k_steps(dim), es);
    const size_t Nt = (size_t)col_tiles(dim), LZ = Nt * 16 + 1;
    const size_t zwords = (size_t)TM * LZ > (size_t)TM * ((size_t)dim + 1)
                              ? (size_t)TM * LZ : (size_t)TM * ((size_t)dim + 1);
    return (3 * (size_t)TM * LS + zwords + 2 * (size_t)TM * Nt) * (size_t)es;
}

// Static LDS of the tiled step body: ids and operations [TM], a mask bitmap
// per lane group, old and new fitness [TM].
inline size_t tile_static_lds(int G, int NCH, int TM, int es) {
    const size_t groups = (size_t)(kTileThreads / G), words = (size_t)((4 * G * NCH + 31) / 32);
    return 2 * 4 * (size_t)TM + 4 * groups * words + 2 * (size_t)es * (size_t)TM;
}

inline bool tile_shape_built(int G, int NCH, int TM) {
#define APO_SHAPE_IS(g, c, t) \
    if (G == (g) && NCH == (c) && TM == (t)) return true;
    APO_TILE_SHAPES(APO_SHAPE_IS)
#undef APO_SHAPE_IS
    return false;
}

inline bool elem_shape_built(int G, int NCH) {
#define APO_SHAPE_IS(g, c) \
    if (G == (g) && NCH == (c)) return true;
    APO_ELEM_SHAPES(APO_SHAPE_IS)
#undef APO_SHAPE_IS
    return false;
}

// A tiled shape the library can launch for this dimension: compiled, and
// its LDS fits one workgroup.
inline bool tile_shape_ok(int dim, int G, int NCH, int TM, int es) {
    if (NCH < 1 || !tile_shape_built(G, NCH, TM)) return false;
    if (4 * G * NCH < dim) return false;          // every coordinate has a lane
    return tile_dynamic_lds(dim, TM, es) + tile_static_lds(G, NCH, TM, es) <= kLdsLimit;
}

// LDS image of a run in the persistent form of apo_run (elementwise step),
// which keeps the run's state there for the whole launch: both position
// buffers [pop][Dp], fitness by id and by rank, the order and the Dr flags,
// and the read-only per-run tables the iterations read (p_dr by rank,
// bounds, shift and, for the thresholding objectives, the 3 x 257 histogram
// tables).  Byte offsets
// from the image's base, each 16-byte aligned.
struct PersistImage {
    size_t x0, x1, f, fs, perm, drf, pdr, lb, ub, sh, htab, total;
};

APO_HD inline PersistImage persist_image(int pop, int Dp, int es, bool hist) {
    PersistImage m;
    size_t o = 0;
    const size_t xb = ((size_t)pop * Dp * es + 15) / 16 * 16;
    const size_t fb = ((size_t)pop * es + 15) / 16 * 16, db = ((size_t)Dp * es + 15) / 16 * 16;
    m.x0 = o; o += xb;
    m.x1 = o; o += xb;
    m.f = o; o += fb;
    m.fs = o; o += fb;
    m.perm = o; o += ((size_t)pop * 4 + 15) / 16 * 16;
    m.drf = o; o += ((size_t)pop + 15) / 16 * 16;
    m.pdr = o; o += ((size_t)pop * 8 + 15) / 16 * 16;
    m.lb = o; o += db;
    m.ub = o; o += db;
    m.sh = o; o += db;
    m.htab = o; o += hist ? (size_t)3 * 257 * 8 : 0;
    m.total = o;
    return m;
}

// Static LDS of the persistent form's sort (the LDS form: 1024 keys and the
// iteration's subset keys) and a margin for the elementwise step's masks.
constexpr size_t kPersistStaticLds = 16384;

// Lanes per protozoan a run takes inside a batch (0: the dimension's own
// count), with one row per lane group.  Rotated separable objectives take
// four lanes up to 64 dimensions and eight up to 128 (64- or 128-row tiles,
// up to four chunks a lane) when that tile fits the LDS (in binary64 it
// does not above 32 dimensions); their results do not depend on the lane
// count (elementwise candidates, set-valued masks, the objective summed from
// the matrix-core tiles in a fixed order).  Rosenbrock's lane sums would
// change with it, so it keeps its own count.
inline int batch_lanes(int dim, bool rotated, bool rosenbrock, int es) {
    if (!rotated || rosenbrock) return 0;
    const int G = (dim > 16 && dim <= 64) ? 4 : (dim > 64 && dim <= 128) ? 8 : 0;
    if (G == 0 || !tile_shape_ok(dim, G, chunks_for(dim, G), tile_rows_wide(G), es)) return 0;
    return G;
}

// Instantiation key of a step launch: equal keys can share one launch.
// Fields: bit 0 binary64, bit 1 tiled form, bit 2 np > 1, bits 3-10 lanes,
// bits 11-14 chunks, bits 15-23 rows; -1 if a field does not fit.
inline int pack_shape(bool fp64, bool tiled, bool np_gt1, int G, int NCH, int TM) {
    if (G < 1 || G > 255 || NCH < 1 || NCH > 15 || TM < 0 || TM > 511) return -1;
    return (fp64 ? 1 : 0) | (tiled ? 2 : 0) | (np_gt1 ? 4 : 0) | (G << 3) | (NCH << 11) |
           (TM << 15);
}

}  // namespace apok
