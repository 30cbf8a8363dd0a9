// apo_api.cpp -- host runtime behind include/apo.h: argument checks, the
// device workspace layout, the schedule tables, launches, HIP-graph replay,
// checkpoint/trace copies and status mapping.
#include "apo.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "apo_internal.h"

using apok::Ctrl;
using apok::Params;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxPop = 65536;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Offsets of every device array inside the workspace (bytes, 256-aligned).
struct Layout {
    size_t gYr, gAb, gan, gP1, gP2, glist, gstat, gcount, gtot, gMb, gMf, gMd, go64, gz64;   // GEMM form
    int Kp, Np;
    size_t X[2], F, perm, Fs, drf, ctrl, p_ah, fscale, cnear, p_dr, lb, ub, shift, rotp, htab, hist,
        best, trY, trF, trOp, total;
    int Dp, Nt, Ks;
};

bool is_threshold(int kind) { return kind == apok::K_KAPUR || kind == apok::K_OTSU; }

// The GEMM form serves rotated objectives of large dimension in binary32 and
// every BF16 handle.
bool gemm_form(int dim, const apo_options &o) {
    if (!o.objective.rot || is_threshold(o.objective.kind)) return false;
    return o.precision == APO_BF16 || (o.precision == APO_FP32 && dim > 512);
}

Layout make_layout(int dim, int pop, const apo_options &o) {
    Layout L;
    std::memset(&L, 0, sizeof(L));
    const size_t es = o.precision == APO_FP64 ? 8 : 4;
    L.Dp = apok::row_stride(dim, (int)es);
    L.Nt = apok::col_tiles(dim);
    L.Ks = apok::k_steps(dim);   // zero-padded so the matrix-core loop runs unguarded
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    for (int b = 0; b < 2; ++b) L.X[b] = take((size_t)pop * L.Dp * es);
    L.F = take((size_t)pop * es);
    L.perm = take((size_t)pop * 4);
    L.Fs = take((size_t)pop * es);
    L.drf = take((size_t)pop);
    L.ctrl = take(sizeof(Ctrl));
    L.p_ah = take((size_t)(o.max_iter + 1) * 8);
    L.fscale = take((size_t)(o.max_iter + 1) * 8);
    L.cnear = take((size_t)(o.max_iter + 1) * 8);
    L.p_dr = take((size_t)pop * 8);
    L.lb = take((size_t)L.Dp * es);
    L.ub = take((size_t)L.Dp * es);
    L.shift = take((size_t)L.Dp * es);
    const bool gf = gemm_form(dim, o);
    L.rotp = (o.objective.rot && !gf) ? take((size_t)L.Ks * L.Nt * 64 * es) : 0;
    if (gf) {
        L.Kp = (dim + 127) / 128 * 128;   // K in groups of four 32-K chunks (BF16 product)
        L.Np = (dim + 127) / 128 * 128;
        const bool bf = o.precision == APO_BF16;
        L.gYr = take((size_t)pop * L.Dp * 4);
        // BF16 A in fragment order, whole 256-row tiles of the product
        L.gAb = bf ? take((size_t)((pop + 255) / 256 * 256) * L.Kp * 2) : 0;
        L.gan = bf ? take((size_t)pop * 4) : 0;
        L.gP1 = take((size_t)pop * (L.Np / 64) * 4);
        L.gP2 = take((size_t)pop * (L.Np / 64) * 4);
        L.glist = take((size_t)pop * 4);
        L.gstat = take((size_t)pop * 4);
        L.gcount = take(4);
        L.gtot = take(8);
        L.gMb = bf ? take((size_t)L.Np * L.Kp * 2) : 0;
        L.gMf = take((size_t)L.Np * L.Kp * 4);
        L.gMd = take((size_t)dim * dim * 8);
        L.go64 = take((size_t)dim * 8);
        L.gz64 = take((size_t)dim * 8);
    }
    L.htab = is_threshold(o.objective.kind) ? take(3 * 257 * 8) : 0;
    L.hist = is_threshold(o.objective.kind) ? take(256 * 8) : 0;
    L.best = take((size_t)(dim + 1) * 8);
    if (o.flags & APO_FLAG_TRACE) {
        L.trY = take((size_t)pop * L.Dp * es);
        L.trF = take((size_t)pop * es);
        L.trOp = take((size_t)pop * 4);
    }
    L.total = off;
    return L;
}

// Rows per workgroup of a single handle's tiled step: wide tiles when the
// run alone still gives every CU a workgroup, or when one wide tile holds the
// whole run; else one MFMA row block.
int single_tile_rows(int dim, int pop, int es) {
    const int G = apok::lanes_for_dim(dim), wide = apok::tile_rows_wide(G);
    if (wide > 16 && pop >= 256 * wide) return wide;
    // one wide tile holds the whole run: the persistent form of apo_run
    if (wide > 16 && pop <= wide && pop <= 256 &&
        apok::tile_shape_ok(dim, G, apok::chunks_for(dim, G), wide, es))
        return wide;
    return 16;
}

int check_args(int32_t dim, const double *lb, const double *ub, int32_t pop, int32_t np,
               double pf_max, const apo_options *opt) {
    if (!opt || !lb || !ub) return APO_E_INVAL;
    if (dim < 1 || pop < 2 || np < 1 || np > apok::kMaxNp) return APO_E_INVAL;
    if (!(pf_max >= 0.0 && pf_max <= 1.0)) return APO_E_INVAL;
    if (opt->max_iter < 1) return APO_E_INVAL;
    if (opt->precision != APO_FP64 && opt->precision != APO_FP32 && opt->precision != APO_BF16)
        return APO_E_INVAL;
    const int kind = opt->objective.kind;
    if (kind < APO_SPHERE || kind > APO_OTSU) return APO_E_INVAL;
    if (opt->precision == APO_BF16 && !opt->objective.rot) return APO_E_INVAL;
    for (int d = 0; d < dim; ++d)
        if (!std::isfinite(lb[d]) || !std::isfinite(ub[d]) || !(lb[d] < ub[d])) return APO_E_INVAL;
    if (is_threshold(kind)) {
        if (!opt->objective.hist || opt->objective.shift || opt->objective.rot) return APO_E_INVAL;
        uint64_t total = 0;
        for (int g = 0; g < 256; ++g) total += opt->objective.hist[g];
        if (total == 0) return APO_E_INVAL;
        for (int d = 0; d < dim; ++d)
            if (lb[d] < 0.0 || ub[d] > 255.0) return APO_E_INVAL;
    } else {
        if (opt->objective.shift)
            for (int d = 0; d < dim; ++d)
                if (!std::isfinite(opt->objective.shift[d])) return APO_E_INVAL;
        if (opt->objective.rot)
            for (size_t i = 0; i < (size_t)dim * dim; ++i)
                if (!std::isfinite(opt->objective.rot[i])) return APO_E_INVAL;
    }
    // sizes the kernels are built for
    if (pop > kMaxPop) return APO_E_UNSUPPORTED;
    const bool tile = opt->objective.rot != nullptr || is_threshold(kind);
    if (gemm_form(dim, *opt)) {
        // separable objectives only (the row sums are taken per column tile)
        if (kind == APO_ROSENBROCK || apok::chunks_for_dim(dim) < 0) return APO_E_UNSUPPORTED;
    } else if (tile) {
        const int lim = is_threshold(kind) ? 512 : (opt->precision == APO_FP64 ? 256 : 512);
        if (dim > lim) return APO_E_UNSUPPORTED;
        const int G = apok::lanes_for_dim(dim);
        const int es = opt->precision == APO_FP64 ? 8 : 4;
        if (!apok::tile_shape_ok(dim, G, apok::chunks_for(dim, G), single_tile_rows(dim, pop, es),
                                 es))
            return APO_E_UNSUPPORTED;
    } else if (!apok::elem_shape_built(apok::lanes_for_dim(dim), apok::chunks_for_dim(dim))) {
        return APO_E_UNSUPPORTED;
    }
    return APO_OK;
}

// The tiled-step shape of a batch member: its batch lane count (or the
// dimension's), one row per lane group, the chunks that cover D.  APO_OK if
// the library has that kernel and its LDS fits, else APO_E_UNSUPPORTED.
struct MemberShape {
    int lanes;   // 0: the dimension's own count
    int G, NCH, rows;
};

int batch_member_shape(const apo_run_desc &d, MemberShape &m) {
    const bool rotated = d.opt.objective.rot != nullptr;
    const int es = d.opt.precision == APO_FP64 ? 8 : 4;
    m.lanes = apok::batch_lanes(d.dim, rotated, d.opt.objective.kind == APO_ROSENBROCK, es);
    m.G = m.lanes ? m.lanes : apok::lanes_for_dim(d.dim);
    m.NCH = apok::chunks_for(d.dim, m.G);
    m.rows = apok::tile_rows_wide(m.G);
    const bool tiled = rotated || is_threshold(d.opt.objective.kind);
    if (!tiled) return APO_OK;   // the elementwise step (shape checked by check_args)
    return apok::tile_shape_ok(d.dim, m.G, m.NCH, m.rows, es) ? APO_OK : APO_E_UNSUPPORTED;
}

template <typename T>
void to_device_row(std::vector<unsigned char> &buf, const double *src, int n, int padded) {
    buf.assign((size_t)padded * sizeof(T), 0);
    T *dst = reinterpret_cast<T *>(buf.data());
    for (int i = 0; i < n; ++i) dst[i] = src ? (T)src[i] : T(0);
}

template <typename T>
void rows_to_double(const unsigned char *src, double *dst, int rows, int dim, int Dp) {
    const T *s = reinterpret_cast<const T *>(src);
    for (int r = 0; r < rows; ++r)
        for (int d = 0; d < dim; ++d) dst[(size_t)r * dim + d] = (double)s[(size_t)r * Dp + d];
}

template <typename T>
void rows_from_double(const double *src, unsigned char *dst, int rows, int dim, int Dp) {
    T *o = reinterpret_cast<T *>(dst);
    for (int r = 0; r < rows; ++r)
        for (int d = 0; d < Dp; ++d) o[(size_t)r * Dp + d] = d < dim ? (T)src[(size_t)r * dim + d] : T(0);
}

}  // namespace

struct apo {
    Params p;
    Layout L;
    bool fp64;
    size_t es;
    int32_t dim, pop, T;
    uint32_t flags;
    hipStream_t stream;
    bool own_stream;
    unsigned char *ws;
    bool own_ws;
    int32_t t;            // host mirror of completed iterations
    bool poisoned;
    hipGraph_t graph[2];          // [0]: one iteration, [1]: kGraphBlock iterations
    hipGraphExec_t graph_exec[2];
    bool graph_tried;
    hipEvent_t ev[4];
    bool have_events;
    bool batch_view;      // a member of a batch: stepped only through the batch
};

#define APO_HIP(h, call)                       \
    do {                                       \
        if ((call) != hipSuccess) {            \
            (h)->poisoned = true;              \
            return APO_E_DEVICE;               \
        }                                      \
    } while (0)


static int destroy_impl(apo_t *h);

// ---------------------------------------------------------------------------
// Batches of runs.  Each member is an ordinary handle whose workspace is a
// slice of the batch workspace and whose stream is the batch stream; the
// batch adds a device table of the members' parameters, the (run, block)
// tables of its launches and the graphs that replay them.
// ---------------------------------------------------------------------------
struct BatchLaunchRec {
    bool rank;                // a sort launch (else a step launch)
    bool fp64;
    int32_t proto;            // a member whose kernel shape the launch uses
    std::vector<int> members; // runs covered, in member order
    size_t lds;
    int nblocks;
    size_t table_off;         // first entry of its (run, block) table
};

struct apo_batch {
    std::vector<apo_t *> runs;
    hipStream_t stream;
    bool own_stream;
    unsigned char *ws;
    bool own_ws;
    size_t runs_bytes;        // the members' workspaces (the state the tuner saves)
    Params *d_params;         // [n] members' parameters (in the workspace)
    int2 *d_blocks;           // (run, block) tables (in the workspace)
    size_t n_entries;
    std::vector<BatchLaunchRec> launches;
    std::vector<hipStream_t> side;     // parallel graph branches of the step launches
    hipEvent_t fork_ev;
    std::vector<hipEvent_t> join_ev;
    int schedule;             // bit 0: parallel step branches; bit 1: interleaved blocks
    hipGraph_t graph[2];
    hipGraphExec_t gexec[2];
    bool graphs_ready;
    bool poisoned;
};

namespace {

// Workspace layout of a batch: the members' workspaces, then the parameter
// table, then the block tables.
struct BatchLayout {
    std::vector<size_t> run_off, run_bytes;
    size_t runs_bytes, params_off, blocks_off, n_entries, total;
};

Params shape_params(const apo_run_desc &d) {
    Params p;
    std::memset(&p, 0, sizeof(p));
    p.dim = d.dim;
    p.pop = d.pop;
    p.np = d.np;
    p.kind = d.opt.objective.kind;
    p.rotated = d.opt.objective.rot != nullptr;
    return p;
}

int batch_layout(int32_t n, const apo_run_desc *runs, BatchLayout &B) {
    if (n < 1 || !runs) return APO_E_INVAL;
    B.run_off.resize(n);
    B.run_bytes.resize(n);
    size_t off = 0, entries = 0;
    for (int i = 0; i < n; ++i) {
        const apo_run_desc &d = runs[i];
        if (d.opt.stream || d.opt.workspace || d.opt.workspace_bytes) return APO_E_INVAL;
        const int chk = check_args(d.dim, d.lb, d.ub, d.pop, d.np, d.pf_max, &d.opt);
        if (chk != APO_OK) return chk;
        if (gemm_form(d.dim, d.opt)) return APO_E_UNSUPPORTED;   // not in batches
        MemberShape ms;
        const int shp = batch_member_shape(d, ms);
        if (shp != APO_OK) return shp;
        const Layout L = make_layout(d.dim, d.pop, d.opt);
        B.run_off[i] = off;
        B.run_bytes[i] = L.total;
        off = align_up(off + L.total, 256);
        const Params sp = shape_params(d);
        entries += (size_t)apok::rank_blocks(sp) + (size_t)apok::step_blocks(sp);
    }
    B.runs_bytes = off;
    B.params_off = off;
    off = align_up(off + (size_t)n * sizeof(Params), 256);
    B.blocks_off = off;
    B.n_entries = entries;
    B.total = align_up(off + entries * sizeof(int2), 256);
    return APO_OK;
}

// The launches of one iteration: a sort per precision, then a step per
// kernel shape, each over its members in member order.
void batch_group_launches(apo_batch *b) {
    b->launches.clear();
    const int n = (int)b->runs.size();
    for (int prec = 0; prec < 2; ++prec) {
        BatchLaunchRec r{};
        r.rank = true;
        r.fp64 = prec == 1;
        for (int i = 0; i < n; ++i)
            if (b->runs[i]->fp64 == r.fp64) r.members.push_back(i);
        if (r.members.empty()) continue;
        r.proto = r.members[0];
        b->launches.push_back(r);
    }
    std::vector<int> shapes;
    for (int i = 0; i < n; ++i) {
        const int sh = apok::step_shape(b->runs[i]->p, b->runs[i]->fp64);
        bool seen = false;
        for (int x : shapes) seen = seen || x == sh;
        if (!seen) shapes.push_back(sh);
    }
    for (int sh : shapes) {
        BatchLaunchRec r{};
        r.rank = false;
        for (int i = 0; i < n; ++i)
            if (apok::step_shape(b->runs[i]->p, b->runs[i]->fp64) == sh) r.members.push_back(i);
        r.proto = r.members[0];
        r.fp64 = b->runs[r.proto]->fp64;
        for (int i : r.members) {
            const size_t l = apok::step_lds_bytes(b->runs[i]->p, b->runs[i]->fp64);
            if (l > r.lds) r.lds = l;
        }
        b->launches.push_back(r);
    }
}

// (run, block) tables of every launch for a schedule: run order (each run's
// blocks together) or interleaved (block 0 of every run, then block 1, ...).
int batch_fill_tables(apo_batch *b, int schedule) {
    std::vector<int2> host;
    host.reserve(b->n_entries);
    for (BatchLaunchRec &r : b->launches) {
        r.table_off = host.size();
        std::vector<int> nb;
        int most = 0;
        for (int i : r.members) {
            const Params &p = b->runs[i]->p;
            nb.push_back(r.rank ? apok::rank_blocks(p) : apok::step_blocks(p));
            if (nb.back() > most) most = nb.back();
        }
        if (schedule & 2) {
            for (int k = 0; k < most; ++k)
                for (size_t m = 0; m < r.members.size(); ++m)
                    if (k < nb[m]) host.push_back(make_int2(r.members[m], k));
        } else {
            for (size_t m = 0; m < r.members.size(); ++m)
                for (int k = 0; k < nb[m]; ++k) host.push_back(make_int2(r.members[m], k));
        }
        r.nblocks = (int)(host.size() - r.table_off);
    }
    if (host.size() > b->n_entries) return APO_E_STATE;
    if (hipMemcpyAsync(b->d_blocks, host.data(), host.size() * sizeof(int2),
                       hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        b->poisoned = true;
        return APO_E_DEVICE;
    }
    return APO_OK;
}

// Enqueues `iters` iterations under the current schedule (on the batch
// stream, or captured from it).
hipError_t batch_enqueue(apo_batch *b, int32_t iters) {
    const bool fork = (b->schedule & 1) != 0;
    for (int32_t it = 0; it < iters; ++it) {
        size_t k = 0;
        for (const BatchLaunchRec &r : b->launches) {
            apok::BatchLaunch bl;
            bl.runs = b->d_params;
            bl.blocks = b->d_blocks + r.table_off;
            bl.nblocks = r.nblocks;
            bl.lds = r.lds;
            hipError_t e;
            if (r.rank) {
                e = apok::launch_rank_batch(bl, r.fp64, b->stream);
                if (e != hipSuccess) return e;
                continue;
            }
            if (!fork) {
                e = apok::launch_step_batch(b->runs[r.proto]->p, r.fp64, bl, b->stream);
                if (e != hipSuccess) return e;
                continue;
            }
            if (k == 0) {
                e = hipEventRecord(b->fork_ev, b->stream);
                if (e != hipSuccess) return e;
            }
            e = hipStreamWaitEvent(b->side[k], b->fork_ev, 0);
            if (e == hipSuccess) {
                ++k;   // side stream k has joined the fork: it must be joined back
                e = apok::launch_step_batch(b->runs[r.proto]->p, r.fp64, bl, b->side[k - 1]);
            }
            if (e == hipSuccess) e = hipEventRecord(b->join_ev[k - 1], b->side[k - 1]);
            if (e != hipSuccess) {
                // join every forked branch back (a capture must not end with
                // unjoined work) and report the first error
                for (size_t j = 0; j < k; ++j) {
                    (void)hipEventRecord(b->join_ev[j], b->side[j]);
                    (void)hipStreamWaitEvent(b->stream, b->join_ev[j], 0);
                }
                return e;
            }
        }
        for (size_t j = 0; j < k; ++j) {
            const hipError_t e = hipStreamWaitEvent(b->stream, b->join_ev[j], 0);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t batch_capture(apo_batch *b, int32_t iters, hipGraph_t *g, hipGraphExec_t *ge) {
    *g = nullptr;
    *ge = nullptr;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t el = batch_enqueue(b, iters);
    e = hipStreamEndCapture(b->stream, g);
    if (el != hipSuccess) e = el;
    if (e == hipSuccess) e = hipGraphInstantiate(ge, *g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (*g) (void)hipGraphDestroy(*g);
        *g = nullptr;
        *ge = nullptr;
    }
    return e;
}

void batch_drop_graphs(apo_batch *b) {
    for (int i = 0; i < 2; ++i) {
        if (b->gexec[i]) (void)hipGraphExecDestroy(b->gexec[i]);
        if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
        b->gexec[i] = nullptr;
        b->graph[i] = nullptr;
    }
    b->graphs_ready = false;
}

int32_t batch_remaining(const apo_batch *b) {
    int32_t rem = 0x7FFFFFFF;
    for (const apo_t *h : b->runs)
        if (h->T - h->t < rem) rem = h->T - h->t;
    return rem;
}

int batch_destroy_impl(apo_batch *b) {
    if (!b) return APO_OK;
    if (b->stream && !b->poisoned) (void)hipStreamSynchronize(b->stream);
    batch_drop_graphs(b);
    for (apo_t *h : b->runs) destroy_impl(h);
    for (hipStream_t s : b->side) (void)hipStreamDestroy(s);
    for (hipEvent_t e : b->join_ev) (void)hipEventDestroy(e);
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    if (b->own_ws && b->ws) (void)hipFree(b->ws);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return APO_OK;
}

}  // namespace

extern "C" {

size_t apo_workspace_bytes(int32_t dim, int32_t pop, const apo_options *opt) {
    if (!opt || dim < 1 || pop < 2 || opt->max_iter < 1) return 0;
    return make_layout(dim, pop, *opt).total;
}

const char *apo_strerror(int status) {
    switch (status) {
    case APO_OK: return "success";
    case APO_E_INVAL: return "invalid argument";
    case APO_E_NOMEM: return "out of memory";
    case APO_E_DEVICE: return "device error (handle poisoned)";
    case APO_E_DONE: return "iteration budget spent";
    case APO_E_STATE: return "handle cannot serve this call";
    case APO_E_UNSUPPORTED: return "sizes outside those the kernels are built for";
    default: return "unknown status";
    }
}

static int destroy_impl(apo_t *h) {
    if (!h) return APO_OK;
    for (int i = 0; i < 2; ++i) {
        if (h->graph_exec[i]) (void)hipGraphExecDestroy(h->graph_exec[i]);
        if (h->graph[i]) (void)hipGraphDestroy(h->graph[i]);
    }
    if (h->have_events)
        for (int i = 0; i < 4; ++i) (void)hipEventDestroy(h->ev[i]);
    if (h->stream && !h->poisoned) (void)hipStreamSynchronize(h->stream);
    if (h->own_ws && h->ws) (void)hipFree(h->ws);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return APO_OK;
}

int apo_destroy(apo_t *h) {
    if (h && h->batch_view) return APO_E_STATE;
    return destroy_impl(h);
}

int apo_create(int32_t dim, const double *lb, const double *ub, int32_t pop, int32_t np,
               double pf_max, uint64_t seed, const apo_options *opt, apo_t **out) {
    if (!out) return APO_E_INVAL;
    *out = nullptr;
    const int chk = check_args(dim, lb, ub, pop, np, pf_max, opt);
    if (chk != APO_OK) return chk;
    const Layout L = make_layout(dim, pop, *opt);
    if (opt->workspace && opt->workspace_bytes < L.total) return APO_E_INVAL;
    const bool gf = gemm_form(dim, *opt);

    apo_t *h = new (std::nothrow) apo_t();
    if (!h) return APO_E_NOMEM;
    std::memset((void *)h, 0, sizeof(*h));
    h->L = L;
    h->fp64 = opt->precision == APO_FP64;
    h->es = h->fp64 ? 8 : 4;
    h->dim = dim;
    h->pop = pop;
    h->T = opt->max_iter;
    h->flags = opt->flags;

    if (opt->stream) {
        h->stream = (hipStream_t)opt->stream;
    } else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
            delete h;
            return APO_E_DEVICE;
        }
        h->own_stream = true;
    }
    if (opt->workspace) {
        h->ws = (unsigned char *)opt->workspace;
    } else {
        if (hipMalloc((void **)&h->ws, L.total) != hipSuccess) {
            h->ws = nullptr;
            destroy_impl(h);
            return APO_E_NOMEM;
        }
        h->own_ws = true;
    }

    Params &p = h->p;
    p.dim = dim;
    p.pop = pop;
    p.np = np;
    p.max_iter = opt->max_iter;
    p.Dp = L.Dp;
    p.kind = opt->objective.kind;
    p.rotated = opt->objective.rot != nullptr;
    p.Nt = L.Nt;
    p.Ks = L.Ks;
    p.rows = single_tile_rows(dim, pop, (int)h->es);
    p.rank_lds = pop <= 256 ? 1 : 0;   // one workgroup ranks the whole run
    p.gemm = gf ? 1 : 0;
    p.trace = (opt->flags & APO_FLAG_TRACE) ? 1 : 0;
    p.seed_lo = (uint32_t)(seed & 0xFFFFFFFFu);
    p.seed_hi = (uint32_t)(seed >> 32);
    p.run = opt->run_id;
    p.pf_max = pf_max;
    unsigned char *ws = h->ws;
    for (int b = 0; b < 2; ++b) {
        p.X[b] = ws + L.X[b];
    }
    p.F = ws + L.F;
    p.perm = (int32_t *)(ws + L.perm);
    p.Fs = ws + L.Fs;
    p.drf = (uint8_t *)(ws + L.drf);
    p.ctrl = (Ctrl *)(ws + L.ctrl);
    p.p_ah = (const double *)(ws + L.p_ah);
    p.fscale = (const double *)(ws + L.fscale);
    p.cnear = (const double *)(ws + L.cnear);
    p.p_dr = (const double *)(ws + L.p_dr);
    p.lb = ws + L.lb;
    p.ub = ws + L.ub;
    p.shift = ws + L.shift;
    p.rotp = (p.rotated && !gf) ? ws + L.rotp : nullptr;
    if (gf) {
        apok::GemmBufs &g = p.gb;
        g.Yr = (float *)(ws + L.gYr);
        g.Ab = L.gAb ? (uint16_t *)(ws + L.gAb) : nullptr;
        g.anorm = L.gan ? (float *)(ws + L.gan) : nullptr;
        g.P1 = (float *)(ws + L.gP1);
        g.P2 = (float *)(ws + L.gP2);
        g.list = (int32_t *)(ws + L.glist);
        g.status = (int32_t *)(ws + L.gstat);
        g.count = (int32_t *)(ws + L.gcount);
        g.total = (unsigned long long *)(ws + L.gtot);
        g.Mb = L.gMb ? (const uint16_t *)(ws + L.gMb) : nullptr;
        g.Mf = (const float *)(ws + L.gMf);
        g.Md = (const double *)(ws + L.gMd);
        g.o64 = (const double *)(ws + L.go64);
        g.z64 = (double *)(ws + L.gz64);
        g.Kp = L.Kp;
        g.Np = L.Np;
        g.bf16 = opt->precision == APO_BF16 ? 1 : 0;
    }
    p.htab = is_threshold(p.kind) ? (const double *)(ws + L.htab) : nullptr;
    if (p.trace) {
        p.trY = ws + L.trY;
        p.trF = ws + L.trF;
        p.trOp = (int32_t *)(ws + L.trOp);
    }

    // Schedule tables, evaluated once with the same expressions as
    // Eqs. (4), (9), (12) and (13) (binary64 on the host, as Algorithm 1
    // initialises the parameters on the CPU); the kernels only read them,
    // so every operation choice is decided on exactly these values.
    const int T = opt->max_iter;
    std::vector<double> p_ah(T + 1), fsc(T + 1), cn(T + 1), pdr(pop);
    for (int t = 0; t <= T; ++t) {
        p_ah[t] = 0.5 * (1.0 + std::cos(((double)t / (double)T) * kPi));
        fsc[t] = 1.0 + std::cos(((double)t / (double)T) * kPi);
        cn[t] = 1.0 - (double)t / (double)T;
    }
    for (int r = 0; r < pop; ++r) {
        const double c = std::cos((1.0 - (double)(r + 1) / (double)pop) * kPi);
        pdr[r] = (opt->flags & APO_FLAG_PDR_PLUS) ? 0.5 * (1.0 + c) : 0.5 * (1.0 - c);
    }

    std::vector<unsigned char> vlb, vub, vsh, vrot;
    if (h->fp64) {
        to_device_row<double>(vlb, lb, dim, L.Dp);
        to_device_row<double>(vub, ub, dim, L.Dp);
        to_device_row<double>(vsh, opt->objective.shift, dim, L.Dp);
    } else {
        to_device_row<float>(vlb, lb, dim, L.Dp);
        to_device_row<float>(vub, ub, dim, L.Dp);
        to_device_row<float>(vsh, opt->objective.shift, dim, L.Dp);
    }
    std::vector<unsigned char> gmb, gmf, gmd, go;
    if (gf) {
        // M rows padded to [Np][Kp] in binary32 and BF16 (round to nearest
        // even), and M and o in binary64 for the elite
        const double *M = opt->objective.rot;
        gmf.assign((size_t)L.Np * L.Kp * 4, 0);
        gmd.assign((size_t)dim * dim * 8, 0);
        go.assign((size_t)dim * 8, 0);
        float *mf = reinterpret_cast<float *>(gmf.data());
        for (int n = 0; n < dim; ++n)
            for (int k = 0; k < dim; ++k) mf[(size_t)n * L.Kp + k] = (float)M[(size_t)n * dim + k];
        std::memcpy(gmd.data(), M, (size_t)dim * dim * 8);
        if (opt->objective.shift) std::memcpy(go.data(), opt->objective.shift, (size_t)dim * 8);
        if (p.gb.bf16) {
            // BF16 M (round to nearest even; M in binary32) in MFMA fragment
            // order: per 16-row group n / 16 and 32-K chunk k / 32 a block of
            // 64 lanes x 8 values, lane n % 16 + 16 ((k % 32) / 8) holding
            // k % 8 = 0..7
            gmb.assign((size_t)L.Np * L.Kp * 2, 0);
            uint16_t *mb = reinterpret_cast<uint16_t *>(gmb.data());
            const size_t kch = (size_t)L.Kp / 32;
            auto bf16_bits = [](float x) {   // finite x: round to nearest even
                uint32_t u;
                std::memcpy(&u, &x, 4);
                u += 0x7FFFu + ((u >> 16) & 1u);
                return (uint16_t)(u >> 16);
            };
            auto bf16_value = [](uint16_t h) {
                const uint32_t u = (uint32_t)h << 16;
                float f;
                std::memcpy(&f, &u, 4);
                return f;
            };
            // row and column sums of |bf16(M) - M| and |M| (binary64: each sum
            // of at most 1024 terms is exact to ~1e-13 relative; the bounds below
            // are rounded up with margin)
            std::vector<double> rd(dim, 0.0), cd(dim, 0.0), ra(dim, 0.0), ca(dim, 0.0);
            for (size_t n = 0; n < (size_t)L.Np; ++n)
                for (size_t k = 0; k < (size_t)L.Kp; ++k) {
                    const float m = mf[n * L.Kp + k];
                    const uint16_t hi = bf16_bits(m);
                    const size_t lane = (n & 15) + 16 * ((k & 31) >> 3);
                    mb[(((n >> 4) * kch + (k >> 5)) * 64 + lane) * 8 + (k & 7)] = hi;
                    if (n < (size_t)dim && k < (size_t)dim) {
                        const double dm = std::fabs((double)m - (double)bf16_value(hi));
                        const double am = std::fabs((double)m);
                        rd[n] += dm;
                        cd[k] += dm;
                        ra[n] += am;
                        ca[k] += am;
                    }
                }
            auto holder = [](const std::vector<double> &r, const std::vector<double> &c) {
                double mr = 0.0, mc = 0.0;
                for (double v : r) mr = v > mr ? v : mr;
                for (double v : c) mc = v > mc ? v : mc;
                return std::sqrt(mr * mc) * (1.0 + 1e-9);
            };
            p.gb.nrm_dM = std::nextafter((float)holder(rd, cd), INFINITY);
            p.gb.nrm_absM = std::nextafter((float)holder(ra, ca), INFINITY);
        }
    }
    if (p.rotated && !gf) {
        // B fragments of M^T for v_mfma 16x16x4: block (ks, nt), lane l holds
        // B[k][n] = M[n][k] with k = Ks (l / 16) + ks, n = 16 nt + l % 16
        // (the kernel reads A in the same k order).
        const size_t cnt = (size_t)L.Ks * L.Nt * 64;
        vrot.assign(cnt * h->es, 0);
        const double *M = opt->objective.rot;
        for (int ks = 0; ks < L.Ks; ++ks)
            for (int nt = 0; nt < L.Nt; ++nt)
                for (int l = 0; l < 64; ++l) {
                    const int k = L.Ks * (l / 16) + ks, n = 16 * nt + l % 16;
                    const double v = (k < dim && n < dim) ? M[(size_t)n * dim + k] : 0.0;
                    const size_t at = ((size_t)ks * L.Nt + nt) * 64 + l;
                    if (h->fp64)
                        reinterpret_cast<double *>(vrot.data())[at] = v;
                    else
                        reinterpret_cast<float *>(vrot.data())[at] = (float)v;
                }
    }

    hipStream_t s = h->stream;
#define CREATE_HIP(call)               \
    do {                               \
        if ((call) != hipSuccess) {    \
            h->poisoned = true;        \
            destroy_impl(h);           \
            return APO_E_DEVICE;       \
        }                              \
    } while (0)
    CREATE_HIP(hipMemsetAsync(ws, 0, L.total, s));
    CREATE_HIP(hipMemcpyAsync(ws + L.p_ah, p_ah.data(), (T + 1) * 8, hipMemcpyHostToDevice, s));
    CREATE_HIP(hipMemcpyAsync(ws + L.fscale, fsc.data(), (T + 1) * 8, hipMemcpyHostToDevice, s));
    CREATE_HIP(hipMemcpyAsync(ws + L.cnear, cn.data(), (T + 1) * 8, hipMemcpyHostToDevice, s));
    CREATE_HIP(hipMemcpyAsync(ws + L.p_dr, pdr.data(), (size_t)pop * 8, hipMemcpyHostToDevice, s));
    CREATE_HIP(hipMemcpyAsync(ws + L.lb, vlb.data(), vlb.size(), hipMemcpyHostToDevice, s));
    CREATE_HIP(hipMemcpyAsync(ws + L.ub, vub.data(), vub.size(), hipMemcpyHostToDevice, s));
    CREATE_HIP(hipMemcpyAsync(ws + L.shift, vsh.data(), vsh.size(), hipMemcpyHostToDevice, s));
    if (p.rotated && !gf)
        CREATE_HIP(hipMemcpyAsync(ws + L.rotp, vrot.data(), vrot.size(), hipMemcpyHostToDevice, s));
    if (gf) {
        CREATE_HIP(hipMemcpyAsync(ws + L.gMf, gmf.data(), gmf.size(), hipMemcpyHostToDevice, s));
        CREATE_HIP(hipMemcpyAsync(ws + L.gMd, gmd.data(), gmd.size(), hipMemcpyHostToDevice, s));
        CREATE_HIP(hipMemcpyAsync(ws + L.go64, go.data(), go.size(), hipMemcpyHostToDevice, s));
        if (p.gb.bf16)
            CREATE_HIP(hipMemcpyAsync(ws + L.gMb, gmb.data(), gmb.size(), hipMemcpyHostToDevice, s));
    }
    if (is_threshold(p.kind)) {
        CREATE_HIP(hipMemcpyAsync(ws + L.hist, opt->objective.hist, 256 * 8, hipMemcpyHostToDevice, s));
        CREATE_HIP(apok::launch_hist_tables(p, (const uint64_t *)(ws + L.hist), s));
    }
    CREATE_HIP(apok::launch_init(p, h->fp64, s));
    CREATE_HIP(hipStreamSynchronize(s));   // host staging buffers go out of scope
#undef CREATE_HIP
    (void)hipGetLastError();
    h->t = 0;
    *out = h;
    return APO_OK;
}

static int launch_iteration(apo_t *h) {
    APO_HIP(h, apok::launch_rank(h->p, h->fp64, h->stream));
    APO_HIP(h, apok::launch_step(h->p, h->fp64, h->stream));
    return APO_OK;
}

int apo_step(apo_t *h) {
    if (!h) return APO_E_INVAL;
    if (h->batch_view) return APO_E_STATE;
    if (h->poisoned) return APO_E_DEVICE;
    if (h->t >= h->T) return APO_E_DONE;
    const int rc = launch_iteration(h);
    if (rc != APO_OK) return rc;
    ++h->t;
    return APO_OK;
}

// Iterations per replay of the block graph: long runs are submitted in
// blocks so the host cost of a graph launch is paid once per block.
static const int32_t kGraphBlock = 16;

// Captures `iters` iterations (rank sort + step, in order) as one graph.
// One iteration is iteration-invariant (the kernels read t from the device
// control block), so the same graph serves every iteration of a run.
static void capture_iterations(apo_t *h, int32_t iters, hipGraph_t *graph,
                               hipGraphExec_t *exec) {
    *graph = nullptr;
    *exec = nullptr;
    if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    hipError_t e = hipSuccess;
    for (int32_t i = 0; i < iters && e == hipSuccess; ++i) {
        e = apok::launch_rank(h->p, h->fp64, h->stream);
        if (e == hipSuccess) e = apok::launch_step(h->p, h->fp64, h->stream);
    }
    hipGraph_t g = nullptr;
    const hipError_t e3 = hipStreamEndCapture(h->stream, &g);
    if (e == hipSuccess && e3 == hipSuccess && g) {
        hipGraphExec_t ge = nullptr;
        if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess) {
            *graph = g;
            *exec = ge;
        } else {
            (void)hipGraphDestroy(g);
        }
    } else if (g) {
        (void)hipGraphDestroy(g);
    }
    (void)hipGetLastError();
}

int apo_run(apo_t *h, int32_t iters) {
    if (!h || iters < 0) return APO_E_INVAL;
    if (h->batch_view) return APO_E_STATE;
    if (h->poisoned) return APO_E_DEVICE;
    int32_t n = h->T - h->t;
    if (iters < n) n = iters;
    if (apok::persist_form(h->p, h->fp64)) {
        // the whole run in one workgroup: all n iterations in one launch
        if (n <= 0) return 0;
        APO_HIP(h, apok::launch_persist(h->p, h->fp64, h->t, n, h->stream));
        h->t += n;
        return n;
    }
    if (!h->graph_tried) {   // apo_run(h, 0) only does this
        h->graph_tried = true;
        capture_iterations(h, 1, &h->graph[0], &h->graph_exec[0]);
        if (h->graph_exec[0] && h->T >= kGraphBlock)
            capture_iterations(h, kGraphBlock, &h->graph[1], &h->graph_exec[1]);
    }
    if (n <= 0) return 0;
    int32_t done = 0;
    while (done < n) {
        if (h->graph_exec[1] && n - done >= kGraphBlock) {
            APO_HIP(h, hipGraphLaunch(h->graph_exec[1], h->stream));
            done += kGraphBlock;
            h->t += kGraphBlock;
        } else if (h->graph_exec[0]) {
            APO_HIP(h, hipGraphLaunch(h->graph_exec[0], h->stream));
            ++done;
            ++h->t;
        } else {
            const int rc = launch_iteration(h);
            if (rc != APO_OK) return rc;
            ++done;
            ++h->t;
        }
    }
    return n;
}

int apo_time_kernels(apo_t *h, int32_t iters, double *avg_us) {
    if (!h || iters < 1 || !avg_us) return APO_E_INVAL;
    if (h->batch_view) return APO_E_STATE;
    if (h->poisoned) return APO_E_DEVICE;
    int32_t n = h->T - h->t;
    if (iters < n) n = iters;
    if (n <= 0) return APO_E_DONE;
    if (!h->have_events) {
        for (int i = 0; i < 4; ++i) APO_HIP(h, hipEventCreate(&h->ev[i]));
        h->have_events = true;
    }
    // each launch records its own start and end events (kernel execution
    // alone, as a kernel trace measures it)
    Params pr = h->p, ps = h->p;
    pr.ev_start = h->ev[0];
    pr.ev_stop = h->ev[1];
    ps.ev_start = h->ev[2];
    ps.ev_stop = h->ev[3];
    double sum_rank = 0.0, sum_step = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        APO_HIP(h, apok::launch_rank(pr, h->fp64, h->stream));
        APO_HIP(h, apok::launch_step(ps, h->fp64, h->stream));
        APO_HIP(h, hipEventSynchronize(h->ev[3]));
        float a = 0.f, b = 0.f;
        APO_HIP(h, hipEventElapsedTime(&a, h->ev[0], h->ev[1]));
        APO_HIP(h, hipEventElapsedTime(&b, h->ev[2], h->ev[3]));
        sum_rank += a;
        sum_step += b;
        ++h->t;
    }
    avg_us[0] = 1000.0 * sum_rank / n;
    avg_us[1] = 1000.0 * sum_step / n;
    return n;
}

int apo_time_gemm_stages(apo_t *h, int32_t iters, double *us) {
    if (!h || iters < 1 || !us) return APO_E_INVAL;
    if (h->batch_view || !h->p.gemm) return APO_E_STATE;
    if (h->poisoned) return APO_E_DEVICE;
    int32_t n = h->T - h->t;
    if (iters < n) n = iters;
    if (n <= 0) return APO_E_DONE;
    // launch order: sort, then stages 0..4; each launch records its own
    // start and end events (kernel execution alone)
    constexpr int kL = 6;
    hipEvent_t ev[2 * kL];
    for (int i = 0; i < 2 * kL; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
            return APO_E_DEVICE;
        }
    const bool bf16 = h->p.gb.bf16 != 0;
    Params q[kL];
    for (int k = 0; k < kL; ++k) {
        q[k] = h->p;
        q[k].ev_start = ev[2 * k];
        q[k].ev_stop = ev[2 * k + 1];
    }
    double sum[kL] = {0, 0, 0, 0, 0, 0};
    int rc = APO_OK;
    for (int32_t it = 0; it < n && rc == APO_OK; ++it) {
        bool ok = apok::launch_rank(q[0], h->fp64, h->stream) == hipSuccess;
        for (int st = 0; ok && st < 5; ++st)
            ok = apok::launch_gemm_stage(q[1 + st], h->p.gb, 0, st, h->stream) == hipSuccess;
        ok = ok && hipStreamSynchronize(h->stream) == hipSuccess;
        for (int k = 0; ok && k < kL; ++k) {
            if (!bf16 && (k == 3 || k == 4)) continue;   // no classification / re-score launch
            float ms = 0.f;
            ok = hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]) == hipSuccess;
            sum[k == 0 ? 5 : k - 1] += 1000.0 * ms;
        }
        if (!ok) {
            h->poisoned = true;
            rc = APO_E_DEVICE;
        } else {
            ++h->t;
        }
    }
    for (int i = 0; i < 2 * kL; ++i) (void)hipEventDestroy(ev[i]);
    if (rc != APO_OK) return rc;
    for (int i = 0; i < kL; ++i) us[i] = sum[i] / n;
    return n;
}

int apo_precision_stats(apo_t *h, int64_t *rescored, int64_t *estimated) {
    if (!h || !rescored || !estimated) return APO_E_INVAL;
    if (h->poisoned) return APO_E_DEVICE;
    *rescored = 0;
    *estimated = 0;
    if (!h->p.gemm || !h->p.gb.bf16) return APO_OK;
    unsigned long long tot = 0;
    APO_HIP(h, hipMemcpyAsync(&tot, h->p.gb.total, 8, hipMemcpyDeviceToHost, h->stream));
    APO_HIP(h, hipStreamSynchronize(h->stream));
    *rescored = (int64_t)tot;
    *estimated = (int64_t)h->pop * (int64_t)h->t;
    return APO_OK;
}

int apo_info(const apo_t *h, int32_t *iter, int64_t *fes) {
    if (!h) return APO_E_INVAL;
    if (iter) *iter = h->t;
    if (fes) *fes = (int64_t)h->pop * ((int64_t)h->t + 1);
    return h->poisoned ? APO_E_DEVICE : APO_OK;
}

int apo_best(apo_t *h, double *x_out, double *f_out, int64_t *fes_out) {
    if (!h) return APO_E_INVAL;
    if (h->poisoned) return APO_E_DEVICE;
    double *d_best = (double *)(h->ws + h->L.best);
    std::vector<double> row((size_t)h->dim + 1);
    APO_HIP(h, apok::launch_best(h->p, h->fp64, h->t & 1, d_best, h->stream));
    if (h->p.gemm)   // the elite's fitness re-scored in binary64
        APO_HIP(h, apok::launch_elite_f64(h->p, h->p.gb, d_best + 1, d_best, h->stream));
    APO_HIP(h, hipMemcpyAsync(row.data(), d_best, row.size() * 8, hipMemcpyDeviceToHost, h->stream));
    APO_HIP(h, hipStreamSynchronize(h->stream));
    if (f_out) *f_out = row[0];
    if (x_out) std::memcpy(x_out, row.data() + 1, (size_t)h->dim * 8);
    if (fes_out) *fes_out = (int64_t)h->pop * ((int64_t)h->t + 1);
    return APO_OK;
}

static int copy_rows_out(apo_t *h, const void *dev, double *host, int rows, int cols, int stride) {
    std::vector<unsigned char> buf((size_t)rows * stride * h->es);
    APO_HIP(h, hipMemcpyAsync(buf.data(), dev, buf.size(), hipMemcpyDeviceToHost, h->stream));
    APO_HIP(h, hipStreamSynchronize(h->stream));
    if (h->fp64)
        rows_to_double<double>(buf.data(), host, rows, cols, stride);
    else
        rows_to_double<float>(buf.data(), host, rows, cols, stride);
    return APO_OK;
}

int apo_get_state(apo_t *h, double *X, double *F, int32_t *iter) {
    if (!h) return APO_E_INVAL;
    if (h->poisoned) return APO_E_DEVICE;
    const int cur = h->t & 1;
    if (X) {
        const int rc = copy_rows_out(h, h->p.X[cur], X, h->pop, h->dim, h->L.Dp);
        if (rc != APO_OK) return rc;
    }
    if (F) {
        const int rc = copy_rows_out(h, h->p.F, F, h->pop, 1, 1);
        if (rc != APO_OK) return rc;
    }
    if (iter) *iter = h->t;
    APO_HIP(h, hipStreamSynchronize(h->stream));
    return APO_OK;
}

int apo_set_state(apo_t *h, const double *X, const double *F, int32_t iter) {
    if (!h || !X || !F || iter < 0 || iter > h->T) return APO_E_INVAL;
    if (h->poisoned) return APO_E_DEVICE;
    const int cur = iter & 1;
    std::vector<unsigned char> xb((size_t)h->pop * h->L.Dp * h->es), fb((size_t)h->pop * h->es);
    if (h->fp64) {
        rows_from_double<double>(X, xb.data(), h->pop, h->dim, h->L.Dp);
        rows_from_double<double>(F, fb.data(), h->pop, 1, 1);
    } else {
        rows_from_double<float>(X, xb.data(), h->pop, h->dim, h->L.Dp);
        rows_from_double<float>(F, fb.data(), h->pop, 1, 1);
    }
    Ctrl c;
    std::memset(&c, 0, sizeof(c));
    c.t = iter;
    c.t_next = iter;
    APO_HIP(h, hipStreamSynchronize(h->stream));
    APO_HIP(h, hipMemcpyAsync(h->p.X[cur], xb.data(), xb.size(), hipMemcpyHostToDevice, h->stream));
    APO_HIP(h, hipMemcpyAsync(h->p.F, fb.data(), fb.size(), hipMemcpyHostToDevice, h->stream));
    APO_HIP(h, hipMemcpyAsync(h->p.ctrl, &c, sizeof(c), hipMemcpyHostToDevice, h->stream));
    APO_HIP(h, hipStreamSynchronize(h->stream));
    h->t = iter;
    return APO_OK;
}

int apo_get_trace(apo_t *h, double *Y, double *Fy, int32_t *op, int32_t *perm) {
    if (!h) return APO_E_INVAL;
    if (h->poisoned) return APO_E_DEVICE;
    if (!h->p.trace) return APO_E_STATE;
    if (Y) {
        const int rc = copy_rows_out(h, h->p.trY, Y, h->pop, h->dim, h->L.Dp);
        if (rc != APO_OK) return rc;
    }
    if (Fy) {
        const int rc = copy_rows_out(h, h->p.trF, Fy, h->pop, 1, 1);
        if (rc != APO_OK) return rc;
    }
    if (op) APO_HIP(h, hipMemcpyAsync(op, h->p.trOp, (size_t)h->pop * 4, hipMemcpyDeviceToHost, h->stream));
    if (perm) APO_HIP(h, hipMemcpyAsync(perm, h->p.perm, (size_t)h->pop * 4, hipMemcpyDeviceToHost, h->stream));
    APO_HIP(h, hipStreamSynchronize(h->stream));
    return APO_OK;
}

int apo_histogram_u8(const uint8_t *d_img, uint64_t n, uint64_t *host_hist, void *stream) {
    if (!host_hist || (!d_img && n > 0) || n >= (1ull << 32)) return APO_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    unsigned char *scratch = nullptr;
    if (hipMalloc((void **)&scratch, apok::histogram_scratch_bytes()) != hipSuccess)
        return APO_E_NOMEM;
    bool ok = apok::launch_histogram(d_img, n, scratch, s) == hipSuccess &&
              hipMemcpyAsync(host_hist, scratch + apok::histogram_out_offset(), 256 * 8,
                             hipMemcpyDeviceToHost, s) == hipSuccess &&
              hipStreamSynchronize(s) == hipSuccess;
    ok = hipFree(scratch) == hipSuccess && ok;
    return ok ? APO_OK : APO_E_DEVICE;
}

int apo_histogram_u8_noalloc(const uint8_t *d_img, uint64_t n, uint64_t *d_hist, void *stream) {
    if (!d_hist || ((uintptr_t)d_hist & 7u) != 0 || (!d_img && n > 0)) return APO_E_INVAL;
    if (n >= (1ull << 32)) return APO_E_UNSUPPORTED;
    return apok::launch_histogram_noalloc(d_img, n, (unsigned long long *)d_hist,
                                          (hipStream_t)stream) == hipSuccess
               ? APO_OK
               : APO_E_DEVICE;
}

size_t apo_batch_workspace_bytes(int32_t n, const apo_run_desc *runs) {
    BatchLayout B;
    return batch_layout(n, runs, B) == APO_OK ? B.total : 0;
}

int apo_batch_create(int32_t n, const apo_run_desc *runs, const apo_batch_options *opt,
                     apo_batch_t **out) {
    if (!out) return APO_E_INVAL;
    *out = nullptr;
    BatchLayout B;
    const int chk = batch_layout(n, runs, B);
    if (chk != APO_OK) return chk;
    if (opt && opt->workspace && opt->workspace_bytes < B.total) return APO_E_INVAL;
    apo_batch *b = new (std::nothrow) apo_batch();
    if (!b) return APO_E_NOMEM;
    if (opt && opt->stream) {
        b->stream = (hipStream_t)opt->stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return APO_E_DEVICE;
        }
        b->own_stream = true;
    }
    if (opt && opt->workspace) {
        b->ws = (unsigned char *)opt->workspace;
    } else {
        if (hipMalloc((void **)&b->ws, B.total) != hipSuccess) {
            b->ws = nullptr;
            batch_destroy_impl(b);
            return APO_E_NOMEM;
        }
        b->own_ws = true;
    }
    b->runs_bytes = B.runs_bytes;
    b->d_params = (Params *)(b->ws + B.params_off);
    b->d_blocks = (int2 *)(b->ws + B.blocks_off);
    b->n_entries = B.n_entries;
    for (int i = 0; i < n; ++i) {
        apo_options o = runs[i].opt;
        o.stream = b->stream;
        o.workspace = b->ws + B.run_off[i];
        o.workspace_bytes = B.run_bytes[i];
        apo_t *h = nullptr;
        const int rc = apo_create(runs[i].dim, runs[i].lb, runs[i].ub, runs[i].pop, runs[i].np,
                                  runs[i].pf_max, runs[i].seed, &o, &h);
        if (rc != APO_OK) {
            batch_destroy_impl(b);
            return rc;
        }
        h->batch_view = true;
        // a batch fills the GPU with runs: fewer, fuller workgroups per run
        // (batch_lanes: fewer lanes per protozoan for rotated separable
        // objectives, one row per lane group; the shape was checked by
        // batch_layout)
        MemberShape ms;
        (void)batch_member_shape(runs[i], ms);
        h->p.lanes = ms.lanes;
        h->p.rows = ms.rows;
        h->p.rank_lds = h->pop <= apok::kRankLdsMax ? 1 : 0;
        b->runs.push_back(h);
    }
    std::vector<Params> hp(n);
    for (int i = 0; i < n; ++i) hp[i] = b->runs[i]->p;
    if (hipMemcpyAsync(b->d_params, hp.data(), (size_t)n * sizeof(Params), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess) {
        b->poisoned = true;
        batch_destroy_impl(b);
        return APO_E_DEVICE;
    }
    batch_group_launches(b);
    size_t steps = 0;
    for (const BatchLaunchRec &r : b->launches) steps += r.rank ? 0 : 1;
    b->side.assign(steps, nullptr);
    b->join_ev.assign(steps, nullptr);
    bool ok = hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) == hipSuccess;
    for (size_t k = 0; ok && k < steps; ++k) {
        ok = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&b->join_ev[k], hipEventDisableTiming) == hipSuccess;
    }
    b->schedule = 0;
    if (!ok || batch_fill_tables(b, b->schedule) != APO_OK) {
        b->poisoned = true;
        batch_destroy_impl(b);
        return APO_E_DEVICE;
    }
    *out = b;
    return APO_OK;
}

int apo_batch_member(apo_batch_t *b, int32_t i, apo_t **run) {
    if (!b || !run || i < 0 || i >= (int32_t)b->runs.size()) return APO_E_INVAL;
    *run = b->runs[i];
    return APO_OK;
}

int apo_batch_run(apo_batch_t *b, int32_t iters) {
    if (!b || iters < 0) return APO_E_INVAL;
    if (b->poisoned) return APO_E_DEVICE;
    for (const apo_t *h : b->runs) {
        if (h->poisoned) return APO_E_DEVICE;
        if (h->t != b->runs[0]->t) return APO_E_STATE;
    }
    int32_t n = batch_remaining(b);
    if (iters < n) n = iters;
    if (n <= 0) return 0;
    if (!b->graphs_ready) {
        b->graphs_ready = true;
        if (batch_capture(b, 1, &b->graph[0], &b->gexec[0]) == hipSuccess &&
            batch_remaining(b) >= kGraphBlock)
            (void)batch_capture(b, kGraphBlock, &b->graph[1], &b->gexec[1]);
        (void)hipGetLastError();
    }
    int32_t done = 0;
    while (done < n) {
        int32_t step;
        hipError_t e;
        if (b->gexec[1] && n - done >= kGraphBlock) {
            e = hipGraphLaunch(b->gexec[1], b->stream);
            step = kGraphBlock;
        } else if (b->gexec[0]) {
            e = hipGraphLaunch(b->gexec[0], b->stream);
            step = 1;
        } else {
            e = batch_enqueue(b, 1);
            step = 1;
        }
        if (e != hipSuccess) {
            b->poisoned = true;
            return APO_E_DEVICE;
        }
        done += step;
        for (apo_t *h : b->runs) h->t += step;
    }
    return n;
}

int apo_batch_tune(apo_batch_t *b, int32_t iters, int32_t *schedule, double *us) {
    if (!b || iters < 1) return APO_E_INVAL;
    if (b->poisoned) return APO_E_DEVICE;
    for (const apo_t *h : b->runs)
        if (h->t != b->runs[0]->t) return APO_E_STATE;
    int32_t n = batch_remaining(b);
    if (iters < n) n = iters;
    if (n < 1) return APO_E_DONE;
    unsigned char *backup = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipMalloc((void **)&backup, b->runs_bytes) != hipSuccess) return APO_E_NOMEM;
    bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
              hipMemcpyAsync(backup, b->ws, b->runs_bytes, hipMemcpyDeviceToDevice,
                             b->stream) == hipSuccess;
    double best = 1e300, t_us[4] = {0, 0, 0, 0};
    int best_s = b->schedule;
    batch_drop_graphs(b);
    for (int sc = 0; ok && sc < 4; ++sc) {
        b->schedule = sc;
        ok = batch_fill_tables(b, sc) == APO_OK;
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        ok = ok && batch_capture(b, n, &g, &ge) == hipSuccess;
        float ms = 0.f;
        for (int rep = 0; ok && rep < 2; ++rep) {   // warm-up, then timed
            ok = hipEventRecord(e0, b->stream) == hipSuccess &&
                 hipGraphLaunch(ge, b->stream) == hipSuccess &&
                 hipEventRecord(e1, b->stream) == hipSuccess &&
                 hipEventSynchronize(e1) == hipSuccess &&
                 hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
                 hipMemcpyAsync(b->ws, backup, b->runs_bytes, hipMemcpyDeviceToDevice,
                                b->stream) == hipSuccess;
        }
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
        t_us[sc] = 1000.0 * ms / n;
        if (ok && t_us[sc] < best) {
            best = t_us[sc];
            best_s = sc;
        }
    }
    ok = ok && hipStreamSynchronize(b->stream) == hipSuccess;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(backup);
    b->schedule = best_s;
    if (!ok || batch_fill_tables(b, best_s) != APO_OK) {
        b->poisoned = true;
        return APO_E_DEVICE;
    }
    if (schedule) *schedule = best_s;
    if (us)
        for (int i = 0; i < 4; ++i) us[i] = t_us[i];
    return APO_OK;
}

int apo_batch_destroy(apo_batch_t *b) { return batch_destroy_impl(b); }

}  // extern "C"
