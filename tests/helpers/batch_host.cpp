// CPU check of the batch runtime (apo_api.cpp compiled for the host, with
// AddressSanitizer): the HIP calls it makes are replaced by stand-ins that
// keep HIP's signatures -- device memory is host memory, streams, events and
// graphs are host objects, stream capture records the launches into the
// graph -- and the kernel launchers are replaced by checks of what each
// launch would run: every (run, block) entry of a batched sort or step
// launch names a member of the batch and one of that run's workgroups, each
// run's workgroups appear exactly once per launch, the runs of a step
// launch share its kernel shape, the launch's LDS covers each of them, and
// a capture ends with every forked stream joined back.  Graph replays
// repeat the checks against the tables current at replay time.
//
// The scenarios create, tune, run and destroy batches one after another in
// one process: the 512-run batched configuration, its subsets by population
// and dimension, and a mixed batch (binary64, elementwise, thresholding,
// np 3).  Prints "ok" and exits 0 when every check passes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "apo.h"
#include "apo_internal.h"

using apok::BatchLaunch;
using apok::Params;

namespace {

int g_fail = 0;
long g_launches = 0, g_replays = 0;
int g_members = 0;   // members of the batch being exercised (its device table size)

#define CHECK(c, ...)                                        \
    do {                                                     \
        if (!(c)) {                                          \
            std::fprintf(stderr, "FAIL %s:%d ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);               \
            std::fprintf(stderr, "\n");                      \
            ++g_fail;                                        \
        }                                                    \
    } while (0)

struct Rec {
    bool rank;
    bool fp64;
    Params proto;
    BatchLaunch b;
};

struct Graph {
    std::vector<Rec> recs;
};

struct Stream {
    Graph *cap = nullptr;        // graph being captured into, if any
    Stream *origin = nullptr;    // the capturing stream this one joined
    long last_launch = 0;        // sequence number of its last captured launch
    long joined_at = 0;          // sequence number when it was last joined back
};

struct Event {
    Stream *src = nullptr;
    long seq = 0;
};

long g_seq = 0;
std::set<Stream *> g_streams;
std::set<Event *> g_events;
std::set<Graph *> g_graphs;
std::set<void *> g_allocs;

Stream *S(hipStream_t s) { return reinterpret_cast<Stream *>(s); }

void check_launch(const Rec &r) {
    const BatchLaunch &b = r.b;
    CHECK(b.nblocks >= 0, "negative block count");
    std::map<int, std::vector<int>> seen;
    for (int i = 0; i < b.nblocks; ++i) {
        const int2 e = b.blocks[i];
        CHECK(e.x >= 0 && e.x < g_members, "entry %d names run %d of %d", i, e.x, g_members);
        if (e.x < 0 || e.x >= g_members) continue;
        const Params &p = b.runs[e.x];
        const int nb = r.rank ? apok::rank_blocks(p) : apok::step_blocks(p);
        CHECK(e.y >= 0 && e.y < nb, "run %d block %d of %d", e.x, e.y, nb);
        seen[e.x].push_back(e.y);
        if (!r.rank) {
            CHECK(apok::step_shape(p, r.fp64) == apok::step_shape(r.proto, r.fp64),
                  "run %d has another kernel shape than the launch", e.x);
            CHECK(b.lds >= apok::step_lds_bytes(p, r.fp64), "launch LDS below run %d's", e.x);
            if (apok::tile_form(p)) {
                const int G = apok::tile_lanes(p);
                CHECK(apok::tile_shape_ok(p.dim, G, apok::tile_chunks(p), apok::tile_rows(p),
                                          r.fp64 ? 8 : 4),
                      "run %d's tile shape is not launchable", e.x);
            }
        }
    }
    for (auto &kv : seen) {
        const Params &p = b.runs[kv.first];
        const int nb = r.rank ? apok::rank_blocks(p) : apok::step_blocks(p);
        std::vector<int> v = kv.second;
        CHECK((int)v.size() == nb, "run %d: %zu of %d workgroups", kv.first, v.size(), nb);
        std::set<int> u(v.begin(), v.end());
        CHECK(u.size() == v.size(), "run %d: a workgroup appears twice", kv.first);
    }
    CHECK(b.lds <= apok::kLdsLimit, "launch LDS %zu above the limit", b.lds);
}

hipError_t record(hipStream_t s, const Rec &r) {
    ++g_launches;
    ++g_seq;
    Stream *st = S(s);
    CHECK(st == nullptr || g_streams.count(st), "launch on a destroyed stream");
    if (st && st->cap) {
        st->cap->recs.push_back(r);
        st->last_launch = g_seq;
    } else {
        check_launch(r);
    }
    return hipSuccess;
}

}  // namespace

// ---------------------------------------------------------------------------
// HIP stand-ins (the calls apo_api.cpp makes).
// ---------------------------------------------------------------------------
extern "C" {
hipError_t hipMalloc(void **ptr, size_t size) {
    *ptr = std::calloc(1, size ? size : 1);
    g_allocs.insert(*ptr);
    return *ptr ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *ptr) {
    if (!ptr) return hipSuccess;
    CHECK(g_allocs.count(ptr), "hipFree of memory not from hipMalloc");
    g_allocs.erase(ptr);
    std::free(ptr);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t s) {
    CHECK(s == nullptr || g_streams.count(S(s)), "copy on a destroyed stream");
    if (n) std::memmove(dst, src, n);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void *dst, int value, size_t n, hipStream_t) {
    std::memset(dst, value, n);
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
    Stream *st = new Stream();
    g_streams.insert(st);
    *s = reinterpret_cast<hipStream_t>(st);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    Stream *st = S(s);
    CHECK(g_streams.count(st), "destroying an unknown stream");
    CHECK(!st->cap, "destroying a stream in capture");
    g_streams.erase(st);
    delete st;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    CHECK(s == nullptr || g_streams.count(S(s)), "sync of a destroyed stream");
    CHECK(s == nullptr || !S(s)->cap, "sync of a capturing stream");
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) {
    Event *ev = new Event();
    g_events.insert(ev);
    *e = reinterpret_cast<hipEvent_t>(ev);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    Event *ev = reinterpret_cast<Event *>(e);
    CHECK(g_events.count(ev), "destroying an unknown event");
    g_events.erase(ev);
    delete ev;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    Event *ev = reinterpret_cast<Event *>(e);
    CHECK(g_events.count(ev), "recording an unknown event");
    ev->src = S(s);
    ev->seq = ++g_seq;
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    CHECK(g_events.count(reinterpret_cast<Event *>(e)), "sync of an unknown event");
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
    // each timing shorter than the one before, so the tuner ends on its
    // last schedule (parallel branches, interleaved blocks)
    static float t = 1.0e6f;
    *ms = (t -= 1.0f);
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
    Stream *st = S(s);
    Event *ev = reinterpret_cast<Event *>(e);
    CHECK(g_streams.count(st) && g_events.count(ev), "wait with unknown stream or event");
    if (ev->src && ev->src->cap && !st->cap) {   // st joins the capture (a fork)
        st->cap = ev->src->cap;
        st->origin = ev->src->origin ? ev->src->origin : ev->src;
        st->last_launch = 0;
        st->joined_at = 0;
    } else if (ev->src && st->cap && ev->src != st && ev->src->origin == st) {
        ev->src->joined_at = ev->seq;   // a forked stream joins back
    }
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    Stream *st = S(s);
    CHECK(g_streams.count(st) && !st->cap, "capture on an unknown or capturing stream");
    Graph *g = new Graph();
    g_graphs.insert(g);
    st->cap = g;
    st->origin = nullptr;
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *graph) {
    Stream *st = S(s);
    CHECK(st->cap && !st->origin, "end of capture on a stream that is not capturing");
    Graph *g = st->cap;
    bool joined = true;
    for (Stream *o : g_streams) {
        if (o == st || o->cap != g) continue;
        if (o->last_launch > o->joined_at) joined = false;
        o->cap = nullptr;
        o->origin = nullptr;
    }
    st->cap = nullptr;
    CHECK(joined, "capture ended with a forked stream not joined back");
    *graph = reinterpret_cast<hipGraph_t>(g);
    return joined ? hipSuccess : hipErrorStreamCaptureUnjoined;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *ge, hipGraph_t g, hipGraphNode_t *, char *,
                               size_t) {
    Graph *src = reinterpret_cast<Graph *>(g);
    CHECK(g_graphs.count(src), "instantiating an unknown graph");
    Graph *x = new Graph(*src);
    g_graphs.insert(x);
    *ge = reinterpret_cast<hipGraphExec_t>(x);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t ge, hipStream_t s) {
    Graph *x = reinterpret_cast<Graph *>(ge);
    CHECK(g_graphs.count(x), "launching a destroyed graph");
    CHECK(g_streams.count(S(s)), "graph launch on a destroyed stream");
    ++g_replays;
    for (const Rec &r : x->recs) check_launch(r);
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    Graph *x = reinterpret_cast<Graph *>(g);
    CHECK(g_graphs.count(x), "destroying an unknown graph");
    g_graphs.erase(x);
    delete x;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t ge) { return hipGraphDestroy(reinterpret_cast<hipGraph_t>(ge)); }
hipError_t hipGetLastError(void) { return hipSuccess; }
}

// ---------------------------------------------------------------------------
// Launcher stand-ins: single-handle launches do nothing; batched launches
// are checked (or recorded into a capture).
// ---------------------------------------------------------------------------
namespace apok {
hipError_t launch_init(const Params &, bool, hipStream_t) { return hipSuccess; }
hipError_t launch_rank(const Params &, bool, hipStream_t) { return hipSuccess; }
hipError_t launch_step(const Params &, bool, hipStream_t) { return hipSuccess; }
hipError_t launch_persist(const Params &, bool, int, int, hipStream_t) { return hipSuccess; }
hipError_t launch_best(const Params &, bool, int, double *, hipStream_t) { return hipSuccess; }
hipError_t launch_hist_tables(const Params &, const uint64_t *, hipStream_t) { return hipSuccess; }
size_t histogram_scratch_bytes() { return kHistScratchBytes; }
hipError_t launch_histogram(const uint8_t *, uint64_t, void *, hipStream_t) { return hipSuccess; }
hipError_t launch_histogram_noalloc(const uint8_t *, uint64_t, unsigned long long *, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_gemm_step(const Params &, const GemmBufs &, int, hipStream_t) { return hipSuccess; }
hipError_t launch_gemm_stage(const Params &, const GemmBufs &, int, int, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_elite_f64(const Params &, const GemmBufs &, const double *, double *, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_rank_batch(const BatchLaunch &b, bool fp64, hipStream_t s) {
    Rec r;
    r.rank = true;
    r.fp64 = fp64;
    std::memset(&r.proto, 0, sizeof(r.proto));
    r.b = b;
    return record(s, r);
}
hipError_t launch_step_batch(const Params &proto, bool fp64, const BatchLaunch &b, hipStream_t s) {
    Rec r;
    r.rank = false;
    r.fp64 = fp64;
    r.proto = proto;
    r.b = b;
    return record(s, r);
}
}  // namespace apok

// ---------------------------------------------------------------------------
// Scenarios.
// ---------------------------------------------------------------------------
namespace {

struct RunSpec {
    int dim, pop, kind, precision, np;
    bool rotated;
};

struct Owned {
    std::vector<std::vector<double>> bufs;
    std::vector<uint64_t> hist;
};

std::vector<apo_run_desc> descs(const std::vector<RunSpec> &rs, Owned &own) {
    std::vector<apo_run_desc> out;
    own.hist.assign(256, 0);
    for (int g = 0; g < 256; ++g) own.hist[g] = (uint64_t)(1 + (g * 37) % 11);
    int i = 0;
    for (const RunSpec &r : rs) {
        const bool thr = r.kind == APO_KAPUR || r.kind == APO_OTSU;
        own.bufs.emplace_back(r.dim, thr ? 0.0 : -100.0);
        const double *lb = own.bufs.back().data();
        own.bufs.emplace_back(r.dim, thr ? 255.0 : 100.0);
        const double *ub = own.bufs.back().data();
        const double *shift = nullptr, *rot = nullptr;
        if (!thr) {
            own.bufs.emplace_back(r.dim, 1.5);
            shift = own.bufs.back().data();
            if (r.rotated) {
                own.bufs.emplace_back((size_t)r.dim * r.dim, 0.0);
                for (int d = 0; d < r.dim; ++d) own.bufs.back()[(size_t)d * r.dim + d] = 1.0;
                rot = own.bufs.back().data();
            }
        }
        apo_run_desc d;
        std::memset(&d, 0, sizeof(d));
        d.dim = r.dim;
        d.lb = lb;
        d.ub = ub;
        d.pop = r.pop;
        d.np = r.np;
        d.pf_max = 0.1;
        d.seed = 1000 + i;
        d.opt.max_iter = 1000;
        d.opt.precision = r.precision;
        d.opt.objective.kind = (apo_obj_kind)r.kind;
        d.opt.objective.shift = shift;
        d.opt.objective.rot = rot;
        d.opt.objective.hist = thr ? own.hist.data() : nullptr;
        d.opt.run_id = (uint32_t)i;
        out.push_back(d);
        ++i;
    }
    return out;
}

void exercise(const char *name, const std::vector<RunSpec> &rs) {
    Owned own;
    std::vector<apo_run_desc> d = descs(rs, own);
    const int n = (int)d.size();
    const size_t bytes = apo_batch_workspace_bytes(n, d.data());
    CHECK(bytes > 0, "%s: workspace size", name);
    if (!bytes) return;
    void *ws = nullptr;
    hipMalloc(&ws, bytes);
    apo_batch_options o;
    std::memset(&o, 0, sizeof(o));
    o.workspace = ws;
    o.workspace_bytes = bytes;
    apo_batch_t *b = nullptr;
    g_members = n;
    const int rc = apo_batch_create(n, d.data(), &o, &b);
    CHECK(rc == APO_OK, "%s: create %d", name, rc);
    if (rc != APO_OK) {
        hipFree(ws);
        return;
    }
    int32_t sched = -1;
    double us[4];
    CHECK(apo_batch_tune(b, 16, &sched, us) == APO_OK, "%s: tune", name);
    CHECK(apo_batch_run(b, 20) == 20, "%s: run 20", name);
    CHECK(apo_batch_run(b, 100) == 100, "%s: run 100", name);
    for (int s = 0; s < 4; ++s) {   // every schedule, then more iterations
        CHECK(apo_batch_tune(b, 16, &sched, us) == APO_OK, "%s: retune", name);
        CHECK(apo_batch_run(b, 17) == 17, "%s: run 17", name);
    }
    apo_t *h = nullptr;
    CHECK(apo_batch_member(b, n - 1, &h) == APO_OK, "%s: member", name);
    int32_t t = -1;
    int64_t fes = 0;
    CHECK(apo_info(h, &t, &fes) == APO_OK && t == 188, "%s: member at t %d", name, t);
    CHECK(apo_batch_destroy(b) == APO_OK, "%s: destroy", name);
    hipFree(ws);
    std::printf("%s: %d runs, schedule %d\n", name, n, sched);
}

}  // namespace

int main() {
    const int dims[] = {10, 20, 50, 100}, pops[] = {64, 256, 1024};
    const int kinds[] = {APO_RASTRIGIN, APO_ROSENBROCK, APO_ACKLEY};
    std::vector<RunSpec> all;
    for (int i = 0; i < 512; ++i) {   // the 512-run batched configuration's mix
        const int c = i % 36;
        all.push_back({dims[c / 9], pops[(c / 3) % 3], kinds[c % 3], APO_FP32, 1, true});
    }
    exercise("all", all);
    for (int ps : pops) {
        std::vector<RunSpec> v;
        for (const RunSpec &r : all)
            if (r.pop == ps) v.push_back(r);
        exercise(("pop" + std::to_string(ps)).c_str(), v);
    }
    for (int dm : dims) {
        std::vector<RunSpec> v;
        for (const RunSpec &r : all)
            if (r.dim == dm) v.push_back(r);
        exercise(("dim" + std::to_string(dm)).c_str(), v);
    }
    std::vector<RunSpec> mixed = {
        {10, 64, APO_RASTRIGIN, APO_FP32, 1, true},   {20, 130, APO_ROSENBROCK, APO_FP32, 1, true},
        {50, 64, APO_ACKLEY, APO_FP32, 1, true},      {100, 130, APO_RASTRIGIN, APO_FP32, 1, true},
        {10, 32, APO_RASTRIGIN, APO_FP64, 1, false},  {4, 70, APO_KAPUR, APO_FP32, 1, false},
        {33, 50, APO_ACKLEY, APO_FP64, 3, false},     {40, 2000, APO_SPHERE, APO_FP32, 1, true},
        {100, 1500, APO_ROSENBROCK, APO_FP64, 2, true}};
    exercise("mixed", mixed);
    exercise("all again", all);
    CHECK(g_streams.empty(), "%zu streams left", g_streams.size());
    CHECK(g_events.empty(), "%zu events left", g_events.size());
    CHECK(g_graphs.empty(), "%zu graphs left", g_graphs.size());
    CHECK(g_allocs.empty(), "%zu allocations left", g_allocs.size());
    std::printf("launches %ld, graph replays %ld\n", g_launches, g_replays);
    if (g_fail) {
        std::printf("FAILED %d checks\n", g_fail);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
