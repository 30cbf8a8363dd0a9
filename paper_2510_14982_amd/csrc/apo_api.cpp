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
    size_t X[2], F, perm, Fs, drf, ctrl, p_ah, fscale, cnear, p_dr, lb, ub, shift, rotp, htab, hist,
        best, trY, trF, trOp, total;
    int Dp, Nt, Ks;
};

bool is_threshold(int kind) { return kind == apok::K_KAPUR || kind == apok::K_OTSU; }

Layout make_layout(int dim, int pop, const apo_options &o) {
    Layout L;
    std::memset(&L, 0, sizeof(L));
    const size_t es = o.precision == APO_FP64 ? 8 : 4;
    L.Dp = (int)align_up((size_t)dim, 64 / es);
    L.Nt = (dim + 15) / 16;
    // k-steps of 4, padded with zeros to 32 (dim <= 128) or a multiple of 8,
    // so the matrix-core loop runs unguarded in blocks of 8
    L.Ks = (dim + 3) / 4;
    L.Ks = L.Ks <= 32 ? 32 : (L.Ks + 7) / 8 * 8;
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
    L.rotp = o.objective.rot ? take((size_t)L.Ks * L.Nt * 64 * es) : 0;
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

int check_args(int32_t dim, const double *lb, const double *ub, int32_t pop, int32_t np,
               double pf_max, const apo_options *opt) {
    if (!opt || !lb || !ub) return APO_E_INVAL;
    if (dim < 1 || pop < 2 || np < 1 || np > apok::kMaxNp) return APO_E_INVAL;
    if (!(pf_max >= 0.0 && pf_max <= 1.0)) return APO_E_INVAL;
    if (opt->max_iter < 1) return APO_E_INVAL;
    if (opt->precision != APO_FP64 && opt->precision != APO_FP32) return APO_E_INVAL;
    const int kind = opt->objective.kind;
    if (kind < APO_SPHERE || kind > APO_OTSU) return APO_E_INVAL;
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
    if (tile) {
        const int lim = is_threshold(kind) ? 512 : (opt->precision == APO_FP64 ? 256 : 512);
        if (dim > lim) return APO_E_UNSUPPORTED;
    } else if (apok::chunks_for_dim(dim) < 0) {
        return APO_E_UNSUPPORTED;
    }
    return APO_OK;
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
    hipEvent_t ev[3];
    bool have_events;
};

#define APO_HIP(h, call)                       \
    do {                                       \
        if ((call) != hipSuccess) {            \
            (h)->poisoned = true;              \
            return APO_E_DEVICE;               \
        }                                      \
    } while (0)

extern "C" {

size_t apo_workspace_bytes(int32_t dim, int32_t pop, int32_t np, const apo_options *opt) {
    if (!opt || dim < 1 || pop < 2 || np < 1 || opt->max_iter < 1) return 0;
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
        for (int i = 0; i < 3; ++i) (void)hipEventDestroy(h->ev[i]);
    if (h->stream && !h->poisoned) (void)hipStreamSynchronize(h->stream);
    if (h->own_ws && h->ws) (void)hipFree(h->ws);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return APO_OK;
}

int apo_destroy(apo_t *h) { return destroy_impl(h); }

int apo_create(int32_t dim, const double *lb, const double *ub, int32_t pop, int32_t np,
               double pf_max, uint64_t seed, const apo_options *opt, apo_t **out) {
    if (!out) return APO_E_INVAL;
    *out = nullptr;
    const int chk = check_args(dim, lb, ub, pop, np, pf_max, opt);
    if (chk != APO_OK) return chk;
    const Layout L = make_layout(dim, pop, *opt);
    if (opt->workspace && opt->workspace_bytes < L.total) return APO_E_INVAL;

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
    p.rotp = p.rotated ? ws + L.rotp : nullptr;
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
    for (int r = 0; r < pop; ++r)
        pdr[r] = 0.5 * (1.0 - std::cos((1.0 - (double)(r + 1) / (double)pop) * kPi));

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
    if (p.rotated) {
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
    if (p.rotated)
        CREATE_HIP(hipMemcpyAsync(ws + L.rotp, vrot.data(), vrot.size(), hipMemcpyHostToDevice, s));
    if (is_threshold(p.kind)) {
        CREATE_HIP(hipMemcpyAsync(ws + L.hist, opt->objective.hist, 256 * 8, hipMemcpyHostToDevice, s));
        CREATE_HIP(apok::launch_hist_tables(p, (const uint64_t *)(ws + L.hist), s));
    }
    CREATE_HIP(apok::launch_init(p, h->fp64, s));
    CREATE_HIP(hipStreamSynchronize(s));   // host staging buffers go out of scope
#undef CREATE_HIP
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
    if (h->poisoned) return APO_E_DEVICE;
    int32_t n = h->T - h->t;
    if (iters < n) n = iters;
    if (n <= 0) return 0;
    if (!h->graph_tried) {
        h->graph_tried = true;
        capture_iterations(h, 1, &h->graph[0], &h->graph_exec[0]);
        if (h->graph_exec[0] && h->T >= kGraphBlock)
            capture_iterations(h, kGraphBlock, &h->graph[1], &h->graph_exec[1]);
    }
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
    if (h->poisoned) return APO_E_DEVICE;
    int32_t n = h->T - h->t;
    if (iters < n) n = iters;
    if (n <= 0) return APO_E_DONE;
    if (!h->have_events) {
        for (int i = 0; i < 3; ++i) APO_HIP(h, hipEventCreate(&h->ev[i]));
        h->have_events = true;
    }
    double sum_rank = 0.0, sum_step = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        APO_HIP(h, hipEventRecord(h->ev[0], h->stream));
        APO_HIP(h, apok::launch_rank(h->p, h->fp64, h->stream));
        APO_HIP(h, hipEventRecord(h->ev[1], h->stream));
        APO_HIP(h, apok::launch_step(h->p, h->fp64, h->stream));
        APO_HIP(h, hipEventRecord(h->ev[2], h->stream));
        APO_HIP(h, hipEventSynchronize(h->ev[2]));
        float a = 0.f, b = 0.f;
        APO_HIP(h, hipEventElapsedTime(&a, h->ev[0], h->ev[1]));
        APO_HIP(h, hipEventElapsedTime(&b, h->ev[1], h->ev[2]));
        sum_rank += a;
        sum_step += b;
        ++h->t;
    }
    avg_us[0] = 1000.0 * sum_rank / n;
    avg_us[1] = 1000.0 * sum_step / n;
    return n;
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

int apo_histogram_u8(const uint8_t *d_img, uint64_t n, uint32_t *d_hist, void *stream) {
    if (!d_hist || (!d_img && n > 0) || n >= (1ull << 32)) return APO_E_INVAL;
    if (apok::launch_histogram(d_img, n, d_hist, (hipStream_t)stream) != hipSuccess)
        return APO_E_DEVICE;
    return APO_OK;
}

}  // extern "C"
