// C ABI of libcaddelag: argument validation, workspace planning and the host
// orchestration of the kernels for each call of include/caddelag.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <initializer_list>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "caddelag.h"
#include "batch.h"
#include "kernels.h"
#include "tune.h"

using cdl::tune_arch;
using cdl::tune_get;
using cdl::tune_key;
using cdl::tune_put;
using cdl::tune_load;
using cdl::tune_save;
using cdl::tune_clear;
using cdl::tune_entries;

struct cdl_timer_rec {
    const char *name;
    hipEvent_t a, b;
};

struct cdl_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // Optional per-kernel timing: HIP events recorded on `stream` around each
    // kernel launch, resolved when the totals are read.
    int solve_depth = 0;   // > 0: total chain depth used by every solve iteration
    bool timing = false;
    std::vector<std::string> timing_only;   // empty: every scope is timed
    std::vector<cdl_timer_rec> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<int64_t, double>> totals;
    std::vector<std::string> names;   // stable order for cdl_timing_read
    // Asynchronous sequences: the last call's key and, once the same call
    // has been seen twice, its captured graph.
    int select_mode = 0;   // 0 bracketed median selection, 1 radix over the matrix only
    std::vector<uint64_t> seq_key;
    hipGraph_t seq_graph = nullptr;
    hipGraphExec_t seq_exec = nullptr;
    hipStream_t side = nullptr;   // second stream of asynchronous sequences (created on first use)
    hipStream_t extra[2] = {nullptr, nullptr};   // third and fourth (one-pass sequences)
    // Pinned host staging for device-to-host reads (grown on demand): a copy
    // into pageable memory is staged by the runtime one copy at a time.
    void *stage = nullptr;
    size_t stage_bytes = 0;
    // Launch-configuration tuning: 1 = time every candidate of a kernel
    // family the first time a shape is met (the process-wide table keeps the
    // fastest); `forced` pins a family's candidate on this context.
    int autotune = 0;
    std::map<std::string, int> forced;
};

// Device scratch of cdl_anomaly_scores_noalloc: a file-scope array that
// every device running the library holds once its code object is loaded
// there.  Host code never uses its name as an address: each device's address
// comes from hipGetSymbolAddress (resolved once per device by
// cdl_ctx_create) and only that pointer reaches kernels.
constexpr size_t kNoAllocScratchBytes = (size_t)160 << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
bool g_scratch_resolved[kMaxDevices];

// Resolves `device`'s address of the scratch array with that device current
// (the caller's current device is restored).  Failure leaves the pointer
// null, which only the allocation-free entry point reports.
void resolve_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices || g_scratch_resolved[device]) return;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (hipSetDevice(device) == hipSuccess) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_ptr[device] = p;
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    g_scratch_resolved[device] = true;
}

void *scratch_ptr(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

hipEvent_t take_event(cdl_ctx *c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

bool timing_selected(const cdl_ctx *c, const char *nm) {
    if (c->timing_only.empty()) return true;
    for (const auto &s : c->timing_only)
        if (s == nm) return true;
    return false;
}

constexpr size_t kStageInitBytes = 4096;

// One device-to-host read: `bytes` from device `src` into host `dst`.
struct HostRead {
    void *dst;
    const void *src;
    size_t bytes;
};

// Enqueues the reads on `stream` into the context's pinned staging buffer,
// synchronises that stream and copies the results out (every read in one
// round trip).
hipError_t read_to_host(cdl_ctx *c, hipStream_t stream, std::initializer_list<HostRead> reads) {
    size_t total = 0;
    for (const auto &r : reads) total += (r.bytes + 255) / 256 * 256;
    if (total > c->stage_bytes) {
        // no copy into the old buffer is pending: every read ends with a sync
        if (c->stage) (void)hipHostFree(c->stage);
        c->stage = nullptr;
        c->stage_bytes = 0;
        void *p = nullptr;
        const hipError_t e = hipHostMalloc(&p, total, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        c->stage = p;
        c->stage_bytes = total;
    }
    size_t off = 0;
    for (const auto &r : reads) {
        const hipError_t e = hipMemcpyAsync((char *)c->stage + off, r.src, r.bytes,
                                            hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) return e;
        off += (r.bytes + 255) / 256 * 256;
    }
    const hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    off = 0;
    for (const auto &r : reads) {
        std::memcpy(r.dst, (const char *)c->stage + off, r.bytes);
        off += (r.bytes + 255) / 256 * 256;
    }
    return hipSuccess;
}

// Brackets one kernel launch (or a fixed group of launches) with events.
struct Timed {
    cdl_ctx *c;
    const char *name;
    hipEvent_t a = nullptr;
    Timed(cdl_ctx *ctx, const char *nm) : c(ctx), name(nm) {
        if (c->timing && timing_selected(c, nm) && (a = take_event(c)) &&
            hipEventRecord(a, c->stream) != hipSuccess) {
            c->pool.push_back(a);
            a = nullptr;
        }
    }
    ~Timed() {
        if (!a) return;
        hipEvent_t b = take_event(c);
        if (!b) {
            c->pool.push_back(a);
            return;
        }
        if (hipEventRecord(b, c->stream) != hipSuccess) {
            c->pool.push_back(a);
            c->pool.push_back(b);
            return;
        }
        c->pending.push_back({name, a, b});
    }
};

void resolve_timers(cdl_ctx *c) {
    if (c->pending.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto &r : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ms = 0.f;
        auto it = c->totals.find(r.name);
        if (it == c->totals.end()) {
            c->names.push_back(r.name);
            it = c->totals.emplace(r.name, std::make_pair((int64_t)0, 0.0)).first;
        }
        it->second.first += 1;
        it->second.second += ms;
        c->pool.push_back(r.a);
        c->pool.push_back(r.b);
    }
    c->pending.clear();
}
} // namespace

namespace {

using namespace cdl;

// Candidate of a tuned kernel family for one shape: the context's forced
// one, else the table's choice, else 0 (*tune: the context tunes and the
// table has no entry yet).
int pick_choice(cdl_ctx *c, const char *family, int prec, int64_t ld, int64_t kp, int ncand,
                bool allow_tune, bool *tune) {
    *tune = false;
    auto f = c->forced.find(family);
    if (f != c->forced.end() && f->second >= 0 && f->second < ncand) return f->second;
    if (ncand <= 1) return 0;
    int ch = 0;
    if (cdl::tune_get(cdl::tune_arch(c->device), cdl::tune_key(family, prec, ld, kp), &ch, nullptr,
                      nullptr) && ch < ncand)
        return ch;
    *tune = allow_tune && c->autotune != 0;
    return 0;
}

// Mean milliseconds of the launches of fn() on the context's stream over
// `reps` timed calls after one untimed call (which takes the first-launch
// costs: code-object load, cold caches); syncs.
template <class F>
hipError_t time_launch(cdl_ctx *c, F &&fn, double *ms, int reps = 3) {
    hipEvent_t a = take_event(c), b = take_event(c);
    hipError_t e = (a && b) ? fn() : hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipEventRecord(a, c->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = fn();
    if (e == hipSuccess) e = hipEventRecord(b, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (a) c->pool.push_back(a);
    if (b) c->pool.push_back(b);
    *ms = (double)t / reps;
    return e;
}

constexpr size_t kAlign = 256;
size_t al(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

size_t esize(int prec) { return prec == 0 ? 8 : prec == 1 ? 4 : 2; }

// Bump allocator over a caller workspace (base == nullptr: size only).
struct Arena {
    char *base;
    size_t off = 0;
    explicit Arena(void *b) : base((char *)b) {}
    template <typename T> T *take(size_t count) {
        T *p = base ? (T *)(base + off) : nullptr;
        off += al(count * sizeof(T));
        return p;
    }
};

struct GraphWs {
    int *flags;
    SelectState *sel;
    unsigned long long *selbuf;
    double *sqn, *Xp, *dpart;
};
GraphWs plan_graph(Arena &a, int64_t n, int64_t T) {
    const int64_t ld = pad_n(n), Tp = pad_t(T);
    GraphWs w;
    w.flags = a.take<int>(64);
    w.sel = a.take<SelectState>(1);
    w.selbuf = a.take<unsigned long long>((size_t)select_buffer_keys(n));
    w.sqn = a.take<double>(ld);
    w.Xp = a.take<double>((size_t)ld * Tp);
    w.dpart = a.take<double>((size_t)(ld / 64) * ld);
    return w;
}

struct ChainBuf {
    double *dmn, *dm, *u, *fro, *fro64;
    float *tail;   // partial tiles of a squaring's last round (nullptr: none)
    char *levels;
    size_t level_bytes;
};
ChainBuf plan_chain(Arena &a, int64_t n, int prec, int depth_max) {
    const int64_t ld = pad_n(n);
    ChainBuf c;
    c.dmn = a.take<double>(ld);
    c.dm = a.take<double>(ld);
    c.u = a.take<double>(ld);
    c.fro = a.take<double>(std::max<int64_t>(sym_tiles64(ld), square_tiles(prec, ld)));
    c.fro64 = a.take<double>(sym_tiles64(ld));
    const size_t tb = square_tail_bytes(prec, ld, n);
    c.tail = tb ? a.take<float>(tb / sizeof(float)) : nullptr;
    c.level_bytes = (size_t)ld * ld * esize(prec);
    c.levels = a.take<char>(c.level_bytes * depth_max);
    return c;
}

struct SolveWs {
    double *Yt, *Xt, *Rt, *V64, *T64, *npart, *mpart, *scal, *mean;
    double *Pt, *Qt, *Zt, *pcg, *dots;   // conjugate-gradient state
    void *Vlo[4];
    void *part;   // split-K partials of the residual and the chain application
};
SolveWs plan_solve(Arena &a, int64_t n, int64_t k, int prec) {
    const int64_t ld = pad_n(n), kp = pad_k(k);
    const size_t panel = (size_t)kp * ld;
    SolveWs w;
    // split-K partials for the largest candidate split counts
    w.part = a.take<char>(panel * std::max<size_t>(8 * (size_t)residual_splits(ld, kp, n, 2),
                                                   4 * (size_t)apply_splits(prec, ld, kp, n, 2)));
    w.Yt = a.take<double>(panel);
    w.Xt = a.take<double>(panel);
    w.Rt = a.take<double>(panel);
    w.V64 = a.take<double>(panel);
    w.T64 = a.take<double>(panel);
    for (int q = 0; q < 4; ++q) w.Vlo[q] = a.take<char>(panel * esize(prec));
    w.npart = a.take<double>((size_t)residual_parts(ld) * kp);
    w.mpart = a.take<double>(residual_tiles(ld, kp));
    w.scal = a.take<double>(kp + 2);
    w.mean = a.take<double>(kp);
    w.Pt = a.take<double>(panel);
    w.Qt = a.take<double>(panel);
    w.Zt = a.take<double>(panel);
    w.pcg = a.take<double>(3 * (size_t)kp);
    w.dots = a.take<double>(2 * (size_t)residual_parts(ld) * kp);
    return w;
}

struct ScoreWs {
    double *Zh, *Zhe, *sq, *part;
    void *topk;
};
ScoreWs plan_score(Arena &a, int64_t m, int64_t k) {
    const int64_t mp = pad_n(m), kp = pad_k(k);
    ScoreWs w;
    w.Zh = a.take<double>((size_t)mp * 2 * kp);
    w.Zhe = a.take<double>((size_t)mp * 2 * kp);
    w.sq = a.take<double>(mp);
    w.part = a.take<double>((size_t)score_tiles_1d(mp) * mp);
    const int64_t cap = topk_scratch_elems(m, CDL_MAX_TOPK);
    w.topk = a.take<char>((size_t)cap * (2 * sizeof(double) + 2 * sizeof(int32_t)));
    return w;
}

struct EdgeWs {
    ScoreWs sw;
    double *tmax, *tau, *cval, *vals;
    int32_t *order;
    int64_t *cidx, *idx;
    unsigned int *count;
    void *tscratch, *cscratch;
    int64_t cap;
};
int64_t edge_cap(int64_t m, int K) {
    const int64_t pairs = m * (m - 1) / 2;
    return std::min<int64_t>(std::max<int64_t>((int64_t)K * 16384, (int64_t)1 << 22), pairs);
}
EdgeWs plan_edges(Arena &a, int64_t m, int64_t k, int K) {
    EdgeWs w;
    w.sw = plan_score(a, m, k);
    const int64_t nt2 = score_tiles_2d(pad_n(m));
    w.tmax = a.take<double>(nt2);
    w.order = a.take<int32_t>(std::max(K, 1));
    w.tscratch = a.take<char>((size_t)topk_scratch_elems(nt2, K) * (2 * sizeof(double) + 2 * sizeof(int32_t)));
    w.tau = a.take<double>(1);
    w.count = a.take<unsigned int>(4);
    w.cap = edge_cap(m, K);
    w.cval = a.take<double>(w.cap);
    w.cidx = a.take<int64_t>(w.cap);
    w.cscratch = a.take<char>((size_t)topk_scratch_elems(w.cap, K) * (2 * sizeof(double) + 2 * sizeof(int64_t)));
    w.vals = a.take<double>(std::max(K, 1));
    w.idx = a.take<int64_t>(std::max(K, 1));
    return w;
}

// Streamed snapshot: the series, one row panel of the distances / weights
// and the solve's kpad x ld panels; nothing of size n x n.  With a stored
// chain level (level_prec >= 0) the solve's panels are those of the stored
// path's solve (plan_solve), the level lives in the caller's chain buffer.
struct StreamWs {
    int *flags;
    SelectState *sel;
    unsigned long long *selbuf;   // keys inside the sampled bracket
    double *sqn, *Xp, *panel;
    double *Yt, *Xt, *Rt, *Ut, *Prod;
    double *npart, *mpart, *scal, *mean, *dinv, *rdeg, *fro, *fro64;
    SolveWs sw;
    int64_t prow;   // rows per panel
};
int64_t stream_panel_rows(int64_t n, int64_t panel_rows) {
    const int64_t ld = pad_n(n);
    int64_t p = panel_rows > 0 ? panel_rows : 32768;
    p = (p + 255) / 256 * 256;
    return std::min(p, ld);
}
StreamWs plan_stream(Arena &a, int64_t n, int64_t T, int64_t k, int64_t panel_rows,
                     int level_prec) {
    const int64_t ld = pad_n(n), Tp = pad_t(T), kp = pad_k(k);
    const size_t kpan = (size_t)kp * ld;
    StreamWs w;
    std::memset(&w, 0, sizeof(w));
    w.prow = stream_panel_rows(n, panel_rows);
    w.flags = a.take<int>(64);
    w.sel = a.take<SelectState>(1);
    w.selbuf = a.take<unsigned long long>((size_t)select_stream_keys(n));
    w.sqn = a.take<double>(ld);
    w.Xp = a.take<double>((size_t)ld * Tp);
    w.panel = a.take<double>((size_t)w.prow * ld);
    w.dinv = a.take<double>(ld);
    w.rdeg = a.take<double>(ld);
    w.fro = a.take<double>(ld);
    w.fro64 = a.take<double>(ld);
    if (level_prec >= 0) {
        w.sw = plan_solve(a, n, k, level_prec);
        w.Yt = w.sw.Yt;
        w.Xt = w.sw.Xt;
        w.Prod = (double *)w.sw.part;
        return w;
    }
    w.Yt = a.take<double>(kpan);
    w.Xt = a.take<double>(kpan);
    w.Rt = a.take<double>(kpan);
    w.Ut = a.take<double>(kpan);
    w.Prod = a.take<double>(kpan);
    w.npart = a.take<double>((size_t)residual_parts(ld) * kp);
    w.mpart = a.take<double>(residual_tiles(ld, kp));
    w.scal = a.take<double>(kp + 2);
    w.mean = a.take<double>(kp);
    return w;
}

cdl_status fail(cdl_ctx *c, cdl_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, CDL_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Stream-ordered graph construction (arguments already checked).
cdl_status graph_enqueue(cdl_ctx *ctx, const double *X, int64_t n, int64_t T, int64_t ldx,
                         double sigma, double *W, double *deg, double *stats, void *ws) {
    Arena a(ws);
    GraphWs w = plan_graph(a, n, T);
    const int64_t ld = pad_n(n), Tp = pad_t(T);
    hipStream_t s = ctx->stream;
    { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w.flags, 256, s)); }
    { Timed t_(ctx, "pad_series"); HIPCHK(launch_pad_series(X, n, T, ldx, w.Xp, ld, Tp, w.sqn, w.flags, s)); }
    // the median's bracket comes from a sample taken from the series, so that
    // the Gram's epilogue can count and gather it (no pass over D2 for it)
    const bool br = sigma <= 0.0 && select_uses_bracket(n, ctx->select_mode == 0);
    if (sigma <= 0.0) { Timed t_(ctx, "select_median"); HIPCHK(launch_select_reset(w.sel, s)); }
    if (br) { Timed t_(ctx, "select_median"); HIPCHK(launch_select_presample(w.Xp, Tp, w.sqn, n, w.sel, w.selbuf, s)); }
    { Timed t_(ctx, "gram_dist"); HIPCHK(launch_gram_dist(w.Xp, Tp, w.sqn, n, ld, W, sigma > 0.0 ? nullptr : w.sel,
                                                          br ? w.selbuf : nullptr, select_buffer_keys(n), s)); }
    if (sigma > 0.0)
        { Timed t_(ctx, "set_sigma"); HIPCHK(launch_set_sigma(sigma, stats, s)); }
    else
        { Timed t_(ctx, "select_median"); HIPCHK(launch_select_median(W, ld, n, w.sel, w.selbuf, br, stats, s)); }
    { Timed t_(ctx, "exp_degree"); HIPCHK(launch_exp_degree(W, ld, n, stats, deg, w.dpart, s)); }
    { Timed t_(ctx, "graph_stats"); HIPCHK(launch_graph_stats(deg, n, stats, s)); }
    return CDL_OK;
}

// Xdst += P1 r, P1 = D^{-1/2} prod_{l<D} (I + S~^{2^l}) D^{-1/2}, for the
// operand V = D^{-1/2} r left in V64 / Vlo[0] by the residual step (FP16: the
// scaled copy is made here).  Levels l >= d are applied as 2^(l-d+1)
// repetitions of the last stored level.  Stream-ordered, no host reads.
cdl_status precondition_enqueue(cdl_ctx *ctx, int prec, int d, int D, const SolveWs &w,
                                const ChainBuf &c, int64_t ld, int64_t n, int64_t kp,
                                bool scaled, const double *inv_vs, double *Xdst,
                                bool allow_tune = true) {
    hipStream_t s = ctx->stream;
    if (scaled) { Timed t_(ctx, "prep_v"); HIPCHK(launch_prep_v2(prec, w.Rt, c.dm, ld, kp, w.scal + kp, w.V64, w.Vlo[0], s)); }
    bool tune = false;
    const int nc = prec == 0 ? 1 : 3;
    int ch = pick_choice(ctx, "apply", prec, ld, kp, nc, allow_tune, &tune);
    if (tune) {
        // one whole application per candidate (split-K product and its
        // reduction, whose reads grow with the split count) into scratch
        // panels: T64 and Vlo[2] take the result, V and X stay untouched
        std::vector<double> ms(nc);
        for (int q = 0; q < nc; ++q)
            HIPCHK(time_launch(ctx, [&] {
                return launch_apply(prec, w.Vlo[0], c.levels, w.Vlo[2], w.T64, ld, n, kp, nullptr,
                                    c.dm, nullptr, (float *)w.part, 0, apply_splits(prec, ld, kp, n, q), s);
            }, &ms[q]));
        ch = cdl::tune_put(cdl::tune_arch(ctx->device), cdl::tune_key("apply", prec, ld, kp), ms);
    }
    const int ns = apply_splits(prec, ld, kp, n, ch);
    int cur = 0;
    for (int l = 0; l < std::min(d, D); ++l) {
        const bool last = l + 1 == D;
        { Timed t_(ctx, "apply"); HIPCHK(launch_apply(prec, w.Vlo[cur], c.levels + c.level_bytes * l, w.Vlo[cur ^ 1],
                            w.V64, ld, n, kp, Xdst, c.dm, last ? inv_vs : nullptr, (float *)w.part, 1, ns, s)); }
        cur ^= 1;
    }
    for (int l = d; l < D; ++l) {
        const int m = 1 << (l - d + 1);
        const void *src = w.Vlo[cur];
        for (int q = 0; q < m; ++q) {
            void *dst = w.Vlo[2 + (q & 1)];
            { Timed t_(ctx, "apply"); HIPCHK(launch_apply(prec, src, c.levels + c.level_bytes * (d - 1), dst, w.T64,
                                ld, n, kp, Xdst, c.dm, nullptr, (float *)w.part, 0, ns, s)); }
            src = dst;
        }
        const bool last = l + 1 == D;
        { Timed t_(ctx, "axpy_v"); HIPCHK(launch_axpy_v(prec, w.T64, ld, kp, w.V64, w.Vlo[cur ^ 1], Xdst, c.dm,
                             last ? inv_vs : nullptr, s)); }
        cur ^= 1;
    }
    return CDL_OK;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }
bool valid_prec(int p) { return p >= 0 && p <= 3; }

// ---- depth model ----------------------------------------------------------

double peak_flops(int prec) {
    switch (prec) {
    case 0: return 78.6e12;
    case 1: return 157.3e12;
    default: return 2.5e15;
    }
}
double unit_roundoff(int prec) {
    switch (prec) {
    case 0: return std::ldexp(1.0, -53);
    case 1: return std::ldexp(1.0, -24);
    case 2: return std::ldexp(1.0, -8);
    default: return std::ldexp(1.0, -11);
    }
}
double iters_for(double c, double tol) {
    if (!(c < 1.0)) return 1e30;
    if (c <= 0.0) return 1.0;
    return std::max(1.0, std::ceil(std::log(tol) / std::log(c)));
}
// Rounding floor of one preconditioner application with levels of the given
// type, relative to the residual it reduces (calibrated on Gaussian-kernel
// graphs at n = 16384: ~8e-4 times the storage unit roundoff; FP32
// accumulation of the products sets a 1e-9 floor).
double apply_floor(int prec) {
    switch (prec) {
    case 0: return 1e-15;
    case 1: return 1e-9;
    default: return std::max(1e-9, 8e-4 * unit_roundoff(prec));
    }
}
// Level applications for total depth D over d stored levels: the stored ones
// once each, level l >= d as 2^(l-d+1) applications of the last stored level.
int applies_for(int d, int D) { return D <= d ? D : d + (1 << (D - d + 1)) - 2; }
// Kernel times of the depth model for n nodes, k columns and level type
// prec: the tuner's measured times of the chosen configurations when its
// table holds this exact shape (split-K products only: their reductions are
// small), else estimates at fixed fractions of the peaks (the FP64 residual
// at 3/4 of the FP64 MFMA peak, applications at half the level type's MFMA
// peak or at the HBM rate, whichever is slower, squarings at half the peak).
struct CostModel {
    double t_res, t_ap, t_sq;
    bool measured_res = false, measured_ap = false, measured_sq = false;
};
CostModel cost_model(int device, int prec, int64_t n, int64_t k) {
    const double nn = (double)n, kk = (double)k;
    CostModel m;
    m.t_res = 2.0 * nn * nn * kk / (78.6e12 * 0.75);
    m.t_ap = std::max(2.0 * nn * nn * kk / (peak_flops(prec) * 0.5), nn * nn * esize(prec) / 4.0e12);
    m.t_sq = nn * nn * nn / (peak_flops(prec) * 0.5);
    const std::string arch = tune_arch(device);
    const int64_t ld = pad_n(n), kp = pad_k(k);
    double ms = 0.0;
    if (tune_get(arch, tune_key("residual", 0, ld, kp), nullptr, &ms, nullptr) && ms > 0.0) {
        m.t_res = ms * 1e-3;
        m.measured_res = true;
    }
    if (prec != 0 && tune_get(arch, tune_key("apply", prec, ld, kp), nullptr, &ms, nullptr) && ms > 0.0) {
        m.t_ap = ms * 1e-3;
        m.measured_ap = true;
    }
    if (tune_get(arch, tune_key("square", prec, ld, 0), nullptr, &ms, nullptr) && ms > 0.0) {
        m.t_sq = ms * 1e-3;
        m.measured_sq = true;
    }
    return m;
}

// Depth for the next iteration: minimise (iterations to gain `need`) x (FP64
// residual + level applications), with contraction max(rho^(2^D), floor).
int choose_depth(int prec, int d, double rho, double need, const CostModel &m) {
    if (!(need < 1.0)) return d;
    const double r = std::min(std::max(rho, 1e-6), 0.999999);
    int best = d;
    double best_cost = 1e300;
    for (int D = 1; D <= d + 3 && D <= 16; ++D) {
        const double c = std::max(std::pow(r, std::ldexp(1.0, D)), apply_floor(prec));
        const double it = iters_for(c, need);
        const double cost = it * (m.t_res + applies_for(d, D) * m.t_ap);
        if (cost < best_cost * (1.0 - 1e-9)) {
            best_cost = cost;
            best = D;
        }
    }
    return best;
}

// Predicted time of one solve that must gain `need` with d stored levels,
// using the best total depth per iteration (same model as choose_depth).
double solve_cost(int prec, int d, double rho, double need, const CostModel &m) {
    const double r = std::min(std::max(rho, 1e-6), 0.999999);
    double best = 1e300;
    for (int D = 1; D <= d + 3 && D <= 16; ++D) {
        const double c = std::max(std::pow(r, std::ldexp(1.0, D)), apply_floor(prec));
        best = std::min(best, iters_for(c, need) * (m.t_res + applies_for(d, D) * m.t_ap));
    }
    return best;
}
// Should the chain with levels 0..l (last Frobenius norm f, spectral estimate
// rho) get level l+1?  Yes when one squaring plus the cheapest solve with
// l+2 stored levels is predicted to beat the cheapest solve with l+1 (model
// times for k = 256 columns, a 1e-8 residual target; deeper levels can
// always be applied by repetition instead).
bool model_wants_square(int prec, int l, double f, double rho, const CostModel &m) {
    (void)f;
    if (!(rho < 1.0 - 1e-9)) return true;   // not contracting yet: keep testing
    const double need = 1e-8;
    return m.t_sq + solve_cost(prec, l + 2, rho, need, m) < solve_cost(prec, l + 1, rho, need, m);
}

} // namespace

extern "C" {

const char *cdl_version(void) { return "caddelag-gfx950 1.0"; }

const char *cdl_status_string(cdl_status s) {
    switch (s) {
    case CDL_OK: return "ok";
    case CDL_E_ARG: return "invalid argument";
    case CDL_E_WORKSPACE: return "workspace too small";
    case CDL_E_NONFINITE: return "non-finite value";
    case CDL_E_GRAPH: return "invalid graph";
    case CDL_E_DIVERGED: return "chain does not contract";
    case CDL_E_NOCONV: return "solve did not converge";
    case CDL_E_HIP: return "HIP runtime error";
    case CDL_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *cdl_last_error(const cdl_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

cdl_status cdl_ctx_create(int device, void *stream, cdl_ctx **out) {
    if (!out) return CDL_E_ARG;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return CDL_E_ARG;
    cdl_ctx *c = new (std::nothrow) cdl_ctx;
    if (!c) return CDL_E_HIP;
    c->device = device;
    c->stream = (hipStream_t)stream;
    resolve_scratch(device);
    // a first pinned staging buffer, so that small read-backs (the
    // allocation-free entry point's flag) never allocate
    void *p = nullptr;
    if (hipHostMalloc(&p, kStageInitBytes, hipHostMallocDefault) == hipSuccess) {
        c->stage = p;
        c->stage_bytes = kStageInitBytes;
    }
    *out = c;
    return CDL_OK;
}

cdl_status cdl_ctx_destroy(cdl_ctx *ctx) {
    if (!ctx) return CDL_OK;
    if (!ctx->pending.empty()) (void)hipStreamSynchronize(ctx->stream);
    for (auto &r : ctx->pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    if (ctx->seq_exec) (void)hipGraphExecDestroy(ctx->seq_exec);
    if (ctx->seq_graph) (void)hipGraphDestroy(ctx->seq_graph);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    for (hipStream_t x : ctx->extra)
        if (x) (void)hipStreamDestroy(x);
    if (ctx->stage) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipHostFree(ctx->stage);
    }
    delete ctx;
    return CDL_OK;
}

cdl_status cdl_ctx_set_solve_depth(cdl_ctx *ctx, int depth) {
    if (!ctx || depth < 0 || depth > 16) return CDL_E_ARG;
    ctx->solve_depth = depth;
    return CDL_OK;
}

cdl_status cdl_ctx_set_select(cdl_ctx *ctx, int mode) {
    if (!ctx || mode < 0 || mode > 1) return CDL_E_ARG;
    ctx->select_mode = mode;
    return CDL_OK;
}

cdl_status cdl_ctx_set_timing(cdl_ctx *ctx, int enable) {
    if (!ctx) return CDL_E_ARG;
    ctx->timing = enable != 0;
    return CDL_OK;
}

cdl_status cdl_ctx_set_timing_only(cdl_ctx *ctx, const char *names) {
    if (!ctx) return CDL_E_ARG;
    ctx->timing_only.clear();
    if (!names) return CDL_OK;
    std::string cur;
    for (const char *p = names;; ++p) {
        if (*p == ',' || *p == '\0') {
            if (!cur.empty()) ctx->timing_only.push_back(cur);
            cur.clear();
            if (!*p) break;
        } else if (*p != ' ') {
            cur.push_back(*p);
        }
    }
    return CDL_OK;
}

cdl_status cdl_timing_reset(cdl_ctx *ctx) {
    if (!ctx) return CDL_E_ARG;
    resolve_timers(ctx);
    ctx->totals.clear();
    ctx->names.clear();
    return CDL_OK;
}

cdl_status cdl_timing_read(cdl_ctx *ctx, int32_t idx, const char **name, int64_t *launches,
                           double *total_ms) {
    if (!ctx || !name || !launches || !total_ms) return CDL_E_ARG;
    resolve_timers(ctx);
    if (idx < 0 || idx >= (int32_t)ctx->names.size()) return CDL_E_ARG;
    const std::string &nm = ctx->names[idx];
    const auto &v = ctx->totals[nm];
    *name = nm.c_str();
    *launches = v.first;
    *total_ms = v.second;
    return CDL_OK;
}

cdl_status cdl_ctx_set_stream(cdl_ctx *ctx, void *stream) {
    if (!ctx) return CDL_E_ARG;
    ctx->stream = (hipStream_t)stream;
    return CDL_OK;
}

cdl_status cdl_ctx_set_autotune(cdl_ctx *ctx, int mode) {
    if (!ctx || mode < 0 || mode > 1) return CDL_E_ARG;
    ctx->autotune = mode;
    return CDL_OK;
}

static bool tuned_family(const char *f) {
    return f && (!std::strcmp(f, "square") || !std::strcmp(f, "apply") || !std::strcmp(f, "residual"));
}

cdl_status cdl_ctx_force_choice(cdl_ctx *ctx, const char *family, int choice) {
    if (!ctx || !tuned_family(family)) return CDL_E_ARG;
    if (choice < 0) ctx->forced.erase(family);
    else ctx->forced[family] = choice;
    return CDL_OK;
}

cdl_status cdl_autotune_lookup(int device, const char *family, cdl_prec prec, int64_t n, int64_t k,
                               int *choice, int *candidates, double *ms) {
    if (!tuned_family(family) || !valid_prec(prec) || n < 2 || n > (1 << 20)) return CDL_E_ARG;
    const bool sq = !std::strcmp(family, "square");
    if (!sq && k < 1) return CDL_E_ARG;
    const std::string key = tune_key(family, prec, pad_n(n), sq ? 0 : pad_k(k));
    if (!tune_get(tune_arch(device), key, choice, ms, candidates)) return CDL_E_UNSUPPORTED;
    return CDL_OK;
}

cdl_status cdl_autotune_load(const char *path) {
    if (!path) return CDL_E_ARG;
    return tune_load(path, nullptr) ? CDL_OK : CDL_E_ARG;
}

cdl_status cdl_autotune_save(const char *path) {
    if (!path) return CDL_E_ARG;
    return tune_save(path, nullptr) ? CDL_OK : CDL_E_ARG;
}

cdl_status cdl_autotune_clear(void) {
    tune_clear();
    return CDL_OK;
}

int32_t cdl_autotune_entries(void) { return tune_entries(); }

int64_t cdl_ld(int64_t n) { return n > 0 ? pad_n(n) : 0; }

cdl_status cdl_k_rp(int64_t n, double eps_rp, int64_t *k) {
    if (!k || n < 2 || !(eps_rp > 0.0 && eps_rp < 1.0)) return CDL_E_ARG;
    *k = (int64_t)std::ceil(std::log((double)n / eps_rp));
    return CDL_OK;
}

cdl_status cdl_device_copy(cdl_ctx *ctx, const void *src, void *dst, size_t bytes) {
    if (!ctx) return CDL_E_ARG;
    if (bytes == 0) return CDL_OK;
    if (!src || !dst || bytes % 16 || !aligned(src, 16) || !aligned(dst, 16))
        return fail(ctx, CDL_E_ARG, "device copy: NULL, unaligned or not a multiple of 16 bytes");
    const char *a = (const char *)src, *b = (const char *)dst;
    if (a < b + bytes && b < a + bytes) return fail(ctx, CDL_E_ARG, "device copy: buffers overlap");
    HIPCHK(launch_copy16(src, dst, bytes, ctx->stream));
    return CDL_OK;
}

cdl_status cdl_level_scale(int64_t n, cdl_prec prec, double *scale) {
    if (!scale || n < 1 || !valid_prec(prec)) return CDL_E_ARG;
    *scale = (double)level_scale(prec, n);
    return CDL_OK;
}

size_t cdl_chain_level_offset(int64_t n, cdl_prec prec) {
    if (n < 2 || !valid_prec(prec)) return 0;
    Arena a(nullptr);
    plan_chain(a, n, prec, 0);
    return a.off;
}

size_t cdl_matrix_bytes(int64_t n, cdl_prec prec) {
    if (n <= 0 || !valid_prec(prec)) return 0;
    const size_t ld = (size_t)pad_n(n);
    return ld * ld * esize(prec);
}

cdl_status cdl_workspace_bytes(int64_t n, int64_t T, int64_t k, int depth_max, cdl_prec prec,
                               size_t *graph, size_t *chain, size_t *solve, size_t *score) {
    if (n < 2 || n > (1 << 20) || T < 1 || k < 1 || depth_max < 1 ||
        depth_max > CDL_MAX_DEPTH || !valid_prec(prec))
        return CDL_E_ARG;
    if (graph) { Arena a(nullptr); plan_graph(a, n, T); *graph = a.off; }
    if (chain) { Arena a(nullptr); plan_chain(a, n, prec, depth_max); *chain = a.off; }
    if (solve) { Arena a(nullptr); plan_solve(a, n, k, prec); *solve = a.off; }
    if (score) { Arena a(nullptr); plan_score(a, n, k); *score = a.off; }
    return CDL_OK;
}

// ---- graph -------------------------------------------------------------------

cdl_status cdl_build_graph(cdl_ctx *ctx, const double *X, int64_t n, int64_t T, int64_t ldx,
                           double sigma, double *W, double *deg, double *stats, void *ws,
                           size_t ws_bytes) {
    if (!ctx) return CDL_E_ARG;
    if (n < 2 || n > (1 << 20)) return fail(ctx, CDL_E_ARG, "n must be in [2, 2^20]");
    if (T < 1 || ldx < T) return fail(ctx, CDL_E_ARG, "need T >= 1 and ldx >= T");
    if (!X || !W || !deg || !stats || !ws) return fail(ctx, CDL_E_ARG, "null pointer");
    if (!aligned(X, 8) || !aligned(W, 16) || !aligned(deg, 8) || !aligned(stats, 8) ||
        !aligned(ws, kAlign))
        return fail(ctx, CDL_E_ARG, "misaligned pointer");
    if (!std::isfinite(sigma)) return fail(ctx, CDL_E_ARG, "sigma must be finite");
    Arena need(nullptr);
    plan_graph(need, n, T);
    if (ws_bytes < need.off) return fail(ctx, CDL_E_WORKSPACE, "graph workspace too small");
    HIPCHK(hipSetDevice(ctx->device));
    return graph_enqueue(ctx, X, n, T, ldx, sigma, W, deg, stats, ws);
}

cdl_status cdl_check_graph(cdl_ctx *ctx, const double *deg, const double *stats, int64_t n,
                           double *host_stats) {
    if (!ctx) return CDL_E_ARG;
    if (!deg || !stats || n < 2) return fail(ctx, CDL_E_ARG, "bad arguments");
    double h[CDL_GRAPH_STATS];
    HIPCHK(read_to_host(ctx, ctx->stream, {{h, stats, sizeof(h)}}));
    if (host_stats) std::memcpy(host_stats, h, sizeof(h));
    for (double v : h)
        if (!std::isfinite(v)) return fail(ctx, CDL_E_NONFINITE, "non-finite weights or degrees");
    if (!(h[2] > 0.0)) return fail(ctx, CDL_E_GRAPH, "a node has zero degree");
    return CDL_OK;
}

cdl_status cdl_graph_from_weights(cdl_ctx *ctx, const double *Win, int64_t n, int64_t ldw,
                                  double *W, double *deg, double *stats, void *ws,
                                  size_t ws_bytes) {
    if (!ctx) return CDL_E_ARG;
    if (n < 2 || n > (1 << 20) || ldw < n) return fail(ctx, CDL_E_ARG, "bad n or ldw");
    if (!Win || !W || !deg || !stats || !ws) return fail(ctx, CDL_E_ARG, "null pointer");
    if (!aligned(Win, 8) || !aligned(W, 16) || !aligned(ws, kAlign))
        return fail(ctx, CDL_E_ARG, "misaligned pointer");
    if (ws_bytes < 256) return fail(ctx, CDL_E_WORKSPACE, "graph workspace too small");
    hipStream_t s = ctx->stream;
    int *flags = (int *)ws;
    const int64_t ld = pad_n(n);
    HIPCHK(hipSetDevice(ctx->device));
    { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(flags, 256, s)); }
    { Timed t_(ctx, "import_weights"); HIPCHK(launch_import_weights(Win, ldw, n, W, ld, deg, flags, s)); }
    { Timed t_(ctx, "set_sigma"); HIPCHK(launch_set_sigma(0.0, stats, s)); }
    { Timed t_(ctx, "graph_stats"); HIPCHK(launch_graph_stats(deg, n, stats, s)); }
    int hf = 0;
    HIPCHK(read_to_host(ctx, s, {{&hf, flags, sizeof(int)}}));
    if (hf & 1) return fail(ctx, CDL_E_NONFINITE, "non-finite weight");
    if (hf & 2) return fail(ctx, CDL_E_GRAPH, "negative weight");
    if (hf & 4) return fail(ctx, CDL_E_GRAPH, "asymmetric weights");
    return cdl_check_graph(ctx, deg, stats, n, nullptr);
}

// ---- chain ---------------------------------------------------------------------

// One squaring (or dense-chain product when A != B) with the tuned tile
// variant; a tuning context times every variant first (each leaves a
// complete, correct output).
static cdl_status square_step(cdl_ctx *ctx, int prec, const void *A, const void *B, void *C,
                              int64_t ld, int64_t n, const ChainBuf &c, bool allow_tune) {
    const bool product = A != B;
    bool tune = false;
    const int nv = square_variants(prec);
    int v = pick_choice(ctx, "square", prec, ld, 0, nv, allow_tune, &tune);
    auto go = [&](int var) {
        return product ? launch_chain_product(prec, A, B, C, ld, n, c.fro, c.tail, var, ctx->stream)
                       : launch_square(prec, A, C, ld, n, c.fro, c.tail, var, ctx->stream);
    };
    if (tune) {
        std::vector<double> ms(nv);
        for (int q = 0; q < nv; ++q) HIPCHK(time_launch(ctx, [&] { return go(q); }, &ms[q]));
        v = cdl::tune_put(cdl::tune_arch(ctx->device), cdl::tune_key("square", prec, ld, 0), ms);
    }
    Timed t_(ctx, product ? "chain_product" : "square");
    HIPCHK(go(v));
    return CDL_OK;
}

static double host_sum(const std::vector<double> &v) {
    double s = 0.0;
    for (double x : v) s += x;
    return s;
}

cdl_status cdl_build_chain(cdl_ctx *ctx, const double *W, const double *deg, const double *stats,
                           int64_t n, cdl_prec prec, int depth, int depth_max, double chain_eps,
                           int lazy, void *chain, size_t chain_bytes, cdl_chain_info *info) {
    if (!ctx) return CDL_E_ARG;
    if (n < 2 || n > (1 << 20)) return fail(ctx, CDL_E_ARG, "bad n");
    if (!valid_prec(prec)) return fail(ctx, CDL_E_ARG, "bad precision");
    if (depth_max < 1 || depth_max > CDL_MAX_DEPTH || depth < 0 || depth > depth_max)
        return fail(ctx, CDL_E_ARG, "need 0 <= depth <= depth_max <= 14, depth_max >= 1");
    if (!W || !deg || !stats || !chain || !info) return fail(ctx, CDL_E_ARG, "null pointer");
    if (!aligned(W, 16) || !aligned(chain, kAlign)) return fail(ctx, CDL_E_ARG, "misaligned pointer");
    Arena need(nullptr);
    plan_chain(need, n, prec, depth_max);
    if (chain_bytes < need.off) return fail(ctx, CDL_E_WORKSPACE, "chain buffer too small");
    Arena a(chain);
    ChainBuf c = plan_chain(a, n, prec, depth_max);
    const int64_t ld = pad_n(n);
    hipStream_t s = ctx->stream;
    const CostModel cm = cost_model(ctx->device, prec, n, 256);
    HIPCHK(hipSetDevice(ctx->device));
    std::memset(info, 0, sizeof(*info));
    info->lazy = lazy ? 1 : 0;
    info->prec = prec;

    { Timed t_(ctx, "chain_prep"); HIPCHK(launch_chain_prep(deg, stats, n, ld, info->lazy, c.dmn, c.dm, c.u, s)); }
    { Timed t_(ctx, "normalize"); HIPCHK(launch_normalize(prec, W, ld, n, c.dmn, c.u, info->lazy, c.levels, c.fro, c.fro64, s)); }
    const int nst = sym_tiles64(ld);
    std::vector<double> part(nst), part64(nst);
    HIPCHK(read_to_host(ctx, s, {{part.data(), c.fro, nst * sizeof(double)},
                              {part64.data(), c.fro64, nst * sizeof(double)}}));
    info->rho_bound = std::sqrt(host_sum(part64));
    double f = std::sqrt(host_sum(part));
    if (!std::isfinite(f)) return fail(ctx, CDL_E_NONFINITE, "non-finite chain level");
    info->fro[0] = f;
    int l = 0;
    double rho = f;
    while (true) {
        rho = std::pow(f, 1.0 / std::ldexp(1.0, l));
        bool more;
        if (depth > 0)
            more = l + 1 < depth;
        else if (chain_eps > 0.0)
            more = l + 1 < depth_max && !(rho < 1.0 && f * f / (1.0 - rho) <= chain_eps);
        else
            more = l + 1 < depth_max && model_wants_square(prec, l, f, rho, cm);
        if (!more) break;
        const int ntl = square_tiles(prec, ld);
        {
            const cdl_status sq = square_step(ctx, prec, c.levels + c.level_bytes * l, c.levels + c.level_bytes * l,
                                              c.levels + c.level_bytes * (l + 1), ld, n, c, true);
            if (sq != CDL_OK) return sq;
        }
        part.resize(ntl);
        HIPCHK(read_to_host(ctx, s, {{part.data(), c.fro, ntl * sizeof(double)}}));
        const double fprev = f;
        f = std::sqrt(host_sum(part));
        if (!std::isfinite(f)) return fail(ctx, CDL_E_NONFINITE, "non-finite chain level");
        ++l;
        info->fro[l] = f;
        // A level whose norm stays >= 1 and no longer shrinks: an eigenvalue of
        // modulus one (a bipartite component) survives every squaring.
        if (f >= 0.999 && f >= 0.999 * fprev && (depth == 0 || l + 1 == depth)) {
            info->depth = l + 1;
            info->rho_hat = std::pow(f, 1.0 / std::ldexp(1.0, l));
            return fail(ctx, CDL_E_DIVERGED,
                        "chain levels do not decay (spectral radius >= 1; bipartite graph? try lazy)");
        }
    }
    info->depth = l + 1;
    info->rho_hat = rho;
    // fro(S~^{2^l})^(1/2^l) bounds rho(S~) from above and tends to it.  When
    // the automatic builder used every allowed level (three or more) and the
    // bound is still >= 1, no contraction was shown.
    if (depth == 0 && l >= 2 && !(rho < 1.0))
        return fail(ctx, CDL_E_DIVERGED,
                    "no contraction shown within depth_max levels (bipartite graph? try lazy)");
    return CDL_OK;
}

cdl_status cdl_chain_densify(cdl_ctx *ctx, int64_t n, void *chain, size_t chain_bytes,
                             cdl_chain_info *info) {
    if (!ctx) return CDL_E_ARG;
    if (!chain || !info || n < 2 || n > (1 << 20)) return fail(ctx, CDL_E_ARG, "bad arguments");
    if (!aligned(chain, kAlign)) return fail(ctx, CDL_E_ARG, "misaligned pointer");
    const int d = info->depth;
    if (d < 1 || d > CDL_MAX_DEPTH || !valid_prec(info->prec)) return fail(ctx, CDL_E_ARG, "invalid chain info");
    if (info->dense_levels != 0) return fail(ctx, CDL_E_ARG, "chain is already dense");
    const int slots = d >= 2 ? d + 1 : 1;
    Arena need(nullptr);
    plan_chain(need, n, info->prec, slots);
    if (chain_bytes < need.off) return fail(ctx, CDL_E_WORKSPACE, "chain buffer needs depth + 1 levels");
    Arena a(chain);
    ChainBuf c = plan_chain(a, n, info->prec, slots);
    const int64_t ld = pad_n(n);
    hipStream_t s = ctx->stream;
    HIPCHK(hipSetDevice(ctx->device));
    auto slot = [&](int l) { return c.levels + c.level_bytes * l; };
    if (d >= 2) {
        // Q_1 = L_0 + L_1 + L_0 L_1 into the spare slot, then
        // Q_{j} = Q_{j-1} + L_j + Q_{j-1} L_j alternating between the spare
        // slot and slot 0 (free once L_0 is consumed); Q ends in slot 0.
        char *spare = slot(d), *cur = spare;
        cdl_status st = square_step(ctx, info->prec, slot(0), slot(1), spare, ld, n, c, true);
        if (st != CDL_OK) return st;
        for (int j = 2; j < d; ++j) {
            char *dst = cur == spare ? slot(0) : spare;
            if ((st = square_step(ctx, info->prec, cur, slot(j), dst, ld, n, c, true)) != CDL_OK) return st;
            cur = dst;
        }
        if (cur != slot(0)) HIPCHK(hipMemcpyAsync(slot(0), cur, c.level_bytes, hipMemcpyDeviceToDevice, s));
    }
    info->dense_levels = d;
    info->depth = 1;
    return CDL_OK;
}

// ---- embedding -------------------------------------------------------------------

// W V for the residual: fills S partial panels of P (summed by the
// reduction); the stored matrix's split-K GEMM or a streamed sweep.
using WProduct = std::function<cdl_status(const double *Vt, double *P, int &S)>;

// The stored matrix's product: split-K FP64 MFMA GEMM.
static WProduct stored_product(cdl_ctx *ctx, const double *W, int64_t n, int64_t k) {
    return [ctx, W, n, k](const double *Vt, double *P, int &S) -> cdl_status {
        const int64_t ld = pad_n(n), kp = pad_k(k);
        bool tune = false;
        int ch = pick_choice(ctx, "residual", 0, ld, kp, 3, true, &tune);
        if (tune) {
            std::vector<double> ms(3);
            for (int q = 0; q < 3; ++q)
                HIPCHK(time_launch(ctx, [&] {
                    return launch_residual_gemm(Vt, W, ld, n, kp, residual_splits(ld, kp, n, q), P,
                                                ctx->stream);
                }, &ms[q]));
            ch = cdl::tune_put(cdl::tune_arch(ctx->device), cdl::tune_key("residual", 0, ld, kp), ms);
        }
        S = residual_splits(ld, kp, n, ch);
        { Timed t_(ctx, "residual"); HIPCHK(launch_residual_gemm(Vt, W, ld, n, kp, S, P, ctx->stream)); }
        return CDL_OK;
    };
}

// The solve from the right-hand sides in w.Yt (X = 0 in w.Xt): norms, the
// refinement iterations and the centred Z.  Syncs once per iteration.
static cdl_status solve_from_rhs(cdl_ctx *ctx, const WProduct &wprod, const double *deg,
                                 const double *stats, int64_t n, const ChainBuf &c,
                                 const cdl_chain_info *ci, int64_t k, cdl_solver solver,
                                 double tol, int max_iter, double *Z, const SolveWs &w,
                                 cdl_solve_info *info) {
    const int prec = ci->prec;
    const int64_t ld = pad_n(n), kp = pad_k(k);
    const size_t panel = (size_t)kp * ld;
    hipStream_t s = ctx->stream;
    const int nparts = residual_parts(ld), ntiles = residual_tiles(ld, kp);
    const int scaled = prec == 3;   // FP16 operands need a power-of-two scale
    { Timed t_(ctx, "residual_init"); HIPCHK(launch_residual_reduce_k(prec, nullptr, 0, w.Yt, w.Xt, deg, c.dm, ld, n, kp, k, w.Rt, w.V64, w.Vlo[0], w.npart, w.mpart, s)); }
    { Timed t_(ctx, "col_norms"); HIPCHK(launch_col_norms2(w.npart, nparts, kp, w.mpart, ntiles, scaled, w.scal, s)); }
    std::vector<double> ynorm(kp), rnorm(kp);
    double hstats[CDL_GRAPH_STATS];
    HIPCHK(read_to_host(ctx, s, {{ynorm.data(), w.scal, kp * sizeof(double)},
                              {hstats, stats, sizeof(hstats)}}));
    for (int64_t r = 0; r < k; ++r)
        if (!std::isfinite(ynorm[r])) return fail(ctx, CDL_E_NONFINITE, "non-finite right-hand side");
    // kappa bounds ||e|| / ||z|| per unit relative residual: the nonzero
    // spectrum of L = D^{1/2} (I - S) D^{1/2} lies in
    // [deg_min (1 - rho), deg_max (1 + rho)], rho = rho(S~) <= ||S~||_F.
    // Lazy levels hold S~' = (I + S)/2 - u u^T: 1 - lambda(S) >= 2 (1 - ||S~'||_F)
    // and <= 2, so kappa = deg_max / (deg_min (1 - ||S~'||_F)).
    const double rb = ci->rho_bound;
    double kappa = INFINITY;
    if (rb < 1.0 && hstats[2] > 0.0)
        kappa = ci->lazy ? hstats[3] / (hstats[2] * (1.0 - rb))
                         : hstats[3] * (1.0 + rb) / (hstats[2] * (1.0 - rb));
    const double target = tol > 0.0 ? tol : (tol < 0.0 ? -tol / kappa : 0.0);
    if (tol < 0.0 && !std::isfinite(kappa))
        return fail(ctx, CDL_E_ARG, "certified tolerance needs ||S~||_F < 1; use tol > 0");
    const double rho_model = std::min(ci->rho_hat, ci->rho_bound);
    const double *inv_vs = w.scal + kp + 1;
    const CostModel cm = cost_model(ctx->device, prec, n, k);

    double rel = 1.0;
    int it = 0;
    bool conv = false;
    const int d = ci->depth;
    auto depth_now = [&]() {
        if (ci->dense_levels > 0) return 1;   // the one stored matrix is the whole product
        return ctx->solve_depth > 0 ? ctx->solve_depth
                                    : (tol == 0.0 ? d : choose_depth(prec, d, rho_model, target / rel, cm));
    };
    auto precondition = [&](int D, double *Xdst) -> cdl_status {
        return precondition_enqueue(ctx, prec, d, D, w, c, ld, n, kp, scaled, inv_vs, Xdst);
    };
    // max_r ||r_r|| / ||y_r|| after the norms kernel; syncs.
    auto residual_check = [&]() -> cdl_status {
        HIPCHK(read_to_host(ctx, s, {{rnorm.data(), w.scal, kp * sizeof(double)}}));
        rel = 0.0;
        for (int64_t r = 0; r < k; ++r) {
            if (!std::isfinite(rnorm[r])) return fail(ctx, CDL_E_NONFINITE, "non-finite residual");
            if (ynorm[r] > 0.0) rel = std::max(rel, rnorm[r] / ynorm[r]);
        }
        if (info && it <= 64) info->history[it - 1] = rel;
        conv = target > 0.0 && rel <= target;
        return CDL_OK;
    };
    cdl_status st = CDL_OK;
    if (solver == CDL_RICHARDSON) {
        // x <- x + P1 (y - L x)  (EstimateSolution with P2 y = P1 L y)
        while (it < max_iter) {
            const int D = depth_now();
            if ((st = precondition(D, w.Xt)) != CDL_OK) return st;
            ++it;
            if (info && it <= 64) info->depth_used[it - 1] = D;
            int S = 0;
            if ((st = wprod(w.Xt, (double *)w.part, S)) != CDL_OK) return st;
            { Timed t_(ctx, "residual_reduce"); HIPCHK(launch_residual_reduce_k(prec, (double *)w.part, S, w.Yt, w.Xt, deg, c.dm, ld, n, kp, k,
                                     w.Rt, w.V64, w.Vlo[0], w.npart, w.mpart, s)); }
            { Timed t_(ctx, "col_norms"); HIPCHK(launch_col_norms2(w.npart, nparts, kp, w.mpart, ntiles, scaled, w.scal, s)); }
            if ((st = residual_check()) != CDL_OK) return st;
            if (conv) break;
        }
    } else {
        // Conjugate gradients preconditioned by P1, per column; x0 = 0, r0 = y.
        double *rho = w.pcg, *alpha = w.pcg + kp, *beta = w.pcg + 2 * kp;
        const size_t pbytes = panel * sizeof(double);
        while (it < max_iter) {
            const int D = depth_now();
            const int first = it == 0;
            { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w.Zt, pbytes, s)); }
            if ((st = precondition(D, w.Zt)) != CDL_OK) return st;
            ++it;
            if (info && it <= 64) info->depth_used[it - 1] = D;
            { Timed t_(ctx, "pcg_vec"); HIPCHK(launch_col_dots(w.Zt, w.Rt, first ? nullptr : w.Zt, w.Qt, ld, kp, w.dots, s)); }
            { Timed t_(ctx, "pcg_vec"); HIPCHK(launch_pcg_scalars(w.dots, ld, kp, 0, first, w.pcg, s)); }
            { Timed t_(ctx, "pcg_vec"); HIPCHK(launch_pcg_dir(w.Zt, w.Pt, beta, ld, kp, first, s)); }
            // q' = -L p
            int S = 0;
            if ((st = wprod(w.Pt, (double *)w.part, S)) != CDL_OK) return st;
            { Timed t_(ctx, "residual_reduce"); HIPCHK(launch_residual_reduce_k(-1, (double *)w.part, S, nullptr, w.Pt, deg, c.dm, ld, n, kp, k,
                                     w.Qt, w.V64, nullptr, w.npart, w.mpart, s)); }
            { Timed t_(ctx, "pcg_vec"); HIPCHK(launch_col_dots(w.Pt, w.Qt, nullptr, nullptr, ld, kp, w.dots, s)); }
            { Timed t_(ctx, "pcg_vec"); HIPCHK(launch_pcg_scalars(w.dots, ld, kp, 1, 0, w.pcg, s)); }
            { Timed t_(ctx, "pcg_update"); HIPCHK(launch_pcg_update(prec, w.Pt, w.Qt, alpha, c.dm, ld, kp, w.Xt, w.Rt, w.V64,
                                       w.Vlo[0], w.npart, w.mpart, s)); }
            { Timed t_(ctx, "col_norms"); HIPCHK(launch_col_norms2(w.npart, nparts, kp, w.mpart, ntiles, scaled, w.scal, s)); }
            if ((st = residual_check()) != CDL_OK) return st;
            if (conv) break;
        }
        (void)rho;
    }
    { Timed t_(ctx, "finalize_z"); HIPCHK(launch_finalize_z2(w.Xt, ld, n, kp, k, w.mean, Z, s)); }
    if (info) {
        info->iterations = it;
        info->converged = conv || tol == 0.0;
        info->rel_residual = rel;
        info->kappa = kappa;
        info->certified_error = kappa * rel + 1e-14;
    }
    if (tol != 0.0 && !conv) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "residual %.3e > target %.3e after %d iterations", rel, target, it);
        return fail(ctx, CDL_E_NOCONV, buf);
    }
    return CDL_OK;
}

// Arguments of one snapshot's solve (k already resolved).
static cdl_status check_solve(cdl_ctx *ctx, const double *W, const double *deg,
                              const double *stats, int64_t n, const void *chain,
                              const cdl_chain_info *ci, int64_t k, cdl_solver solver,
                              int max_iter, const double *Z, const void *ws, size_t ws_bytes) {
    if (n < 2 || n > (1 << 20)) return fail(ctx, CDL_E_ARG, "bad n");
    if (!W || !deg || !stats || !chain || !ci || !Z || !ws) return fail(ctx, CDL_E_ARG, "null pointer");
    if (!aligned(W, 16) || !aligned(chain, kAlign) || !aligned(ws, kAlign) || !aligned(Z, 8))
        return fail(ctx, CDL_E_ARG, "misaligned pointer");
    if (k < 1 || k > (int64_t)1 << 20) return fail(ctx, CDL_E_ARG, "k must be in [1, 2^20]");
    if (ci->depth < 1 || ci->depth > CDL_MAX_DEPTH || !valid_prec(ci->prec) ||
        ci->dense_levels < 0 || ci->dense_levels > CDL_MAX_DEPTH || (ci->dense_levels > 0 && ci->depth != 1))
        return fail(ctx, CDL_E_ARG, "invalid chain info");
    if (max_iter < 1 || max_iter > 64) return fail(ctx, CDL_E_ARG, "max_iter must be in [1, 64]");
    if (solver != CDL_RICHARDSON && solver != CDL_PCG) return fail(ctx, CDL_E_ARG, "bad solver");
    Arena need(nullptr);
    plan_solve(need, n, k, ci->prec);
    if (ws_bytes < need.off) return fail(ctx, CDL_E_WORKSPACE, "solve workspace too small");
    return CDL_OK;
}

cdl_status cdl_solve_embedding(cdl_ctx *ctx, const double *W, const double *deg,
                               const double *stats, const int32_t *gid, int64_t n,
                               const void *chain, const cdl_chain_info *ci, int64_t k,
                               double eps_rp, uint64_t seed, cdl_solver solver, double tol,
                               int max_iter, double *Z, void *ws, size_t ws_bytes,
                               cdl_solve_info *info) {
    if (!ctx) return CDL_E_ARG;
    if (k <= 0 && cdl_k_rp(n, eps_rp, &k) != CDL_OK)
        return fail(ctx, CDL_E_ARG, "need n >= 2 and 0 < eps_rp < 1 when k <= 0");
    cdl_status st = check_solve(ctx, W, deg, stats, n, chain, ci, k, solver, max_iter, Z, ws, ws_bytes);
    if (st != CDL_OK) return st;
    Arena a(ws);
    SolveWs w = plan_solve(a, n, k, ci->prec);
    Arena ac((void *)chain);
    ChainBuf c = plan_chain(ac, n, ci->prec, ci->depth);
    const int64_t ld = pad_n(n), kp = pad_k(k);
    const size_t panel = (size_t)kp * ld;
    hipStream_t s = ctx->stream;
    HIPCHK(hipSetDevice(ctx->device));
    if (info) std::memset(info, 0, sizeof(*info));

    { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w.Yt, panel * sizeof(double), s)); }
    { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w.Xt, panel * sizeof(double), s)); }
    { Timed t_(ctx, "rhs"); HIPCHK(launch_rhs(W, ld, n, gid, k, kp, seed, w.Yt, s)); }
    return solve_from_rhs(ctx, stored_product(ctx, W, n, k), deg, stats, n, c, ci, k, solver, tol,
                          max_iter, Z, w, info);
}

cdl_status cdl_solve_embedding_pair(cdl_ctx *ctx, const double *W0, const double *deg0,
                                    const double *stats0, const void *chain0,
                                    const cdl_chain_info *ci0, const double *W1,
                                    const double *deg1, const double *stats1,
                                    const void *chain1, const cdl_chain_info *ci1,
                                    const int32_t *gid, int64_t n, int64_t k, uint64_t seed,
                                    cdl_solver solver, double tol, int max_iter, double *Z0,
                                    double *Z1, void *ws0, void *ws1, size_t ws_bytes,
                                    cdl_solve_info *info0, cdl_solve_info *info1) {
    if (!ctx) return CDL_E_ARG;
    cdl_status st = check_solve(ctx, W0, deg0, stats0, n, chain0, ci0, k, solver, max_iter, Z0, ws0, ws_bytes);
    if (st == CDL_OK)
        st = check_solve(ctx, W1, deg1, stats1, n, chain1, ci1, k, solver, max_iter, Z1, ws1, ws_bytes);
    if (st != CDL_OK) return st;
    if (W0 == W1 || ws0 == ws1 || Z0 == Z1) return fail(ctx, CDL_E_ARG, "the two snapshots need their own W, Z and workspace");
    Arena a0(ws0), a1(ws1);
    SolveWs w0 = plan_solve(a0, n, k, ci0->prec), w1 = plan_solve(a1, n, k, ci1->prec);
    Arena ac0((void *)chain0), ac1((void *)chain1);
    ChainBuf c0 = plan_chain(ac0, n, ci0->prec, ci0->depth), c1 = plan_chain(ac1, n, ci1->prec, ci1->depth);
    const int64_t ld = pad_n(n), kp = pad_k(k);
    const size_t pbytes = (size_t)kp * ld * sizeof(double);
    hipStream_t s = ctx->stream;
    HIPCHK(hipSetDevice(ctx->device));
    if (info0) std::memset(info0, 0, sizeof(*info0));
    if (info1) std::memset(info1, 0, sizeof(*info1));
    { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w0.Yt, pbytes, s)); }
    { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w0.Xt, pbytes, s)); }
    { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w1.Yt, pbytes, s)); }
    { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w1.Xt, pbytes, s)); }
    { Timed t_(ctx, "rhs_pair"); HIPCHK(launch_rhs_pair(W0, W1, ld, n, gid, k, kp, seed, w0.Yt, w1.Yt, s)); }
    st = solve_from_rhs(ctx, stored_product(ctx, W0, n, k), deg0, stats0, n, c0, ci0, k, solver,
                        tol, max_iter, Z0, w0, info0);
    if (st != CDL_OK) return st;
    return solve_from_rhs(ctx, stored_product(ctx, W1, n, k), deg1, stats1, n, c1, ci1, k, solver,
                          tol, max_iter, Z1, w1, info1);
}

// ---- right-hand sides alone ----------------------------------------------------

cdl_status cdl_rhs_workspace_bytes(int64_t n, int64_t k, int pair, size_t *bytes) {
    if (n < 2 || n > (1 << 20) || k < 1 || k > ((int64_t)1 << 20) || !bytes) return CDL_E_ARG;
    Arena a(nullptr);
    a.take<double>((size_t)pad_k(k) * pad_n(n) * (pair ? 2 : 1));
    *bytes = a.off;
    return CDL_OK;
}

cdl_status cdl_rhs(cdl_ctx *ctx, const double *W0, const double *W1, const int32_t *gid,
                   int64_t n, int64_t k, uint64_t seed, double *Y0, double *Y1, void *ws,
                   size_t ws_bytes) {
    if (!ctx) return CDL_E_ARG;
    if (n < 2 || n > (1 << 20)) return fail(ctx, CDL_E_ARG, "n must be in [2, 2^20]");
    if (k < 1 || k > (int64_t)1 << 20) return fail(ctx, CDL_E_ARG, "k must be in [1, 2^20]");
    if (!W0 || !Y0 || !ws || (W1 == nullptr) != (Y1 == nullptr))
        return fail(ctx, CDL_E_ARG, "null pointer (W1 and Y1 go together)");
    if (!aligned(W0, 16) || (W1 && !aligned(W1, 16)) || !aligned(Y0, 8) || (Y1 && !aligned(Y1, 8)) ||
        !aligned(ws, kAlign))
        return fail(ctx, CDL_E_ARG, "misaligned pointer");
    size_t need = 0;
    cdl_rhs_workspace_bytes(n, k, W1 != nullptr, &need);
    if (ws_bytes < need) return fail(ctx, CDL_E_WORKSPACE, "right-hand-side workspace too small");
    const int64_t ld = pad_n(n), kp = pad_k(k);
    Arena a(ws);
    double *Yt0 = a.take<double>((size_t)kp * ld);
    double *Yt1 = W1 ? a.take<double>((size_t)kp * ld) : nullptr;
    hipStream_t s = ctx->stream;
    HIPCHK(hipSetDevice(ctx->device));
    if (W1) {
        Timed t_(ctx, "rhs_pair");
        HIPCHK(launch_rhs_pair(W0, W1, ld, n, gid, k, kp, seed, Yt0, Yt1, s));
    } else {
        Timed t_(ctx, "rhs");
        HIPCHK(launch_rhs(W0, ld, n, gid, k, kp, seed, Yt0, s));
    }
    HIPCHK(launch_transpose(Yt0, ld, n, k, Y0, s));
    if (W1) HIPCHK(launch_transpose(Yt1, ld, n, k, Y1, s));
    return CDL_OK;
}

// ---- streamed snapshots ---------------------------------------------------------

cdl_status cdl_stream_workspace_bytes(int64_t n, int64_t T, int64_t k, int64_t panel_rows,
                                      int level_prec, size_t *bytes) {
    if (n < 2 || n > (1 << 20) || T < 1 || k < 1 || k > ((int64_t)1 << 20) || panel_rows < 0 ||
        !bytes || level_prec < -1 || level_prec > 3)
        return CDL_E_ARG;
    Arena a(nullptr);
    plan_stream(a, n, T, k, panel_rows, level_prec);
    *bytes = a.off;
    return CDL_OK;
}

cdl_status cdl_stream_embedding(cdl_ctx *ctx, const double *X, int64_t n, int64_t T,
                                int64_t ldx, double sigma, const int32_t *gid, int64_t k,
                                uint64_t seed, double tol, int max_iter, int64_t panel_rows,
                                int level_prec, void *chain, size_t chain_bytes,
                                cdl_chain_info *chain_info, double *deg, double *stats,
                                double *Z, void *ws, size_t ws_bytes, cdl_solve_info *info) {
    if (!ctx) return CDL_E_ARG;
    if (n < 2 || n > (1 << 20)) return fail(ctx, CDL_E_ARG, "n must be in [2, 2^20]");
    if (T < 1 || ldx < T) return fail(ctx, CDL_E_ARG, "need T >= 1 and ldx >= T");
    if (k < 1 || k > ((int64_t)1 << 20)) return fail(ctx, CDL_E_ARG, "k must be in [1, 2^20]");
    if (!X || !deg || !stats || !Z || !ws) return fail(ctx, CDL_E_ARG, "null pointer");
    if (!aligned(X, 8) || !aligned(deg, 8) || !aligned(stats, 8) || !aligned(Z, 8) ||
        !aligned(ws, kAlign))
        return fail(ctx, CDL_E_ARG, "misaligned pointer");
    if (!std::isfinite(sigma) || !std::isfinite(tol)) return fail(ctx, CDL_E_ARG, "sigma and tol must be finite");
    if (max_iter < 1 || max_iter > 64) return fail(ctx, CDL_E_ARG, "max_iter must be in [1, 64]");
    if (panel_rows < 0) return fail(ctx, CDL_E_ARG, "panel_rows must be >= 0");
    if (level_prec < -1 || level_prec > 3) return fail(ctx, CDL_E_ARG, "bad level type");
    const bool stored_level = level_prec >= 0;
    if (stored_level) {
        if (!chain || !aligned(chain, kAlign)) return fail(ctx, CDL_E_ARG, "a stored level needs an aligned chain buffer");
        Arena cneed(nullptr);
        plan_chain(cneed, n, level_prec, 1);
        if (chain_bytes < cneed.off) return fail(ctx, CDL_E_WORKSPACE, "chain buffer too small");
    }
    Arena need(nullptr);
    plan_stream(need, n, T, k, panel_rows, level_prec);
    if (ws_bytes < need.off) return fail(ctx, CDL_E_WORKSPACE, "stream workspace too small");
    HIPCHK(hipSetDevice(ctx->device));
    if (info) std::memset(info, 0, sizeof(*info));
    if (chain_info) std::memset(chain_info, 0, sizeof(*chain_info));
    Arena a(ws);
    const StreamWs w = plan_stream(a, n, T, k, panel_rows, level_prec);
    const int64_t ld = pad_n(n), Tp = pad_t(T), kp = pad_k(k), P = w.prow;
    const size_t kbytes = (size_t)kp * ld * sizeof(double);
    hipStream_t s = ctx->stream;

    { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w.flags, 256, s)); }
    { Timed t_(ctx, "pad_series"); HIPCHK(launch_pad_series(X, n, T, ldx, w.Xp, ld, Tp, w.sqn, w.flags, s)); }
    int hflag = 0;
    HIPCHK(read_to_host(ctx, s, {{&hflag, w.flags, sizeof(int)}}));
    if (hflag) return fail(ctx, CDL_E_NONFINITE, "non-finite node series");

    // Bandwidth: exact lower median of the upper-triangle distances.  One
    // sweep over the recomputed upper row panels counts the keys below a
    // sampled bracket and gathers those inside; the radix passes then run over
    // the gathered keys.  If the bracket misses the rank (or the buffer
    // overflows), one 12-bit digit per sweep from the top bit instead.
    if (sigma > 0.0) {
        { Timed t_(ctx, "set_sigma"); HIPCHK(launch_set_sigma(sigma, stats, s)); }
    } else {
        const int64_t cap = select_stream_keys(n);
        { Timed t_(ctx, "stream_select"); HIPCHK(launch_select_start_top(w.sel, n, s)); }
        int src = 0, mode = 0;
        if (ctx->select_mode == 0) {   // 1: the digit sweeps only (cdl_ctx_set_select)
            { Timed t_(ctx, "stream_select"); HIPCHK(launch_select_sample_x(w.Xp, Tp, w.sqn, n, w.sel, s)); }
            for (int64_t r0 = 0; r0 < n; r0 += P) {
                const int64_t rows = std::min(P, ld - r0);
                { Timed t_(ctx, "stream_gram_upper"); HIPCHK(launch_gram_panel(w.Xp, Tp, w.sqn, n, ld, r0, rows, false, w.panel, nullptr, s)); }
                { Timed t_(ctx, "stream_select"); HIPCHK(launch_select_bracket_panel(w.panel, ld, n, r0, std::min(r0 + rows, n), w.sel, w.selbuf, cap, s)); }
            }
            { Timed t_(ctx, "stream_select"); HIPCHK(launch_select_check(w.sel, cap, stats, s)); }
            HIPCHK(read_to_host(ctx, s, {{&src, &w.sel->src, sizeof(int)}, {&mode, &w.sel->mode, sizeof(int)}}));
        }
        if (src == 1 && mode != 2) {
            // at most 6 digit passes resolve 64 bits; the collect pass is one more
            for (int p = 0; p < 7; ++p)
                { Timed t_(ctx, "stream_select"); HIPCHK(launch_select_buffer_pass(w.sel, w.selbuf, cap, stats, s)); }
            HIPCHK(read_to_host(ctx, s, {{&mode, &w.sel->mode, sizeof(int)}}));
        }
        for (int digit = 0; digit < 7 && mode != 2; ++digit) {
            for (int64_t r0 = 0; r0 < n; r0 += P) {
                const int64_t rows = std::min(P, ld - r0);
                { Timed t_(ctx, "stream_gram_upper"); HIPCHK(launch_gram_panel(w.Xp, Tp, w.sqn, n, ld, r0, rows, false, w.panel, nullptr, s)); }
                { Timed t_(ctx, "stream_select"); HIPCHK(launch_select_panel(w.panel, ld, n, r0, std::min(r0 + rows, n), w.sel, s)); }
            }
            { Timed t_(ctx, "stream_select"); HIPCHK(launch_select_pick(w.sel, stats, s)); }
            HIPCHK(read_to_host(ctx, s, {{&mode, &w.sel->mode, sizeof(int)}}));
        }
        if (mode != 2) return fail(ctx, CDL_E_HIP, "median selection did not finish");
    }

    // Weights, degrees and right-hand sides: one sweep over the full row panels.
    { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w.Yt, kbytes, s)); }
    { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w.Xt, kbytes, s)); }
    for (int64_t r0 = 0; r0 < n; r0 += P) {
        const int64_t rows = std::min(P, ld - r0);
        { Timed t_(ctx, "stream_gram"); HIPCHK(launch_gram_panel(w.Xp, Tp, w.sqn, n, ld, r0, rows, true, w.panel, nullptr, s)); }
        { Timed t_(ctx, "stream_exp"); HIPCHK(launch_exp_rows(w.panel, ld, n, r0, rows, stats, deg, nullptr, nullptr, s)); }
        { Timed t_(ctx, "rhs"); HIPCHK(launch_rhs_rows(w.panel, ld, n, r0, std::min(r0 + rows, n), gid, k, kp, seed, w.Yt, s)); }
    }
    { Timed t_(ctx, "graph_stats"); HIPCHK(launch_graph_stats(deg, n, stats, s)); }
    if (stored_level) {
        // Level 0 of the chain is stored in the level type (the FP64 weights
        // are not): one more sweep normalises each recomputed panel into it.
        // The solve is then the stored path's (level applications, repeated
        // for deeper levels), with the FP64 residual's product W X taken by a
        // streamed sweep.
        double hst[CDL_GRAPH_STATS];
        HIPCHK(read_to_host(ctx, s, {{hst, stats, sizeof(hst)}}));
        for (double v : hst)
            if (!std::isfinite(v)) return fail(ctx, CDL_E_NONFINITE, "non-finite weights or degrees");
        if (!(hst[2] > 0.0)) return fail(ctx, CDL_E_GRAPH, "a node has zero degree");
        Arena ac(chain);
        const ChainBuf c = plan_chain(ac, n, level_prec, 1);
        { Timed t_(ctx, "chain_prep"); HIPCHK(launch_chain_prep(deg, stats, n, ld, 0, c.dmn, c.dm, c.u, s)); }
        for (int64_t r0 = 0; r0 < n; r0 += P) {
            const int64_t rows = std::min(P, ld - r0);
            { Timed t_(ctx, "stream_gram_exp"); HIPCHK(launch_gram_panel(w.Xp, Tp, w.sqn, n, ld, r0, rows, true, w.panel, stats, s)); }
            { Timed t_(ctx, "stream_normalize"); HIPCHK(launch_normalize_rows(level_prec, w.panel, ld, n, r0, rows, c.dmn, c.u, 0, c.levels,
                                                w.fro + r0, w.fro64 + r0, s)); }
        }
        std::vector<double> f1(n), f2(n);
        HIPCHK(read_to_host(ctx, s, {{f1.data(), w.fro, n * sizeof(double)}, {f2.data(), w.fro64, n * sizeof(double)}}));
        cdl_chain_info ci;
        std::memset(&ci, 0, sizeof(ci));
        ci.prec = (cdl_prec)level_prec;
        ci.lazy = 0;
        ci.depth = 1;
        ci.fro[0] = std::sqrt(host_sum(f1));
        ci.rho_bound = std::sqrt(host_sum(f2));
        ci.rho_hat = ci.fro[0];
        if (chain_info) *chain_info = ci;
        if (!std::isfinite(ci.fro[0])) return fail(ctx, CDL_E_NONFINITE, "non-finite chain level");
        const WProduct sweep = [&](const double *Vt, double *Pp, int &S) -> cdl_status {
            S = 1;
            for (int64_t r0 = 0; r0 < n; r0 += P) {
                const int64_t rows = std::min(P, ld - r0);
                { Timed t_(ctx, "stream_gram_exp"); HIPCHK(launch_gram_panel(w.Xp, Tp, w.sqn, n, ld, r0, rows, true, w.panel, stats, s)); }
                { Timed t_(ctx, "stream_product"); HIPCHK(launch_panel_product(Vt, w.panel, ld, n, kp, r0, rows, Pp, s)); }
            }
            return CDL_OK;
        };
        return solve_from_rhs(ctx, sweep, deg, stats, n, c, &ci, k, CDL_RICHARDSON, tol, max_iter,
                              Z, w.sw, info);
    }
    { Timed t_(ctx, "stream_prep"); HIPCHK(launch_stream_prep(deg, n, ld, w.dinv, w.rdeg, s)); }
    const int nparts = residual_parts(ld), ntiles = residual_tiles(ld, kp);
    // R = Y (X = 0) and the norms of Y's columns
    { Timed t_(ctx, "residual_init"); HIPCHK(launch_residual_reduce(nullptr, 0, w.Yt, w.Xt, deg, w.rdeg, ld, n, kp, k, w.Rt, w.npart, w.mpart, s)); }
    { Timed t_(ctx, "col_norms"); HIPCHK(launch_col_norms2(w.npart, nparts, kp, w.mpart, ntiles, 0, w.scal, s)); }
    std::vector<double> ynorm(kp), rnorm(kp);
    double hstats[CDL_GRAPH_STATS];
    HIPCHK(read_to_host(ctx, s, {{ynorm.data(), w.scal, kp * sizeof(double)}, {hstats, stats, sizeof(hstats)}}));
    for (double v : hstats)
        if (!std::isfinite(v)) return fail(ctx, CDL_E_NONFINITE, "non-finite weights or degrees");
    if (!(hstats[2] > 0.0)) return fail(ctx, CDL_E_GRAPH, "a node has zero degree");
    for (int64_t r = 0; r < k; ++r)
        if (!std::isfinite(ynorm[r])) return fail(ctx, CDL_E_NONFINITE, "non-finite right-hand side");

    // One sweep: Prod = W V over the recomputed full row panels.  The first
    // sweep also collects the row norms of S for the certificate (separate
    // exponential kernel); the others take the weights straight from the
    // Gram epilogue.
    auto product_sweep = [&](const double *Vt, bool frob) -> cdl_status {
        for (int64_t r0 = 0; r0 < n; r0 += P) {
            const int64_t rows = std::min(P, ld - r0);
            if (frob) {
                { Timed t_(ctx, "stream_gram"); HIPCHK(launch_gram_panel(w.Xp, Tp, w.sqn, n, ld, r0, rows, true, w.panel, nullptr, s)); }
                { Timed t_(ctx, "stream_exp"); HIPCHK(launch_exp_rows(w.panel, ld, n, r0, rows, stats, nullptr, w.dinv, w.fro + r0, s)); }
            } else {
                { Timed t_(ctx, "stream_gram_exp"); HIPCHK(launch_gram_panel(w.Xp, Tp, w.sqn, n, ld, r0, rows, true, w.panel, stats, s)); }
            }
            { Timed t_(ctx, "stream_product"); HIPCHK(launch_panel_product(Vt, w.panel, ld, n, kp, r0, rows, w.Prod, s)); }
        }
        return CDL_OK;
    };

    double kappa = INFINITY, rb = INFINITY, target = tol > 0.0 ? tol : 0.0, rel = 1.0;
    int it = 0;
    bool conv = false;
    cdl_status st = CDL_OK;
    while (it < max_iter) {
        // X += P1 R, P1 = D^{-1} + D^{-1} W D^{-1}
        { Timed t_(ctx, "stream_scale"); HIPCHK(launch_stream_scale(w.Rt, w.rdeg, ld, kp, w.Ut, s)); }
        if ((st = product_sweep(w.Ut, it == 0)) != CDL_OK) return st;
        { Timed t_(ctx, "stream_update"); HIPCHK(launch_stream_update(w.Ut, w.Prod, w.rdeg, ld, kp, w.Xt, s)); }
        if (it == 0) {
            // ||S~||_F^2 = ||S||_F^2 - 1 for the deflated S~ = S - u u^T
            std::vector<double> fro(n);
            HIPCHK(read_to_host(ctx, s, {{fro.data(), w.fro, n * sizeof(double)}}));
            const double f2 = host_sum(fro) - 1.0;
            rb = std::sqrt(std::max(f2, 0.0));
            if (rb < 1.0) kappa = hstats[3] * (1.0 + rb) / (hstats[2] * (1.0 - rb));
            if (tol < 0.0) {
                if (!std::isfinite(kappa))
                    return fail(ctx, CDL_E_ARG, "certified tolerance needs ||S~||_F < 1; use tol > 0");
                target = -tol / kappa;
            }
        }
        ++it;
        if (info && it <= 64) info->depth_used[it - 1] = 1;
        // R = Y - D X + W X
        if ((st = product_sweep(w.Xt, false)) != CDL_OK) return st;
        { Timed t_(ctx, "residual"); HIPCHK(launch_residual_reduce(w.Prod, 1, w.Yt, w.Xt, deg, w.rdeg, ld, n, kp, k, w.Rt, w.npart, w.mpart, s)); }
        { Timed t_(ctx, "col_norms"); HIPCHK(launch_col_norms2(w.npart, nparts, kp, w.mpart, ntiles, 0, w.scal, s)); }
        HIPCHK(read_to_host(ctx, s, {{rnorm.data(), w.scal, kp * sizeof(double)}}));
        rel = 0.0;
        for (int64_t r = 0; r < k; ++r) {
            if (!std::isfinite(rnorm[r])) return fail(ctx, CDL_E_NONFINITE, "non-finite residual");
            if (ynorm[r] > 0.0) rel = std::max(rel, rnorm[r] / ynorm[r]);
        }
        if (info && it <= 64) info->history[it - 1] = rel;
        if (target > 0.0 && rel <= target) {
            conv = true;
            break;
        }
    }
    { Timed t_(ctx, "finalize_z"); HIPCHK(launch_finalize_z2(w.Xt, ld, n, kp, k, w.mean, Z, s)); }
    if (info) {
        info->iterations = it;
        info->converged = conv || tol == 0.0;
        info->rel_residual = rel;
        info->kappa = kappa;
        info->certified_error = kappa * rel + 1e-14;
    }
    if (tol != 0.0 && !conv) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "residual %.3e > target %.3e after %d iterations", rel, target, it);
        return fail(ctx, CDL_E_NOCONV, buf);
    }
    return CDL_OK;
}

// ---- scores -----------------------------------------------------------------------

static cdl_status check_map(cdl_ctx *ctx, const int32_t *map, int64_t m, int64_t n) {
    if (!map) return m == n ? CDL_OK : fail(ctx, CDL_E_ARG, "identity map needs m == n");
    std::vector<int32_t> h(m);
    HIPCHK(read_to_host(ctx, ctx->stream, {{h.data(), map, m * sizeof(int32_t)}}));
    for (int32_t v : h)
        if (v < 0 || v >= n) return fail(ctx, CDL_E_ARG, "map entry out of range");
    return CDL_OK;
}

// Argument checks shared by both score entry points (everything but the
// workspace and the map entries).
static cdl_status check_scores(cdl_ctx *ctx, const double *Z0, const double *W0,
                               const double *stats0, int64_t n0, const double *Z1,
                               const double *W1, const double *stats1, int64_t n1, int64_t k,
                               const int32_t *map0, const int32_t *map1, int64_t m,
                               cdl_score_mode mode, double *F, int32_t top_k,
                               int32_t *top_idx) {
    if (!ctx) return CDL_E_ARG;
    if (n0 < 2 || n1 < 2 || m < 1 || m > std::min(n0, n1) || k < 1)
        return fail(ctx, CDL_E_ARG, "bad sizes");
    if (!Z0 || !Z1 || !stats0 || !stats1 || !F) return fail(ctx, CDL_E_ARG, "null pointer");
    if (mode != CDL_SCORE_UNWEIGHTED && mode != CDL_SCORE_DELTA_A) return fail(ctx, CDL_E_ARG, "bad mode");
    if (mode == CDL_SCORE_DELTA_A && (!W0 || !W1)) return fail(ctx, CDL_E_ARG, "weighted mode needs W0, W1");
    if (top_k < 0 || top_k > CDL_MAX_TOPK || top_k > m || (top_k > 0 && !top_idx))
        return fail(ctx, CDL_E_ARG, "bad top_k");
    if (!aligned(Z0, 8) || !aligned(Z1, 8)) return fail(ctx, CDL_E_ARG, "misaligned pointer");
    if ((map0 == nullptr) != (map1 == nullptr)) return fail(ctx, CDL_E_ARG, "give both maps or neither");
    return CDL_OK;
}

// The score kernels over workspace `ws` (plan_score layout); `timed`: bracket
// them with the context's timing events.
static cdl_status score_enqueue(cdl_ctx *ctx, bool timed, const double *Z0, const double *W0,
                                const double *stats0, int64_t n0, const double *Z1,
                                const double *W1, const double *stats1, int64_t n1, int64_t k,
                                const int32_t *map0, const int32_t *map1, int64_t m,
                                cdl_score_mode mode, double *F, int32_t top_k, int32_t *top_idx,
                                void *ws) {
    Arena a(ws);
    ScoreWs w = plan_score(a, m, k);
    const int64_t mp = pad_n(m), kp = pad_k(k);
    hipStream_t s = ctx->stream;
    auto scope = [&](const char *nm, auto &&fn) -> hipError_t {
        if (!timed) return fn();
        Timed t_(ctx, nm);
        return fn();
    };
    HIPCHK(scope("build_zhat", [&] { return launch_build_zhat(Z0, Z1, map0, map1, m, mp, k, kp, stats0, stats1, w.Zh, w.Zhe, w.sq, s); }));
    HIPCHK(scope("score", [&] { return launch_score(w.Zh, w.Zhe, kp, w.sq, m, mp, W0, pad_n(n0), W1, pad_n(n1), map0, map1,
                                                    mode == CDL_SCORE_DELTA_A, w.part, nullptr, s); }));
    HIPCHK(scope("score_reduce", [&] { return launch_score_reduce(w.part, score_tiles_1d(mp), m, mp, F, s); }));
    if (top_k > 0) HIPCHK(scope("topk", [&] { return launch_topk(F, m, top_k, w.topk, top_idx, s); }));
    return CDL_OK;
}

cdl_status cdl_anomaly_scores(cdl_ctx *ctx, const double *Z0, const double *W0,
                              const double *stats0, int64_t n0, const double *Z1,
                              const double *W1, const double *stats1, int64_t n1, int64_t k,
                              const int32_t *map0, const int32_t *map1, int64_t m,
                              cdl_score_mode mode, double *F, int32_t top_k, int32_t *top_idx,
                              void *ws, size_t ws_bytes) {
    cdl_status st0 = check_scores(ctx, Z0, W0, stats0, n0, Z1, W1, stats1, n1, k, map0, map1, m,
                                  mode, F, top_k, top_idx);
    if (st0 != CDL_OK) return st0;
    if (!ws) return fail(ctx, CDL_E_ARG, "null pointer");
    if (!aligned(ws, kAlign)) return fail(ctx, CDL_E_ARG, "misaligned pointer");
    Arena need(nullptr);
    plan_score(need, m, k);
    if (ws_bytes < need.off) return fail(ctx, CDL_E_WORKSPACE, "score workspace too small");
    HIPCHK(hipSetDevice(ctx->device));
    cdl_status st = check_map(ctx, map0, m, n0);
    if (st != CDL_OK) return st;
    st = check_map(ctx, map1, m, n1);
    if (st != CDL_OK) return st;
    return score_enqueue(ctx, true, Z0, W0, stats0, n0, Z1, W1, stats1, n1, k, map0, map1, m, mode,
                         F, top_k, top_idx, ws);
}

cdl_status cdl_anomaly_scores_noalloc(cdl_ctx *ctx, const double *Z0, const double *W0,
                                      const double *stats0, int64_t n0, const double *Z1,
                                      const double *W1, const double *stats1, int64_t n1,
                                      int64_t k, const int32_t *map0, const int32_t *map1,
                                      int64_t m, cdl_score_mode mode, double *F, int32_t top_k,
                                      int32_t *top_idx) {
    cdl_status st = check_scores(ctx, Z0, W0, stats0, n0, Z1, W1, stats1, n1, k, map0, map1, m,
                                 mode, F, top_k, top_idx);
    if (st != CDL_OK) return st;
    Arena need(nullptr);
    plan_score(need, m, k);
    int *flag = (int *)nullptr;
    const size_t bytes = need.off + kAlign;   // the workspace, then the map flag
    if (bytes > kNoAllocScratchBytes) {
        char buf[200];
        std::snprintf(buf, sizeof(buf), "m = %lld, k = %lld need %zu bytes of scratch; the fixed "
                      "device scratch holds %zu", (long long)m, (long long)k, bytes,
                      kNoAllocScratchBytes);
        return fail(ctx, CDL_E_WORKSPACE, buf);
    }
    char *ws = (char *)scratch_ptr(ctx->device);
    if (!ws) return fail(ctx, CDL_E_HIP, "the device scratch of this device has no address");
    if (map0 && (!ctx->stage || ctx->stage_bytes < kAlign))
        return fail(ctx, CDL_E_HIP, "no pinned staging buffer for the map check");
    flag = (int *)(ws + need.off);
    HIPCHK(hipSetDevice(ctx->device));
    if (map0) {
        int bad = 0;
        HIPCHK(launch_check_maps(map0, map1, m, n0, n1, flag, ctx->stream));
        HIPCHK(read_to_host(ctx, ctx->stream, {{&bad, flag, sizeof(int)}}));
        if (bad) return fail(ctx, CDL_E_ARG, "map entry out of range");
    }
    return score_enqueue(ctx, false, Z0, W0, stats0, n0, Z1, W1, stats1, n1, k, map0, map1, m,
                         mode, F, top_k, top_idx, ws);
}

cdl_status cdl_edges_workspace_bytes(int64_t m, int64_t k, int32_t top_k, size_t *bytes) {
    if (m < 2 || m > (1 << 20) || k < 1 || top_k < 1 || top_k > CDL_MAX_TOPK ||
        top_k > m * (m - 1) / 2 || !bytes)
        return CDL_E_ARG;
    Arena a(nullptr);
    plan_edges(a, m, k, top_k);
    *bytes = a.off;
    return CDL_OK;
}

cdl_status cdl_anomaly_edges(cdl_ctx *ctx, const double *Z0, const double *W0,
                             const double *stats0, int64_t n0, const double *Z1,
                             const double *W1, const double *stats1, int64_t n1, int64_t k,
                             const int32_t *map0, const int32_t *map1, int64_t m,
                             cdl_score_mode mode, double *F, int32_t top_k, int32_t *edge_a,
                             int32_t *edge_b, double *edge_val, void *ws, size_t ws_bytes) {
    if (!ctx) return CDL_E_ARG;
    if (n0 < 2 || n1 < 2 || m < 2 || m > std::min(n0, n1) || k < 1)
        return fail(ctx, CDL_E_ARG, "bad sizes");
    if (!Z0 || !Z1 || !stats0 || !stats1 || !F || !ws || !edge_a || !edge_b || !edge_val)
        return fail(ctx, CDL_E_ARG, "null pointer");
    if (mode != CDL_SCORE_UNWEIGHTED && mode != CDL_SCORE_DELTA_A) return fail(ctx, CDL_E_ARG, "bad mode");
    if (mode == CDL_SCORE_DELTA_A && (!W0 || !W1)) return fail(ctx, CDL_E_ARG, "weighted mode needs W0, W1");
    if (top_k < 1 || top_k > CDL_MAX_TOPK || top_k > m * (m - 1) / 2)
        return fail(ctx, CDL_E_ARG, "bad top_k");
    if (!aligned(ws, kAlign) || !aligned(Z0, 8) || !aligned(Z1, 8)) return fail(ctx, CDL_E_ARG, "misaligned pointer");
    if ((map0 == nullptr) != (map1 == nullptr)) return fail(ctx, CDL_E_ARG, "give both maps or neither");
    Arena need(nullptr);
    plan_edges(need, m, k, top_k);
    if (ws_bytes < need.off) return fail(ctx, CDL_E_WORKSPACE, "edge workspace too small");
    HIPCHK(hipSetDevice(ctx->device));
    cdl_status st = check_map(ctx, map0, m, n0);
    if (st != CDL_OK) return st;
    st = check_map(ctx, map1, m, n1);
    if (st != CDL_OK) return st;
    Arena a(ws);
    EdgeWs e = plan_edges(a, m, k, top_k);
    ScoreWs &w = e.sw;
    const int64_t mp = pad_n(m), kp = pad_k(k);
    const int weighted = mode == CDL_SCORE_DELTA_A;
    hipStream_t s = ctx->stream;
    { Timed t_(ctx, "build_zhat"); HIPCHK(launch_build_zhat(Z0, Z1, map0, map1, m, mp, k, kp, stats0, stats1, w.Zh, w.Zhe, w.sq, s)); }
    { Timed t_(ctx, "score"); HIPCHK(launch_score(w.Zh, w.Zhe, kp, w.sq, m, mp, W0, pad_n(n0), W1, pad_n(n1), map0, map1,
                        weighted, w.part, e.tmax, s)); }
    { Timed t_(ctx, "score_reduce"); HIPCHK(launch_score_reduce(w.part, score_tiles_1d(mp), m, mp, F, s)); }
    const int nt2 = score_tiles_2d(mp);
    { Timed t_(ctx, "topk"); HIPCHK(launch_topk(e.tmax, nt2, top_k, e.tscratch, e.order, s)); }
    { Timed t_(ctx, "edge_collect"); HIPCHK(launch_edge_collect(w.Zh, w.Zhe, kp, w.sq, m, mp, W0, pad_n(n0), W1, pad_n(n1),
                               map0, map1, weighted, e.tmax, e.order, top_k, e.tau, e.cap,
                               e.count, e.cval, e.cidx, s)); }
    { Timed t_(ctx, "topk"); HIPCHK(launch_topk64(e.cval, e.cidx, e.cap, e.count, top_k, e.cscratch, edge_val, e.idx, s)); }
    { Timed t_(ctx, "edge_split"); HIPCHK(launch_edge_split(e.idx, m, top_k, edge_a, edge_b, s)); }
    unsigned int cnt = 0;
    HIPCHK(read_to_host(ctx, s, {{&cnt, e.count, sizeof(cnt)}}));
    if ((int64_t)cnt > e.cap)
        return fail(ctx, CDL_E_UNSUPPORTED, "more than " + std::to_string(e.cap) +
                                                " edges reach the K-th edge score (massive ties)");
    return CDL_OK;
}

// ---- sequence ------------------------------------------------------------------------

} // extern "C"

namespace {
struct SeqPlan {
    int64_t nmax = 0, Tmax = 0, mmax = 0, ntot = 0, nsnap = 0;
};
SeqPlan seq_plan(int32_t n_snap, const cdl_snapshot *sn) {
    SeqPlan p;
    for (int t = 0; t < n_snap; ++t) {
        p.nmax = std::max(p.nmax, sn[t].n);
        p.Tmax = std::max(p.Tmax, sn[t].T);
        p.ntot += sn[t].n;
    }
    p.mmax = p.nmax;
    p.nsnap = n_snap;
    return p;
}

// Common nodes of snapshots y and x (ascending global id): row indices.
void common_maps(const cdl_snapshot &y, const cdl_snapshot &x, std::vector<int32_t> &m0,
                 std::vector<int32_t> &m1) {
    m0.clear();
    m1.clear();
    int64_t i = 0, j = 0;
    while (i < y.n && j < x.n) {
        if (y.gid_host[i] == x.gid_host[j]) { m0.push_back((int32_t)i); m1.push_back((int32_t)j); ++i; ++j; }
        else if (y.gid_host[i] < x.gid_host[j]) ++i;
        else ++j;
    }
}

// Chain with a fixed number of levels, no host reads.
cdl_status chain_enqueue(cdl_ctx *ctx, const double *W, const double *deg, const double *stats,
                         int64_t n, int prec, int depth, void *chain) {
    Arena a(chain);
    ChainBuf c = plan_chain(a, n, prec, depth);
    const int64_t ld = pad_n(n);
    hipStream_t s = ctx->stream;
    { Timed t_(ctx, "chain_prep"); HIPCHK(launch_chain_prep(deg, stats, n, ld, 0, c.dmn, c.dm, c.u, s)); }
    { Timed t_(ctx, "normalize"); HIPCHK(launch_normalize(prec, W, ld, n, c.dmn, c.u, 0, c.levels, c.fro, c.fro64, s)); }
    for (int l = 0; l + 1 < depth; ++l) {
        const cdl_status sq = square_step(ctx, prec, c.levels + c.level_bytes * l, c.levels + c.level_bytes * l,
                                          c.levels + c.level_bytes * (l + 1), ld, n, c, false);
        if (sq != CDL_OK) return sq;
    }
    return CDL_OK;
}

// Richardson with exactly `iters` applications of the full stored chain, no
// host reads: the same kernels, in the same order, as cdl_solve_embedding
// with tol = 0.  ||y_r|| and the final ||r_r|| go to ynorm / rnorm (device).
cdl_status solve_enqueue_fixed(cdl_ctx *ctx, const double *W, const double *deg,
                               const int32_t *gid, int64_t n, const void *chain, int prec,
                               int depth, int64_t k, uint64_t seed, int iters, double *Z,
                               void *ws, double *ynorm, double *rnorm) {
    Arena a(ws);
    SolveWs w = plan_solve(a, n, k, prec);
    Arena ac((void *)chain);
    ChainBuf c = plan_chain(ac, n, prec, depth);
    const int64_t ld = pad_n(n), kp = pad_k(k);
    const size_t panel = (size_t)kp * ld;
    hipStream_t s = ctx->stream;
    const int nparts = residual_parts(ld), ntiles = residual_tiles(ld, kp);
    const bool scaled = prec == 3;
    { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w.Yt, panel * sizeof(double), s)); }
    { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w.Xt, panel * sizeof(double), s)); }
    { Timed t_(ctx, "rhs"); HIPCHK(launch_rhs(W, ld, n, gid, k, kp, seed, w.Yt, s)); }
    { Timed t_(ctx, "residual_init"); HIPCHK(launch_residual_k(prec, w.Xt, W, w.Yt, deg, c.dm, ld, n, kp, k, 1, (double *)w.part, w.Rt, w.V64, w.Vlo[0], w.npart, w.mpart, s)); }
    { Timed t_(ctx, "col_norms"); HIPCHK(launch_col_norms2(w.npart, nparts, kp, w.mpart, ntiles, scaled, w.scal, s)); }
    HIPCHK(hipMemcpyAsync(ynorm, w.scal, kp * sizeof(double), hipMemcpyDeviceToDevice, s));
    const double *inv_vs = w.scal + kp + 1;
    for (int it = 0; it < iters; ++it) {
        cdl_status st = precondition_enqueue(ctx, prec, depth, depth, w, c, ld, n, kp, scaled, inv_vs, w.Xt, false);
        if (st != CDL_OK) return st;
        { Timed t_(ctx, "residual"); HIPCHK(launch_residual_k(prec, w.Xt, W, w.Yt, deg, c.dm, ld, n, kp, k, 0, (double *)w.part, w.Rt,
                                 w.V64, w.Vlo[0], w.npart, w.mpart, s)); }
        { Timed t_(ctx, "col_norms"); HIPCHK(launch_col_norms2(w.npart, nparts, kp, w.mpart, ntiles, scaled, w.scal, s)); }
    }
    HIPCHK(hipMemcpyAsync(rnorm, w.scal, kp * sizeof(double), hipMemcpyDeviceToDevice, s));
    { Timed t_(ctx, "finalize_z"); HIPCHK(launch_finalize_z2(w.Xt, ld, n, kp, k, w.mean, Z, s)); }
    return CDL_OK;
}
// ---- one-pass sequences (CDL_SEQ_BATCHED) ------------------------------------
// Every snapshot's weights, chain, solve workspace and embedding and every
// pair's score workspace are resident at once, so each kernel family of the
// chain squarings, the refinement iterations and the scores runs as one
// grouped launch over all snapshots (pairs).

size_t put(Arena &a, size_t bytes) {
    const size_t o = a.off;
    a.take<char>(bytes);
    return o;
}

struct BatchLayout {
    std::vector<size_t> W, deg, st, chain, solve, Z, score, gws;
    size_t maps = 0, snaps = 0, pairs = 0, prefix = 0, gsnaps = 0, gprefix = 0, flags = 0,
           ynorm = 0, rel = 0, status = 0, total = 0;
};
// Streams of a one-pass sequence's right-hand sides: the context's stream,
// its second stream and two more.
constexpr int kSeqStreams = 4;
constexpr int kBatchTables = 10;   // prefix tables of the grouped launches

BatchLayout batch_layout(int32_t n_snap, const cdl_snapshot *sn, const cdl_seq_params *q) {
    BatchLayout L;
    Arena a(nullptr);
    const int depth = std::max(q->depth, 1);
    int64_t ntot = 0;
    for (int t = 0; t < n_snap; ++t) {
        const int64_t n = sn[t].n, ld = pad_n(n);
        ntot += n;
        L.W.push_back(put(a, (size_t)ld * ld * sizeof(double)));
        L.deg.push_back(put(a, (size_t)ld * sizeof(double)));
        L.st.push_back(put(a, CDL_GRAPH_STATS * sizeof(double)));
        Arena c(nullptr);
        plan_chain(c, n, q->prec, depth);
        L.chain.push_back(put(a, c.off));
        Arena w(nullptr);
        plan_solve(w, n, q->k, q->prec);
        L.solve.push_back(put(a, w.off));
        L.Z.push_back(put(a, (size_t)n * q->k * sizeof(double)));
        Arena g(nullptr);
        plan_graph(g, n, sn[t].T);
        L.gws.push_back(put(a, g.off));
    }
    for (int t = 1; t < n_snap; ++t) {
        Arena w(nullptr);
        plan_score(w, std::min(sn[t - 1].n, sn[t].n), q->k);
        L.score.push_back(put(a, w.off));
    }
    const int64_t kp = pad_k(q->k);
    L.maps = put(a, 2 * (size_t)ntot * sizeof(int32_t));
    L.snaps = put(a, (size_t)n_snap * sizeof(cdl::BatchSnap));
    L.pairs = put(a, (size_t)n_snap * sizeof(cdl::BatchPair));
    L.prefix = put(a, (size_t)kBatchTables * (n_snap + 1) * sizeof(int));
    L.gsnaps = put(a, (size_t)n_snap * sizeof(cdl::GraphSnap));
    L.gprefix = put(a, (size_t)cdl::kGraphTables * (n_snap + 1) * sizeof(int));
    L.flags = put(a, 2 * (size_t)n_snap * sizeof(int));
    L.ynorm = put(a, (size_t)n_snap * kp * sizeof(double));
    L.rel = put(a, (size_t)n_snap * sizeof(double));
    L.status = put(a, (size_t)n_snap * CDL_GRAPH_STATS * sizeof(double));
    L.total = a.off;
    return L;
}

size_t seq_bytes(const SeqPlan &p, const cdl_seq_params *q) {
    const int dmax = q->depth > 0 ? q->depth : q->depth_max;
    size_t g = 0, c = 0, so = 0, sc = 0;
    cdl_workspace_bytes(p.nmax, p.Tmax, q->k, dmax, q->prec, &g, &c, &so, &sc);
    const size_t ld = (size_t)pad_n(p.nmax);
    size_t tot = 0;
    tot += 2 * al(ld * ld * sizeof(double));                    // W ping-pong
    tot += 2 * al(ld * sizeof(double));                          // deg
    tot += 2 * al(CDL_GRAPH_STATS * sizeof(double));             // stats
    tot += 2 * al((size_t)p.nmax * q->k * sizeof(double));       // Z ping-pong
    tot += 2 * al((size_t)p.mmax * sizeof(int32_t));             // maps
    tot += g + c + so + sc;
    tot += 2 * al((size_t)p.ntot * sizeof(int32_t));             // all pair maps (async)
    tot += al((size_t)p.nsnap * (CDL_GRAPH_STATS + 2 * pad_k(q->k)) * sizeof(double));   // status
    if (q->flags & CDL_SEQ_ASYNC) {
        // two streams: a third set of per-snapshot state, a second set of workspaces
        tot += al(ld * ld * sizeof(double)) + al(ld * sizeof(double)) +
               al(CDL_GRAPH_STATS * sizeof(double)) + al((size_t)p.nmax * q->k * sizeof(double));
        tot += g + c + so + sc;
    }
    return tot;
}
} // namespace

static void sync_side_streams(cdl_ctx *ctx) {
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    for (hipStream_t x : ctx->extra)
        if (x) (void)hipStreamSynchronize(x);
}

// Runs enqueue(s0, s1) eagerly on the context's stream and its second
// stream; with use_graph, the second call with the same key is captured into
// a HIP graph (both streams forked and joined inside the capture) and later
// calls with that key replay it in one launch.
static cdl_status run_sequence(cdl_ctx *ctx, bool use_graph, const std::vector<uint64_t> &key,
                               const std::function<cdl_status(hipStream_t, hipStream_t)> &enqueue,
                               cdl_seq_info *info) {
    const bool timing = ctx->timing;
    hipStream_t s = ctx->stream;
    cdl_status st = CDL_OK;
    if (!use_graph) {
        // eager two-stream enqueue; a later graph call starts its key afresh
        ctx->seq_key.clear();
        if ((st = enqueue(s, ctx->side)) != CDL_OK) {
            sync_side_streams(ctx);
            return st;
        }
    } else if (key == ctx->seq_key && ctx->seq_exec) {
        HIPCHK(hipGraphLaunch(ctx->seq_exec, s));
        if (info) info->graph_launches = 1;
    } else if (key == ctx->seq_key) {
        // second identical call: capture the enqueue into a graph, on a
        // private stream (the caller's may be the null stream, which
        // cannot be captured), then launch it on the caller's stream
        hipStream_t cap = nullptr, cap2 = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        const hipError_t e2 = hipStreamCreateWithFlags(&cap2, hipStreamNonBlocking);
        if (e2 != hipSuccess) {
            (void)hipStreamDestroy(cap);
            HIPCHK(e2);
        }
        const hipError_t eb = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (eb != hipSuccess) {
            (void)hipStreamDestroy(cap);
            (void)hipStreamDestroy(cap2);
            HIPCHK(eb);
        }
        ctx->timing = false;
        st = enqueue(cap, cap2);   // cap2 joins the capture through the fork event
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(cap, &g);
        ctx->stream = s;
        ctx->timing = timing;
        (void)hipStreamDestroy(cap);
        (void)hipStreamDestroy(cap2);
        if (st != CDL_OK || ec != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            ctx->seq_key.clear();
            if (st != CDL_OK) return st;
            HIPCHK(ec);
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(g);
            HIPCHK(ei);
        }
        ctx->seq_graph = g;
        ctx->seq_exec = ex;
        HIPCHK(hipGraphLaunch(ex, s));
        if (info) info->graph_launches = 1;
    } else {
        if (ctx->seq_exec) (void)hipGraphExecDestroy(ctx->seq_exec);
        if (ctx->seq_graph) (void)hipGraphDestroy(ctx->seq_graph);
        ctx->seq_exec = nullptr;
        ctx->seq_graph = nullptr;
        ctx->seq_key = key;
        if ((st = enqueue(s, ctx->side)) != CDL_OK) {
            sync_side_streams(ctx);   // nothing may stay in flight on the side streams
            return st;
        }
    }
    return CDL_OK;
}

// CDL_SEQ_BATCHED: grouped launches over all snapshots build the graphs
// (padding, distance Gram, exact median, weights, degrees, statistics) and
// the level-0 chains; the right-hand sides rotate over four streams; then,
// on the context's stream, grouped
// launches over all snapshots run the squarings (one per level), the
// initial residuals and every refinement iteration (the applications level
// by level, the FP64 residual product and its reduction, the norms and the
// device-side convergence test: converged snapshots skip their workgroups),
// the centred embeddings, and grouped launches over all pairs the scores;
// top-K per pair.  Nothing is read back until the end.
static cdl_status score_sequence_batched(cdl_ctx *ctx, int32_t n_snap, const cdl_snapshot *sn,
                                         const cdl_seq_params *q, double *const *F,
                                         int32_t *const *top_idx, void *ws,
                                         cdl_seq_info *info) {
    using cdl::BatchPair;
    using cdl::BatchSnap;
    const int P = n_snap, NP = n_snap - 1;
    const int depth = q->depth, prec = q->prec;
    const int64_t k = q->k, kp = pad_k(k);
    const bool scaled = prec == 3;
    const BatchLayout L = batch_layout(n_snap, sn, q);
    char *base = (char *)ws;
    if (info) std::memset(info, 0, sizeof(*info));
    hipStream_t s = ctx->stream;
    HIPCHK(hipSetDevice(ctx->device));
    // host tables: snapshot and pair descriptors, prefix tables, maps
    std::vector<BatchSnap> hs(P);
    std::vector<ChainBuf> chains(P);
    std::vector<SolveWs> solves(P);
    // Split-K counts for the grouped launches: one count S for the whole group,
    // the smallest power of two that gives the group at least two workgroups
    // per CU (the per-snapshot counts fill the chip with one snapshot alone and
    // multiply the partial sums' traffic when many snapshots share a launch),
    // clamped per snapshot to what its length and its workspace allow.
    auto ap_split = [&](int t, int S) {
        const int64_t n = sn[t].n, ld = pad_n(n);
        return std::min(cdl::apply_splits_fixed(prec, n, S), apply_splits(prec, ld, kp, n, 2));
    };
    auto res_split = [&](int t, int S) {
        const int64_t n = sn[t].n, ld = pad_n(n);
        return std::min(cdl::residual_splits_fixed(n, S), residual_splits(ld, kp, n, 2));
    };
    constexpr int64_t kGroupWgs = 2 * 256;
    int Sa = 1, Sr = 1;
    auto ap_tiles = [&](int S) {
        int64_t c = 0;
        for (int t = 0; t < P; ++t) c += cdl::apply_gemm_tiles(pad_n(sn[t].n), kp, ap_split(t, S));
        return c;
    };
    auto res_tiles = [&](int S) {
        int64_t c = 0;
        for (int t = 0; t < P; ++t) c += cdl::residual_gemm_tiles(pad_n(sn[t].n), kp, res_split(t, S));
        return c;
    };
    while (Sa < 256 && ap_tiles(Sa) < kGroupWgs && ap_tiles(2 * Sa) > ap_tiles(Sa)) Sa *= 2;
    while (Sr < 256 && res_tiles(Sr) < kGroupWgs && res_tiles(2 * Sr) > res_tiles(Sr)) Sr *= 2;
    // a choice pinned on the context (cdl_ctx_force_choice) keeps the
    // per-snapshot split counts, so that the grouped launches compute exactly
    // the per-snapshot path's partial sums
    auto pinned = [&](const char *fam) {
        auto f = ctx->forced.find(fam);
        return f != ctx->forced.end() && f->second >= 0 && f->second < 3 ? f->second : -1;
    };
    const int pin_ap = pinned("apply"), pin_res = pinned("residual");
    for (int t = 0; t < P; ++t) {
        const int64_t n = sn[t].n, ld = pad_n(n);
        Arena ac(base + L.chain[t]);
        chains[t] = plan_chain(ac, n, prec, depth);
        Arena aw(base + L.solve[t]);
        solves[t] = plan_solve(aw, n, k, prec);
        const ChainBuf &c = chains[t];
        const SolveWs &w = solves[t];
        BatchSnap &d = hs[t];
        d.n = n;
        d.ld = ld;
        d.W = (const double *)(base + L.W[t]);
        d.deg = (const double *)(base + L.deg[t]);
        d.levels = c.levels;
        d.level_bytes = (int64_t)c.level_bytes;
        d.dm = c.dm;
        d.fro = c.fro;
        d.inv_scale = 1.0f / level_scale(prec, n);
        d.Yt = w.Yt;
        d.Xt = w.Xt;
        d.Rt = w.Rt;
        d.V64 = w.V64;
        d.Vlo[0] = w.Vlo[0];
        d.Vlo[1] = w.Vlo[1];
        d.Pap = (float *)w.part;
        d.Pres = (double *)w.part;
        d.npart = w.npart;
        d.mpart = w.mpart;
        d.scal = w.scal;
        d.ap_splits = pin_ap >= 0 ? apply_splits(prec, ld, kp, n, pin_ap) : ap_split(t, Sa);
        d.res_splits = pin_res >= 0 ? residual_splits(ld, kp, n, pin_res) : res_split(t, Sr);
    }
    std::vector<BatchPair> hp(NP);
    std::vector<int32_t> hm, m0, m1;
    std::vector<int64_t> mcnt(NP);
    int32_t *maps = (int32_t *)(base + L.maps);
    for (int t = 1; t < P; ++t) {
        common_maps(sn[t - 1], sn[t], m0, m1);
        const int64_t m = (int64_t)m0.size();
        if (m < 2) return fail(ctx, CDL_E_GRAPH, "consecutive snapshots share fewer than two nodes");
        BatchPair &r = hp[t - 1];
        r.m = m;
        r.mpad = pad_n(m);
        r.Z0 = (const double *)(base + L.Z[t - 1]);
        r.Z1 = (const double *)(base + L.Z[t]);
        r.map0 = maps + hm.size();
        r.map1 = r.map0 + m;
        hm.insert(hm.end(), m0.begin(), m0.end());
        hm.insert(hm.end(), m1.begin(), m1.end());
        r.stats0 = (const double *)(base + L.st[t - 1]);
        r.stats1 = (const double *)(base + L.st[t]);
        r.W0 = (const double *)(base + L.W[t - 1]);
        r.W1 = (const double *)(base + L.W[t]);
        r.ld0 = pad_n(sn[t - 1].n);
        r.ld1 = pad_n(sn[t].n);
        Arena as(base + L.score[t - 1]);
        const ScoreWs sw = plan_score(as, m, k);
        r.Zh = sw.Zh;
        r.Zhe = sw.Zhe;
        r.sq = sw.sq;
        r.part = sw.part;
        r.F = F[t - 1];
        mcnt[t - 1] = m;
    }
    // prefix tables: 0 squaring, 1 apply product, 2 apply update, 3 residual
    // product, 4 residual reduction, 5 FP16 operand, 6 signature rows,
    // 7 score tiles, 8 score reduction
    std::vector<int> pre((size_t)kBatchTables * (P + 1), 0);
    auto table = [&](int id) { return pre.data() + (size_t)id * (P + 1); };
    auto fill = [&](int id, int cnt, const std::function<int(int)> &f) {
        int *tb = table(id);
        tb[0] = 0;
        for (int i = 0; i < cnt; ++i) tb[i + 1] = tb[i] + f(i);
        return tb[cnt];
    };
    const int tot_sq = fill(0, P, [&](int t) { return square_tiles(prec, hs[t].ld); });
    const int tot_ag = fill(1, P, [&](int t) { return apply_gemm_tiles(hs[t].ld, kp, hs[t].ap_splits); });
    // element-wise kernels stride over at most 256 workgroups per snapshot, so
    // that the launches after every snapshot has converged stay cheap
    constexpr int kEltWgs = 256;
    const int tot_ar = fill(2, P, [&](int t) { return apply_reduce_blocks(hs[t].ld, kp, kEltWgs); });
    const int tot_rg = fill(3, P, [&](int t) { return residual_gemm_tiles(hs[t].ld, kp, hs[t].res_splits); });
    const int tot_rr = fill(4, P, [&](int t) { return (int)std::min<int64_t>(hs[t].ld / 256 * kp, kEltWgs); });
    const int tot_pv = fill(5, P, [&](int t) { return apply_reduce_blocks(hs[t].ld, kp, kEltWgs); });
    const int tot_zh = fill(6, NP, [&](int t) { return (int)hp[t].mpad; });
    const int tot_sc = fill(7, NP, [&](int t) { return score_tiles_2d(hp[t].mpad); });
    const int tot_sr = fill(8, NP, [&](int t) { return (int)((hp[t].m + 63) / 64); });
    BatchSnap *dsnap = (BatchSnap *)(base + L.snaps);
    BatchPair *dpair = (BatchPair *)(base + L.pairs);
    int *dpre = (int *)(base + L.prefix);
    auto dtable = [&](int id) { return dpre + (size_t)id * (P + 1); };
    HIPCHK(hipMemcpyAsync(maps, hm.data(), hm.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dsnap, hs.data(), hs.size() * sizeof(BatchSnap), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dpair, hp.data(), hp.size() * sizeof(BatchPair), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dpre, pre.data(), pre.size() * sizeof(int), hipMemcpyHostToDevice, s));
    // the graph build and level-0 chains of all snapshots: descriptors and
    // prefix tables of the grouped launches
    std::vector<cdl::GraphSnap> hg(P);
    std::vector<int> gpre((size_t)cdl::kGraphTables * (P + 1), 0), gtot(cdl::kGraphTables, 0);
    for (int t = 0; t < P; ++t) {
        const int64_t n = sn[t].n, ld = pad_n(n);
        Arena ag(base + L.gws[t]);
        const GraphWs gw = plan_graph(ag, n, sn[t].T);
        cdl::GraphSnap &g = hg[t];
        g.X = sn[t].X;
        g.n = n;
        g.T = sn[t].T;
        g.ldx = sn[t].ldx;
        g.Tp = pad_t(sn[t].T);
        g.ld = ld;
        g.Xp = gw.Xp;
        g.sqn = gw.sqn;
        g.flags = gw.flags;
        g.W = (double *)hs[t].W;
        g.deg = (double *)hs[t].deg;
        g.stats = (double *)(base + L.st[t]);
        g.sel = gw.sel;
        g.buf = gw.selbuf;
        g.cap = select_buffer_keys(n);
        g.dpart = gw.dpart;
        g.dmn = chains[t].dmn;
        g.dm = chains[t].dm;
        g.u = chains[t].u;
        g.level0 = chains[t].levels;
        g.fro = chains[t].fro;
        g.fro64 = chains[t].fro64;
        g.scale = (double)level_scale(prec, n);
        const bool br = cdl::select_uses_bracket(n, ctx->select_mode == 0);
        g.bracket = br ? 1 : 0;
        for (int tb = 0; tb < cdl::kGraphTables; ++tb) {
            int *row = gpre.data() + (size_t)tb * (P + 1);
            row[t + 1] = row[t] + cdl::graph_table_count(tb, n, ld, br);
        }
    }
    for (int tb = 0; tb < cdl::kGraphTables; ++tb) gtot[tb] = gpre[(size_t)tb * (P + 1) + P];
    cdl::GraphSnap *dgs = (cdl::GraphSnap *)(base + L.gsnaps);
    int *dgpre = (int *)(base + L.gprefix);
    HIPCHK(hipMemcpyAsync(dgs, hg.data(), hg.size() * sizeof(cdl::GraphSnap), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dgpre, gpre.data(), gpre.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    int *done = (int *)(base + L.flags), *iters = done + P;
    double *ynorm = (double *)(base + L.ynorm), *rel = (double *)(base + L.rel);
    double *status = (double *)(base + L.status);
    if (!ctx->side) HIPCHK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    for (hipStream_t &x : ctx->extra)
        if (!x) HIPCHK(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    // fork (one event on the first stream) and join (one per other stream)
    hipEvent_t evs[kSeqStreams] = {};
    struct EvGuard {
        hipEvent_t *v;
        ~EvGuard() { for (int i = 0; i < kSeqStreams; ++i) if (v[i]) (void)hipEventDestroy(v[i]); }
    } ev_guard{evs};
    for (auto &e : evs) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    const int weighted = q->mode == CDL_SCORE_DELTA_A;

    auto enqueue = [&](hipStream_t s0, hipStream_t s1) -> cdl_status {
        // the two extra streams join a capture through the fork event like s1
        hipStream_t ss[kSeqStreams] = {s0, s1, ctx->extra[0], ctx->extra[1]};
        cdl_status st = CDL_OK;
        // graphs and level-0 chains: grouped launches over all snapshots
        { Timed t_(ctx, "graph_grouped"); HIPCHK(cdl::launch_graph_grouped(dgs, dgpre, gtot.data(), P, q->sigma, s0)); }
        { Timed t_(ctx, "chain_level0"); HIPCHK(cdl::launch_chain_level0_grouped(prec, dgs, dgpre, gtot.data(), P, s0)); }
        // right-hand sides per snapshot over the streams
        HIPCHK(hipEventRecord(evs[0], s0));
        for (int b = 1; b < kSeqStreams; ++b) HIPCHK(hipStreamWaitEvent(ss[b], evs[0], 0));
        for (int t = 0; t < P && st == CDL_OK; ++t) {
            hipStream_t es = ss[t % kSeqStreams];
            ctx->stream = es;
            const cdl_snapshot &x = sn[t];
            const double *W = hs[t].W;
            double *stats = (double *)(base + L.st[t]);
            const SolveWs &w = solves[t];
            const size_t panel = (size_t)kp * hs[t].ld * sizeof(double);
            { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w.Yt, panel, es)); }
            { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(w.Xt, panel, es)); }
            { Timed t_(ctx, "rhs"); HIPCHK(launch_rhs(W, hs[t].ld, x.n, x.gid, k, kp, q->seed, w.Yt, es)); }
            HIPCHK(hipMemcpyAsync(status + (size_t)t * CDL_GRAPH_STATS, stats,
                                  CDL_GRAPH_STATS * sizeof(double), hipMemcpyDeviceToDevice, es));
        }
        ctx->stream = s0;
        for (int b = 1; b < kSeqStreams; ++b) {
            HIPCHK(hipEventRecord(evs[b], ss[b]));
            HIPCHK(hipStreamWaitEvent(s0, evs[b], 0));
        }
        if (st != CDL_OK) return st;
        for (int l = 0; l + 1 < depth; ++l)
            { Timed t_(ctx, "square"); HIPCHK(cdl::launch_square_grouped(prec, dsnap, dtable(0), P, tot_sq, l, s0)); }
        // done and iteration flags (their region is rounded up to 256 bytes)
        { Timed t_(ctx, "fill_zero"); HIPCHK(launch_fill_zero(done, (2 * (size_t)P * sizeof(int) + 15) / 16 * 16, s0)); }
        { Timed t_(ctx, "residual_init"); HIPCHK(cdl::launch_residual_grouped(prec, dsnap, dtable(3), tot_rg, dtable(4), tot_rr, P, kp, k, 1, done, s0)); }
        { Timed t_(ctx, "col_norms"); HIPCHK(cdl::launch_norms_grouped(dsnap, P, kp, k, scaled, q->tol, 1, ynorm, rel, done, iters, s0)); }
        for (int it = 0; it < q->max_iter; ++it) {
            if (scaled) { Timed t_(ctx, "prep_v"); HIPCHK(cdl::launch_prep_grouped(prec, dsnap, dtable(5), tot_pv, P, kp, done, s0)); }
            int cur = 0;
            for (int l = 0; l < depth; ++l) {
                { Timed t_(ctx, "apply"); HIPCHK(cdl::launch_apply_grouped(prec, dsnap, dtable(1), tot_ag, dtable(2), tot_ar, P, kp, l, cur, 1,
                                                                     l + 1 == depth, done, s0)); }
                cur ^= 1;
            }
            { Timed t_(ctx, "residual"); HIPCHK(cdl::launch_residual_grouped(prec, dsnap, dtable(3), tot_rg, dtable(4), tot_rr, P, kp, k, 0, done, s0)); }
            { Timed t_(ctx, "col_norms"); HIPCHK(cdl::launch_norms_grouped(dsnap, P, kp, k, scaled, q->tol, 0, ynorm, rel, done, iters, s0)); }
        }
        for (int t = 0; t < P; ++t)
            { Timed t_(ctx, "finalize_z"); HIPCHK(launch_finalize_z2(solves[t].Xt, hs[t].ld, sn[t].n, kp, k, solves[t].mean,
                                                             (double *)(base + L.Z[t]), s0)); }
        { Timed t_(ctx, "score"); HIPCHK(cdl::launch_score_grouped(dpair, dtable(6), tot_zh, dtable(7), tot_sc, dtable(8), tot_sr, NP, k, kp,
                                                             weighted, s0)); }
        if (top_idx && q->top_k > 0)
            for (int t = 0; t < NP; ++t) {
                Arena as(base + L.score[t]);
                const ScoreWs sw = plan_score(as, mcnt[t], k);
                const int32_t K = std::min<int32_t>(q->top_k, (int32_t)mcnt[t]);
                Timed t_(ctx, "topk");
                HIPCHK(launch_topk(F[t], mcnt[t], K, sw.topk, top_idx[t], s0));
            }
        return CDL_OK;
    };
    // the key of a graph: buffers, shapes, parameters, global ids
    std::vector<uint64_t> key = {(uint64_t)n_snap, (uint64_t)(uintptr_t)ws, (uint64_t)L.total,
                                 (uint64_t)q->k, q->seed, (uint64_t)q->prec, (uint64_t)q->depth,
                                 (uint64_t)q->max_iter, (uint64_t)q->mode, (uint64_t)q->top_k,
                                 (uint64_t)q->flags};
    uint64_t bits;
    std::memcpy(&bits, &q->sigma, sizeof(bits));
    key.push_back(bits);
    std::memcpy(&bits, &q->tol, sizeof(bits));
    key.push_back(bits);
    for (int t = 0; t < n_snap; ++t) {
        uint64_t h = 1469598103934665603ull;
        for (int64_t i = 0; i < sn[t].n; ++i) h = (h ^ (uint32_t)sn[t].gid_host[i]) * 1099511628211ull;
        key.insert(key.end(), {(uint64_t)(uintptr_t)sn[t].X, (uint64_t)sn[t].n, (uint64_t)sn[t].T,
                               (uint64_t)sn[t].ldx, (uint64_t)(uintptr_t)sn[t].gid, h,
                               (uint64_t)(uintptr_t)(t + 1 < n_snap ? F[t] : nullptr),
                               (uint64_t)(uintptr_t)(t + 1 < n_snap && top_idx ? top_idx[t] : nullptr)});
        key.insert(key.end(), {(uint64_t)hs[t].ap_splits, (uint64_t)hs[t].res_splits});
    }
    cdl_status st = run_sequence(ctx, (q->flags & CDL_SEQ_GRAPH) != 0, key, enqueue, info);
    if (st != CDL_OK) return st;
    // one read-back: graph statistics, final residuals, iterations
    std::vector<double> hst((size_t)P * CDL_GRAPH_STATS), hrel(P);
    std::vector<int> hit(P), hdone(P);
    HIPCHK(read_to_host(ctx, s, {{hst.data(), status, hst.size() * sizeof(double)},
                                 {hrel.data(), rel, hrel.size() * sizeof(double)},
                                 {hdone.data(), done, hdone.size() * sizeof(int)},
                                 {hit.data(), iters, hit.size() * sizeof(int)}}));
    double worst = 0.0;
    int most = 0;
    for (int t = 0; t < P; ++t) {
        const double *h = hst.data() + (size_t)t * CDL_GRAPH_STATS;
        for (int q2 = 0; q2 < CDL_GRAPH_STATS; ++q2)
            if (!std::isfinite(h[q2])) return fail(ctx, CDL_E_NONFINITE, "snapshot " + std::to_string(t) + ": non-finite weights or degrees");
        if (!(h[2] > 0.0)) return fail(ctx, CDL_E_GRAPH, "snapshot " + std::to_string(t) + ": a node has zero degree");
        if (!std::isfinite(hrel[t])) return fail(ctx, CDL_E_NONFINITE, "snapshot " + std::to_string(t) + ": non-finite residual");
        worst = std::max(worst, hrel[t]);
        most = std::max(most, hit[t]);
    }
    if (info) {
        info->pairs = NP;
        info->max_iterations = most;
        info->max_rel_residual = worst;
    }
    if (q->tol > 0.0 && worst > q->tol)
        return fail(ctx, CDL_E_NOCONV, "residual " + std::to_string(worst) + " above tol after max_iter iterations");
    return CDL_OK;
}

extern "C" {

cdl_status cdl_sequence_workspace_bytes(int32_t n_snap, const cdl_snapshot *snaps,
                                        const cdl_seq_params *p, size_t *bytes) {
    if (n_snap < 2 || !snaps || !p || !bytes || p->k < 1) return CDL_E_ARG;
    for (int t = 0; t < n_snap; ++t)
        if (snaps[t].n < 2 || snaps[t].T < 1) return CDL_E_ARG;
    *bytes = (p->flags & CDL_SEQ_BATCHED) ? batch_layout(n_snap, snaps, p).total
                                           : seq_bytes(seq_plan(n_snap, snaps), p);
    return CDL_OK;
}

cdl_status cdl_score_sequence(cdl_ctx *ctx, int32_t n_snap, const cdl_snapshot *sn,
                              const cdl_seq_params *q, double *const *F, int32_t *const *top_idx,
                              void *ws, size_t ws_bytes, cdl_seq_info *info) {
    if (!ctx) return CDL_E_ARG;
    if (n_snap < 2 || !sn || !q || !F || !ws) return fail(ctx, CDL_E_ARG, "bad arguments");
    for (int t = 0; t < n_snap; ++t) {
        if (!sn[t].X || !sn[t].gid || !sn[t].gid_host || sn[t].n < 2)
            return fail(ctx, CDL_E_ARG, "bad snapshot");
        for (int64_t i = 1; i < sn[t].n; ++i)
            if (sn[t].gid_host[i] <= sn[t].gid_host[i - 1])
                return fail(ctx, CDL_E_ARG, "global ids must be strictly increasing");
        if (sn[t].gid_host[sn[t].n - 1] >= (1 << 20) || sn[t].gid_host[0] < 0)
            return fail(ctx, CDL_E_ARG, "global ids must be in [0, 2^20)");
    }
    const SeqPlan plan = seq_plan(n_snap, sn);
    const bool async = (q->flags & CDL_SEQ_ASYNC) != 0;
    const bool batched = (q->flags & CDL_SEQ_BATCHED) != 0;
    if ((q->flags & ~(CDL_SEQ_ASYNC | CDL_SEQ_GRAPH | CDL_SEQ_BATCHED)) != 0 ||
        ((q->flags & (CDL_SEQ_GRAPH | CDL_SEQ_BATCHED)) && !async))
        return fail(ctx, CDL_E_ARG, "bad sequence flags");
    if (ws_bytes < (batched ? batch_layout(n_snap, sn, q).total : seq_bytes(plan, q)))
        return fail(ctx, CDL_E_WORKSPACE, "sequence workspace too small");
    if (async) {
        // the enqueue helpers check nothing: every argument is checked here
        if (q->depth < 1 || q->depth > CDL_MAX_DEPTH || q->solver != CDL_RICHARDSON || !(q->tol >= 0.0))
            return fail(ctx, CDL_E_ARG, "CDL_SEQ_ASYNC needs 1 <= depth <= 14, Richardson and tol >= 0");
        if (q->k < 1 || q->k > ((int64_t)1 << 20) || !valid_prec(q->prec) || q->max_iter < 1 ||
            q->max_iter > 64 || (q->mode != CDL_SCORE_UNWEIGHTED && q->mode != CDL_SCORE_DELTA_A) ||
            q->top_k < 0 || q->top_k > CDL_MAX_TOPK || !std::isfinite(q->sigma))
            return fail(ctx, CDL_E_ARG, "bad sequence parameters");
        if (!aligned(ws, kAlign)) return fail(ctx, CDL_E_ARG, "misaligned workspace");
        for (int t = 0; t < n_snap; ++t) {
            if (sn[t].n > (1 << 20) || sn[t].T < 1 || sn[t].ldx < sn[t].T || !aligned(sn[t].X, 8) ||
                !aligned(sn[t].gid, 4))
                return fail(ctx, CDL_E_ARG, "bad snapshot");
            if (t + 1 < n_snap && (!F[t] || !aligned(F[t], 8) || (q->top_k > 0 && top_idx && !top_idx[t])))
                return fail(ctx, CDL_E_ARG, "bad output pointer");
        }
        if (batched) {
            if (q->prec == CDL_FP64) return fail(ctx, CDL_E_ARG, "CDL_SEQ_BATCHED needs FP32, BF16 or FP16 levels");
            if (n_snap > 4096) return fail(ctx, CDL_E_ARG, "CDL_SEQ_BATCHED takes at most 4096 snapshots");
            return score_sequence_batched(ctx, n_snap, sn, q, F, top_idx, ws, info);
        }
    }
    const int dmax = q->depth > 0 ? q->depth : q->depth_max;
    size_t gB = 0, cB = 0, soB = 0, scB = 0;
    cdl_workspace_bytes(plan.nmax, plan.Tmax, q->k, dmax, q->prec, &gB, &cB, &soB, &scB);
    Arena a(ws);
    const size_t ld = (size_t)pad_n(plan.nmax);
    double *Wb[2] = {a.take<double>(ld * ld), a.take<double>(ld * ld)};
    double *degb[2] = {a.take<double>(ld), a.take<double>(ld)};
    double *stb[2] = {a.take<double>(CDL_GRAPH_STATS), a.take<double>(CDL_GRAPH_STATS)};
    double *Zb[2] = {a.take<double>((size_t)plan.nmax * q->k), a.take<double>((size_t)plan.nmax * q->k)};
    int32_t *mapb[2] = {a.take<int32_t>(plan.mmax), a.take<int32_t>(plan.mmax)};
    char *gws = a.take<char>(gB), *cws = a.take<char>(cB), *sows = a.take<char>(soB), *scws = a.take<char>(scB);
    int32_t *maps_all = a.take<int32_t>(2 * (size_t)plan.ntot);
    const int64_t kp = pad_k(q->k);
    double *status = a.take<double>((size_t)n_snap * (CDL_GRAPH_STATS + 2 * kp));
    if (async) {
        if (info) std::memset(info, 0, sizeof(*info));
        hipStream_t s = ctx->stream;
        HIPCHK(hipSetDevice(ctx->device));
        // per-snapshot state rotates over three sets (snapshot t + 3 reuses t's
        // only after every reader of t's set is done); workspaces per stream
        double *W3[3] = {Wb[0], Wb[1], a.take<double>(ld * ld)};
        double *deg3[3] = {degb[0], degb[1], a.take<double>(ld)};
        double *st3[3] = {stb[0], stb[1], a.take<double>(CDL_GRAPH_STATS)};
        double *Z3[3] = {Zb[0], Zb[1], a.take<double>((size_t)plan.nmax * q->k)};
        char *gws2[2] = {gws, a.take<char>(gB)}, *cws2[2] = {cws, a.take<char>(cB)};
        char *sows2[2] = {sows, a.take<char>(soB)}, *scws2[2] = {scws, a.take<char>(scB)};
        if (!ctx->side) HIPCHK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
        std::vector<hipEvent_t> ev(n_snap + 1, nullptr);
        struct EvGuard {
            std::vector<hipEvent_t> &v;
            ~EvGuard() { for (hipEvent_t e : v) if (e) (void)hipEventDestroy(e); }
        } ev_guard{ev};
        for (auto &e : ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        // all common-node maps, uploaded before anything is enqueued
        std::vector<int32_t> hm, m0, m1;
        std::vector<int64_t> moff(n_snap, 0), mcnt(n_snap, 0);
        for (int t = 1; t < n_snap; ++t) {
            common_maps(sn[t - 1], sn[t], m0, m1);
            if ((int64_t)m0.size() < 2) return fail(ctx, CDL_E_GRAPH, "consecutive snapshots share fewer than two nodes");
            moff[t] = (int64_t)hm.size();
            mcnt[t] = (int64_t)m0.size();
            hm.insert(hm.end(), m0.begin(), m0.end());
            hm.insert(hm.end(), m1.begin(), m1.end());
        }
        HIPCHK(hipMemcpyAsync(maps_all, hm.data(), hm.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        // the key of this call: buffers, shapes, parameters, global ids
        std::vector<uint64_t> key = {(uint64_t)n_snap, (uint64_t)(uintptr_t)ws, (uint64_t)ws_bytes,
                                     (uint64_t)q->k, q->seed, (uint64_t)q->prec, (uint64_t)q->depth,
                                     (uint64_t)q->max_iter, (uint64_t)q->mode, (uint64_t)q->top_k};
        uint64_t sb;
        std::memcpy(&sb, &q->sigma, sizeof(sb));
        key.push_back(sb);
        for (int t = 0; t < n_snap; ++t) {
            uint64_t h = 1469598103934665603ull;
            for (int64_t i = 0; i < sn[t].n; ++i) h = (h ^ (uint32_t)sn[t].gid_host[i]) * 1099511628211ull;
            key.insert(key.end(), {(uint64_t)(uintptr_t)sn[t].X, (uint64_t)sn[t].n, (uint64_t)sn[t].T,
                                   (uint64_t)sn[t].ldx, (uint64_t)(uintptr_t)sn[t].gid, h,
                                   (uint64_t)(uintptr_t)(t + 1 < n_snap ? F[t] : nullptr),
                                   (uint64_t)(uintptr_t)(t + 1 < n_snap && top_idx ? top_idx[t] : nullptr)});
        }
        // Snapshot t runs on stream t % 2 (the second joins after a fork
        // event), then scores pair (t - 1, t) once snapshot t - 1 and its own
        // score are done (event ev[t - 1]); ev[t] marks the end of both.
        // Consecutive snapshots therefore overlap.  s0 joins s1 at the end.
        auto enqueue = [&](hipStream_t s0, hipStream_t s1) -> cdl_status {
            hipStream_t ss[2] = {s0, s1};
            HIPCHK(hipEventRecord(ev[n_snap], s0));
            HIPCHK(hipStreamWaitEvent(s1, ev[n_snap], 0));
            cdl_status st = CDL_OK;
            for (int t = 0; t < n_snap && st == CDL_OK; ++t) {
                const int si = t & 1, b = t % 3;
                hipStream_t es = ss[si];
                ctx->stream = es;
                const cdl_snapshot &x = sn[t];
                st = graph_enqueue(ctx, x.X, x.n, x.T, x.ldx, q->sigma, W3[b], deg3[b], st3[b], gws2[si]);
                if (st != CDL_OK) break;
                double *stat_t = status + (size_t)t * (CDL_GRAPH_STATS + 2 * kp);
                if (hipMemcpyAsync(stat_t, st3[b], CDL_GRAPH_STATS * sizeof(double), hipMemcpyDeviceToDevice, es) != hipSuccess) {
                    st = fail(ctx, CDL_E_HIP, "status copy failed");
                    break;
                }
                if ((st = chain_enqueue(ctx, W3[b], deg3[b], st3[b], x.n, q->prec, q->depth, cws2[si])) != CDL_OK) break;
                if ((st = solve_enqueue_fixed(ctx, W3[b], deg3[b], x.gid, x.n, cws2[si], q->prec, q->depth, q->k, q->seed,
                                              q->max_iter, Z3[b], sows2[si], stat_t + CDL_GRAPH_STATS,
                                              stat_t + CDL_GRAPH_STATS + kp)) != CDL_OK)
                    break;
                if (t > 0) {
                    if (hipStreamWaitEvent(es, ev[t - 1], 0) != hipSuccess) {
                        st = fail(ctx, CDL_E_HIP, "event wait failed");
                        break;
                    }
                    const int pb = (t - 1) % 3;
                    const cdl_snapshot &y = sn[t - 1];
                    const int64_t m = mcnt[t], mp = pad_n(m);
                    const int32_t *mp0 = maps_all + moff[t], *mp1 = mp0 + m;
                    Arena as(scws2[si]);
                    ScoreWs w = plan_score(as, m, q->k);
                    const int32_t K = top_idx ? std::min<int32_t>(q->top_k, (int32_t)m) : 0;
                    const int weighted = q->mode == CDL_SCORE_DELTA_A;
                    hipError_t e = hipSuccess;
                    { Timed t_(ctx, "build_zhat"); e = launch_build_zhat(Z3[pb], Z3[b], mp0, mp1, m, mp, q->k, kp, st3[pb], st3[b], w.Zh, w.Zhe, w.sq, es); }
                    if (e == hipSuccess) { Timed t_(ctx, "score"); e = launch_score(w.Zh, w.Zhe, kp, w.sq, m, mp, W3[pb], pad_n(y.n), W3[b], pad_n(x.n),
                                        mp0, mp1, weighted, w.part, nullptr, es); }
                    if (e == hipSuccess) { Timed t_(ctx, "score_reduce"); e = launch_score_reduce(w.part, score_tiles_1d(mp), m, mp, F[t - 1], es); }
                    if (e == hipSuccess && K > 0) { Timed t_(ctx, "topk"); e = launch_topk(F[t - 1], m, K, w.topk, top_idx[t - 1], es); }
                    if (e != hipSuccess) {
                        st = fail(ctx, CDL_E_HIP, std::string("score launch: ") + hipGetErrorString(e));
                        break;
                    }
                }
                if (hipEventRecord(ev[t], es) != hipSuccess) st = fail(ctx, CDL_E_HIP, "event record failed");
            }
            ctx->stream = s0;
            // join: s0 waits for the last snapshot on s1 (the last on s0 is in order)
            const int last1 = (n_snap - 1) & 1 ? n_snap - 1 : n_snap - 2;
            if (hipStreamWaitEvent(s0, ev[last1 >= 1 ? last1 : n_snap], 0) != hipSuccess && st == CDL_OK)
                st = fail(ctx, CDL_E_HIP, "event wait failed");
            return st;
        };
        cdl_status st = run_sequence(ctx, (q->flags & CDL_SEQ_GRAPH) != 0, key, enqueue, info);
        if (st != CDL_OK) return st;
        // one read-back for the whole sequence: graph checks and residuals
        std::vector<double> hs((size_t)n_snap * (CDL_GRAPH_STATS + 2 * kp));
        HIPCHK(read_to_host(ctx, s, {{hs.data(), status, hs.size() * sizeof(double)}}));
        double worst = 0.0;
        for (int t = 0; t < n_snap; ++t) {
            const double *h = hs.data() + (size_t)t * (CDL_GRAPH_STATS + 2 * kp);
            for (int q2 = 0; q2 < CDL_GRAPH_STATS; ++q2)
                if (!std::isfinite(h[q2])) return fail(ctx, CDL_E_NONFINITE, "snapshot " + std::to_string(t) + ": non-finite weights or degrees");
            if (!(h[2] > 0.0)) return fail(ctx, CDL_E_GRAPH, "snapshot " + std::to_string(t) + ": a node has zero degree");
            double rel = 0.0;
            for (int64_t r = 0; r < q->k; ++r) {
                const double yn = h[CDL_GRAPH_STATS + r], rn = h[CDL_GRAPH_STATS + kp + r];
                if (!std::isfinite(rn)) return fail(ctx, CDL_E_NONFINITE, "snapshot " + std::to_string(t) + ": non-finite residual");
                if (yn > 0.0) rel = std::max(rel, rn / yn);
            }
            worst = std::max(worst, rel);
        }
        if (info) {
            info->pairs = n_snap - 1;
            info->max_iterations = q->max_iter;
            info->max_rel_residual = worst;
        }
        if (q->tol > 0.0 && worst > q->tol)
            return fail(ctx, CDL_E_NOCONV, "residual " + std::to_string(worst) + " above tol after the fixed iterations");
        return CDL_OK;
    }
    if (info) std::memset(info, 0, sizeof(*info));
    hipStream_t s = ctx->stream;
    for (int t = 0; t < n_snap; ++t) {
        const int b = t & 1;
        const cdl_snapshot &x = sn[t];
        cdl_status st = cdl_build_graph(ctx, x.X, x.n, x.T, x.ldx, q->sigma, Wb[b], degb[b], stb[b], gws, gB);
        if (st == CDL_OK) st = cdl_check_graph(ctx, degb[b], stb[b], x.n, nullptr);
        cdl_chain_info ci;
        if (st == CDL_OK)
            st = cdl_build_chain(ctx, Wb[b], degb[b], stb[b], x.n, q->prec, q->depth, dmax, q->chain_eps,
                                 0, cws, cB, &ci);
        cdl_solve_info si;
        if (st == CDL_OK)
            st = cdl_solve_embedding(ctx, Wb[b], degb[b], stb[b], x.gid, x.n, cws, &ci, q->k, 0.0, q->seed,
                                     q->solver, q->tol, q->max_iter, Zb[b], sows, soB, &si);
        if (st != CDL_OK) {
            ctx->err = "snapshot " + std::to_string(t) + ": " + ctx->err;
            return st;
        }
        if (info) {
            info->max_iterations = std::max(info->max_iterations, si.iterations);
            info->max_rel_residual = std::max(info->max_rel_residual, si.rel_residual);
        }
        if (t == 0) continue;
        // common nodes of (t-1, t) in ascending global id order
        const cdl_snapshot &y = sn[t - 1];
        std::vector<int32_t> m0, m1;
        common_maps(y, x, m0, m1);
        const int64_t m = (int64_t)m0.size();
        if (m < 2) return fail(ctx, CDL_E_GRAPH, "consecutive snapshots share fewer than two nodes");
        HIPCHK(hipMemcpyAsync(mapb[0], m0.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(mapb[1], m1.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, s));
        const int pb = b ^ 1;
        const int32_t K = top_idx ? std::min<int32_t>(q->top_k, (int32_t)m) : 0;
        st = cdl_anomaly_scores(ctx, Zb[pb], Wb[pb], stb[pb], y.n, Zb[b], Wb[b], stb[b], x.n, q->k,
                                mapb[0], mapb[1], m, q->mode, F[t - 1], K,
                                top_idx ? top_idx[t - 1] : nullptr, scws, scB);
        if (st != CDL_OK) return st;
        HIPCHK(hipStreamSynchronize(s));   // host maps are reused next pair
        if (info) info->pairs += 1;
    }
    return CDL_OK;
}

} // extern "C"
