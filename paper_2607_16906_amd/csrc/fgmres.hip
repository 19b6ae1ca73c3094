// Host driver of restarted flexible GMRES (Algorithm 1 with the bookkeeping of Section 4).
//
// Everything numerical runs in device kernels; the host only enqueues them. A restart
// cycle is captured once into a HIP graph (its m Arnoldi steps and the cycle end) and
// replayed for every cycle of the same length: every kernel of a step first reads the
// device flag `stop` (set when the Givens estimate reaches tol, on breakdown or on a
// non-finite value) and returns at once when it is set, so steps past the end of a cycle
// cost one empty launch each. The cycle ends with the least-squares update of x and the
// FP64 true residual that starts the next cycle; the host then reads the device state
// once (the only synchronisation per cycle).
//
// Instantiated cycle graphs are kept between calls: a later solve with the same problem,
// network, options, vectors and workspace (and cycle length) replays the kept graph instead of
// capturing and instantiating it again (about 1.7 ms of host time for a 30-step cycle with the
// network). A kept graph only holds addresses, so new values in b, x0, the weights or the
// coefficients are seen; it is dropped when its problem or network is destroyed.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>

#include "krylov.h"
#include "net.h"
#include "problem.h"

namespace hz {

uint64_t next_handle_uid() {
    static std::atomic<uint64_t> next{1};
    return next.fetch_add(1);
}

// ------------------------------------------------------------------ kept cycle graphs

// Everything a captured cycle depends on. Zero-filled before use and compared bytewise.
struct GraphKey {
    uint64_t puid, nuid, tgen;
    int32_t steps, fuse, m, maxit, krylov, net_prec, ortho, pad;
    double tol;
    const void* b;
    const void* x;
    const void* ws;
    uint64_t ws_len;
};
struct GraphKeyLess {
    bool operator()(const GraphKey& a, const GraphKey& b) const { return std::memcmp(&a, &b, sizeof a) < 0; }
};
struct KeptGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    bool busy = false;      // in use by a running solve (a second caller captures its own)
    uint64_t last = 0;      // use stamp (the least recent free entry is dropped when full)
};
constexpr size_t GRAPH_CACHE_MAX = 32;

// Heap-held and never freed: no graph is destroyed by static destructors after the runtime.
static std::mutex& graph_mu() {
    static std::mutex* m = new std::mutex();
    return *m;
}
static std::map<GraphKey, KeptGraph, GraphKeyLess>& graph_cache() {
    static auto* c = new std::map<GraphKey, KeptGraph, GraphKeyLess>();
    return *c;
}
static uint64_t graph_stamp = 0;

static void destroy_graph(hipGraph_t g, hipGraphExec_t e) {
    if (e) (void)hipGraphExecDestroy(e);
    if (g) (void)hipGraphDestroy(g);
}

void fgmres_graph_cache_evict(uint64_t uid) {
    if (uid == 0) return;
    std::lock_guard<std::mutex> lk(graph_mu());
    auto& c = graph_cache();
    for (auto it = c.begin(); it != c.end();) {
        if (it->first.puid == uid || it->first.nuid == uid) {
            destroy_graph(it->second.g, it->second.e);
            it = c.erase(it);
        } else {
            ++it;
        }
    }
}

// The graph a solve is using: kept in the cache (released at the end) or owned (destroyed).
struct GraphUse {
    GraphKey key{};
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    bool kept = false;
    void release() {
        if (!e && !g) return;
        if (kept) {
            std::lock_guard<std::mutex> lk(graph_mu());
            auto it = graph_cache().find(key);
            if (it != graph_cache().end()) it->second.busy = false;
        } else {
            destroy_graph(g, e);
        }
        g = nullptr;
        e = nullptr;
        kept = false;
    }
    ~GraphUse() { release(); }
};

// A free kept graph for this key, marked busy; false when there is none.
static bool graph_acquire(const GraphKey& k, GraphUse& u) {
    std::lock_guard<std::mutex> lk(graph_mu());
    auto it = graph_cache().find(k);
    if (it == graph_cache().end() || it->second.busy) return false;
    it->second.busy = true;
    it->second.last = ++graph_stamp;
    u.key = k;
    u.g = it->second.g;
    u.e = it->second.e;
    u.kept = true;
    return true;
}

// Keep a freshly instantiated graph (busy) if there is room, dropping the least recently used
// free entry when full; otherwise the solve owns it.
static void graph_keep(const GraphKey& k, GraphUse& u) {
    std::lock_guard<std::mutex> lk(graph_mu());
    auto& c = graph_cache();
    if (c.count(k)) return;   // another caller keeps one for this key (busy): own this one
    if (c.size() >= GRAPH_CACHE_MAX) {
        auto victim = c.end();
        for (auto it = c.begin(); it != c.end(); ++it)
            if (!it->second.busy && (victim == c.end() || it->second.last < victim->second.last)) victim = it;
        if (victim == c.end()) return;
        destroy_graph(victim->second.g, victim->second.e);
        c.erase(victim);
    }
    KeptGraph kg;
    kg.g = u.g;
    kg.e = u.e;
    kg.busy = true;
    kg.last = ++graph_stamp;
    c.emplace(k, kg);
    u.key = k;
    u.kept = true;
}

struct FgmresLayout {
    KrylovBufs kb;
    void* V;          // (m+1) x n Krylov vectors
    void* Z;          // m x n preconditioned vectors (NULL: Z = V)
    double2* r64;     // n, FP64 residual
    double* rpart;    // stencil block partials
    void* net_ws;
    size_t net_ws_bytes;
    size_t total;
};

static FgmresLayout fgmres_layout(const hz_problem* p, const no_net* net, const hz_opts* o, void* base,
                                  size_t cap) {
    FgmresLayout L{};
    const int64_t n = p->n;
    const int m = o->m;
    const bool c128 = o->krylov == HZ_C128;
    const size_t es = c128 ? sizeof(double2) : sizeof(float2);
    Split sp = krylov_split(n);
    Carver c(base, cap);
    L.kb.st = c.take<SolveState>(1);
    L.kb.R = c.take<double2>((size_t)(m + 1) * m);
    L.kb.cs = c.take<double>(m);
    L.kb.sn = c.take<double2>(m);
    L.kb.g = c.take<double2>(m + 1);
    L.kb.y = c.take<double2>(m);
    const bool lag = o->ortho == 1;
    L.kb.h1 = c.take<double2>(lag ? 2 * m + 4 : m + 2);
    L.kb.h2 = c.take<double2>(m + 2);
    L.kb.ldp = lag ? 2 * m + 4 : m + 2;
    if (lag) {
        L.kb.pend = c.take<double2>(m + 1);
        L.kb.colb = c.take<double2>(m + 1);
        L.kb.coef = c.take<double2>(2 * m + 2);
        L.kb.lag_sc = c.take<double>(4);
    }
    L.kb.part = c.take<double2>((size_t)sp.nblk * L.kb.ldp);
    L.kb.hist_cap = std::max(o->maxit, 1);
    L.kb.hist = c.take<double>(L.kb.hist_cap);
    L.rpart = c.take<double>(stencil_blocks(p));
    L.r64 = c.take<double2>(n);
    L.V = c.take<char>(es * n * (m + 1));
    L.Z = net ? c.take<char>(es * n * m) : nullptr;
    if (net) {
        int Hp, Wp;
        net_padded_dims(net, p, &Hp, &Wp);
        L.net_ws_bytes = net_fwd_ws_bytes(net, Hp, Wp, 1, o->net_prec);
        L.net_ws = c.take<char>(L.net_ws_bytes);
    }
    L.total = c.off + 256;
    return L;
}

static int check_opts(const hz_opts* o, const no_net* net, const hz_problem* p) {
    HZ_CHECK_ARG(o, "fgmres: NULL options");
    HZ_CHECK_ARG(o->m >= 1 && o->m <= 4096, "fgmres: m must be in [1, 4096]");
    HZ_CHECK_ARG(o->maxit >= 1, "fgmres: maxit must be >= 1");
    HZ_CHECK_ARG(o->tol > 0, "fgmres: tol must be > 0");
    HZ_CHECK_ARG(o->krylov == HZ_C64 || o->krylov == HZ_C128, "fgmres: krylov must be HZ_C64 or HZ_C128");
    HZ_CHECK_ARG(!net || o->net_prec == NO_BF16 || o->net_prec == NO_FP32 || o->net_prec == NO_FP64,
                 "fgmres: bad net_prec");
    HZ_CHECK_ARG(!o->hist_host || o->hist_len >= 0, "fgmres: bad hist_len");
    HZ_CHECK_ARG(o->ortho == 0 || (o->ortho == 1 && net), "fgmres: ortho must be 0, or 1 with a network");
    HZ_CHECK_ARG(!(o->ortho == 1 && p && is_spectral(p)), "fgmres: the spectral operator runs with ortho = 0");
    return HZ_OK;
}

// The launches of one restart cycle (steps Arnoldi steps, then the cycle end).
static int cycle_launches(const hz_problem* p, const no_net* net, const hz_opts* o, const FgmresLayout& L,
                          KrylovBufs& kb, const double2* b, double2* x, int steps, hipStream_t s) {
    const int64_t n = p->n;
    const bool c128 = o->krylov == HZ_C128;
    const size_t es = c128 ? sizeof(double2) : sizeof(float2);
    const int* stop = &kb.st->stop;
    Split sp = krylov_split(n);
    const int nres = stencil_blocks(p);
    auto vcol = [&](int i) { return (void*)((char*)L.V + es * n * i); };
    auto zcol = [&](int i) { return L.Z ? (void*)((char*)L.Z + es * n * i) : vcol(i); };
    for (int j = 0; j < steps; ++j) {
        // z_j = N(v_j); for j >= 1 the network's input pass first completes v_j = w / h_{j,j-1}
        if (net)
            HZ_TRY(net_precond(net, p, o->net_prec, c128, vcol(j), zcol(j), L.net_ws, L.net_ws_bytes, stop, s, true,
                               j > 0 ? &kb.st->inv_h : nullptr));
        // w = A z_j, written into the slot of v_{j+1}, with the first Gram-Schmidt sums
        void* w = vcol(j + 1);
        HZ_TRY(launch_stencil_dots(p, c128, zcol(j), L.V, n, j + 1, w, sp, kb.part, kb.ldp, stop, s));
        HZ_TRY(launch_finalize(kb.part, sp.nblk, kb.ldp, j + 2, kb.h1, stop, s));
        HZ_TRY(launch_update(c128, L.V, n, j + 1, kb.h1, w, n, sp, kb.part, kb.ldp, 1, stop, s));
        HZ_TRY(launch_finalize(kb.part, sp.nblk, kb.ldp, j + 1, kb.h2, stop, s));
        HZ_TRY(launch_update(c128, L.V, n, j + 1, kb.h2, w, n, sp, kb.part, kb.ldp, 2, stop, s));
        HZ_TRY(launch_arnoldi_finish(kb, j, sp.nblk, true, s));
        // without a network the next step's matvec reads v_{j+1} directly
        if (!net) HZ_TRY(launch_scale(c128, w, n, &kb.st->inv_h, stop, s));
    }
    HZ_TRY(launch_backsolve(kb, s));
    HZ_TRY(launch_xupdate(c128, zcol(0), n, x, n, kb, s));
    HZ_TRY(launch_resid64(p, b, x, L.r64, L.rpart, nullptr, s));
    HZ_TRY(launch_cycle_start(kb, L.rpart, nres, s));
    HZ_TRY(launch_cast_scale(c128, L.r64, vcol(0), n, kb.st, s));
    return HZ_OK;
}

// One restart cycle with delayed reorthogonalisation (ortho = 1): per step the network on the
// once-projected vector v~_j (slot j; v_0 is normalised), w = A z_j into slot j + 1 with the
// sums [Q, v~]^H [v~, w] and ||w||^2 in one reduction, the Hessenberg step (completes column
// j - 1, forms column j's first pass) and one update pass (q_j into slot j, the next v~ into slot
// j + 1); after the last step one more reduction completes the last column.
static int cycle_launches_lag(const hz_problem* p, const no_net* net, const hz_opts* o, const FgmresLayout& L,
                              KrylovBufs& kb, const double2* b, double2* x, int steps, hipStream_t s) {
    const int64_t n = p->n;
    const bool c128 = o->krylov == HZ_C128;
    const size_t es = c128 ? sizeof(double2) : sizeof(float2);
    const int* stop = &kb.st->stop;
    Split sp = krylov_split(n);
    const int nres = stencil_blocks(p);
    auto vcol = [&](int i) { return (void*)((char*)L.V + es * n * i); };
    auto zcol = [&](int i) { return (void*)((char*)L.Z + es * n * i); };
    // the previous step's update pass leaves ||v~_j||^2 as block partials in slot 0 of part
    const NormParts np{kb.part, sp.nblk, kb.ldp, kb.lag_sc};
    for (int j = 0; j < steps; ++j) {
        HZ_TRY(net_precond(net, p, o->net_prec, c128, vcol(j), zcol(j), L.net_ws, L.net_ws_bytes, stop, s, j == 0,
                           nullptr, j > 0 ? &np : nullptr));
        HZ_TRY(launch_stencil_dots(p, c128, zcol(j), L.V, n, j + 1, vcol(j + 1), sp, kb.part, kb.ldp, stop, s, true));
        HZ_TRY(launch_finalize(kb.part, sp.nblk, kb.ldp, 2 * j + 3, kb.h1, stop, s));
        HZ_TRY(launch_arnoldi_lag(kb, j, false, s));
        HZ_TRY(launch_update_lag(c128, L.V, n, j, kb.coef, n, sp, kb.part, kb.ldp, stop, s));
    }
    // complete the last column: [Q, v~]^H v~ with v~ in slot steps
    HZ_TRY(launch_dots(c128, L.V, n, steps + 1, vcol(steps), n, sp, kb.part, kb.ldp, false, stop, s));
    HZ_TRY(launch_finalize(kb.part, sp.nblk, kb.ldp, steps + 1, kb.h1, stop, s));
    HZ_TRY(launch_arnoldi_lag(kb, steps, true, s));
    HZ_TRY(launch_backsolve(kb, s));
    HZ_TRY(launch_xupdate(c128, zcol(0), n, x, n, kb, s));
    HZ_TRY(launch_resid64(p, b, x, L.r64, L.rpart, nullptr, s));
    HZ_TRY(launch_cycle_start(kb, L.rpart, nres, s));
    HZ_TRY(launch_cast_scale(c128, L.r64, vcol(0), n, kb.st, s));
    return HZ_OK;
}

static int solve_on(const hz_problem* p, const no_net* net, const hz_opts* o, const double2* b, double2* x,
                    FgmresLayout& L, hz_info* info, hipStream_t s, GraphUse& gu) {
    const int64_t n = p->n;
    const int m = o->m;
    const bool c128 = o->krylov == HZ_C128;
    KrylovBufs& kb = L.kb;
    Split sp = krylov_split(n);
    const int nres = stencil_blocks(p);

    PhaseTimer pt;
    HZ_TRY(pt.create());
    HZ_HIP(hipEventRecord(pt.ev[0], s));
    // pick the fastest launch variant of every network layer at this size (first call only)
    if (net) HZ_TRY(net_autotune(net, p, o->net_prec, L.net_ws, L.net_ws_bytes, s));
    // ||b||, then the first true residual and v_1
    HZ_TRY(launch_norm_partials(true, b, n, sp, kb.part, kb.ldp, 0, nullptr, s));
    HZ_TRY(launch_init_state(kb, sp.nblk, o->tol, m, s));
    HZ_TRY(launch_resid64(p, b, x, L.r64, L.rpart, nullptr, s));
    HZ_TRY(launch_cycle_start(kb, L.rpart, nres, s));
    HZ_TRY(launch_cast_scale(c128, L.r64, L.V, n, kb.st, s));

    HZ_HIP(hipEventRecord(pt.ev[1], s));
    SolveState hs{};
    HZ_HIP(hipMemcpyAsync(&hs, kb.st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    HZ_TRY(pt.add(HZ_PHASE_SETUP));
    if (hs.bnorm == 0.0 && !(hs.flags & FL_NONFINITE)) HZ_HIP(hipMemsetAsync(x, 0, sizeof(double2) * n, s));
    int graph_steps = -1;
    while (!(hs.flags & (FL_CONVERGED | FL_NONFINITE | FL_BREAKDOWN)) && hs.its < o->maxit) {
        const int steps = std::min(m, o->maxit - hs.its);
        // one cycle = one graph launch; the graph of a cycle length is captured once (and kept
        // for later solves with the same arguments)
        if (steps != graph_steps) {
            gu.release();
            GraphKey k;
            std::memset(&k, 0, sizeof k);
            k.puid = p->uid;
            k.nuid = net ? net->uid : 0;
            k.tgen = net ? net->tune_gen.load() : 0;
            k.steps = steps;
            k.fuse = net ? net->fuse_up : -1;
            k.m = o->m;
            k.maxit = o->maxit;
            k.krylov = (int32_t)o->krylov;
            k.net_prec = net ? (int32_t)o->net_prec : -1;
            k.ortho = o->ortho;
            k.tol = o->tol;
            k.b = b;
            k.x = x;
            k.ws = L.kb.st;   // the workspace base (the layout's first buffer)
            k.ws_len = L.total;
            if (!graph_acquire(k, gu)) {
                const auto t0 = std::chrono::steady_clock::now();
                HZ_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                const int crc = o->ortho == 1 ? cycle_launches_lag(p, net, o, L, kb, b, x, steps, s)
                                              : cycle_launches(p, net, o, L, kb, b, x, steps, s);
                const hipError_t e = hipStreamEndCapture(s, &gu.g);
                if (crc != HZ_OK) return crc;
                HZ_HIP(e);
                HZ_HIP(hipGraphInstantiate(&gu.e, gu.g, nullptr, nullptr, 0));
                graph_keep(k, gu);
                pt.ms[HZ_PHASE_BUILD] +=
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            }
            graph_steps = steps;
        }
        HZ_HIP(hipEventRecord(pt.ev[0], s));
        HZ_HIP(hipGraphLaunch(gu.e, s));
        HZ_HIP(hipEventRecord(pt.ev[1], s));
        HZ_HIP(hipMemcpyAsync(&hs, kb.st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
        HZ_HIP(hipStreamSynchronize(s));
        HZ_TRY(pt.add(HZ_PHASE_CYCLES));
    }
    for (int i = 0; i < HZ_PHASE_TOTAL; ++i) info->phase_ms[i] = pt.ms[i];
    if (o->hist_host && o->hist_len > 0) {
        const int cnt = std::min(std::min(hs.its, o->hist_len), kb.hist_cap);
        if (cnt > 0) {
            HZ_HIP(hipMemcpyAsync(o->hist_host, kb.hist, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
            HZ_HIP(hipStreamSynchronize(s));
        }
    }
    info->its = hs.its;
    info->cycles = hs.cycles;
    info->est_relres = hs.est;
    info->true_relres = hs.true_rel;
    if (hs.flags & FL_NONFINITE) {
        info->status = HZ_ERR_NONFINITE;
        set_error("fgmres_solve: non-finite value in the input or an iterate");
    } else if (hs.flags & FL_CONVERGED) {
        info->status = HZ_OK;
    } else if (hs.flags & FL_BREAKDOWN) {
        info->status = HZ_ERR_BREAKDOWN;
        set_error("fgmres_solve: breakdown (preconditioned vectors lost rank)");
    } else {
        info->status = HZ_NOT_CONVERGED;
    }
    return info->status;
}

}  // namespace hz

using namespace hz;

extern "C" size_t fgmres_workspace_size(const hz_problem* p, const no_net* net, const hz_opts* o) {
    clear_error();
    if (!p || check_opts(o, net, p) != HZ_OK) return 0;
    return fgmres_layout(p, net, o, nullptr, 0).total;
}

// The solve runs on a stream owned by the call (graph capture needs a non-default stream),
// ordered after the caller's pending work and before anything the caller enqueues later.
extern "C" int fgmres_solve(const hz_problem* p, const no_net* net, const hz_opts* o, const void* b_dev,
                            void* x_dev, void* ws, size_t ws_bytes, hz_info* info, void* stream) {
    clear_error();
    const auto t_call = std::chrono::steady_clock::now();
    HZ_CHECK_ARG(p && b_dev && x_dev && ws && info, "fgmres_solve: NULL argument");
    std::memset(info->phase_ms, 0, sizeof info->phase_ms);
    HZ_TRY(check_opts(o, net, p));
    FgmresLayout L = fgmres_layout(p, net, o, ws, ws_bytes);
    if (L.total > ws_bytes) {
        set_error("fgmres_solve: workspace too small");
        return HZ_ERR_WORKSPACE;
    }
    hipStream_t user = (hipStream_t)stream, s;
    hipEvent_t ev;
    HZ_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(s);
        set_error("fgmres_solve: hipEventCreate failed");
        return HZ_ERR_HIP;
    }
    int rc = HZ_ERR_HIP;
    {
        GraphUse gu;   // released (kept graph) or destroyed (owned) after the stream drains
        if (hipEventRecord(ev, user) == hipSuccess && hipStreamWaitEvent(s, ev, 0) == hipSuccess)
            rc = solve_on(p, net, o, (const double2*)b_dev, (double2*)x_dev, L, info, s, gu);
        else
            set_error("fgmres_solve: stream ordering failed");
        if (hipEventRecord(ev, s) != hipSuccess || hipStreamWaitEvent(user, ev, 0) != hipSuccess) rc = HZ_ERR_HIP;
        (void)hipStreamSynchronize(s);
    }
    (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(s);
    info->phase_ms[HZ_PHASE_TOTAL] =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_call).count();
    return rc;
}

