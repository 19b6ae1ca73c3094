// Ragged batch of FGMRES solves (Algorithm 1 for many independent systems at once).
//
// The systems advance in lockstep: at every Arnoldi step one launch per step kernel covers
// every active system, each block reading its (system, tile) from a job table and the
// system's buffers from a descriptor table. Every system keeps its own device state (stop
// flag, Hessenberg, Givens, residual history); a system whose Givens estimate reaches tol
// idles (its blocks return at once) until the cycle ends. At the end of every cycle the
// host reads all states once, drops the systems that finished, and rebuilds the tables if
// the active set changed. A cycle's launches are captured once into a HIP graph and replayed
// while the active set and the cycle length stay the same; the work runs on a stream owned
// by the call, ordered after and before the caller's stream with events.
#include <algorithm>
#include <cstring>
#include <vector>

#include "krylov.h"
#include "krylov_impl.h"
#include "net_impl.h"
#include "problem.h"
#include "stencil_impl.h"

namespace hz {

template <typename C> struct scalar_of;
template <> struct scalar_of<float2> { using type = float; };
template <> struct scalar_of<double2> { using type = double; };

// Per-system descriptor (device table).
struct KDesc {
    void* V;              // (m+1) x n Krylov vectors
    void* Z;              // m x n preconditioned vectors (== V without a network)
    double2* x;
    const double2* b;
    double2* r64;
    int64_t n, per;
    int nblk, ldp;
    double2* part;        // [nblk][ldp]
    double* rpart;        // stencil-tile partials
    int nres;
    SolveState* st;
    double2 *R, *sn, *g, *y, *h1, *h2;
    double *cs, *hist;
    int nxt, nyt, Hp, Wp;
    const float* k2f;
    const double* k2d;
    const float2 *fE_f, *fW_f, *fN_f, *fS_f, *dx_f, *dy_f;
    const double2 *fE_d, *fW_d, *fN_d, *fS_d, *dx_d, *dy_d;
    const double *cnd, *sigx, *sigy;
    void* X;              // packed network input
    const void* D0;       // decoder level-0 output
    double2* npart;       // ||v||^2 partials (network input scale)
    double* sc;           // (s, 1/s)
};

// ------------------------------------------------------------------ kernels

template <typename T>
__global__ __launch_bounds__(256) void kb_stencil(const TileJob* __restrict__ jobs, const KDesc* __restrict__ kd,
                                                  int src, int dst, int use_z) {
    using C = cplx_t<T>;
    const TileJob jb = jobs[blockIdx.x];
    const KDesc& d = kd[jb.sys];
    if (d.st->stop) return;
    const C* u = (const C*)(use_z ? d.Z : d.V) + (int64_t)src * d.n;
    C* y = (C*)d.V + (int64_t)dst * d.n;
    if constexpr (sizeof(T) == 4)
        stencil_tile<float, ST_PLAIN>(u, y, nullptr, d.k2f, d.fE_f, d.fW_f, d.fN_f, d.fS_f, d.dx_f, d.dy_f, 0, d.nxt,
                                      d.nyt, nullptr, jb.tx0, jb.ty0);
    else
        stencil_tile<double, ST_PLAIN>(u, y, nullptr, d.k2d, d.fE_d, d.fW_d, d.fN_d, d.fS_d, d.dx_d, d.dy_d, 0, d.nxt,
                                       d.nyt, nullptr, jb.tx0, jb.ty0);
}

// FP64 true residual r = b - A x with per-tile ||r||^2 partials (job.c0 = tile index in the system).
__global__ __launch_bounds__(256) void kb_resid(const TileJob* __restrict__ jobs, const KDesc* __restrict__ kd) {
    const TileJob jb = jobs[blockIdx.x];
    const KDesc& d = kd[jb.sys];
    stencil_tile<double, ST_RESID>(d.x, d.r64, d.b, d.k2d, d.fE_d, d.fW_d, d.fN_d, d.fS_d, d.dx_d, d.dy_d, 0, d.nxt,
                                   d.nyt, d.rpart + jb.c0, jb.tx0, jb.ty0);
}

// Krylov range jobs: job.c0 = block index b of the system, points [b * per, (b + 1) * per).
#define KB_RANGE                                              \
    const TileJob jb = jobs[blockIdx.x];                      \
    const KDesc& d = kd[jb.sys];                              \
    const int64_t p0 = (int64_t)jb.c0 * d.per;                \
    const int64_t p1 = min(d.n, p0 + d.per);

template <typename C>
__global__ __launch_bounds__(KT) void kb_norm(const TileJob* __restrict__ jobs, const KDesc* __restrict__ kd,
                                              int what, int col) {
    KB_RANGE
    if (what == 0) {   // ||b||^2 into part slot 0 (b is FP64)
        norm_body((const double2*)d.b, p0, p1, d.part + (int64_t)jb.c0 * d.ldp);
    } else {           // ||v_col||^2 into the network-scale partials
        if (d.st->stop) return;
        norm_body((const C*)d.V + (int64_t)col * d.n, p0, p1, d.npart + jb.c0);
    }
}

template <typename C>
__global__ __launch_bounds__(KT) void kb_dots(const TileJob* __restrict__ jobs, const KDesc* __restrict__ kd, int nv) {
    KB_RANGE
    if (d.st->stop) return;
    const C* V = (const C*)d.V;
    const C* w = V + (int64_t)nv * d.n;
    double2* mine = d.part + (int64_t)jb.c0 * d.ldp;
    dots_body(V, d.n, nv, w, p0, p1, mine);
    norm_body(w, p0, p1, mine + nv);
}

template <typename C, int MODE>
__global__ __launch_bounds__(KT) void kb_update(const TileJob* __restrict__ jobs, const KDesc* __restrict__ kd,
                                                int nv) {
    KB_RANGE
    if (d.st->stop) return;
    const C* V = (const C*)d.V;
    C* w = (C*)d.V + (int64_t)nv * d.n;
    const double2* h = MODE == 1 ? d.h1 : d.h2;
    update_body(V, d.n, nv, h, w, p0, p1);
    __syncthreads();   // the sweeps below may read points written by other threads of the block
    double2* mine = d.part + (int64_t)jb.c0 * d.ldp;
    if (MODE == 1) dots_body(V, d.n, nv, (const C*)w, p0, p1, mine);
    if (MODE == 2) norm_body((const C*)w, p0, p1, mine);
}

// per-system reductions: one block of 256 threads per active system
// block (system, value)
__global__ __launch_bounds__(KT) void kb_finalize(const KDesc* __restrict__ kd, const int* __restrict__ act,
                                                  int which) {
    const KDesc& d = kd[act[blockIdx.x]];
    if (d.st->stop) return;
    double2* out = which == 1 ? d.h1 : d.h2;
    const double2 v = block_sum_slot(d.part, d.nblk, d.ldp, blockIdx.y);
    if (threadIdx.x == 0) out[blockIdx.y] = v;
}

__global__ void kb_arnoldi_finish(const KDesc* __restrict__ kd, const int* __restrict__ act, int j) {
    const KDesc& d = kd[act[blockIdx.x]];
    arnoldi_finish_body(d.st, d.R, d.cs, d.sn, d.g, d.h1, d.h2, d.part, d.nblk, d.ldp, j, d.hist);
}

template <typename C>
__global__ __launch_bounds__(KT) void kb_scale(const TileJob* __restrict__ jobs, const KDesc* __restrict__ kd,
                                               int col) {
    KB_RANGE
    if (d.st->stop) return;
    C* v = (C*)d.V + (int64_t)col * d.n;
    const double s = d.st->inv_h;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += KT) {
        const C a = v[p];
        v[p] = from_d2<C>(double2{a.x * s, a.y * s});
    }
}

__global__ void kb_init_state(const KDesc* __restrict__ kd, const int* __restrict__ act, double tol, int m,
                              int maxit) {
    const KDesc& d = kd[act[blockIdx.x]];
    init_state_body(d.st, d.part, d.nblk, d.ldp, tol, m, maxit);
}

__global__ void kb_cycle_start(const KDesc* __restrict__ kd, const int* __restrict__ act, int m) {
    const KDesc& d = kd[act[blockIdx.x]];
    cycle_start_body(d.st, d.rpart, d.nres, d.g, m);
}

__global__ void kb_backsolve(const KDesc* __restrict__ kd, const int* __restrict__ act) {
    const KDesc& d = kd[act[blockIdx.x]];
    backsolve_body(d.st, d.R, d.g, d.y);
}

template <typename C>
__global__ __launch_bounds__(KT) void kb_xupdate(const TileJob* __restrict__ jobs, const KDesc* __restrict__ kd) {
    KB_RANGE
    const int k = d.st->k;
    if (k == 0) return;
    const C* Z = (const C*)d.Z;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += KT) {
        double2 a = d.x[p];
        for (int i = 0; i < k; ++i) {
            const C z = Z[(int64_t)i * d.n + p];
            const double2 yi = d.y[i];
            a.x += (double)z.x * yi.x - (double)z.y * yi.y;
            a.y += (double)z.x * yi.y + (double)z.y * yi.x;
        }
        d.x[p] = a;
    }
}

template <typename C>
__global__ __launch_bounds__(KT) void kb_cast_scale(const TileJob* __restrict__ jobs, const KDesc* __restrict__ kd) {
    KB_RANGE
    if (d.st->stop) return;
    const double s = d.st->inv_beta;
    C* v = (C*)d.V;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += KT) {
        const double2 a = d.r64[p];
        v[p] = from_d2<C>(double2{a.x * s, a.y * s});
    }
}

// network input scale s = ||v|| / sqrt(n)
__global__ void kb_scale_factor(const KDesc* __restrict__ kd, const int* __restrict__ act) {
    const KDesc& d = kd[act[blockIdx.x]];
    if (d.st->stop) return;
    double a = 0;
    for (int q = threadIdx.x; q < d.nblk; q += 64) a += d.npart[q].x;
    a = wave_sum(a);
    if (threadIdx.x == 0) {
        const double s = sqrt(a / (double)d.n);
        d.sc[0] = s;
        d.sc[1] = s > 0 ? 1.0 / s : 0.0;
    }
}

// pack jobs: job.c0 = block of 256 padded pixels
template <class P, typename C>
__global__ void kb_pack(const TileJob* __restrict__ jobs, const KDesc* __restrict__ kd, int col, int in_ch) {
    using T = typename P::T;
    const TileJob jb = jobs[blockIdx.x];
    const KDesc& d = kd[jb.sys];
    if (d.st->stop) return;
    const int64_t idx = (int64_t)jb.c0 * 256 + threadIdx.x;
    if (idx >= (int64_t)d.Hp * d.Wp) return;
    const int yy = (int)(idx / d.Wp), xx = (int)(idx % d.Wp);
    T out[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) out[c] = P::cvt(0);
    if (yy < d.nyt && xx < d.nxt) {
        const int64_t g = (int64_t)yy * d.nxt + xx;
        const double is = d.sc[1];
        const C a = ((const C*)d.V)[(int64_t)col * d.n + g];
        out[0] = P::cvt((typename P::Acc)((double)a.x * is));
        out[1] = P::cvt((typename P::Acc)((double)a.y * is));
        if (in_ch == 5) {
            out[2] = P::cvt((typename P::Acc)d.cnd[g]);
            out[3] = P::cvt((typename P::Acc)d.sigx[xx]);
            out[4] = P::cvt((typename P::Acc)d.sigy[yy]);
        }
    }
    T* dst = (T*)d.X + idx * 8;
#pragma unroll
    for (int c = 0; c < 8; ++c) dst[c] = out[c];
}

// head: z_col = s (out_0 + i out_1) over the system's grid points (range jobs)
template <class P, typename C>
__global__ __launch_bounds__(KT) void kb_head(const TileJob* __restrict__ jobs, const KDesc* __restrict__ kd, int col,
                                              const typename P::T* __restrict__ wh,
                                              const typename P::Acc* __restrict__ bh, int cin_p) {
    using Acc = typename P::Acc;
    KB_RANGE
    if (d.st->stop) return;
    const typename P::T* D = (const typename P::T*)d.D0;
    C* z = (C*)d.Z + (int64_t)col * d.n;
    const double s = d.sc[0];
    for (int64_t p = p0 + threadIdx.x; p < p1; p += KT) {
        const int yy = (int)(p / d.nxt), xx = (int)(p % d.nxt);
        const typename P::T* q = D + ((int64_t)yy * d.Wp + xx) * cin_p;
        Acc o0 = bh[0], o1 = bh[1];
        for (int c = 0; c < cin_p; ++c) {
            const Acc dv = P::val(q[c]);
            o0 += dv * P::val(wh[c]);
            o1 += dv * P::val(wh[cin_p + c]);
        }
        z[p] = from_d2<C>(double2{s * (double)o0, s * (double)o1});
    }
}

// ------------------------------------------------------------------ host side

struct SysLayout {
    int64_t n;
    Split sp;
    int nres;
    int Hp, Wp;
    KDesc d;
    FwdBufs fb;
};

struct BatchTables {
    KDesc* kd;          // nsys
    int* act;           // nsys
    TileJob *vjobs, *stjobs, *pjobs;
    std::vector<LayerIO*> io;      // per layer, nsys
    std::vector<TileJob*> cjobs;   // per layer
    size_t vcap, stcap, pcap;
    std::vector<size_t> ccap;
};

template <class P>
static int64_t layer_jobs_cap(const no_net* net, const std::vector<SysLayout>& S, int li, int level, bool convT) {
    const Layer& ly = net->layers[li];
    int64_t tiles = 0;
    for (const SysLayout& sl : S) {
        const int H = sl.Hp >> level, W = sl.Wp >> level;
        tiles += convT ? (int64_t)H * ((W + 63) / 64) : (int64_t)((W + 15) / 16) * ((H + 7) / 8);
    }
    return tiles * (ly.cout_p / 16);
}

// levels of the layers in flat order: enc l a, enc l b, ..., up l (input level l+1), dec l a, dec l b, head
static void layer_levels(const no_net* net, std::vector<int>& lvl, std::vector<int>& role) {
    const int lv = net->a.levels;
    for (int l = 0; l < lv; ++l) {
        lvl.push_back(l); role.push_back(0);   // enc a
        lvl.push_back(l); role.push_back(1);   // enc b
    }
    for (int l = lv - 2; l >= 0; --l) {
        lvl.push_back(l + 1); role.push_back(2);   // up (input level l+1)
        lvl.push_back(l); role.push_back(3);       // dec a
        lvl.push_back(l); role.push_back(4);       // dec b
    }
    lvl.push_back(0); role.push_back(5);           // head
}

// whether the 1x1 head runs in the epilogue of the last 3x3 layer (a decoder's second layer whose
// 16, 32 or 64 output channels one block covers)
static bool head_fused(const no_net* net) {
    const int nl = (int)net->layers.size();
    if (net->a.levels < 2 || nl < 2) return false;
    const int cp = net->layers[nl - 2].cout_p;
    return (cp == 16 || cp == 32 || cp == 64) && net->layers[nl - 1].cin_p == cp;
}

template <class P>
struct BatchPlan {
    std::vector<SysLayout> S;
    BatchTables t;
    size_t total;
};

template <class P>
static BatchPlan<P> batch_layout(int nsys, const hz_problem* const* probs, const no_net* net, const hz_opts* o,
                                 void* base, size_t cap) {
    BatchPlan<P> B;
    const int m = o->m;
    const bool c128 = o->krylov == HZ_C128;
    const size_t es = c128 ? sizeof(double2) : sizeof(float2);
    Carver c(base, cap);
    B.S.resize(nsys);
    for (int s = 0; s < nsys; ++s) {
        const hz_problem* p = probs[s];
        SysLayout& L = B.S[s];
        KDesc& d = L.d;
        memset(&d, 0, sizeof(d));
        L.n = p->n;
        L.sp = krylov_split(p->n);
        L.nres = stencil_blocks(p);
        d.n = p->n;
        d.per = L.sp.per_block;
        d.nblk = L.sp.nblk;
        d.ldp = m + 2;
        d.st = c.take<SolveState>(1);
        d.R = c.take<double2>((size_t)(m + 1) * m);
        d.cs = c.take<double>(m);
        d.sn = c.take<double2>(m);
        d.g = c.take<double2>(m + 1);
        d.y = c.take<double2>(m);
        d.h1 = c.take<double2>(m + 2);
        d.h2 = c.take<double2>(m + 2);
        d.part = c.take<double2>((size_t)d.nblk * d.ldp);
        d.hist = c.take<double>(std::max(o->maxit, 1));
        d.rpart = c.take<double>(L.nres);
        d.nres = L.nres;
        d.r64 = c.take<double2>(p->n);
        d.V = c.take<char>(es * p->n * (m + 1));
        d.Z = net ? (void*)c.take<char>(es * p->n * m) : d.V;
        d.nxt = p->nxt;
        d.nyt = p->nyt;
        d.k2f = p->k2f;
        d.k2d = p->k2d;
        d.fE_f = p->fE_f; d.fW_f = p->fW_f; d.fN_f = p->fN_f; d.fS_f = p->fS_f; d.dx_f = p->dx_f; d.dy_f = p->dy_f;
        d.fE_d = p->fE_d; d.fW_d = p->fW_d; d.fN_d = p->fN_d; d.fS_d = p->fS_d; d.dx_d = p->dx_d; d.dy_d = p->dy_d;
        d.cnd = p->cnd;
        d.sigx = p->sigx;
        d.sigy = p->sigy;
        if (net) {
            net_padded_dims(net, p, &L.Hp, &L.Wp);
            d.Hp = L.Hp;
            d.Wp = L.Wp;
            Carver sub(c.base ? c.base + align_up(c.off, 256) : nullptr, c.base ? cap - align_up(c.off, 256) : 0);
            L.fb = fwd_layout<P>(net, L.Hp, L.Wp, 1, sub.base, sub.cap);
            c.off = align_up(c.off, 256) + L.fb.total;
            d.X = L.fb.X;
            d.D0 = net->a.levels > 1 ? L.fb.D[0] : L.fb.E[0];
            d.npart = L.fb.part;
            d.sc = L.fb.sc;
        }
    }
    // tables (sized for the whole batch; the active set only shrinks)
    BatchTables& t = B.t;
    t.kd = c.take<KDesc>(nsys);
    t.act = c.take<int>(nsys);
    t.vcap = t.stcap = t.pcap = 0;
    for (const SysLayout& L : B.S) {
        t.vcap += L.sp.nblk;
        t.stcap += L.nres;
        t.pcap += ((int64_t)L.Hp * L.Wp + 255) / 256;
    }
    t.vjobs = c.take<TileJob>(t.vcap);
    t.stjobs = c.take<TileJob>(t.stcap);
    t.pjobs = c.take<TileJob>(std::max<size_t>(t.pcap, 1));
    if (net) {
        std::vector<int> lvl, role;
        layer_levels(net, lvl, role);
        const int nl = (int)net->layers.size();
        t.io.resize(nl);
        t.cjobs.resize(nl);
        t.ccap.resize(nl);
        for (int li = 0; li < nl - 1; ++li) {
            t.io[li] = c.take<LayerIO>(nsys);
            t.ccap[li] = (size_t)layer_jobs_cap<P>(net, B.S, li, lvl[li], role[li] == 2);
            t.cjobs[li] = c.take<TileJob>(t.ccap[li]);
        }
    }
    B.total = c.off + 256;
    return B;
}

// Host copies of the tables for the given active set; returns the job counts.
template <class P>
struct HostTables {
    std::vector<KDesc> kd;
    std::vector<int> act;
    std::vector<TileJob> vjobs, stjobs, pjobs;
    std::vector<std::vector<LayerIO>> io;
    std::vector<std::vector<TileJob>> cjobs;
    std::vector<int> tn, rpw;
    std::vector<char> ws;   // layer in the weight-stationary form
};

// Launch form of a 3x3 layer over a ragged batch with `tiles` 16 x 16 pixel tiles in all: in BF16
// the weight-stationary form with 32-channel blocks where it applies (layers of at most two input
// chunks), with enough tiles per block to pipeline them and enough blocks to fill the GPU, else
// 16 x 16 tiles with 32-channel blocks; FP32 / FP64 keep 8 x 16 tiles (conv3_batch_tn).
template <class P>
static void batch_conv3_form(const Layer& ly, int c1, int64_t tiles16, int64_t tiles8, bool head, int& tn, int& rpw,
                             int& tpb) {
    tpb = 0;
    if (std::is_same<P, PolBF16>::value && ly.cout_p % 32 == 0) {
        const int64_t ncb = ly.cout_p / WSJ_TN;
        if (ws_jobs_ok<P>(ly.cin_p - c1, c1, ly.cout_p) && (!head || ly.cout_p == WSJ_TN)) {
            int t = 32;
            while (t > 4 && (tiles16 + t - 1) / t * ncb < 1024) t /= 2;
            if ((tiles16 + t - 1) / t * ncb >= 256) {
                tn = WSJ_TN;
                rpw = WSJ_RPW;
                tpb = t;
                return;
            }
        }
        if (!head && tiles16 * (ly.cout_p / 32) >= 512) {
            tn = 32;
            rpw = 4;
            return;
        }
    }
    tn = head ? ly.cout_p : conv3_batch_tn(ly.cout_p, tiles8);
    rpw = 2;
}

template <class P>
static void build_tables(const BatchPlan<P>& B, const no_net* net, const std::vector<int>& active, HostTables<P>& h) {
    const int nsys = (int)B.S.size();
    h.kd.resize(nsys);
    for (int s = 0; s < nsys; ++s) h.kd[s] = B.S[s].d;
    h.act = active;
    h.vjobs.clear();
    h.stjobs.clear();
    h.pjobs.clear();
    for (int s : active) {
        const SysLayout& L = B.S[s];
        for (int b = 0; b < L.sp.nblk; ++b) h.vjobs.push_back(TileJob{s, b, 0, 0});
        const int tx = (L.d.nxt + 63) / 64, ty = (L.d.nyt + 15) / 16;
        for (int jy = 0; jy < ty; ++jy)
            for (int ix = 0; ix < tx; ++ix) h.stjobs.push_back(TileJob{s, jy * tx + ix, jy * 16, ix * 64});
        if (net) {
            const int64_t np = ((int64_t)L.Hp * L.Wp + 255) / 256;
            for (int64_t b = 0; b < np; ++b) h.pjobs.push_back(TileJob{s, (int)b, 0, 0});
        }
    }
    if (!net) return;
    std::vector<int> lvl, role;
    layer_levels(net, lvl, role);
    const int nl = (int)net->layers.size();
    h.io.assign(nl, std::vector<LayerIO>(nsys));
    h.cjobs.assign(nl, {});
    h.tn.assign(nl, 16);
    h.rpw.assign(nl, 2);
    h.ws.assign(nl, 0);
    for (int li = 0; li < nl - 1; ++li) {
        const Layer& ly = net->layers[li];
        const int l = lvl[li];
        const bool convT = role[li] == 2;
        int64_t tiles = 0, tiles16 = 0;
        for (int s : active) {
            const int H = B.S[s].Hp >> l, W = B.S[s].Wp >> l;
            tiles += convT ? (int64_t)H * ((W + 63) / 64) : (int64_t)((W + 15) / 16) * ((H + 7) / 8);
            tiles16 += (int64_t)((W + 15) / 16) * ((H + 15) / 16);
        }
        const bool fhead = li == nl - 2 && head_fused(net);
        int tn = 16, rpw = 2, tpb = 0;
        if (convT) {
            tn = convT2_batch_tn(ly.cout_p);
            // weight-stationary form where the input channels fit one stage: 4-32 row segments per
            // job, while that still gives at least 256 jobs
            if (convT2_ws_ok<P>(ly.cin_p, ly.cout_p, tn)) {
                const int64_t ncb = ly.cout_p / tn;
                int t = 32;
                while (t > 4 && (tiles + t - 1) / t * ncb < 1024) t /= 2;
                if ((tiles + t - 1) / t * ncb >= 256) tpb = t;
            }
        } else {
            batch_conv3_form<P>(ly, ly.cat_cp ? ly.cin_p - ly.cat_cp : 0, tiles16, tiles, fhead, tn, rpw, tpb);
        }
        h.tn[li] = tn;
        h.rpw[li] = rpw;
        h.ws[li] = tpb > 0;
        for (int s = 0; s < nsys; ++s) {
            const FwdBufs& fb = B.S[s].fb;
            LayerIO& io = h.io[li][s];
            memset(&io, 0, sizeof(io));
            io.H = B.S[s].Hp >> l;
            io.W = B.S[s].Wp >> l;
            io.stop = &B.S[s].d.st->stop;
            const int lv = net->a.levels;
            switch (role[li]) {
                case 0: io.x0 = l == 0 ? fb.X : fb.P[l]; io.y = fb.T1[l]; break;
                case 1: io.x0 = fb.T1[l]; io.y = fb.E[l]; io.ypool = l + 1 < lv ? fb.P[l + 1] : nullptr; break;
                case 2: io.x0 = l == lv - 1 ? fb.E[l] : fb.D[l]; io.y = fb.U[l - 1]; break;
                case 3: io.x0 = fb.E[l]; io.x1 = fb.U[l]; io.y = fb.T1d[l]; break;
                case 4: io.x0 = fb.T1d[l]; io.y = fb.D[l]; break;
            }
            if (fhead) {
                const KDesc& d = B.S[s].d;
                io.y = nullptr;
                io.z = d.Z;
                io.zld = d.n;
                io.nxt = d.nxt;
                io.nyt = d.nyt;
                io.sc = d.sc;
            }
        }
        // channel blocks of one tile are neighbours in the job order (the kernel maps each XCD
        // to a contiguous range of jobs, so they share the tile's input in one L2)
        for (int s : active) {
            const int H = B.S[s].Hp >> l, W = B.S[s].Wp >> l;
            if (convT && tpb > 0) {   // (sys, first channel, first segment, end segment)
                const int nt = H * ((W + 63) / 64);
                for (int t0 = 0; t0 < nt; t0 += tpb)
                    for (int co = 0; co < ly.cout_p; co += tn)
                        h.cjobs[li].push_back(TileJob{s, co, t0, std::min(nt, t0 + tpb)});
            } else if (convT) {
                for (int iy = 0; iy < H; ++iy)
                    for (int ix = 0; ix < W; ix += 64)
                        for (int co = 0; co < ly.cout_p; co += tn) h.cjobs[li].push_back(TileJob{s, co, iy, ix});
            } else if (tpb > 0) {   // (sys, first channel, first tile, end tile), tiles of 4 rpw x 16
                const int nt = ((W + 15) / 16) * ((H + 4 * rpw - 1) / (4 * rpw));
                for (int t0 = 0; t0 < nt; t0 += tpb)
                    for (int co = 0; co < ly.cout_p; co += tn)
                        h.cjobs[li].push_back(TileJob{s, co, t0, std::min(nt, t0 + tpb)});
            } else {
                for (int ty = 0; ty < H; ty += 4 * rpw)
                    for (int tx = 0; tx < W; tx += 16)
                        for (int co = 0; co < ly.cout_p; co += tn) h.cjobs[li].push_back(TileJob{s, co, ty, tx});
            }
        }
    }
}

template <class P>
static int upload_tables(const BatchPlan<P>& B, const HostTables<P>& h, hipStream_t s) {
    const BatchTables& t = B.t;
    HZ_HIP(hipMemcpyAsync(t.kd, h.kd.data(), sizeof(KDesc) * h.kd.size(), hipMemcpyHostToDevice, s));
    HZ_HIP(hipMemcpyAsync(t.act, h.act.data(), sizeof(int) * h.act.size(), hipMemcpyHostToDevice, s));
    HZ_HIP(hipMemcpyAsync(t.vjobs, h.vjobs.data(), sizeof(TileJob) * h.vjobs.size(), hipMemcpyHostToDevice, s));
    HZ_HIP(hipMemcpyAsync(t.stjobs, h.stjobs.data(), sizeof(TileJob) * h.stjobs.size(), hipMemcpyHostToDevice, s));
    if (!h.pjobs.empty())
        HZ_HIP(hipMemcpyAsync(t.pjobs, h.pjobs.data(), sizeof(TileJob) * h.pjobs.size(), hipMemcpyHostToDevice, s));
    for (size_t li = 0; li < h.cjobs.size(); ++li) {
        if (h.cjobs[li].empty()) continue;
        HZ_HIP(hipMemcpyAsync(t.io[li], h.io[li].data(), sizeof(LayerIO) * h.io[li].size(), hipMemcpyHostToDevice, s));
        HZ_HIP(hipMemcpyAsync(t.cjobs[li], h.cjobs[li].data(), sizeof(TileJob) * h.cjobs[li].size(),
                              hipMemcpyHostToDevice, s));
    }
    HZ_HIP(hipStreamSynchronize(s));   // the host vectors may change after this call
    return HZ_OK;
}

template <class P, typename C>
static int net_step(const BatchPlan<P>& B, const HostTables<P>& h, const no_net* net, int col, hipStream_t s) {
    const BatchTables& t = B.t;
    const int nact = (int)h.act.size();
    const int nv = (int)h.vjobs.size();
    hipLaunchKernelGGL((kb_norm<C>), dim3(nv), dim3(KT), 0, s, t.vjobs, t.kd, 1, col);
    hipLaunchKernelGGL(kb_scale_factor, dim3(nact), dim3(64), 0, s, t.kd, t.act);
    hipLaunchKernelGGL((kb_pack<P, C>), dim3((unsigned)h.pjobs.size()), dim3(256), 0, s, t.pjobs, t.kd, col,
                       net->a.in_ch);
    HZ_LAUNCH_CHECK();
    std::vector<int> lvl, role;
    layer_levels(net, lvl, role);
    const int nl = (int)net->layers.size();
    const bool fhead = head_fused(net);
    const Layer& lh = net->layers.back();
    for (int li = 0; li < nl - 1; ++li) {
        const Layer& ly = net->layers[li];
        const int nj = (int)h.cjobs[li].size();
        const bool hd = fhead && li == nl - 2;
        if (role[li] == 2 && h.ws[li]) {
            HZ_TRY(launch_convT2_ws_jobs<P>(t.cjobs[li], nj, t.io[li], packed_w<P>(net, ly), packed_b<P>(net, ly),
                                            ly.cin_p, ly.cout_p, h.tn[li], s));
        } else if (h.ws[li]) {
            const int c1 = ly.cat_cp ? ly.cin_p - ly.cat_cp : 0;
            const bool pool = role[li] == 1 && lvl[li] + 1 < net->a.levels;
            HZ_TRY(launch_conv3_ws_jobs<P>(t.cjobs[li], nj, t.io[li], packed_w<P>(net, ly), packed_b<P>(net, ly),
                                           ly.cin_p - c1, c1, ly.cout_p, pool, hd ? packed_w<P>(net, lh) : nullptr,
                                           hd ? packed_b<P>(net, lh) : nullptr, col, std::is_same<C, double2>::value,
                                           s));
        } else if (hd) {
            HZ_TRY(launch_conv3_jobs_head<P>(t.cjobs[li], nj, t.io[li], packed_w<P>(net, ly), packed_b<P>(net, ly),
                                             ly.cin_p, 0, ly.cout_p, packed_w<P>(net, lh), packed_b<P>(net, lh), col,
                                             std::is_same<C, double2>::value, s));
        } else if (role[li] == 2) {
            HZ_TRY(launch_convT2_jobs<P>(t.cjobs[li], nj, t.io[li], packed_w<P>(net, ly), packed_b<P>(net, ly), ly.cin_p,
                                         ly.cout_p, h.tn[li], s));
        } else {
            const int c1 = ly.cat_cp ? ly.cin_p - ly.cat_cp : 0;
            const bool pool = role[li] == 1 && lvl[li] + 1 < net->a.levels;
            HZ_TRY(launch_conv3_jobs<P>(t.cjobs[li], nj, t.io[li], packed_w<P>(net, ly), packed_b<P>(net, ly),
                                        ly.cin_p - c1, c1, ly.cout_p, h.tn[li], h.rpw[li], pool, s));
        }
    }
    if (!fhead) {
        hipLaunchKernelGGL((kb_head<P, C>), dim3(nv), dim3(KT), 0, s, t.vjobs, t.kd, col, packed_w<P>(net, lh),
                           packed_b<P>(net, lh), lh.cin_p);
        HZ_LAUNCH_CHECK();
    }
    return HZ_OK;
}

template <class P, typename C>
static int cycle_launches(const BatchPlan<P>& B, const HostTables<P>& h, const no_net* net, int m, int steps,
                          hipStream_t s) {
    const BatchTables& t = B.t;
    const int nact = (int)h.act.size();
    const int nv = (int)h.vjobs.size(), nst = (int)h.stjobs.size();
    using T = typename scalar_of<C>::type;
    for (int j = 0; j < steps; ++j) {
        if (net) HZ_TRY((net_step<P, C>(B, h, net, j, s)));
        hipLaunchKernelGGL((kb_stencil<T>), dim3(nst), dim3(256), 0, s, t.stjobs, t.kd, j, j + 1, net ? 1 : 0);
        hipLaunchKernelGGL((kb_dots<C>), dim3(nv), dim3(KT), 0, s, t.vjobs, t.kd, j + 1);
        hipLaunchKernelGGL(kb_finalize, dim3(nact, j + 2), dim3(KT), 0, s, t.kd, t.act, 1);
        hipLaunchKernelGGL((kb_update<C, 1>), dim3(nv), dim3(KT), 0, s, t.vjobs, t.kd, j + 1);
        hipLaunchKernelGGL(kb_finalize, dim3(nact, j + 1), dim3(KT), 0, s, t.kd, t.act, 2);
        hipLaunchKernelGGL((kb_update<C, 2>), dim3(nv), dim3(KT), 0, s, t.vjobs, t.kd, j + 1);
        hipLaunchKernelGGL(kb_arnoldi_finish, dim3(nact), dim3(64), 0, s, t.kd, t.act, j);
        hipLaunchKernelGGL((kb_scale<C>), dim3(nv), dim3(KT), 0, s, t.vjobs, t.kd, j + 1);
        HZ_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(kb_backsolve, dim3(nact), dim3(64), 0, s, t.kd, t.act);
    hipLaunchKernelGGL((kb_xupdate<C>), dim3(nv), dim3(KT), 0, s, t.vjobs, t.kd);
    hipLaunchKernelGGL(kb_resid, dim3(nst), dim3(256), 0, s, t.stjobs, t.kd);
    hipLaunchKernelGGL(kb_cycle_start, dim3(nact), dim3(64), 0, s, t.kd, t.act, m);
    hipLaunchKernelGGL((kb_cast_scale<C>), dim3(nv), dim3(KT), 0, s, t.vjobs, t.kd);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

template <class P, typename C>
static int solve_batched(int nsys, const hz_problem* const* probs, const no_net* net, const hz_opts* o,
                         const void* const* bv, void* const* xv, void* ws, size_t ws_bytes, hz_info* info,
                         hipStream_t user) {
    BatchPlan<P> B = batch_layout<P>(nsys, probs, net, o, ws, ws_bytes);
    if (B.total > ws_bytes) {
        set_error("fgmres_solve_batched: workspace too small");
        return HZ_ERR_WORKSPACE;
    }
    for (int s = 0; s < nsys; ++s) {
        B.S[s].d.b = (const double2*)bv[s];
        B.S[s].d.x = (double2*)xv[s];
    }
    // own stream, ordered after the caller's work
    hipStream_t s;
    hipEvent_t ev;
    HZ_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    HZ_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    int rc = HZ_OK;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    PhaseTimer pt;
    do {
        if ((rc = pt.create()) != HZ_OK) break;
        if (hipEventRecord(ev, user) != hipSuccess || hipStreamWaitEvent(s, ev, 0) != hipSuccess ||
            hipEventRecord(pt.ev[0], s) != hipSuccess) {
            rc = HZ_ERR_HIP;
            break;
        }
        std::vector<int> active(nsys);
        for (int i = 0; i < nsys; ++i) active[i] = i;
        HostTables<P> h;
        build_tables<P>(B, net, active, h);
        if ((rc = upload_tables<P>(B, h, s)) != HZ_OK) break;
        const BatchTables& t = B.t;
        const int nv = (int)h.vjobs.size(), nst = (int)h.stjobs.size();
        hipLaunchKernelGGL((kb_norm<C>), dim3(nv), dim3(KT), 0, s, t.vjobs, t.kd, 0, 0);
        hipLaunchKernelGGL(kb_init_state, dim3(nsys), dim3(64), 0, s, t.kd, t.act, o->tol, o->m, std::max(o->maxit, 1));
        hipLaunchKernelGGL(kb_resid, dim3(nst), dim3(256), 0, s, t.stjobs, t.kd);
        hipLaunchKernelGGL(kb_cycle_start, dim3(nsys), dim3(64), 0, s, t.kd, t.act, o->m);
        hipLaunchKernelGGL((kb_cast_scale<C>), dim3(nv), dim3(KT), 0, s, t.vjobs, t.kd);
        if (hipGetLastError() != hipSuccess) {
            rc = HZ_ERR_HIP;
            break;
        }
        std::vector<SolveState> hs(nsys);
        auto read_states = [&]() -> int {
            for (int i = 0; i < nsys; ++i)
                if (hipMemcpyAsync(&hs[i], B.S[i].d.st, sizeof(SolveState), hipMemcpyDeviceToHost, s) != hipSuccess)
                    return HZ_ERR_HIP;
            return hipStreamSynchronize(s) == hipSuccess ? HZ_OK : HZ_ERR_HIP;
        };
        if (hipEventRecord(pt.ev[1], s) != hipSuccess) {
            rc = HZ_ERR_HIP;
            break;
        }
        if ((rc = read_states()) != HZ_OK || (rc = pt.add(HZ_PHASE_SETUP)) != HZ_OK) break;
        for (int i = 0; i < nsys; ++i)
            if (hs[i].bnorm == 0.0 && !(hs[i].flags & FL_NONFINITE))
                if (hipMemsetAsync(B.S[i].d.x, 0, sizeof(double2) * B.S[i].n, s) != hipSuccess) rc = HZ_ERR_HIP;
        if (rc != HZ_OK) break;
        int graph_steps = -1;
        bool tables_dirty = false;
        while (true) {
            std::vector<int> next;
            int steps = 0;
            for (int i : active) {
                const SolveState& q = hs[i];
                if (q.flags & (FL_CONVERGED | FL_NONFINITE | FL_BREAKDOWN)) continue;
                if (q.its >= o->maxit) continue;
                next.push_back(i);
                steps = std::max(steps, std::min(o->m, o->maxit - q.its));
            }
            if (next.empty()) break;
            if (next != active) {
                active = next;
                build_tables<P>(B, net, active, h);
                if ((rc = upload_tables<P>(B, h, s)) != HZ_OK) break;
                tables_dirty = true;
            }
            if (tables_dirty || steps != graph_steps || !exec) {
                const auto t0 = std::chrono::steady_clock::now();
                if (exec) (void)hipGraphExecDestroy(exec);
                if (graph) (void)hipGraphDestroy(graph);
                exec = nullptr;
                graph = nullptr;
                if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                    rc = HZ_ERR_HIP;
                    break;
                }
                int crc = cycle_launches<P, C>(B, h, net, o->m, steps, s);
                hipError_t e = hipStreamEndCapture(s, &graph);
                if (crc != HZ_OK || e != hipSuccess ||
                    hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                    rc = crc != HZ_OK ? crc : HZ_ERR_HIP;
                    if (rc == HZ_ERR_HIP) set_error("fgmres_solve_batched: graph capture failed");
                    break;
                }
                graph_steps = steps;
                tables_dirty = false;
                pt.ms[HZ_PHASE_BUILD] +=
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            }
            if (hipEventRecord(pt.ev[0], s) != hipSuccess || hipGraphLaunch(exec, s) != hipSuccess ||
                hipEventRecord(pt.ev[1], s) != hipSuccess) {
                rc = HZ_ERR_HIP;
                break;
            }
            if ((rc = read_states()) != HZ_OK || (rc = pt.add(HZ_PHASE_CYCLES)) != HZ_OK) break;
        }
        if (rc != HZ_OK) break;
        for (int i = 0; i < nsys; ++i) {
            const SolveState& q = hs[i];
            hz_info& f = info[i];
            f.its = q.its;
            f.cycles = q.cycles;
            f.est_relres = q.est;
            f.true_relres = q.true_rel;
            for (int k = 0; k < HZ_PHASE_TOTAL; ++k) f.phase_ms[k] = pt.ms[k];
            if (q.flags & FL_NONFINITE) f.status = HZ_ERR_NONFINITE;
            else if (q.flags & FL_CONVERGED) f.status = HZ_OK;
            else if (q.flags & FL_BREAKDOWN) f.status = HZ_ERR_BREAKDOWN;
            else f.status = HZ_NOT_CONVERGED;
        }
        if (hipEventRecord(ev, s) != hipSuccess || hipStreamWaitEvent(user, ev, 0) != hipSuccess) rc = HZ_ERR_HIP;
    } while (0);
    if (rc == HZ_ERR_HIP && hz_last_error()[0] == 0) set_error("fgmres_solve_batched: HIP error");
    (void)hipStreamSynchronize(s);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(s);
    if (rc != HZ_OK) return rc;
    int worst = HZ_OK;
    for (int i = 0; i < nsys; ++i) {
        const int st = info[i].status;
        if (st < 0 && (worst >= 0 || st < worst)) worst = st;
        else if (st == HZ_NOT_CONVERGED && worst == HZ_OK) worst = HZ_NOT_CONVERGED;
    }
    return worst;
}

static int check_batch(int nsys, const hz_problem* const* probs, const no_net* net, const hz_opts* o) {
    HZ_CHECK_ARG(nsys >= 1 && probs && o, "fgmres_solve_batched: bad arguments");
    HZ_CHECK_ARG(o->m >= 1 && o->m <= 4096 && o->maxit >= 1 && o->tol > 0, "fgmres_solve_batched: bad options");
    HZ_CHECK_ARG(o->krylov == HZ_C64 || o->krylov == HZ_C128, "fgmres_solve_batched: bad krylov precision");
    HZ_CHECK_ARG(!net || o->net_prec == NO_BF16 || o->net_prec == NO_FP32 || o->net_prec == NO_FP64,
                 "fgmres_solve_batched: bad net_prec");
    HZ_CHECK_ARG(o->ortho == 0, "fgmres_solve_batched: only ortho = 0 (CGS with one reorthogonalisation)");
    HZ_CHECK_ARG(!net || net->a.kind == NO_ARCH_UNET3, "fgmres_solve_batched: the UNET3 network only");
    for (int s = 0; s < nsys; ++s) HZ_CHECK_ARG(probs[s], "fgmres_solve_batched: NULL problem");
    for (int s = 0; s < nsys; ++s)
        HZ_CHECK_ARG(!is_spectral(probs[s]), "fgmres_solve_batched: finite-difference problems only");
    return HZ_OK;
}

}  // namespace hz

using namespace hz;

extern "C" size_t fgmres_batched_workspace_size(int nsys, const hz_problem* const* probs, const no_net* net,
                                                const hz_opts* o) {
    clear_error();
    if (check_batch(nsys, probs, net, o) != HZ_OK) return 0;
    switch (net ? o->net_prec : NO_FP32) {
        case NO_BF16: return batch_layout<PolBF16>(nsys, probs, net, o, nullptr, 0).total;
        case NO_FP32: return batch_layout<PolF32>(nsys, probs, net, o, nullptr, 0).total;
        default: return batch_layout<PolF64>(nsys, probs, net, o, nullptr, 0).total;
    }
}

extern "C" int fgmres_solve_batched(int nsys, const hz_problem* const* probs, const no_net* net, const hz_opts* o,
                                    const void* const* b, void* const* x, void* ws, size_t ws_bytes, hz_info* info,
                                    void* stream) {
    clear_error();
    const auto t_call = std::chrono::steady_clock::now();
    HZ_TRY(check_batch(nsys, probs, net, o));
    HZ_CHECK_ARG(b && x && ws && info, "fgmres_solve_batched: NULL argument");
    for (int s = 0; s < nsys; ++s) HZ_CHECK_ARG(b[s] && x[s], "fgmres_solve_batched: NULL vector");
    for (int s = 0; s < nsys; ++s) std::memset(info[s].phase_ms, 0, sizeof info[s].phase_ms);
    hipStream_t st = (hipStream_t)stream;
    const bool c128 = o->krylov == HZ_C128;
    int rc;
    switch (net ? o->net_prec : NO_FP32) {
        case NO_BF16:
            rc = c128 ? solve_batched<PolBF16, double2>(nsys, probs, net, o, b, x, ws, ws_bytes, info, st)
                      : solve_batched<PolBF16, float2>(nsys, probs, net, o, b, x, ws, ws_bytes, info, st);
            break;
        case NO_FP32:
            rc = c128 ? solve_batched<PolF32, double2>(nsys, probs, net, o, b, x, ws, ws_bytes, info, st)
                      : solve_batched<PolF32, float2>(nsys, probs, net, o, b, x, ws, ws_bytes, info, st);
            break;
        default:
            rc = c128 ? solve_batched<PolF64, double2>(nsys, probs, net, o, b, x, ws, ws_bytes, info, st)
                      : solve_batched<PolF64, float2>(nsys, probs, net, o, b, x, ws, ws_bytes, info, st);
    }
    const double total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_call).count();
    for (int s = 0; s < nsys; ++s) info[s].phase_ms[HZ_PHASE_TOTAL] = total;
    return rc;
}
